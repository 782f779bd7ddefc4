// fl_stencil.h -- device functions of the Wilson hopping stencil (spin
// projection in the chiral basis, link multiplication, one site of H).
// See fl_dslash.hip for the derivation of the projection formulas.
#pragma once
#include "fl_common.h"

template <int MU, int S, typename R>
__device__ __forceinline__ void project(const cx<R> p[12], cx<R> h[6])
{
    const R s = (R)S;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cx<R> u0 = p[a], u1 = p[3 + a], l0 = p[6 + a], l1 = p[9 + a];
        if (MU == 0) {
            h[a] = u0 - s * ti(l1);
            h[3 + a] = u1 - s * ti(l0);
        } else if (MU == 1) {
            h[a] = u0 - s * l1;
            h[3 + a] = u1 + s * l0;
        } else if (MU == 2) {
            h[a] = u0 - s * ti(l0);
            h[3 + a] = u1 + s * ti(l1);
        } else {
            h[a] = u0 + s * l0;
            h[3 + a] = u1 + s * l1;
        }
    }
}

template <int MU, int S, typename R>
__device__ __forceinline__ void accumulate(cx<R> acc[12], const cx<R> w[6])
{
    const R s = (R)S;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cx<R> w0 = w[a], w1 = w[3 + a];
        acc[a] = acc[a] + w0;
        acc[3 + a] = acc[3 + a] + w1;
        if (MU == 0) {
            acc[6 + a] = acc[6 + a] + s * ti(w1);
            acc[9 + a] = acc[9 + a] + s * ti(w0);
        } else if (MU == 1) {
            acc[6 + a] = acc[6 + a] + s * w1;
            acc[9 + a] = acc[9 + a] - s * w0;
        } else if (MU == 2) {
            acc[6 + a] = acc[6 + a] + s * ti(w0);
            acc[9 + a] = acc[9 + a] - s * ti(w1);
        } else {
            acc[6 + a] = acc[6 + a] + s * w0;
            acc[9 + a] = acc[9 + a] + s * w1;
        }
    }
}

// acc += c * v as two FMAs
template <typename R>
__device__ __forceinline__ cx<R> caxpy(cx<R> acc, R c, cx<R> v)
{
    return cx<R>{fma(c, v.re, acc.re), fma(c, v.im, acc.im)};
}

// acc += c * (full 4-spinor of the projected product w), the hop's scalar
// factor c (boundary sign, storage scales) folded into the FMAs
template <int MU, int S, typename R>
__device__ __forceinline__ void accumulate_scaled(cx<R> acc[12], const cx<R> w[6], R c)
{
    const R cs = (R)S * c;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cx<R> w0 = w[a], w1 = w[3 + a];
        acc[a] = caxpy(acc[a], c, w0);
        acc[3 + a] = caxpy(acc[3 + a], c, w1);
        if (MU == 0) {
            acc[6 + a] = caxpy(acc[6 + a], cs, ti(w1));
            acc[9 + a] = caxpy(acc[9 + a], cs, ti(w0));
        } else if (MU == 1) {
            acc[6 + a] = caxpy(acc[6 + a], cs, w1);
            acc[9 + a] = caxpy(acc[9 + a], -cs, w0);
        } else if (MU == 2) {
            acc[6 + a] = caxpy(acc[6 + a], cs, ti(w0));
            acc[9 + a] = caxpy(acc[9 + a], -cs, ti(w1));
        } else {
            acc[6 + a] = caxpy(acc[6 + a], cs, w0);
            acc[9 + a] = caxpy(acc[9 + a], cs, w1);
        }
    }
}

// w = U h (two spin components)
template <typename R>
__device__ __forceinline__ void link_mul(const cx<R> U[3][3], const cx<R> h[6], cx<R> w[6])
{
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cx<R> acc = U[a][0] * h[3 * sp];
            acc = cmad(acc, U[a][1], h[3 * sp + 1]);
            acc = cmad(acc, U[a][2], h[3 * sp + 2]);
            w[3 * sp + a] = acc;
        }
}

// w = U^+ h
template <typename R>
__device__ __forceinline__ void link_adj_mul(const cx<R> U[3][3], const cx<R> h[6], cx<R> w[6])
{
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cx<R> acc = cjmul(U[0][a], h[3 * sp]);
            acc = cjmad(acc, U[1][a], h[3 * sp + 1]);
            acc = cjmad(acc, U[2][a], h[3 * sp + 2]);
            w[3 * sp + a] = acc;
        }
}

// Where the stencil reads its input spinor field and links from: plain
// pointers (FP64 fields, any lane layout) or per-wave buffer views (scalar
// resources) of a field stored in format S.  spinor() returns the site's
// values up to a common factor, which it returns.
template <typename R, class LK>
struct PtrSrc {
    static constexpr R LINK_UNIT = LK::UNIT;
    const typename SpinorFmt<R>::V *in;
    const typename LK::V *gauge;
    int Vh;
    template <int MU>
    __device__ __forceinline__ R spinor(int i, cx<R> s[12]) const
    {
        SpinorFmt<R>::load(in, Vh, i, s);
        return (R)1;
    }
    __device__ __forceinline__ void link(int mu, int par, int i, cx<R> U[3][3]) const
    {
        link_load<LK>(gauge + (size_t)(mu * 2 + par) * LK::NC * Vh, Vh, i, U);
    }
};

template <typename S, class LK>
struct BufSrc {
    typedef typename SpinorFmt<S>::R R;
    static constexpr R LINK_UNIT = LK::UNIT;
    Buf in, gauge;
    int Vh;
    template <int MU>
    __device__ __forceinline__ R spinor(int i, cx<R> s[12]) const
    {
        return SpinorFmt<S>::load_raw(in, Vh, i, s);
    }
    __device__ __forceinline__ void link(int mu, int par, int i, cx<R> U[3][3]) const
    {
        link_load<LK>(gauge, Vh, (mu * 2 + par) * LK::NC * Vh * LK::ESZ, i, U);
    }
};

template <int MU, bool DAG, typename R, class SRC>
__device__ __forceinline__ void hop_dir(int p, int i, int nf, int nb, R sf, R sb, const SRC &src, cx<R> acc[12])
{
    constexpr int SF = DAG ? 1 : -1;
    constexpr int SB = DAG ? -1 : 1;
    cx<R> psi[12], h[6], w[6], U[3][3];
    // forward hop: U_mu(x) psi(x + mu), link stored with the output parity
    const R cf = src.template spinor<MU>(nf, psi);
    project<MU, SF>(psi, h);
    src.link(MU, p, i, U);
    link_mul(U, h, w);
    accumulate_scaled<MU, SF>(acc, w, sf * cf * SRC::LINK_UNIT);
    // backward hop: U_mu(x - mu)^+ psi(x - mu), link stored at the neighbour
    const R cb = src.template spinor<MU>(nb, psi);
    project<MU, SB>(psi, h);
    src.link(MU, 1 - p, nb, U);
    link_adj_mul(U, h, w);
    accumulate_scaled<MU, SB>(acc, w, sb * cb * SRC::LINK_UNIT);
}

template <bool DAG, typename R, class SRC>
__device__ __forceinline__ void hop_site(const LatGeom &g, int p, int i, const Coord &c, const SRC &src,
                                         cx<R> acc[12])
{
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = cx<R>{(R)0, (R)0};
    const int Lh0 = g.Lh0, xh = c.x >> 1;
    {   // x
        int xf = (c.x + 1 == g.L[0]) ? 0 : c.x + 1;
        int xb = (c.x == 0) ? g.L[0] - 1 : c.x - 1;
        hop_dir<0, DAG, R>(p, i, (xf >> 1) + Lh0 * c.rest, (xb >> 1) + Lh0 * c.rest, (R)1, (R)1, src, acc);
    }
    const int Ly = g.L[1], Lz = g.L[2], Lt = g.L[3];
    {   // y
        int yf = (c.y + 1 == Ly) ? 0 : c.y + 1;
        int yb = (c.y == 0) ? Ly - 1 : c.y - 1;
        int zt = Ly * (c.z + Lz * c.t);
        hop_dir<1, DAG, R>(p, i, xh + Lh0 * (yf + zt), xh + Lh0 * (yb + zt), (R)1, (R)1, src, acc);
    }
    {   // z
        int zf = (c.z + 1 == Lz) ? 0 : c.z + 1;
        int zb = (c.z == 0) ? Lz - 1 : c.z - 1;
        int base = xh + Lh0 * c.y;
        int s = Lh0 * Ly;
        hop_dir<2, DAG, R>(p, i, base + s * (zf + Lz * c.t), base + s * (zb + Lz * c.t), (R)1, (R)1, src, acc);
    }
    {   // t, with the boundary factor on the hops that wrap
        int tf = c.t + 1, tb = c.t - 1;
        R sf = (R)1, sb = (R)1;
        if (tf == Lt) { tf = 0; sf = (R)g.bc_t; }
        if (tb < 0) { tb = Lt - 1; sb = (R)g.bc_t; }
        int base = xh + Lh0 * (c.y + Ly * c.z);
        int s = Lh0 * Ly * Lz;
        hop_dir<3, DAG, R>(p, i, base + s * tf, base + s * tb, sf, sb, src, acc);
    }
}

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

// ---------------------------------------------------------------------------
// Packed 16-bit integer form of one hop, for fields stored as 16-bit fixed
// point: the spin projection runs as packed int16 adds on the stored
// integers and the colour product as exact int16 dot products summed in
// int32 (v_dot2_i32_i16), converted to FP32 once per product component.
// The fields store at most 16383 in magnitude, so no projected component
// leaves the int16 range (|u| + |l| <= 32766), and the links are staged at
// half scale, round(16383.5 u), which keeps every three-term sum of a
// product row below sqrt(6) * 32766 * 16384 < 2^31
// (Cauchy-Schwarz over the 6 reals of a unit row of U or U^+ and the 6
// reals of a projected colour vector).  Each staged entry carries the two
// int16 pairs that give the real and the imaginary part of its product with
// a colour component directly, so a lane forms no conjugate or swapped copy
// of anything.  A complex number is one 32-bit word, real part in the low
// half.
// ---------------------------------------------------------------------------
// the projection of project<MU, S> on the stored integers; i z = swp(z) * (-1, 1)
template <int MU, int S>
__device__ __forceinline__ void project_i16(const s2 p[12], s2 h[6])
{
    constexpr short s = (short)S, n = (short)-S;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const s2 u0 = p[a], u1 = p[3 + a], l0 = p[6 + a], l1 = p[9 + a];
        if (MU == 0) {
            h[a] = mad_swp(l1, (s2){s, n}, u0);      // u0 - s i l1
            h[3 + a] = mad_swp(l0, (s2){s, n}, u1);  // u1 - s i l0
        } else if (MU == 1) {
            h[a] = u0 + l1 * (s2){n, n};
            h[3 + a] = u1 + l0 * (s2){s, s};
        } else if (MU == 2) {
            h[a] = mad_swp(l0, (s2){s, n}, u0);      // u0 - s i l0
            h[3 + a] = mad_swp(l1, (s2){n, s}, u1);  // u1 + s i l1
        } else {
            h[a] = u0 + l0 * (s2){s, s};
            h[3 + a] = u1 + l1 * (s2){s, s};
        }
    }
}

// w = M h for the staged link forms of M (U or U^+): words 2e, 2e + 1 of
// entry e = 3a + b hold the pairs whose dot products with h_b give the real
// and imaginary parts of M_ab h_b
__device__ __forceinline__ void link_mul_i16(const unsigned L[18], const s2 h[6], cx<float> w[6])
{
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            int re = sdot2_first(as_s2(L[6 * a]), h[3 * sp]);
            int im = sdot2_first(as_s2(L[6 * a + 1]), h[3 * sp]);
#pragma unroll
            for (int b = 1; b < 3; ++b) {
                re = __builtin_amdgcn_sdot2(as_s2(L[6 * a + 2 * b]), h[3 * sp + b], re, false);
                im = __builtin_amdgcn_sdot2(as_s2(L[6 * a + 2 * b + 1]), h[3 * sp + b], im, false);
            }
            w[3 * sp + a] = cx<float>{(float)re, (float)im};
        }
}

// Where the stencil reads its input spinor field and links from: plain
// pointers (FP64 fields, any lane layout) or per-wave buffer views (scalar
// resources) of a field stored in format S.  spinor() returns the site's
// values up to a common factor, which it returns.
template <typename R, class LK>
struct PtrSrc {
    static constexpr bool PACKED_I16 = false;
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
    static constexpr bool PACKED_I16 = false;
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
    if constexpr (SRC::PACKED_I16) {
        // spinor_i16 returns the stored integers and the factor that turns
        // them (times the staged link integers) into values
        s2 psi[12], h[6];
        unsigned L[18];
        cx<float> w[6];
        const float cf = src.template spinor_i16<MU>(nf, psi);
        project_i16<MU, SF>(psi, h);
        src.link_i16(2 * MU, L);
        link_mul_i16(L, h, w);
        accumulate_scaled<MU, SF>(acc, w, sf * cf);
        const float cb = src.template spinor_i16<MU>(nb, psi);
        project_i16<MU, SB>(psi, h);
        src.link_i16(2 * MU + 1, L);
        link_mul_i16(L, h, w);
        accumulate_scaled<MU, SB>(acc, w, sb * cb);
    } else {
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

// ---------------------------------------------------------------------------
// Packed integer hop of one site with its neighbour loads issued PF
// directions ahead of their use (direction slot D = 2 mu + 0 forward / 1
// backward, in the order of hop_site).  Each step projects the spinor of
// its slot, then refills that register slot with the spinor of slot D + PF
// before the colour product, so PF loads are in flight while a wave computes.
// The source must read every neighbour from memory (no LDS windows).
// Measured at 16^3x32 with 384 right-hand sides: PF = 2 (100 VGPRs, 4 waves
// per SIMD) 848-854 us per launch, PF = 3 or 4 and the compiler's own
// schedule (about one direction ahead, 64 VGPRs, 8 waves) 870-913 us;
// capping PF = 2 at 5 or 6 waves per SIMD (fewer registers, one colour row
// of the link at a time) 910-936 us.
// ---------------------------------------------------------------------------
template <int D, bool DAG, int PF, class SRC>
__device__ __forceinline__ void pk_step(const SRC &src, const int nb[8], const float bf[8], s2 (&buf)[PF][12],
                                        float (&cf)[PF], cx<float> acc[12])
{
    constexpr int MU = D >> 1;
    constexpr int SGN = (D & 1) ? (DAG ? -1 : 1) : (DAG ? 1 : -1);
    s2 h[6];
    project_i16<MU, SGN>(buf[D % PF], h);
    const float f = bf[D] * cf[D % PF];
    if constexpr (D + PF < 8) {
        cf[(D + PF) % PF] = src.template spinor_i16<3>(nb[D + PF], buf[(D + PF) % PF]);
        __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the work that hides them
    }
    unsigned L[18];
    src.link_i16(D, L);
    cx<float> w[6];
    link_mul_i16(L, h, w);
    accumulate_scaled<MU, SGN>(acc, w, f);
}

template <bool DAG, int PF, class SRC>
__device__ __forceinline__ void hop_site_pk(const LatGeom &g, const Coord &c, const SRC &src, cx<float> acc[12])
{
    int nb[8];
    float bf[8];
    const int Lh0 = g.Lh0, Ly = g.L[1], Lz = g.L[2], Lt = g.L[3], xh = c.x >> 1;
    {
        const int xf = (c.x + 1 == g.L[0]) ? 0 : c.x + 1, xb = (c.x == 0) ? g.L[0] - 1 : c.x - 1;
        nb[0] = (xf >> 1) + Lh0 * c.rest;
        nb[1] = (xb >> 1) + Lh0 * c.rest;
    }
    {
        const int yf = (c.y + 1 == Ly) ? 0 : c.y + 1, yb = (c.y == 0) ? Ly - 1 : c.y - 1;
        const int zt = Ly * (c.z + Lz * c.t);
        nb[2] = xh + Lh0 * (yf + zt);
        nb[3] = xh + Lh0 * (yb + zt);
    }
    {
        const int zf = (c.z + 1 == Lz) ? 0 : c.z + 1, zb = (c.z == 0) ? Lz - 1 : c.z - 1;
        const int base = xh + Lh0 * c.y, s = Lh0 * Ly;
        nb[4] = base + s * (zf + Lz * c.t);
        nb[5] = base + s * (zb + Lz * c.t);
    }
    {
        int tf = c.t + 1, tb = c.t - 1;
        bf[6] = 1.0f;
        bf[7] = 1.0f;
        if (tf == Lt) { tf = 0; bf[6] = (float)g.bc_t; }
        if (tb < 0) { tb = Lt - 1; bf[7] = (float)g.bc_t; }
        const int base = xh + Lh0 * (c.y + Ly * c.z), s = Lh0 * Ly * Lz;
        nb[6] = base + s * tf;
        nb[7] = base + s * tb;
    }
#pragma unroll
    for (int d = 0; d < 6; ++d) bf[d] = 1.0f;
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = cx<float>{0.0f, 0.0f};
    s2 buf[PF][12];
    float cf[PF];
#pragma unroll
    for (int d = 0; d < PF; ++d) cf[d] = src.template spinor_i16<3>(nb[d], buf[d]);
    __builtin_amdgcn_sched_barrier(0);
    pk_step<0, DAG, PF>(src, nb, bf, buf, cf, acc);
    pk_step<1, DAG, PF>(src, nb, bf, buf, cf, acc);
    pk_step<2, DAG, PF>(src, nb, bf, buf, cf, acc);
    pk_step<3, DAG, PF>(src, nb, bf, buf, cf, acc);
    pk_step<4, DAG, PF>(src, nb, bf, buf, cf, acc);
    pk_step<5, DAG, PF>(src, nb, bf, buf, cf, acc);
    pk_step<6, DAG, PF>(src, nb, bf, buf, cf, acc);
    pk_step<7, DAG, PF>(src, nb, bf, buf, cf, acc);
}

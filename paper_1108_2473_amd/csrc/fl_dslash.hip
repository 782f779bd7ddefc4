// fl_dslash.hip -- the Wilson hopping stencil on one checkerboard parity.
//
//   (H psi)(x) = sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu) ]
//
// with the time-boundary hop multiplied by bc_t; D = 1 - kappa H and the
// Schur operator of the even sites is Dhat = 1 - kappa^2 H_eo H_oe.  The
// dagger form swaps the two projectors (H^+ = g5 H g5).
//
// Each projector (1 -/+ g_mu) has rank 2: in the chiral basis the product
// with a 4-spinor psi = (u, l) is (h, M h) with a 2-spinor h and a fixed 2x2
// matrix M, so only 2 colour vectors are multiplied by the link (spin
// projection) and the lower half is rebuilt from the product.  With
// g_k = [[0, -i s_k], [i s_k, 0]] and g_4 = [[0, 1], [1, 0]]:
//   (1 + s g_k) psi = (u - s i s_k l,  s i s_k h)
//   (1 + s g_4) psi = (u + s l,        s h)
// and i s_1 (a, b) = (i b, i a), i s_2 (a, b) = (b, -a), i s_3 (a, b) = (i a, -i b).
//
// One lane computes one output site of one right-hand side; a wavefront is
// 64 consecutive sites of one right-hand side and a workgroup RT such waves
// (RT right-hand sides of the same 64 sites, which share the link loads in
// L1).  The epilogue fuses the vector update and the reductions that the
// Krylov iteration needs right after the operator.
#include <type_traits>

#include "fl_host.h"
#include "fl_stencil.h"

namespace {

// An own-site operand of the epilogue (x, y): read once by this kernel, so
// 16-bit and FP32 fields are loaded non-temporally and leave L2 to the
// neighbour spinors that other workgroups still read (the dagger hop that
// updates z, which reads two such fields, at 16^3x32 with 384 right-hand
// sides: 1235 instead of 1276 us per launch with 16-bit fields, 2223
// instead of 2358 us with FP32 fields)
template <typename S, typename R>
__device__ __forceinline__ void load_once(const Buf &b, int Vh, int i, cx<R> s[12])
{
    if constexpr (std::is_same<S, H16>::value) {
        v4f v[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = __builtin_amdgcn_raw_buffer_load_b128(b.r, i * 16, c * Vh * 16, LD_STREAM);
        const float sc =
            __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(b.r, i * 4, 3 * Vh * 16, LD_STREAM));
        SpinorFmt<H16>::unpack(v, s);
#pragma unroll
        for (int k = 0; k < 12; ++k) s[k] = cx<float>{s[k].re * sc, s[k].im * sc};
    } else if constexpr (std::is_same<S, float>::value) {
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const v4f v = __builtin_amdgcn_raw_buffer_load_b128(b.r, i * 16, c * Vh * 16, LD_STREAM);
            s[2 * c] = cx<float>{v.x, v.y};
            s[2 * c + 1] = cx<float>{v.z, v.w};
        }
    } else {
        SpinorFmt<S>::load(b, Vh, i, s);
    }
}

// S: storage format of the fields (SpinorFmt<S>), arithmetic in SpinorFmt<S>::R.
// The reductions use the values as stored (after any rounding of the format).
template <typename S, int EPI, typename R>
__device__ __forceinline__ void epilogue(const DslashArgs &a, const TileInfo &T, const LatGeom &g, int rhs,
                                         const cx<R> acc[12], R &q0, R &q1, R &q2)
{
    typedef SpinorFmt<S> F;
    const R cb = (R)a.cb[T.lat];
    if constexpr (std::is_same<S, H16>::value && !(EPI & (EPI_XPAY | EPI_DOTX_NORM | EPI_DOTY))) {
        // 16-bit result cb * acc: cb enters the site scale, not the values
        unsigned w[12];
        const float sc =
            F::template store_words<ST_STREAM>(spinor_buf<S>(a.out[T.lat], g.Vh, rhs), g.Vh, T.site, acc, w, cb);
        if (EPI & EPI_NORM) q2 += h16_norm2(w, sc);
        return;
    }
    cx<R> out[12], xv[12];
    if (EPI & EPI_XPAY) {
        load_once<S, R>(spinor_buf<S>(a.x[T.lat], g.Vh, rhs), g.Vh, T.site, xv);
        const R ca = (R)a.ca[T.lat];
        if (ca == (R)1) {
#pragma unroll
            for (int k = 0; k < 12; ++k) out[k] = cx<R>{fma(cb, acc[k].re, xv[k].re), fma(cb, acc[k].im, xv[k].im)};
        } else {
#pragma unroll
            for (int k = 0; k < 12; ++k) out[k] = ca * xv[k] + cb * acc[k];
        }
    } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) out[k] = cb * acc[k];
    }
    if constexpr ((EPI & EPI_CGZ) != 0) {
        // out = y - alpha (x + cb acc), y the field this launch overwrites (own site only)
        cx<R> yv[12];
        load_once<S, R>(spinor_buf<S>(a.y[T.lat], g.Vh, rhs), g.Vh, T.site, yv);
        const R al = (R)a.st[T.sys].alpha[0];
#pragma unroll
        for (int k = 0; k < 12; ++k) out[k] = cx<R>{fma(-al, out[k].re, yv[k].re), fma(-al, out[k].im, yv[k].im)};
    }
    if constexpr ((EPI & (EPI_SUBY16 | EPI_SUBY32)) != 0 && std::is_same<S, double>::value) {
        // y in the iteration's format: its values (16-bit: the decoded ones)
        // widen to FP64 exactly
        typedef typename std::conditional<(EPI & EPI_SUBY16) != 0, H16, float>::type Y;
        cx<float> yl[12];
        SpinorFmt<Y>::load(spinor_buf<Y>(a.y[T.lat], g.Vh, rhs), g.Vh, T.site, yl);
#pragma unroll
        for (int k = 0; k < 12; ++k) out[k] = out[k] - cx<double>{(double)yl[k].re, (double)yl[k].im};
        if constexpr ((EPI & EPI_ACCX) != 0) {
            // the solution moves by the same values at this site: w += y,
            // then y = 0 (the accumulation of a reliable update)
            cx<double> h[12];
            SpinorFmt<double>::load(spinor_buf<double>(a.w[T.lat], g.Vh, rhs), g.Vh, T.site, h);
#pragma unroll
            for (int k = 0; k < 12; ++k) h[k] = h[k] + cx<double>{(double)yl[k].re, (double)yl[k].im};
            store_result<double>(spinor_buf<double>(a.w[T.lat], g.Vh, rhs), g.Vh, T.site, h);
            cx<float> z[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) z[k] = cx<float>{0.0f, 0.0f};
            store_result<Y>(spinor_buf<Y>(a.y[T.lat], g.Vh, rhs), g.Vh, T.site, z);
        }
    }
    if constexpr (std::is_same<S, H16>::value && !(EPI & (EPI_DOTX_NORM | EPI_DOTY))) {
        // 16-bit result without dot products: stored as words, its norm
        // summed from the stored integers (no decode back to FP32)
        unsigned w[12];
        const float sc = F::template store_words<ST_STREAM>(spinor_buf<S>(a.out[T.lat], g.Vh, rhs), g.Vh, T.site,
                                                           out, w);
        if (EPI & EPI_NORM) q2 += h16_norm2(w, sc);
        return;
    }
    store_result<S>(spinor_buf<S>(a.out[T.lat], g.Vh, rhs), g.Vh, T.site, out);
    if (EPI & EPI_DOTX_NORM) {
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            cx<R> d = cjmul(out[k], xv[k]);
            q0 += d.re;
            q1 += d.im;
            q2 += out[k].re * out[k].re + out[k].im * out[k].im;
        }
    }
    if (EPI & EPI_DOTY) {
        cx<R> yv[12];
        load_once<S, R>(spinor_buf<S>(a.y[T.lat], g.Vh, rhs), g.Vh, T.site, yv);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            cx<R> d = cjmul(yv[k], out[k]);
            q0 += d.re;
            q1 += d.im;
        }
    }
    if (EPI & EPI_NORM) {
#pragma unroll
        for (int k = 0; k < 12; ++k) q2 += out[k].re * out[k].re + out[k].im * out[k].im;
    }
}

template <int EPI, typename R>
__device__ __forceinline__ void reduce_partials(const DslashArgs &a, const TileInfo &T, R q0, R q1, R q2)
{
    if (EPI & (EPI_DOTY | EPI_DOTX_NORM | EPI_NORM)) {
        double s0 = wave_sum((double)q0), s1 = wave_sum((double)q1), s2 = wave_sum((double)q2);
        constexpr int which = ((EPI & (EPI_DOTY | EPI_DOTX_NORM)) ? 3 : 0) | ((EPI & (EPI_DOTX_NORM | EPI_NORM)) ? 4 : 0);
        write_partials(a.partial, a.slot0, a.nsys, T.sys, a.B.nsb_max, T.sb, s0, s1, s2, which);
    }
}

template <typename S, class LK, bool DAG, int EPI>
__global__ __launch_bounds__(sizeof(typename SpinorFmt<S>::R) == 8 ? 512 : 1024) void k_dslash(DslashArgs a)
{
    typedef typename SpinorFmt<S>::R R;
    TileInfo T = tile_info(a.B);
    if (!T.valid_rhs) return;
    if (a.mask && !a.mask[T.sys]) return;  // wave-uniform: one wave = one right-hand side
    const LatGeom &g = a.B.lat[T.lat];
    const int rhs = __builtin_amdgcn_readfirstlane(T.rhs);
    R q0 = 0, q1 = 0, q2 = 0;
    if (T.valid_site) {
        Coord c = cb_coords(g, a.par, T.site);
        BufSrc<S, LK> src;
        src.in = spinor_buf<S>(a.in[T.lat], g.Vh, rhs);
        src.gauge = make_buf(a.gauge[T.lat], (unsigned)(8u * LK::NC * LK::ESZ * (unsigned)g.Vh));
        src.Vh = g.Vh;
        cx<R> acc[12];
        hop_site<DAG, R>(g, a.par, T.site, c, src, acc);
        epilogue<S, EPI>(a, T, g, rhs, acc, q0, q1, q2);
    }
    reduce_partials<EPI>(a, T, q0, q1, q2);
}

// a 16-bit or FP32 field read into FP64 arithmetic: its values (16-bit: the
// stored integers times the site scale, rounded to FP32 exactly as every
// other reader of the field decodes them) widen to FP64 without rounding
template <typename Y>
struct WideSrc {
    static constexpr bool PACKED_I16 = false;
    static constexpr double LINK_UNIT = LinkF64R18::UNIT;
    Buf in, gauge;
    int Vh;
    template <int MU>
    __device__ __forceinline__ double spinor(int i, cx<double> s[12]) const
    {
        cx<float> f[12];
        SpinorFmt<Y>::load(in, Vh, i, f);
#pragma unroll
        for (int k = 0; k < 12; ++k) s[k] = cx<double>{(double)f[k].re, (double)f[k].im};
        return 1.0;
    }
    __device__ __forceinline__ void link(int mu, int par, int i, cx<double> U[3][3]) const
    {
        link_load<LinkF64R18>(gauge, Vh, (mu * 2 + par) * LinkF64R18::NC * Vh * LinkF64R18::ESZ, i, U);
    }
};

template <typename Y, bool DAG>
__global__ __launch_bounds__(512) void k_dslash_wide(DslashArgs a)
{
    typedef LinkF64R18 LK;
    TileInfo T = tile_info(a.B);
    if (!T.valid_rhs) return;
    if (a.mask && !a.mask[T.sys]) return;  // wave-uniform
    const LatGeom &g = a.B.lat[T.lat];
    const int rhs = __builtin_amdgcn_readfirstlane(T.rhs);
    double q0 = 0, q1 = 0, q2 = 0;
    if (T.valid_site) {
        Coord c = cb_coords(g, a.par, T.site);
        WideSrc<Y> src;
        src.in = spinor_buf<Y>(a.in[T.lat], g.Vh, rhs);
        src.gauge = make_buf(a.gauge[T.lat], (unsigned)(8u * LK::NC * LK::ESZ * (unsigned)g.Vh));
        src.Vh = g.Vh;
        cx<double> acc[12];
        hop_site<DAG, double>(g, a.par, T.site, c, src, acc);
        epilogue<double, EPI_PLAIN>(a, T, g, rhs, acc, q0, q1, q2);
    }
}

template <typename S, class LK, bool SLINK, bool WIN = true>
struct LdsSrc {
    typedef typename SpinorFmt<S>::R R;
    static constexpr bool PACKED_I16 = false;
    static constexpr R LINK_UNIT = LK::UNIT;
    Buf in, gauge;
    int Vh, wlo, wsz, wsmax, p, lane;
    const unsigned char *win;
    const typename LK::SV *lk;
    template <int MU>
    __device__ __forceinline__ R spinor(int i, cx<R> s[12]) const
    {
        if (WIN && MU < 2)
            return SpinorFmt<S>::lds_load_raw(win, wsmax, i - wlo, s);
        else
            return SpinorFmt<S>::load_raw(in, Vh, i, s);
    }
    __device__ __forceinline__ void link(int mu, int par, int i, cx<R> U[3][3]) const
    {
        if (SLINK) {
            const int dslot = 2 * mu + (par == p ? 0 : 1);
            typename LK::SV w[LK::SNC];
#pragma unroll
            for (int c = 0; c < LK::SNC; ++c) w[c] = lk[(dslot * LK::SNC + c) * FL_WAVE + lane];
            LK::unpack_staged(w, U);
        } else {
            link_load<LK>(gauge, Vh, (mu * 2 + par) * LK::NC * Vh * LK::ESZ, i, U);
        }
    }
};

// Source of the packed integer hop (16-bit fields, lds modes 3 and 4): x/y
// neighbours from the wave's LDS window (mode 3) or from memory like the
// z/t neighbours (mode 4), links from the workgroup's half-scale staging.
// The factor returned with a site's integers is its scale times the staged
// link unit.
template <bool WIN>
struct LdsSrcQ16 {
    static constexpr bool PACKED_I16 = true;
    Buf in;
    int Vh, wlo, wsmax, lane;
    const unsigned char *win;
    const unsigned *lk;
    template <int MU>
    __device__ __forceinline__ float spinor_i16(int i, s2 p[12]) const
    {
        constexpr float k = LinkQ16R12::HALF_UNIT;
        if (WIN && MU < 2)
            return k * SpinorFmt<H16>::lds_load_i16(win, wsmax, i - wlo, p);
        else
            return k * SpinorFmt<H16>::load_i16(in, Vh, i, p);
    }
    __device__ __forceinline__ void link_i16(int dslot, unsigned L[18]) const
    {
#pragma unroll
        for (int c = 0; c < LinkQ16R12::PK_SNC; ++c) L[c] = lk[(dslot * LinkQ16R12::PK_SNC + c) * FL_WAVE + lane];
    }
};

// checkerboard index of the backward neighbour x - mu of site (p, i)
__device__ __forceinline__ int back_neighbour(const LatGeom &g, const Coord &c, int mu)
{
    const int Lh0 = g.Lh0, Ly = g.L[1], Lz = g.L[2], Lt = g.L[3], xh = c.x >> 1;
    if (mu == 0) {
        int xb = (c.x == 0) ? g.L[0] - 1 : c.x - 1;
        return (xb >> 1) + Lh0 * c.rest;
    } else if (mu == 1) {
        int yb = (c.y == 0) ? Ly - 1 : c.y - 1;
        return xh + Lh0 * (yb + Ly * (c.z + Lz * c.t));
    } else if (mu == 2) {
        int zb = (c.z == 0) ? Lz - 1 : c.z - 1;
        return xh + Lh0 * (c.y + Ly * (zb + Lz * c.t));
    }
    int tb = (c.t == 0) ? Lt - 1 : c.t - 1;
    return xh + Lh0 * (c.y + Ly * (c.z + Lz * tb));
}

// SLINK: links staged in LDS; PK (16-bit fields only, with SLINK): the
// packed integer hop with half-scale staged links;
// NOWIN: no neighbour windows (x/y neighbours from memory like z/t); with
// SLINK and without PK the LDS holds the staged links only, so that more
// workgroups fit a CU than with the windows
template <typename S, class LK, bool DAG, int EPI, bool SLINK, bool PK = false, bool NOWIN = false>
__global__ __launch_bounds__(sizeof(typename SpinorFmt<S>::R) == 8 ? 512 : 1024) void k_dslash_lds(DslashArgs a)
{
    static_assert(!PK || (SLINK && std::is_same<LK, LinkQ16R12>::value), "packed hop needs staged Q16 links");
    typedef typename SpinorFmt<S>::R R;
    typedef typename LK::V LV;
    typedef typename LK::SV LSV;
    constexpr int SB = SpinorFmt<S>::SITE_BYTES;
    extern __shared__ unsigned char smem[];
    TileInfo T = tile_info(a.B);
    const LatGeom &g = a.B.lat[T.lat];
    const int Vh = g.Vh;
    const int lane = threadIdx.x % FL_WAVE;
    const int wave = threadIdx.x / FL_WAVE;
    const int i0 = T.sb * FL_WAVE;
    const int plane = g.Lh0 * g.L[1];  // sites of one (z, t) plane
    const int wlo = (i0 / plane) * plane;
    const int wsz = min(Vh, (min(i0 + FL_WAVE, Vh) - 1) / plane * plane + plane) - wlo;
    const int wsmax = a.wsmax;
    // wsmax is a multiple of 4, so that every window starts 16-byte aligned
    unsigned char *win = smem + (size_t)wave * SB * wsmax;
    LSV *lk = (LSV *)(NOWIN ? smem : smem + (size_t)a.B.RT * SB * wsmax);
    const bool live = T.valid_rhs && !(a.mask && !a.mask[T.sys]);
    const int rhs = __builtin_amdgcn_readfirstlane(T.valid_rhs ? T.rhs : 0);
    const Buf gbuf = make_buf(a.gauge[T.lat], (unsigned)(8u * LK::NC * LK::ESZ * (unsigned)Vh));
    Buf ibuf = spinor_buf<S>(a.in[T.lat], Vh, rhs);
    if (SLINK) {
        // the 8 links (4 forward at the site, 4 backward at the neighbour) of
        // the block's 64 sites, shared by all its right-hand sides
        for (int k = threadIdx.x; k < 8 * FL_WAVE; k += blockDim.x) {
            // one direction slot per wave (64 consecutive k)
            const int dslot = __builtin_amdgcn_readfirstlane(k / FL_WAVE), s = k % FL_WAVE, mu = dslot >> 1;
            const int site = i0 + s;
            LV v[LK::NC];
            if (site < Vh) {
                int idx = site, par = a.par;
                if (dslot & 1) {
                    Coord c = cb_coords(g, a.par, site);
                    idx = back_neighbour(g, c, mu);
                    par = 1 - a.par;
                }
#pragma unroll
                for (int cc = 0; cc < LK::NC; ++cc)
                    v[cc] = LK::buf_get(gbuf, idx * LK::ESZ, ((mu * 2 + par) * LK::NC + cc) * Vh * LK::ESZ);
            } else {
#pragma unroll
                for (int cc = 0; cc < LK::NC; ++cc) v[cc] = LV{};
            }
            if constexpr (PK) {
                LSV w[LK::PK_SNC];
                if (dslot & 1)
                    LK::template stage_pk<true>(v, w);
                else
                    LK::template stage_pk<false>(v, w);
#pragma unroll
                for (int cc = 0; cc < LK::PK_SNC; ++cc) lk[(dslot * LK::PK_SNC + cc) * FL_WAVE + s] = w[cc];
            } else {
                LSV w[LK::SNC];
                LK::stage(v, w);
#pragma unroll
                for (int cc = 0; cc < LK::SNC; ++cc) lk[(dslot * LK::SNC + cc) * FL_WAVE + s] = w[cc];
            }
        }
    }
    if (live && !NOWIN)
        for (int j = lane; j < wsz; j += FL_WAVE) {
            SpinorFmt<S>::to_lds(ibuf, Vh, wlo + j, win, wsmax, j);
        }
    __syncthreads();
    if (!live) return;
    R q0 = 0, q1 = 0, q2 = 0;
    if (T.valid_site) {
        Coord c = cb_coords(g, a.par, T.site);
        cx<R> acc[12];
        if constexpr (PK) {
            LdsSrcQ16<!NOWIN> src;
            src.in = ibuf;
            src.Vh = Vh;
            src.wlo = wlo;
            src.wsmax = wsmax;
            src.lane = lane;
            src.win = win;
            src.lk = (const unsigned *)lk;
            if constexpr (NOWIN)
                hop_site_pk<DAG, 2>(g, c, src, acc);  // neighbour loads two directions ahead
            else
                hop_site<DAG, R>(g, a.par, T.site, c, src, acc);
        } else {
            LdsSrc<S, LK, SLINK, !NOWIN> src;
            src.in = ibuf;
            src.gauge = gbuf;
            src.Vh = Vh;
            src.wlo = wlo;
            src.wsz = wsz;
            src.wsmax = wsmax;
            src.p = a.par;
            src.lane = lane;
            src.win = win;
            src.lk = lk;
            hop_site<DAG, R>(g, a.par, T.site, c, src, acc);
        }
        epilogue<S, EPI>(a, T, g, rhs, acc, q0, q1, q2);
    }
    reduce_partials<EPI>(a, T, q0, q1, q2);
}

template <typename S, class LK>
size_t dslash_lds_bytes_t(int RT, int wsmax, int lds)
{
    // modes: 1 windows, 2 windows + staged links, 3 (16-bit) windows + packed
    // staged links, 4 staged links only (packed for 16-bit fields)
    constexpr bool Q16 = std::is_same<LK, LinkQ16R12>::value;
    size_t b = lds == 4 ? 0 : (size_t)RT * SpinorFmt<S>::SITE_BYTES * wsmax;
    if (lds == 2 || (lds == 4 && !Q16)) b += (size_t)8 * LK::SNC * FL_WAVE * sizeof(typename LK::SV);
    if constexpr (Q16)
        if (lds >= 3) b += (size_t)8 * LK::PK_SNC * FL_WAVE * sizeof(typename LK::SV);
    return b;
}

constexpr size_t FP32_HOP_LDS_CAP = 70 * 1024;

template <typename S, class LK, bool DAG, int EPI>
void launch_one(const DslashArgs &a, dim3 grid, dim3 block, hipStream_t s)
{
    if (a.lds == 0) {
        hipLaunchKernelGGL((k_dslash<S, LK, DAG, EPI>), grid, block, 0, s, a);
    } else {
        size_t shm = dslash_lds_bytes_t<S, LK>(a.B.RT, a.wsmax, a.lds);
        if constexpr (std::is_same<LK, LinkQ16R12>::value) {
            if (a.lds == 3) {
                hipLaunchKernelGGL((k_dslash_lds<S, LK, DAG, EPI, true, true>), grid, block, shm, s, a);
                return;
            }
            if (a.lds == 4) {
                hipLaunchKernelGGL((k_dslash_lds<S, LK, DAG, EPI, true, true, true>), grid, block, shm, s, a);
                return;
            }
        } else if (a.lds == 4) {
            // FP32 fields: at most two workgroups per CU (the LDS request
            // reserves a third of the CU's 160 KB), so that the neighbour
            // spinors of the tiles in flight stay within each XCD's L2:
            // 1518 instead of 1586 us per H_oe launch at 16^3x32 with 384
            // right-hand sides (three workgroups by registers; one: 1637 us)
            if constexpr (std::is_same<S, float>::value) shm = std::max(shm, (size_t)FP32_HOP_LDS_CAP);
            hipLaunchKernelGGL((k_dslash_lds<S, LK, DAG, EPI, true, false, true>), grid, block, shm, s, a);
            return;
        }
        if (a.lds >= 2)
            hipLaunchKernelGGL((k_dslash_lds<S, LK, DAG, EPI, true>), grid, block, shm, s, a);
        else
            hipLaunchKernelGGL((k_dslash_lds<S, LK, DAG, EPI, false>), grid, block, shm, s, a);
    }
}

template <typename S, class LK, bool DAG>
void dispatch_epi(const DslashArgs &a, int epi, dim3 grid, dim3 block, hipStream_t s)
{
    switch (epi) {
    case EPI_PLAIN: launch_one<S, LK, DAG, EPI_PLAIN>(a, grid, block, s); break;
    case EPI_XPAY: launch_one<S, LK, DAG, EPI_XPAY>(a, grid, block, s); break;
    case EPI_XPAY | EPI_NORM: launch_one<S, LK, DAG, EPI_XPAY | EPI_NORM>(a, grid, block, s); break;
    case EPI_XPAY | EPI_DOTY: launch_one<S, LK, DAG, EPI_XPAY | EPI_DOTY>(a, grid, block, s); break;
    case EPI_XPAY | EPI_DOTX_NORM: launch_one<S, LK, DAG, EPI_XPAY | EPI_DOTX_NORM>(a, grid, block, s); break;
    case EPI_NORM: launch_one<S, LK, DAG, EPI_NORM>(a, grid, block, s); break;
    case EPI_XPAY | EPI_NORM | EPI_CGZ: launch_one<S, LK, DAG, EPI_XPAY | EPI_NORM | EPI_CGZ>(a, grid, block, s); break;
    case EPI_XPAY | EPI_NORM | EPI_SUBY16:
        if constexpr (std::is_same<S, double>::value)
            launch_one<S, LK, DAG, EPI_XPAY | EPI_NORM | EPI_SUBY16>(a, grid, block, s);
        else
            launch_unsupported("hopping epilogue: 16-bit subtraction needs FP64 fields");
        break;
    case EPI_XPAY | EPI_NORM | EPI_SUBY16 | EPI_ACCX:
        if constexpr (std::is_same<S, double>::value)
            launch_one<S, LK, DAG, EPI_XPAY | EPI_NORM | EPI_SUBY16 | EPI_ACCX>(a, grid, block, s);
        else
            launch_unsupported("hopping epilogue: 16-bit subtraction needs FP64 fields");
        break;
    case EPI_XPAY | EPI_NORM | EPI_SUBY32 | EPI_ACCX:
        if constexpr (std::is_same<S, double>::value)
            launch_one<S, LK, DAG, EPI_XPAY | EPI_NORM | EPI_SUBY32 | EPI_ACCX>(a, grid, block, s);
        else
            launch_unsupported("hopping epilogue: FP32 subtraction needs FP64 fields");
        break;
    default: launch_unsupported("hopping epilogue"); break;
    }
}

template <typename S, class LK>
void dispatch_dag(const DslashArgs &a, bool dag, int epi, dim3 grid, dim3 block, hipStream_t s)
{
    if (dag)
        dispatch_epi<S, LK, true>(a, epi, grid, block, s);
    else
        dispatch_epi<S, LK, false>(a, epi, grid, block, s);
}

}  // namespace

size_t dslash_lds_bytes(LinkFormat fmt, int RT, int wsmax, int lds)
{
    if (lds == 0) return 0;
    switch (fmt) {
    case LINK_F64_R18: return dslash_lds_bytes_t<double, LinkF64R18>(RT, wsmax, lds);
    case LINK_F32_R18: return dslash_lds_bytes_t<float, LinkF32R18>(RT, wsmax, lds);
    case LINK_F32_R12: return dslash_lds_bytes_t<float, LinkF32R12>(RT, wsmax, lds);
    case LINK_Q16_R12: return dslash_lds_bytes_t<H16, LinkQ16R12>(RT, wsmax, lds);
    default: return dslash_lds_bytes_t<float, LinkBF16R12>(RT, wsmax, lds);
    }
}

bool dslash_epi_supported(int epi)
{
    return epi == EPI_PLAIN || epi == EPI_XPAY || epi == (EPI_XPAY | EPI_NORM) ||
           epi == (EPI_XPAY | EPI_DOTY) || epi == (EPI_XPAY | EPI_DOTX_NORM) || epi == EPI_NORM ||
           epi == (EPI_XPAY | EPI_NORM | EPI_SUBY16) || epi == (EPI_XPAY | EPI_NORM | EPI_CGZ) ||
           epi == (EPI_XPAY | EPI_NORM | EPI_SUBY16 | EPI_ACCX) || epi == (EPI_XPAY | EPI_NORM | EPI_SUBY32 | EPI_ACCX);
}

void launch_dslash_wide(const DslashArgs &a, VecFormat yf, bool dag, hipStream_t s)
{
    if (a.B.ntiles == 0) return;
    dim3 grid(a.B.ntiles), block(FL_WAVE * a.B.RT);
    if (yf == VEC_H16) {
        if (dag)
            hipLaunchKernelGGL((k_dslash_wide<H16, true>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((k_dslash_wide<H16, false>), grid, block, 0, s, a);
    } else if (yf == VEC_F32) {
        if (dag)
            hipLaunchKernelGGL((k_dslash_wide<float, true>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((k_dslash_wide<float, false>), grid, block, 0, s, a);
    } else {
        launch_unsupported("widening hop: input format");
    }
}

void launch_dslash(LinkFormat fmt, const DslashArgs &a, bool dag, int epi, hipStream_t s)
{
    dim3 grid(a.B.ntiles), block(FL_WAVE * a.B.RT);
    if (a.B.ntiles == 0) return;
    if (!dslash_epi_supported(epi)) {
        launch_unsupported("hopping epilogue");
        return;
    }
    switch (fmt) {
    case LINK_F64_R18: dispatch_dag<double, LinkF64R18>(a, dag, epi, grid, block, s); break;
    case LINK_F32_R18: dispatch_dag<float, LinkF32R18>(a, dag, epi, grid, block, s); break;
    case LINK_F32_R12: dispatch_dag<float, LinkF32R12>(a, dag, epi, grid, block, s); break;
    case LINK_BF16_R12: dispatch_dag<float, LinkBF16R12>(a, dag, epi, grid, block, s); break;
    case LINK_Q16_R12: dispatch_dag<H16, LinkQ16R12>(a, dag, epi, grid, block, s); break;
    default: launch_unsupported("hopping link format"); break;
    }
}

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
#include "fl_host.h"
#include "fl_stencil.h"

namespace {

template <typename R, class LK, bool DAG, int EPI>
__global__ __launch_bounds__(sizeof(R) == 8 ? 512 : 1024) void k_dslash(DslashArgs a)
{
    typedef typename SpinorFmt<R>::V SV;
    TileInfo T = tile_info(a.B);
    if (!T.valid_rhs) return;
    if (a.mask && !a.mask[T.sys]) return;  // wave-uniform: one wave = one right-hand side
    const LatGeom &g = a.B.lat[T.lat];
    const int rhs = __builtin_amdgcn_readfirstlane(T.rhs);
    const size_t fs = (size_t)SpinorFmt<R>::NC * g.Vh;
    const unsigned fbytes = (unsigned)(fs * sizeof(SV));
    R q0 = 0, q1 = 0, q2 = 0;
    if (T.valid_site) {
        Coord c = cb_coords(g, a.par, T.site);
        BufSrc<R, LK> src;
        src.in = make_buf((const SV *)a.in[T.lat] + rhs * fs, fbytes);
        src.gauge = make_buf(a.gauge[T.lat], (unsigned)(8u * LK::NC * LK::ESZ * (unsigned)g.Vh));
        src.Vh = g.Vh;
        cx<R> acc[12];
        hop_site<DAG, R>(g, a.par, T.site, c, src, acc);
        const R cb = (R)a.cb[T.lat];
        cx<R> out[12];
        if (EPI & EPI_XPAY) {
            cx<R> xv[12];
            SpinorFmt<R>::load(make_buf((const SV *)a.x[T.lat] + rhs * fs, fbytes), g.Vh, T.site, xv);
            const R ca = (R)a.ca[T.lat];
            if (ca == (R)1) {
#pragma unroll
                for (int k = 0; k < 12; ++k)
                    out[k] = cx<R>{fma(cb, acc[k].re, xv[k].re), fma(cb, acc[k].im, xv[k].im)};
            } else {
#pragma unroll
                for (int k = 0; k < 12; ++k) out[k] = ca * xv[k] + cb * acc[k];
            }
            if (EPI & EPI_DOTX_NORM) {
#pragma unroll
                for (int k = 0; k < 12; ++k) {
                    cx<R> d = cjmul(out[k], xv[k]);
                    q0 += d.re;
                    q1 += d.im;
                    q2 += out[k].re * out[k].re + out[k].im * out[k].im;
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < 12; ++k) out[k] = cb * acc[k];
        }
        SpinorFmt<R>::store(make_buf((SV *)a.out[T.lat] + rhs * fs, fbytes), g.Vh, T.site, out);
        if (EPI & EPI_DOTY) {
            cx<R> yv[12];
            SpinorFmt<R>::load(make_buf((const SV *)a.y[T.lat] + rhs * fs, fbytes), g.Vh, T.site, yv);
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
    if (EPI & (EPI_DOTY | EPI_DOTX_NORM | EPI_NORM)) {
        double s0 = wave_sum((double)q0), s1 = wave_sum((double)q1), s2 = wave_sum((double)q2);
        if (threadIdx.x % FL_WAVE == 0) {
            const int ns = a.nsys, nb = a.B.nsb_max;
            if (EPI & (EPI_DOTY | EPI_DOTX_NORM)) {
                a.partial[pidx(a.slot0, ns, T.sys, nb, T.sb)] = s0;
                a.partial[pidx(a.slot0 + 1, ns, T.sys, nb, T.sb)] = s1;
            }
            if (EPI & (EPI_DOTX_NORM | EPI_NORM))
                a.partial[pidx(a.slot0 + 2, ns, T.sys, nb, T.sb)] = s2;
        }
    }
}

template <typename R, class LK, bool DAG>
void dispatch_epi(const DslashArgs &a, int epi, dim3 grid, dim3 block, hipStream_t s)
{
    switch (epi) {
    case EPI_PLAIN: hipLaunchKernelGGL((k_dslash<R, LK, DAG, EPI_PLAIN>), grid, block, 0, s, a); break;
    case EPI_XPAY: hipLaunchKernelGGL((k_dslash<R, LK, DAG, EPI_XPAY>), grid, block, 0, s, a); break;
    case EPI_XPAY | EPI_NORM:
        hipLaunchKernelGGL((k_dslash<R, LK, DAG, EPI_XPAY | EPI_NORM>), grid, block, 0, s, a);
        break;
    case EPI_XPAY | EPI_DOTY:
        hipLaunchKernelGGL((k_dslash<R, LK, DAG, EPI_XPAY | EPI_DOTY>), grid, block, 0, s, a);
        break;
    case EPI_XPAY | EPI_DOTX_NORM:
        hipLaunchKernelGGL((k_dslash<R, LK, DAG, EPI_XPAY | EPI_DOTX_NORM>), grid, block, 0, s, a);
        break;
    case EPI_NORM: hipLaunchKernelGGL((k_dslash<R, LK, DAG, EPI_NORM>), grid, block, 0, s, a); break;
    default: break;
    }
}

template <typename R, class LK>
void dispatch_dag(const DslashArgs &a, bool dag, int epi, dim3 grid, dim3 block, hipStream_t s)
{
    if (dag)
        dispatch_epi<R, LK, true>(a, epi, grid, block, s);
    else
        dispatch_epi<R, LK, false>(a, epi, grid, block, s);
}

}  // namespace

bool dslash_epi_supported(int epi)
{
    return epi == EPI_PLAIN || epi == EPI_XPAY || epi == (EPI_XPAY | EPI_NORM) ||
           epi == (EPI_XPAY | EPI_DOTY) || epi == (EPI_XPAY | EPI_DOTX_NORM) || epi == EPI_NORM;
}

void launch_dslash(LinkFormat fmt, const DslashArgs &a, bool dag, int epi, hipStream_t s)
{
    dim3 grid(a.B.ntiles), block(FL_WAVE * a.B.RT);
    if (a.B.ntiles == 0) return;
    switch (fmt) {
    case LINK_F64_R18: dispatch_dag<double, LinkF64R18>(a, dag, epi, grid, block, s); break;
    case LINK_F32_R18: dispatch_dag<float, LinkF32R18>(a, dag, epi, grid, block, s); break;
    case LINK_F32_R12: dispatch_dag<float, LinkF32R12>(a, dag, epi, grid, block, s); break;
    case LINK_BF16_R12: dispatch_dag<float, LinkBF16R12>(a, dag, epi, grid, block, s); break;
    }
}

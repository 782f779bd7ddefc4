// fl_blas.hip -- vector updates, reductions and per-system scalar steps of
// the batched Krylov solvers.
//
// BiCGStab (van der Vorst 1992) is run independently for every right-hand
// side of a batch (no block method: the low-precision map of each source
// must not depend on the rest of the batch).  The iteration is split into
//   v = Dhat p (+ <r0, v>)      -> alpha = rho / <r0, v>
//   s = r - alpha v
//   t = Dhat s (+ <t, s>, |t|^2) -> omega = <t, s> / |t|^2
//   x += alpha p + omega s, r = s - omega t (+ <r0, r>, |r|^2)
//                               -> beta = (rho'/rho)(alpha/omega)
//   p = r + beta (p - omega v)
// with the operator launches in fl_dslash.hip carrying the reductions in
// their epilogue.  Reductions are two-stage and deterministic: each
// wavefront writes one partial per 64-site block, and one workgroup per
// system sums the partials in a fixed order.
#include "fl_host.h"

namespace {

// per-wave buffer view of right-hand side `rhs` of a field stored as
// SpinorFmt<S> (one resource per field, built in scalar registers)
template <typename S>
__device__ __forceinline__ Buf fbuf(const void *base, const LatGeom &g, int rhs)
{
    return spinor_buf<S>(base, g.Vh, rhs);
}

template <typename R>
__device__ __forceinline__ cx<R> cpx_of(const double *v)
{
    return cx<R>{(R)v[0], (R)v[1]};
}

// S: storage format of the iteration vectors, arithmetic in SpinorFmt<S>::R
template <typename S, int OP>
__global__ __launch_bounds__(sizeof(typename SpinorFmt<S>::R) == 8 ? 512 : 1024) void k_blas(BlasArgs a)
{
    typedef typename SpinorFmt<S>::R R;
    TileInfo T = tile_info(a.B);
    if (!T.valid_rhs) return;
    if (OP == OP_CG_PX) {
        // a system that stopped in this iteration still owes its x update
        if (!a.mask[T.sys] && a.st[T.sys].xstamp != a.stamp) return;
    } else if (a.mask && !a.mask[T.sys]) {
        return;
    }
    const LatGeom &g = a.B.lat[T.lat];
    const int l = T.lat, i = T.site, Vh = g.Vh;
    const int rhs = __builtin_amdgcn_readfirstlane(T.rhs);
    typedef SpinorFmt<S> F;
    typedef SpinorFmt<double> F64;
    R q0 = 0, q1 = 0, q2 = 0;
    if (T.valid_site) {
        if (OP == OP_BICG_S) {
            const SysState &st = a.st[T.sys];
            cx<R> al = cpx_of<R>(st.alpha);
            cx<R> r[12], v[12];
            F::load(fbuf<S>(a.f[0][l], g, rhs), Vh, i, r);
            F::load(fbuf<S>(a.f[1][l], g, rhs), Vh, i, v);
#pragma unroll
            for (int k = 0; k < 12; ++k) r[k] = cmsub(r[k], al, v[k]);
            store_result<S>(fbuf<S>(a.f[2][l], g, rhs), Vh, i, r);
        } else if (OP == OP_BICG_XR) {
            const SysState &st = a.st[T.sys];
            cx<R> al = cpx_of<R>(st.alpha), om = cpx_of<R>(st.omega);
            cx<R> x[12], p[12], s[12], t[12], r0[12];
            F::load(fbuf<S>(a.f[0][l], g, rhs), Vh, i, x);
            F::load(fbuf<S>(a.f[1][l], g, rhs), Vh, i, p);
            F::load(fbuf<S>(a.f[2][l], g, rhs), Vh, i, s);
            F::load(fbuf<S>(a.f[3][l], g, rhs), Vh, i, t);
            F::load(fbuf<S>(a.f[5][l], g, rhs), Vh, i, r0);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                x[k] = cmad(cmad(x[k], al, p[k]), om, s[k]);
                s[k] = cmsub(s[k], om, t[k]);  // new r
            }
            store_result<S>(fbuf<S>(a.f[0][l], g, rhs), Vh, i, x);
            store_result<S>(fbuf<S>(a.f[4][l], g, rhs), Vh, i, s);  // reductions of the stored values
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                cx<R> d = cjmul(r0[k], s[k]);
                q0 += d.re;
                q1 += d.im;
                q2 += s[k].re * s[k].re + s[k].im * s[k].im;
            }
        } else if (OP == OP_BICG_P) {
            const SysState &st = a.st[T.sys];
            cx<R> be = cpx_of<R>(st.beta), om = cpx_of<R>(st.omega);
            cx<R> p[12], r[12], v[12];
            F::load(fbuf<S>(a.f[0][l], g, rhs), Vh, i, p);
            F::load(fbuf<S>(a.f[1][l], g, rhs), Vh, i, r);
            F::load(fbuf<S>(a.f[2][l], g, rhs), Vh, i, v);
#pragma unroll
            for (int k = 0; k < 12; ++k) p[k] = cmad(r[k], be, cmsub(p[k], om, v[k]));
            store_result<S>(fbuf<S>(a.f[0][l], g, rhs), Vh, i, p);
        } else if (OP == OP_HI_TO_LO) {
            cx<double> h[12];
            cx<R> lo[12], r0[12];
            F64::load(fbuf<double>(a.f[1][l], g, rhs), Vh, i, h);
#pragma unroll
            for (int k = 0; k < 12; ++k) lo[k] = cx<R>{(R)h[k].re, (R)h[k].im};
            store_result<S>(fbuf<S>(a.f[0][l], g, rhs), Vh, i, lo);
            if (a.flag) {
                store_result<S>(fbuf<S>(a.f[2][l], g, rhs), Vh, i, lo);
                store_result<S>(fbuf<S>(a.f[3][l], g, rhs), Vh, i, lo);
                cx<R> z[12];
#pragma unroll
                for (int k = 0; k < 12; ++k) z[k] = cx<R>{(R)0, (R)0};
                store_result<S>(fbuf<S>(a.f[4][l], g, rhs), Vh, i, z);
#pragma unroll
                for (int k = 0; k < 12; ++k) r0[k] = lo[k];
            } else {
                F::load(fbuf<S>(a.f[2][l], g, rhs), Vh, i, r0);
            }
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                cx<R> d = cjmul(r0[k], lo[k]);
                q0 += d.re;
                q1 += d.im;
                q2 += lo[k].re * lo[k].re + lo[k].im * lo[k].im;
            }
        } else if (OP == OP_ACC_HI) {
            cx<double> h[12];
            cx<R> lo[12];
            F64::load(fbuf<double>(a.f[0][l], g, rhs), Vh, i, h);
            F::load(fbuf<S>(a.f[1][l], g, rhs), Vh, i, lo);
#pragma unroll
            for (int k = 0; k < 12; ++k) h[k] = h[k] + cx<double>{(double)lo[k].re, (double)lo[k].im};
            store_result<double>(fbuf<double>(a.f[0][l], g, rhs), Vh, i, h);
            if (a.flag) {
#pragma unroll
                for (int k = 0; k < 12; ++k) lo[k] = cx<R>{(R)0, (R)0};
                store_result<S>(fbuf<S>(a.f[1][l], g, rhs), Vh, i, lo);
            }
        } else if (OP == OP_SUB_HI) {
            cx<double> u[12], w[12];
            F64::load(fbuf<double>(a.f[1][l], g, rhs), Vh, i, u);
            F64::load(fbuf<double>(a.f[2][l], g, rhs), Vh, i, w);
#pragma unroll
            for (int k = 0; k < 12; ++k) u[k] = u[k] - w[k];
            store_result<double>(fbuf<double>(a.f[0][l], g, rhs), Vh, i, u);
        } else if (OP == OP_NORM) {
            cx<R> f[12];
            F::load(fbuf<S>(a.f[0][l], g, rhs), Vh, i, f);
#pragma unroll
            for (int k = 0; k < 12; ++k) q2 += f[k].re * f[k].re + f[k].im * f[k].im;
        } else if (OP == OP_ZERO) {
            cx<R> z[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) z[k] = cx<R>{(R)0, (R)0};
            store_result<S>(fbuf<S>(a.f[0][l], g, rhs), Vh, i, z);
        } else if (OP == OP_DOT) {
            cx<R> u[12], w[12];
            F::load(fbuf<S>(a.f[0][l], g, rhs), Vh, i, u);
            F::load(fbuf<S>(a.f[1][l], g, rhs), Vh, i, w);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                cx<R> d = cjmul(u[k], w[k]);
                q0 += d.re;
                q1 += d.im;
            }
        } else if (OP == OP_CG_FIXP) {
            const cx<R> c = {(R)a.st[T.sys].beta[0], (R)a.st[T.sys].beta[1]};
            cx<R> p[12], z[12];
            F::load(fbuf<S>(a.f[0][l], g, rhs), Vh, i, p);
            F::load(fbuf<S>(a.f[1][l], g, rhs), Vh, i, z);
#pragma unroll
            for (int k = 0; k < 12; ++k) p[k] = cmad(p[k], c, z[k]);
            store_result<S>(fbuf<S>(a.f[0][l], g, rhs), Vh, i, p);
        } else if (OP == OP_CG_R) {
            const R al = (R)a.st[T.sys].alpha[0];
            cx<R> r[12], q[12];
            F::load(fbuf<S>(a.f[0][l], g, rhs), Vh, i, r);
            F::load(fbuf<S>(a.f[1][l], g, rhs), Vh, i, q);
#pragma unroll
            for (int k = 0; k < 12; ++k) r[k] = cx<R>{fma(-al, q[k].re, r[k].re), fma(-al, q[k].im, r[k].im)};
            store_result<S>(fbuf<S>(a.f[0][l], g, rhs), Vh, i, r);
#pragma unroll
            for (int k = 0; k < 12; ++k) q2 += r[k].re * r[k].re + r[k].im * r[k].im;
        } else if (OP == OP_CG_P) {
            const R be = (R)a.st[T.sys].beta[0];
            cx<R> p[12], z[12];
            F::load(fbuf<S>(a.f[0][l], g, rhs), Vh, i, p);
            F::load(fbuf<S>(a.f[1][l], g, rhs), Vh, i, z);
#pragma unroll
            for (int k = 0; k < 12; ++k) p[k] = cx<R>{fma(be, p[k].re, z[k].re), fma(be, p[k].im, z[k].im)};
            store_result<S>(fbuf<S>(a.f[0][l], g, rhs), Vh, i, p);
        } else if (OP == OP_CG_PX) {
            // wave-uniform: one wave is one system
            const SysState &st = a.st[T.sys];
            const bool xu = st.xstamp == a.stamp, pu = a.mask[T.sys] != 0;
            cx<R> p[12];
            F::load(fbuf<S>(a.f[0][l], g, rhs), Vh, i, p);
            if (xu) {
                const R al = (R)st.alpha[0];
                cx<R> x[12];
                F::load(fbuf<S>(a.f[2][l], g, rhs), Vh, i, x);
#pragma unroll
                for (int k = 0; k < 12; ++k) x[k] = cx<R>{fma(al, p[k].re, x[k].re), fma(al, p[k].im, x[k].im)};
                store_result<S>(fbuf<S>(a.f[2][l], g, rhs), Vh, i, x);
            }
            if (pu) {
                const R be = (R)st.beta[0];
                cx<R> z[12];
                F::load(fbuf<S>(a.f[1][l], g, rhs), Vh, i, z);
#pragma unroll
                for (int k = 0; k < 12; ++k) p[k] = cx<R>{fma(be, p[k].re, z[k].re), fma(be, p[k].im, z[k].im)};
                store_result<S>(fbuf<S>(a.f[0][l], g, rhs), Vh, i, p);
            }
        }
    }
    if (OP == OP_BICG_XR || OP == OP_HI_TO_LO || OP == OP_NORM || OP == OP_CG_R || OP == OP_DOT) {
        double s0 = wave_sum((double)q0), s1 = wave_sum((double)q1), s2 = wave_sum((double)q2);
        constexpr int which = (OP == OP_BICG_XR || OP == OP_HI_TO_LO) ? 7 : (OP == OP_DOT ? 3 : 4);
        write_partials(a.partial, a.slot0, a.nsys, T.sys, a.B.nsb_max, T.sb, s0, s1, s2, which);
    }
}

template <typename S>
void dispatch(const BlasArgs &a, dim3 grid, dim3 block, hipStream_t s)
{
    switch (a.op) {
    case OP_BICG_S: hipLaunchKernelGGL((k_blas<S, OP_BICG_S>), grid, block, 0, s, a); break;
    case OP_BICG_XR: hipLaunchKernelGGL((k_blas<S, OP_BICG_XR>), grid, block, 0, s, a); break;
    case OP_BICG_P: hipLaunchKernelGGL((k_blas<S, OP_BICG_P>), grid, block, 0, s, a); break;
    case OP_HI_TO_LO: hipLaunchKernelGGL((k_blas<S, OP_HI_TO_LO>), grid, block, 0, s, a); break;
    case OP_ACC_HI: hipLaunchKernelGGL((k_blas<S, OP_ACC_HI>), grid, block, 0, s, a); break;
    case OP_SUB_HI: hipLaunchKernelGGL((k_blas<S, OP_SUB_HI>), grid, block, 0, s, a); break;
    case OP_NORM: hipLaunchKernelGGL((k_blas<S, OP_NORM>), grid, block, 0, s, a); break;
    case OP_ZERO: hipLaunchKernelGGL((k_blas<S, OP_ZERO>), grid, block, 0, s, a); break;
    case OP_CG_R: hipLaunchKernelGGL((k_blas<S, OP_CG_R>), grid, block, 0, s, a); break;
    case OP_CG_P: hipLaunchKernelGGL((k_blas<S, OP_CG_P>), grid, block, 0, s, a); break;
    case OP_CG_PX: hipLaunchKernelGGL((k_blas<S, OP_CG_PX>), grid, block, 0, s, a); break;
    case OP_DOT: hipLaunchKernelGGL((k_blas<S, OP_DOT>), grid, block, 0, s, a); break;
    case OP_CG_FIXP: hipLaunchKernelGGL((k_blas<S, OP_CG_FIXP>), grid, block, 0, s, a); break;
    default: launch_unsupported("vector operation"); break;
    }
}

// ---------------------------------------------------------------------------
// per-system scalar steps: one workgroup per system sums the partials of
// the six slots in a fixed order, then lane 0 advances the recurrence
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool finite_d(double v) { return v == v && v - v == 0.0; }

// one step of a system's scalar recurrence on a local copy of its state
__device__ __forceinline__ void scal_step(const ScalArgs &a, const double P[6], SysState &s, int &act)
{
    switch (a.step) {
    case SC_ALPHA: {
        double den = P[0] * P[0] + P[1] * P[1];
        if (!(den > 0) || !finite_d(den)) {
            s.flags |= ST_BREAK;
            act = 0;
            break;
        }
        // alpha = rho / r0v
        s.alpha[0] = (s.rho[0] * P[0] + s.rho[1] * P[1]) / den;
        s.alpha[1] = (s.rho[1] * P[0] - s.rho[0] * P[1]) / den;
        break;
    }
    case SC_OMEGA: {
        double tt = P[2];
        if (tt > 0 && finite_d(tt)) {
            s.omega[0] = P[0] / tt;
            s.omega[1] = P[1] / tt;
        } else if (tt == 0) {
            s.omega[0] = s.omega[1] = 0;
        } else {
            s.flags |= ST_BREAK;
            act = 0;
        }
        break;
    }
    case SC_BETA: {
        double rho_n[2] = {P[0], P[1]};
        double rr = P[2];
        s.iter += 1;
        if (!finite_d(rr) || !finite_d(rho_n[0]) || !finite_d(rho_n[1])) {
            s.flags |= ST_BREAK;
            act = 0;
            break;
        }
        s.rr = rr;
        if (rr > s.rmax2) s.rmax2 = rr;
        if (rr < s.delta2 * s.rmax2) s.flags |= ST_WANT_UPD;
        if (rr <= s.stop2) {
            s.flags |= ST_CONV_ITER;
            act = 0;
        } else if (s.iter >= s.max_iter) {
            s.flags |= ST_MAXIT;
            act = 0;
        }
        double om2 = s.omega[0] * s.omega[0] + s.omega[1] * s.omega[1];
        double rh2 = s.rho[0] * s.rho[0] + s.rho[1] * s.rho[1];
        if (act && (!(om2 > 0) || !(rh2 > 0))) {
            s.flags |= ST_BREAK;
            act = 0;
        }
        if (om2 > 0 && rh2 > 0) {
            // beta = (rho_n / rho) * (alpha / omega)
            double q[2] = {(rho_n[0] * s.rho[0] + rho_n[1] * s.rho[1]) / rh2,
                           (rho_n[1] * s.rho[0] - rho_n[0] * s.rho[1]) / rh2};
            double w[2] = {(s.alpha[0] * s.omega[0] + s.alpha[1] * s.omega[1]) / om2,
                           (s.alpha[1] * s.omega[0] - s.alpha[0] * s.omega[1]) / om2};
            s.beta[0] = q[0] * w[0] - q[1] * w[1];
            s.beta[1] = q[0] * w[1] + q[1] * w[0];
        }
        s.rho[0] = rho_n[0];
        s.rho[1] = rho_n[1];
        break;
    }
    case SC_RESET:
        s.tr2 = P[2];
        s.rho[0] = P[3];
        s.rho[1] = P[4];
        s.rr = P[5];
        s.rmax2 = P[5];
        s.flags &= ~(ST_CONV_ITER | ST_WANT_UPD);
        break;
    case SC_INIT:
        s.rho[0] = P[3];
        s.rho[1] = P[4];
        s.rr = P[5];
        s.rmax2 = P[5];
        s.flags = 0;
        s.alpha[0] = s.omega[0] = 1;
        s.alpha[1] = s.omega[1] = 0;
        s.beta[0] = s.beta[1] = 0;
        if (P[5] <= s.stop2) {
            s.flags |= ST_CONV_ITER;
            act = 0;
        } else {
            act = 1;
        }
        break;
    case SC_CG_INIT:  // slot 2: |z|^2 with z = Dhat^+ r; slot 5: |r|^2
        s.zz = P[2];
        s.rr = P[5];
        s.beta[0] = s.beta[1] = 0;
        s.flags &= ST_MAXIT;
        if (P[5] <= s.stop2 || !(P[2] > 0)) {
            s.flags |= ST_CONV_ITER;
            act = 0;
        } else {
            act = 1;
        }
        break;
    case SC_CG_ALPHA:  // slot 2: |q|^2 with q = Dhat p
        if (!(P[2] > 0) || !finite_d(P[2])) {
            s.flags |= ST_BREAK;
            act = 0;
        } else {
            s.alpha[0] = s.zz / P[2];
        }
        break;
    case SC_CG_BETA: {  // slot 2: |z'|^2 of the updated z = Dhat^+ r; slot 5: |r|^2 if carried
        // Without a carried r: |r - alpha q|^2 = |r|^2 - 2 alpha Re<q, r>
        // + alpha^2 |q|^2 with <q, r> = <p, Dhat^+ r> = <p, z> = |z|^2 (CG;
        // restored at every residual replacement) and alpha = |z|^2 / |q|^2.
        // The recurrence holds to the rounding of the low-precision operator
        // relative to |r|^2 at the last replacement, so below 1e-6 of that
        // value it is no longer trusted: it still asks for a replacement
        // (far below the delta trigger) but claims no convergence
        double zn = P[2], rr = a.carried_r ? P[5] : s.rr - s.alpha[0] * s.zz;
        const bool trusted = a.carried_r || rr > 1e-6 * s.rmax2;
        s.xstamp = a.stamp;  // r moved by alpha q in this iteration: x moves by alpha p
        s.iter += 1;
        s.rr = rr;
        if (!finite_d(zn) || !finite_d(rr)) {
            s.flags |= ST_BREAK;
            act = 0;
            break;
        }
        s.beta[0] = zn / s.zz;
        s.zz = zn;
        if (rr > s.rmax2) s.rmax2 = rr;
        if (rr < s.delta2 * s.rmax2 || !trusted) s.flags |= ST_WANT_UPD;
        if (trusted && rr <= s.stop2) {
            s.flags |= ST_CONV_ITER;
            act = 0;
        } else if (s.iter >= s.max_iter) {
            s.flags |= ST_MAXIT;
            act = 0;
        }
        break;
    }
    case SC_CG_REZ: {  // after a residual replacement that keeps p: slot 2 |z|^2, z = Dhat^+ r;
                       // slots 0, 1 <z, p>; slot 5 |r|^2
        // CG's step length alpha = |z|^2 / |Dhat p|^2 assumes <z, p> = |z|^2,
        // which holds for the iteration's own z but not for the replaced one;
        // p += c z with c = (|z|^2 - <z, p>) / |z|^2 restores it
        s.zz = P[2];
        s.rr = P[5];
        s.rmax2 = P[5];
        s.flags &= ~(ST_CONV_ITER | ST_WANT_UPD);
        const double zz = P[2] > 0 ? P[2] : 1.0;
        s.beta[0] = (P[2] - P[0]) / zz;
        s.beta[1] = -P[1] / zz;
        if (!(P[2] > 0) || !finite_d(P[2])) {
            s.flags |= ST_BREAK;
            act = 0;
        }
        break;
    }
    default: break;
    }
}

// the partial-sum slots each scalar step reads (bit k: slot k)
__device__ __forceinline__ int scal_slots(int step)
{
    switch (step) {
    case SC_ALPHA: return 0x03;     // <r0, v>
    case SC_OMEGA: return 0x07;     // <t, s>, |t|^2
    case SC_BETA: return 0x07;      // <r0, r>, |r|^2
    case SC_RESET: return 0x3c;     // |rh|^2, <r0, r>, |r|^2
    case SC_INIT: return 0x38;      // <r0, r>, |r|^2
    case SC_CG_INIT: return 0x24;   // |z|^2, |r|^2
    case SC_CG_ALPHA: return 0x04;  // |q|^2
    case SC_CG_BETA: return 0x24;   // |z|^2, |r|^2 (if carried)
    case SC_CG_REZ: return 0x27;    // <z, p>, |z|^2, |r|^2
    default: return 0x3f;
    }
}

__global__ __launch_bounds__(256) void k_scal(ScalArgs a)
{
    const int sys = blockIdx.x;
    if (a.mask) {
        if (!a.mask[sys]) return;
    } else if (!a.active[sys]) {
        return;
    }
    int l = 0;
    for (int k = 1; k < FL_MAXLAT; ++k)
        if (k < a.B.nlat && sys >= a.B.lat[k].sys0) l = k;
    const int nsb = a.B.lat[l].nsb, nb = a.B.nsb_max;
    __shared__ double red[6][256];
    __shared__ SysState snew;
    // only the slots this step reads (the same for the whole block)
    const int used = scal_slots(a.step);
    for (int slot = 0; slot < 6; ++slot) {
        if (!((used >> slot) & 1)) continue;
        double acc = 0;
        for (int sb = threadIdx.x; sb < nsb; sb += 256) acc += a.partial[pidx(slot, a.nsys, sys, nb, sb)];
        red[slot][threadIdx.x] = acc;
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int slot = 0; slot < 6; ++slot)
                if ((used >> slot) & 1) red[slot][threadIdx.x] += red[slot][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x >= FL_WAVE) return;
    if (threadIdx.x == 0) {
        double P[6];
        for (int slot = 0; slot < 6; ++slot) P[slot] = ((used >> slot) & 1) ? red[slot][0] : 0.0;
        SysState s = a.st[sys];
        const int act0 = a.active[sys];
        int act = act0;
        scal_step(a, P, s, act);
        snew = s;
        if (act != act0) a.active[sys] = act;
    }
    // the flag store completes before the state is written as one store
    // instruction of 8-byte words, one per lane, which ends the kernel
    store_drain();
    constexpr int NW = (int)(sizeof(SysState) / 8);
    static_assert(sizeof(SysState) % 8 == 0, "SysState is written in 8-byte words");
    if ((int)threadIdx.x < NW)
        ((unsigned long long *)(a.st + sys))[threadIdx.x] = ((const unsigned long long *)&snew)[threadIdx.x];
}

}  // namespace

void launch_blas(VecFormat vf, const BlasArgs &a, hipStream_t s)
{
    if (a.B.ntiles == 0) return;
    dim3 grid(a.B.ntiles), block(FL_WAVE * a.B.RT);
    if (vf == VEC_F64)
        dispatch<double>(a, grid, block, s);
    else if (vf == VEC_F32)
        dispatch<float>(a, grid, block, s);
    else
        dispatch<H16>(a, grid, block, s);
}

void launch_scalars(const ScalArgs &a, hipStream_t s)
{
    if (a.nsys == 0) return;
    if (a.step < SC_ALPHA || a.step > SC_CG_REZ) {
        launch_unsupported("scalar step");
        return;
    }
    hipLaunchKernelGGL(k_scal, dim3(a.nsys), dim3(256), 0, s, a);
}

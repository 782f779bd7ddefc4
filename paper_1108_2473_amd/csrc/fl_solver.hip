// fl_solver.hip -- batched even-odd Schur solves.
//
// Every right-hand side of every lattice in the batch runs its own Krylov
// recurrence (BiCGStab, or CG on the normal equations of the Schur
// operator Dhat = 1 - kappa^2 H_eo H_oe); all of them advance together, one
// kernel launch per stage covering the whole batch, with per-system scalars
// kept on the device.  The host looks at the per-system state every few
// iterations only.
//
// Precision: the iteration runs in FP64, or in FP32 vectors with FP32 or
// bfloat16 links.  In the low-precision modes the solution is accumulated
// in FP64 and the FP64 residual bhat - Dhat x is recomputed, replacing the
// iteration's residual, whenever the latter has dropped by `delta` since the
// previous replacement and when the iteration believes it has converged
// (reliable updates; van der Vorst and Ye 2000 on residual replacement).
// A system is finished only when that FP64 residual meets the stopping rule
// |D x - b| <= tol |b| of the paper (Sec. III; for the Schur system the full
// residual equals the even-site residual).  Truncated (LP) solves stop on
// the low-precision iteration's own residual, with no FP64 step.
#include <cmath>
#include <cstring>

#include "fl_host.h"

namespace {

struct MF {  // one field per lattice
    void *p[FL_MAXLAT] = {nullptr, nullptr, nullptr, nullptr};
};

// a host array in the context's page-locked staging block: transfers of the
// per-system state and masks between host checks are then DMA copies
// without a pageable bounce (a block is rewritten only after the stream has
// been synchronised past its last transfer, which every host check does)
template <typename T>
struct PinArr {
    T *p = nullptr;
    size_t n = 0;
    T &operator[](size_t i) { return p[i]; }
    const T &operator[](size_t i) const { return p[i]; }
    T *data() { return p; }
    size_t size() const { return n; }
    void assign(size_t m, const T &v)
    {
        for (size_t i = 0; i < m && i < n; ++i) p[i] = v;
    }
};

struct Solver {
    SolveBatch &sb;
    const fl_solver_params &prm;
    BatchGeom B;    // launches in the iteration precision
    BatchGeom B64;  // FP64 launches (reliable updates): at most 8 waves per workgroup
    int nsys = 0;
    LinkFormat fmt;
    VecFormat vf;  // storage of the iteration vectors
    bool lo64;     // iteration vectors in FP64
    hipStream_t st;
    fl_ctx *c0;
    MF RH, T64, R, R0, P, V, S, T, XL, TMP, XH, BH;
    const void *gauge_lo[FL_MAXLAT], *gauge_hi[FL_MAXLAT];
    double kap2[FL_MAXLAT];
    double *partial = nullptr;
    SysState *dst = nullptr;
    int stamp = 0;  // CGNR iteration stamp
    int flip = 0;   // sweep direction of the next launch (BatchGeom::rev)
    int *active = nullptr, *mask = nullptr;
    PinArr<SysState> hst;
    PinArr<int> hact, hmask, hm2;  // hm2: the masks of restarts and CGNR replacements
    std::vector<long long> active_count;  // per lattice, at the last check

    Solver(SolveBatch &b, const fl_solver_params &p) : sb(b), prm(p) {}

    double lo_bytes_per_site_rhs() const { return (double)vec_site_bytes(vf); }

    void dslash(LinkFormat f, bool lo, int par, const MF &in, const MF &out, const MF *x, const MF *y,
                double ca, const double *cbv, int epi, int slot0, const int *msk, bool dag, int pslot,
                const MF *w = nullptr)
    {
        DslashArgs a;
        std::memset(&a, 0, sizeof(a));
        a.B = f == LINK_F64_R18 ? B64 : B;
        a.par = par;
        a.slot0 = slot0;
        a.nsys = nsys;
        a.mask = msk;
        a.partial = partial;
        a.st = dst;
        for (int l = 0; l < B.nlat; ++l) {
            a.in[l] = in.p[l];
            a.out[l] = out.p[l];
            a.x[l] = x ? x->p[l] : nullptr;
            a.y[l] = y ? y->p[l] : nullptr;
            a.w[l] = w ? w->p[l] : nullptr;
            a.gauge[l] = lo ? gauge_lo[l] : gauge_hi[l];
            a.ca[l] = ca;
            a.cb[l] = cbv ? cbv[l] : 1.0;
        }
        a.B.rev = flip;
        flip ^= 1;
        dslash_config(c0, f, a);
        if (pslot >= 0) prof_begin(c0, pslot);
        launch_dslash(f, a, dag, epi, st);
        if (pslot >= 0) prof_end(c0, pslot, 0.0);
    }

    void blas(VecFormat f, int op, std::initializer_list<const MF *> fields, int flag, int slot0, const int *msk,
              int pslot = -1)
    {
        BlasArgs a;
        std::memset(&a, 0, sizeof(a));
        a.B = f == VEC_F64 ? B64 : B;
        a.op = op;
        a.flag = flag;
        a.slot0 = slot0;
        a.nsys = nsys;
        a.mask = msk;
        a.partial = partial;
        a.st = dst;
        a.stamp = stamp;
        int k = 0;
        for (const MF *f : fields) {
            for (int l = 0; l < B.nlat; ++l) a.f[k][l] = f->p[l];
            ++k;
        }
        a.B.rev = flip;
        flip ^= 1;
        if (pslot >= 0) prof_begin(c0, pslot);
        launch_blas(f, a, st);
        if (pslot >= 0) prof_end(c0, pslot, 0.0);
    }

    void scal(int step, const int *msk)
    {
        ScalArgs a;
        a.B = B;
        a.step = step;
        a.nsys = nsys;
        a.active = active;
        a.mask = msk;
        a.partial = partial;
        a.st = dst;
        a.stamp = stamp;
        a.carried_r = prm.truncated != 0;
        launch_scalars(a, st);
    }

    double neg_k2[FL_MAXLAT], pos_k2[FL_MAXLAT];

    // Dhat (or Dhat^+) applied in the iteration precision: out = in - k^2 H_eo H_oe in;
    // p1, p2: profiling slots of the two hops (-1: none)
    void schur_lo(const MF &in, const MF &out, int epi_extra, const MF *y, int slot0, bool dag, int p1 = -1,
                  int p2 = -1)
    {
        dslash(fmt, true, 1, in, TMP, nullptr, nullptr, 1.0, nullptr, EPI_PLAIN, 0, active, dag, p1);
        dslash(fmt, true, 0, TMP, out, &in, y, 1.0, neg_k2, EPI_XPAY | epi_extra, slot0, active, dag, p2);
    }

    // one BiCGStab iteration for every active system
    void bicg_iteration()
    {
        const VecFormat lf = vf;
        schur_lo(P, V, EPI_DOTY, &R0, 0, false, FL_PROF_DSLASH);   // v = Dhat p, <r0, v>
        scal(SC_ALPHA, nullptr);
        blas(lf, OP_BICG_S, {&R, &V, &S}, 0, 0, active);          // s = r - alpha v
        schur_lo(S, T, EPI_DOTX_NORM, nullptr, 0, false, -1, FL_PROF_DSLASH_END);  // t = Dhat s, <t, s>, |t|^2
        scal(SC_OMEGA, nullptr);
        blas(lf, OP_BICG_XR, {&XL, &P, &S, &T, &R, &R0}, 0, 0, active, FL_PROF_BLAS_UPDATE);
        scal(SC_BETA, nullptr);
        blas(lf, OP_BICG_P, {&P, &R, &V}, 0, 0, active);          // p = r + beta (p - omega v)
    }

    // CGNR on the Schur system: p, q = Dhat p and the normal residual
    // z = Dhat^+ r.  Solves accepted on the FP64 residual carry z itself,
    // z -= alpha Dhat^+ q, fused into the epilogue of the second hop of
    // Dhat^+ (the residual r = b - Dhat x is formed only at a replacement;
    // |r|^2 follows from the scalars): one vector pass of r -= alpha q (three
    // fields) fewer per iteration.  Truncated solves, which stop on their
    // own residual with no FP64 check, carry r and form z = Dhat^+ r.
    void cg_iteration()
    {
        const VecFormat lf = vf;
        ++stamp;
        // q = Dhat p with |q|^2 (slot 2)
        dslash(fmt, true, 1, P, TMP, nullptr, nullptr, 1.0, nullptr, EPI_PLAIN, 0, active, false, FL_PROF_DSLASH);
        dslash(fmt, true, 0, TMP, V, &P, nullptr, 1.0, neg_k2, EPI_XPAY | EPI_NORM, 0, active, false, -1);
        scal(SC_CG_ALPHA, nullptr);
        if (prm.truncated) {
            blas(lf, OP_CG_R, {&R, &V}, 0, 3, active);  // r -= alpha q, |r|^2 -> slot 5
            // z = Dhat^+ r with |z|^2 (slot 2)
            dslash(fmt, true, 1, R, TMP, nullptr, nullptr, 1.0, nullptr, EPI_PLAIN, 0, active, true, -1);
            dslash(fmt, true, 0, TMP, S, &R, nullptr, 1.0, neg_k2, EPI_XPAY | EPI_NORM, 0, active, true,
                   FL_PROF_DSLASH_END);
        } else {
            // z -= alpha Dhat^+ q in the epilogue of the second hop, with |z|^2 (slot 2)
            dslash(fmt, true, 1, V, TMP, nullptr, nullptr, 1.0, nullptr, EPI_PLAIN, 0, active, true, -1);
            dslash(fmt, true, 0, TMP, S, &V, &S, 1.0, neg_k2, EPI_XPAY | EPI_NORM | EPI_CGZ, 0, active, true,
                   FL_PROF_DSLASH_END);
        }
        scal(SC_CG_BETA, nullptr);
        // x += alpha p (also for a system that stopped in SC_CG_BETA), then p = z + beta p
        blas(lf, OP_CG_PX, {&P, &S, &XL}, 0, 0, active, FL_PROF_BLAS_UPDATE);
    }

    // FP64 residual of the masked systems: rh = bh - Dhat xh (|rh|^2 -> slot 2),
    // then the iteration residual r = lo(rh) with <r0, r>, |r|^2 (slots 3..5);
    // init = 1 also restarts the recurrence (r0 = p = r, xl = 0).
    // With FP32 or 16-bit iteration vectors rh = bh - Dhat xh holds between
    // replacements, and the update is rh -= Dhat xl (FP64 arithmetic on the
    // values of xl, the same values that xh += xl adds), which reads xl
    // instead of xh in the first hop and needs no rh = bh - xh pass.  Its
    // rounding is relative to |Dhat xl|, about the residual of the previous
    // replacement, where rh = bh - Dhat xh computed afresh carries an error of
    // the FP64 rounding of |b| whatever the residual: far below tol, but at
    // |r| ~ 1e-8 |b| a perturbation of 1e-8 |r| in a direction unrelated to
    // the Krylov space, which BiCGStab's <r0, r> recurrences amplify.  The
    // carried residual keeps the rounding of every update, relative to the
    // size of each xl: bf16 links, whose operator error (~4e-3) lets
    // BiCGStab's iterate swing far between replacements, and restarts after a
    // breakdown recompute rh from xh instead (the stopping rule on the full
    // operator is checked separately by the callers)
    void replace_residual(const int *msk, int init)
    {
        const bool carry = vf != VEC_F64 && fmt != LINK_BF16_R12 && !init;
        if (carry) {
            DslashArgs a;
            std::memset(&a, 0, sizeof(a));
            a.B = B64;
            a.par = 1;
            a.nsys = nsys;
            a.mask = msk;
            a.partial = partial;
            for (int l = 0; l < B.nlat; ++l) {
                a.in[l] = XL.p[l];
                a.out[l] = T64.p[l];
                a.gauge[l] = gauge_hi[l];
                a.ca[l] = 1.0;
                a.cb[l] = 1.0;
            }
            launch_dslash_wide(a, vf, false, st);                      // t = H_oe xl
            // rh += k^2 H_eo t - xl, and in the same epilogue xh += xl, xl = 0
            dslash(LINK_F64_R18, false, 0, T64, RH, &RH, &XL, 1.0, pos_k2,
                   EPI_XPAY | EPI_NORM | (vf == VEC_H16 ? EPI_SUBY16 : EPI_SUBY32) | EPI_ACCX, 0, msk, false, -1,
                   &XH);
        } else {
            blas(vf, OP_ACC_HI, {&XH, &XL}, 1, 0, msk);                // xh += xl, xl = 0
            blas(VEC_F64, OP_SUB_HI, {&RH, &BH, &XH}, 0, 0, msk);      // rh = bh - xh
            dslash(LINK_F64_R18, false, 1, XH, T64, nullptr, nullptr, 1.0, nullptr, EPI_PLAIN, 0, msk, false,
                   -1);
            dslash(LINK_F64_R18, false, 0, T64, RH, &RH, nullptr, 1.0, pos_k2, EPI_XPAY | EPI_NORM, 0, msk, false,
                   -1);
        }
        blas(vf, OP_HI_TO_LO, {&R, &RH, &R0, &P, &XL}, init, 3, msk);
    }

    fl_status prepare();
    fl_status run(std::vector<SysResult> &res);
    fl_status apply(bool dag);
};

// precision, batch geometry and workspace of the batch
fl_status Solver::prepare()
{
    c0 = sb.ctx[0];
    st = c0->stream;
    if (prm.inner_prec == FL_PREC_F64) {
        fmt = LINK_F64_R18;
    } else if (prm.inner_prec == FL_PREC_F32) {
        fmt = prm.gauge_reals == 18 ? LINK_F32_R18 : LINK_F32_R12;
    } else if (prm.inner_prec == FL_PREC_BF16) {
        fmt = LINK_BF16_R12;
    } else {
        fmt = LINK_Q16_R12;
    }
    vf = vec_format(fmt);
    lo64 = vf == VEC_F64;
    if (fmt == LINK_F32_R12 || fmt == LINK_BF16_R12 || fmt == LINK_Q16_R12)
        for (int l = 0; l < sb.nlat; ++l)
            if (!sb.ctx[l]->su3)
                return set_err(c0, FL_ERR_ARG, "12-real link storage needs SU(3) links; use gauge_reals = 18");
    int minr = 1 << 30;
    for (int l = 0; l < sb.nlat; ++l) minr = std::min(minr, std::max(1, sb.nrhs[l]));
    int RT, G;
    tile_shape(c0, fmt, minr, &RT, &G);
    B = batch_geom(sb.ctx, sb.nrhs, sb.nlat, RT, G);
    // the FP64 kernels are built for at most 512 threads per workgroup
    B64 = RT > 8 ? batch_geom(sb.ctx, sb.nrhs, sb.nlat, 8, G) : B;
    nsys = 0;
    for (int l = 0; l < sb.nlat; ++l) nsys += sb.nrhs[l];
    if (nsys == 0) return FL_OK;

    // workspace
    const size_t lob = vec_site_bytes(vf);
    for (int l = 0; l < sb.nlat; ++l) {
        fl_ctx *c = sb.ctx[l];
        size_t n = (size_t)sb.nrhs[l] * c->Vh;
        RH.p[l] = ws_get(c, WS_RH, n * 192);
        T64.p[l] = ws_get(c, WS_T64, n * 192);
        R.p[l] = ws_get(c, WS_R, n * lob);
        R0.p[l] = ws_get(c, WS_R0, n * lob);
        P.p[l] = ws_get(c, WS_P, n * lob);
        V.p[l] = ws_get(c, WS_V, n * lob);
        S.p[l] = ws_get(c, WS_S, n * lob);
        T.p[l] = ws_get(c, WS_T, n * lob);
        XL.p[l] = ws_get(c, WS_XL, n * lob);
        TMP.p[l] = ws_get(c, WS_TMP, n * lob);
        XH.p[l] = sb.xh[l];
        BH.p[l] = (void *)sb.bh[l];
        for (void *q : {RH.p[l], T64.p[l], R.p[l], R0.p[l], P.p[l], V.p[l], S.p[l], T.p[l], XL.p[l], TMP.p[l]})
            if (!q) return set_err(c, FL_ERR_NOMEM, "device allocation failed (solver vectors)");
        gauge_lo[l] = links(c, fmt);
        gauge_hi[l] = links(c, LINK_F64_R18);
        if (!gauge_lo[l] || !gauge_hi[l]) return set_err(c, FL_ERR_NOMEM, "device allocation failed (links)");
        neg_k2[l] = -c->kappa * c->kappa;
        pos_k2[l] = c->kappa * c->kappa;
    }
    partial = (double *)ws_get(c0, WS_PART, sizeof(double) * 6 * (size_t)nsys * B.nsb_max);
    // [SysState x nsys][active x nsys] in one block, laid out like the
    // page-locked host copy below, so one transfer fetches both at a check
    dst = (SysState *)ws_get(c0, WS_STATE, (sizeof(SysState) + sizeof(int)) * nsys);
    active = dst ? (int *)(dst + nsys) : nullptr;
    mask = (int *)ws_get(c0, WS_MASK, sizeof(int) * nsys);
    if (!partial || !dst || !active || !mask) return set_err(c0, FL_ERR_NOMEM, "device allocation failed");
    {
        // [SysState x nsys][hact][hmask][hm2], SysState is 8-byte aligned
        const size_t ns = (size_t)nsys;
        char *h = (char *)pinned_get(c0, sizeof(SysState) * ns + 3 * sizeof(int) * ns + 64);
        if (!h) return set_err(c0, FL_ERR_NOMEM, "page-locked host allocation failed");
        hst.p = (SysState *)h;
        hst.n = ns;
        int *ip = (int *)(h + sizeof(SysState) * ns);
        hact.p = ip;
        hmask.p = ip + ns;
        hm2.p = ip + 2 * ns;
        hact.n = hmask.n = hm2.n = ns;
    }
    return hip_check(c0, hipMemsetAsync(partial, 0, sizeof(double) * 6 * (size_t)nsys * B.nsb_max, st), "memset");
}

// xh = Dhat bh (dag: Dhat^+ bh) with the operator and vectors in the
// iteration precision: bh rounded to the iteration format, the two hops of
// the Schur operator, the result widened to FP64
fl_status Solver::apply(bool dag)
{
    fl_status e;
    if ((e = prepare())) return e;
    if (nsys == 0) return FL_OK;
    hact.assign(nsys, 1);
    if ((e = hip_check(c0, hipMemcpyAsync(active, hact.data(), sizeof(int) * nsys, hipMemcpyHostToDevice, st),
                       "upload active")))
        return e;
    for (int l = 0; l < sb.nlat; ++l) {
        size_t n = (size_t)sb.nrhs[l] * sb.ctx[l]->Vh * 192;
        if ((e = hip_check(c0, hipMemcpyAsync(RH.p[l], BH.p[l], n, hipMemcpyDeviceToDevice, st), "copy b")))
            return e;
        if ((e = hip_check(c0, hipMemsetAsync(XH.p[l], 0, n, st), "memset x"))) return e;
    }
    blas(vf, OP_HI_TO_LO, {&R, &RH, &R0, &P, &XL}, 0, 3, nullptr);  // r = lo(b)
    schur_lo(R, V, 0, nullptr, 0, dag);
    blas(vf, OP_ACC_HI, {&XH, &V}, 0, 0, nullptr);  // xh = v
    if ((e = hip_check(c0, hipStreamSynchronize(st), "apply Schur operator"))) return e;
    return hip_check(c0, hipGetLastError(), "apply Schur operator");
}

fl_status Solver::run(std::vector<SysResult> &res)
{
    fl_status e;
    if ((e = prepare())) return e;
    if (nsys == 0) return FL_OK;
    if ((int)sb.bnorm.size() != nsys) return set_err(c0, FL_ERR_ARG, "internal: bnorm size");
    const int solver = prm.solver;

    // initial state
    const double tol = prm.tol;
    const bool trunc = prm.truncated != 0;
    // default trigger: a decade per replacement; 16-bit storage drifts
    // faster and needs one replacement per factor ~3 (measured at 16^3x32:
    // 386 CGNR iterations at 0.3, 417 at 0.1, no convergence at 0.05)
    double delta = prm.delta > 0 && prm.delta < 1 ? prm.delta : (vf == VEC_H16 ? 0.3 : 0.1);
    hst.assign(nsys, SysState());
    for (int k = 0; k < nsys; ++k) {
        SysState &s = hst[k];
        std::memset(&s, 0, sizeof(s));
        double bn = sb.bnorm[k];
        // accepted 1 % below tol: the callers recompute the residual on the
        // full operator after the solve, and that FP64 recomputation differs
        // from the Schur residual by rounding (~1e-4 of tol |b| at 16^3x32)
        const double acc = trunc ? tol : 0.99 * tol;
        s.tstop2 = (acc * bn) * (acc * bn);
        // the iteration aims a little below the target so that the FP64 check passes
        s.stop2 = trunc ? s.tstop2 : 0.25 * s.tstop2;
        s.delta2 = (lo64 || trunc) ? 0.0 : delta * delta;
        s.max_iter = prm.max_iter > 0 ? prm.max_iter : 20000;
    }
    if ((e = hip_check(c0, hipMemcpyAsync(dst, hst.data(), sizeof(SysState) * nsys, hipMemcpyHostToDevice, st),
                       "upload state")))
        return e;
    for (int l = 0; l < sb.nlat; ++l) {
        size_t n = (size_t)sb.nrhs[l] * sb.ctx[l]->Vh * 192;
        if ((e = hip_check(c0, hipMemsetAsync(XH.p[l], 0, n, st), "memset x"))) return e;
        if ((e = hip_check(c0, hipMemcpyAsync(RH.p[l], BH.p[l], n, hipMemcpyDeviceToDevice, st), "copy b")))
            return e;
    }
    blas(vf, OP_HI_TO_LO, {&R, &RH, &R0, &P, &XL}, 1, 3, nullptr);  // r = r0 = p = lo(b), xl = 0
    hact.assign(nsys, 1);
    hmask.assign(nsys, 0);
    if ((e = hip_check(c0, hipMemcpyAsync(active, hact.data(), sizeof(int) * nsys, hipMemcpyHostToDevice, st),
                       "upload active")))
        return e;
    auto cg_start = [&](const int *msk) {
        // z = Dhat^+ r (|z|^2 -> slot 2); |r|^2 already in slot 5; p = z
        dslash(fmt, true, 1, R, TMP, nullptr, nullptr, 1.0, nullptr, EPI_PLAIN, 0, msk, true, -1);
        dslash(fmt, true, 0, TMP, S, &R, nullptr, 1.0, neg_k2, EPI_XPAY | EPI_NORM, 0, msk, true, -1);
        scal(SC_CG_INIT, msk);
        blas(vf, OP_ZERO, {&P}, 0, 0, msk);
        blas(vf, OP_CG_P, {&P, &S}, 0, 0, msk);  // SC_CG_INIT sets beta = 0: p = z
    };
    auto cg_rez = [&](const int *msk) {
        // reliable update that keeps p: z = Dhat^+ r for the replaced r
        // (|z|^2 -> slot 2, |r|^2 already in slot 5, <z, p> -> slots 0, 1),
        // new |z|^2 for alpha, and p += c z so that <z, p> = |z|^2 again
        // (without it, a replaced residual that has moved away from the
        // recursive one, as it does when an iteration gains a lot between
        // two host checks, derails the recurrence)
        dslash(fmt, true, 1, R, TMP, nullptr, nullptr, 1.0, nullptr, EPI_PLAIN, 0, msk, true, -1);
        dslash(fmt, true, 0, TMP, S, &R, nullptr, 1.0, neg_k2, EPI_XPAY | EPI_NORM, 0, msk, true, -1);
        blas(vf, OP_DOT, {&S, &P}, 0, 0, msk);
        scal(SC_CG_REZ, msk);
        blas(vf, OP_CG_FIXP, {&P, &S}, 0, 0, msk);
    };
    if (solver == FL_SOLVER_CGNR) {
        cg_start(nullptr);
    } else {
        scal(SC_INIT, nullptr);
    }

    res.assign(nsys, SysResult());
    std::vector<int> done(nsys, 0), restarts(nsys, 0);
    // the host looks at the state every `chunk` iterations; for CGNR the
    // chunk (at most 16) follows the convergence rate so that a check comes
    // about once per replacement trigger (delta): rarely on slowly
    // converging systems (fewer FP64 replacements and host round trips;
    // 16^3x32 at kappa 0.1596: 15 instead of 17 replacements per system),
    // often on fast ones (a replacement far behind its trigger costs
    // iterations)
    int chunk = trunc ? 4 : (solver == FL_SOLVER_CGNR ? 16 : 8);
    std::vector<double> rr_prev(nsys, 0.0);
    std::vector<int> act_start(nsys, 0);
    active_count.assign(sb.nlat, 0);
    int ndone = 0;
    auto sys_lat = [&](int k) {
        int l = 0;
        for (int q = 1; q < B.nlat; ++q)
            if (k >= B.lat[q].sys0) l = q;
        return l;
    };
    // vector fields each profiled kernel reads or writes once per site and
    // system: the first hop its input and output; the hop that ends the
    // iteration also its own-site operands (CGNR: q and z; truncated CGNR
    // and BiCGStab: r resp. s); the vector update x and p (CGNR: p, z and x
    // read, x and p written; BiCGStab: x, p, s, t, r0 read, x and r written).
    // Links are counted for the hops only.
    const int prof_slot[3] = {FL_PROF_DSLASH, FL_PROF_DSLASH_END, FL_PROF_BLAS_UPDATE};
    const int prof_fields[3] = {2, (solver == FL_SOLVER_CGNR && !trunc) ? 4 : 3,
                                solver == FL_SOLVER_CGNR ? 5 : 7};
    size_t prof_mark[3];
    for (int k = 0; k < 3; ++k) prof_mark[k] = c0->prof[prof_slot[k]].ev.size();
    auto account_prof = [&]() {
        for (int k = 0; k < 3; ++k) {
            ProfSlot &ps = c0->prof[prof_slot[k]];
            if (!ps.on) continue;
            size_t nnew = ps.ev.size() - prof_mark[k];
            prof_mark[k] = ps.ev.size();
            if (!nnew) continue;
            // algorithmic bytes of one hopping launch: every link once per
            // lattice, plus each field read or written once for the systems
            // still iterating (counted at the end of the chunk: a lower bound)
            double bytes = 0;
            for (int l = 0; l < B.nlat; ++l) {
                const double lb = (double)link_bytes(fmt);
                bytes += (k < 2 ? 8.0 * lb * B.lat[l].Vh : 0.0) +
                         prof_fields[k] * lo_bytes_per_site_rhs() * B.lat[l].Vh * active_count[l];
            }
            ps.bytes += bytes * nnew;
        }
    };

    while (ndone < nsys) {
        // check the state every chunk of iterations
        bool any_active = false;
        for (int k = 0; k < nsys; ++k) any_active |= (hact[k] != 0);
        act_start.assign(hact.data(), hact.data() + nsys);
        if (any_active)
            for (int it = 0; it < chunk; ++it) {
                if (solver == FL_SOLVER_CGNR)
                    cg_iteration();
                else
                    bicg_iteration();
            }
        // state and active flags in one transfer (adjacent on both sides)
        if ((e = hip_check(c0, hipMemcpyAsync(hst.data(), dst, (sizeof(SysState) + sizeof(int)) * nsys,
                                              hipMemcpyDeviceToHost, st),
                           "download state")))
            return e;
        if ((e = hip_check(c0, hipStreamSynchronize(st), "sync"))) return e;
        if ((e = hip_check(c0, hipGetLastError(), "solver launch"))) return e;
        for (int l = 0; l < sb.nlat; ++l) active_count[l] = 0;
        for (int k = 0; k < nsys; ++k)
            if (hact[k]) active_count[sys_lat(k)]++;
        account_prof();

        if (solver == FL_SOLVER_CGNR && !trunc && any_active) {
            // per-iteration factor of |r|^2 of the fastest system that iterated
            // the whole chunk, where its estimate is trusted (the scalar
            // recurrence above 1e-6 of its value at the last replacement);
            // next chunk ~ log(delta^2) / log(factor)
            double fmin = 1.0;
            const int nch = chunk;
            for (int k = 0; k < nsys; ++k)
                if (act_start[k] && hact[k] && !done[k] && rr_prev[k] > 0 && hst[k].rr > 1e-6 * hst[k].rmax2 &&
                    hst[k].rr < rr_prev[k])
                    fmin = std::min(fmin, std::pow(hst[k].rr / rr_prev[k], 1.0 / nch));
            if (fmin < 1.0)
                chunk = std::min(16, std::max(2, (int)std::floor(std::log(delta * delta) / std::log(fmin))));
        }
        if (trunc && any_active) {
            // truncated solves stop on the device (a system leaves the active
            // set in the scalar step that meets its residual), so the host
            // only has to notice that all have stopped: the next check comes
            // when the slowest system still iterating is expected to stop
            // (launches after that run with no active system and do no work)
            double need = 0.0;
            bool est = false;
            const int nch = chunk;
            for (int k = 0; k < nsys; ++k)
                if (act_start[k] && hact[k] && !done[k] && rr_prev[k] > 0 && hst[k].rr > 0 &&
                    hst[k].rr < rr_prev[k]) {
                    const double f = std::pow(hst[k].rr / rr_prev[k], 1.0 / nch);
                    if (f < 1.0) {
                        need = std::max(need, std::log(hst[k].stop2 / hst[k].rr) / std::log(f));
                        est = true;
                    }
                }
            if (est) chunk = std::min(16, std::max(2, (int)std::ceil(need)));
        }

        bool any_upd = false, any_restart = false;
        std::vector<int> final_upd(nsys, 0), restart(nsys, 0);
        for (int k = 0; k < nsys; ++k) {
            hmask[k] = 0;
            if (done[k]) continue;
            const int f = hst[k].flags;
            if (trunc) {
                if (f & (ST_CONV_ITER | ST_MAXIT | ST_BREAK)) {
                    done[k] = 1;
                    ++ndone;
                    res[k].converged = (f & ST_CONV_ITER) ? 1 : 0;
                    res[k].flags = f;
                }
                continue;
            }
            if (f & ST_BREAK) {
                if (restarts[k] < 4 && hst[k].iter < hst[k].max_iter) {
                    restart[k] = 1;
                    any_restart = true;
                    restarts[k]++;
                } else {
                    final_upd[k] = 1;
                    hmask[k] = 1;
                    any_upd = true;
                }
            } else if (f & (ST_CONV_ITER | ST_WANT_UPD | ST_MAXIT)) {
                hmask[k] = 1;
                any_upd = true;
                if (f & ST_MAXIT) final_upd[k] = 1;
            }
        }
        if (any_restart) {
            // breakdown: fresh recurrence from the current FP64 iterate
            for (int k = 0; k < nsys; ++k) hm2[k] = restart[k];
            if ((e = hip_check(c0, hipMemcpyAsync(mask, hm2.data(), sizeof(int) * nsys, hipMemcpyHostToDevice, st),
                               "upload mask")))
                return e;
            replace_residual(mask, 1);
            if ((e = hip_check(c0, hipMemcpyAsync(hst.data(), dst, sizeof(SysState) * nsys, hipMemcpyDeviceToHost, st),
                               "download state")))
                return e;
            if ((e = hip_check(c0, hipStreamSynchronize(st), "sync"))) return e;
            if ((e = hip_check(c0, hipGetLastError(), "solver launch"))) return e;
            for (int k = 0; k < nsys; ++k)
                if (restart[k]) {
                    hst[k].flags = 0;
                    res[k].updates++;
                }
            if ((e = hip_check(c0, hipMemcpyAsync(dst, hst.data(), sizeof(SysState) * nsys, hipMemcpyHostToDevice, st),
                               "upload state")))
                return e;
            if (solver == FL_SOLVER_CGNR)
                cg_start(mask);
            else
                scal(SC_INIT, mask);
            if ((e = hip_check(c0, hipMemcpyAsync(hact.data(), active, sizeof(int) * nsys, hipMemcpyDeviceToHost, st),
                               "download active")))
                return e;
            if ((e = hip_check(c0, hipStreamSynchronize(st), "sync"))) return e;
            if ((e = hip_check(c0, hipGetLastError(), "solver launch"))) return e;
        }
        if (any_upd) {
            if ((e = hip_check(c0, hipMemcpyAsync(mask, hmask.data(), sizeof(int) * nsys, hipMemcpyHostToDevice, st),
                               "upload mask")))
                return e;
            replace_residual(mask, 0);
            scal(SC_RESET, mask);
            if ((e = hip_check(c0, hipMemcpyAsync(hst.data(), dst, sizeof(SysState) * nsys, hipMemcpyDeviceToHost, st),
                               "download state")))
                return e;
            if ((e = hip_check(c0, hipStreamSynchronize(st), "sync"))) return e;
            if ((e = hip_check(c0, hipGetLastError(), "solver launch"))) return e;
            for (int k = 0; k < nsys; ++k) {
                if (!hmask[k]) continue;
                res[k].updates++;
                const SysState &s = hst[k];
                bool ok = s.tr2 <= s.tstop2;
                const bool out_of_cycles = prm.max_outer > 0 && res[k].updates >= prm.max_outer;
                if (ok || final_upd[k] || s.iter >= s.max_iter || out_of_cycles) {
                    done[k] = 1;
                    ++ndone;
                    hact[k] = 0;
                    res[k].converged = ok ? 1 : 0;
                    res[k].flags = s.flags | ((final_upd[k] || (!ok && out_of_cycles)) ? ST_MAXIT : 0);
                } else {
                    hact[k] = 1;
                }
            }
            if (solver == FL_SOLVER_CGNR) {
                // CGNR continues from the replaced residual with the same
                // search direction: z = Dhat^+ r and |z|^2 are recomputed
                for (int k = 0; k < nsys; ++k) hm2[k] = hmask[k] && hact[k];
                if ((e = hip_check(c0, hipMemcpyAsync(mask, hm2.data(), sizeof(int) * nsys, hipMemcpyHostToDevice, st),
                                   "upload mask")))
                    return e;
                cg_rez(mask);
            }
            if ((e = hip_check(c0, hipMemcpyAsync(active, hact.data(), sizeof(int) * nsys, hipMemcpyHostToDevice, st),
                               "upload active")))
                return e;
        }
        for (int k = 0; k < nsys; ++k) rr_prev[k] = hst[k].rr;
        // a system with nothing left to do must not spin the loop
        if (!any_upd && !any_restart) {
            bool progressing = false;
            for (int k = 0; k < nsys; ++k) progressing |= (!done[k] && hact[k]);
            if (!progressing)
                for (int k = 0; k < nsys; ++k)
                    if (!done[k]) {
                        done[k] = 1;
                        ++ndone;
                        res[k].flags = hst[k].flags;
                    }
        }
    }
    if (trunc) {
        // the LP solution is the low-precision iterate
        blas(vf, OP_ACC_HI, {&XH, &XL}, 0, 0, nullptr);
    }
    fl_status out = FL_OK;
    for (int k = 0; k < nsys; ++k) {
        const SysState &s = hst[k];
        res[k].iters = s.iter;
        double bn = sb.bnorm[k] > 0 ? sb.bnorm[k] : 1.0;
        res[k].true_resid = trunc ? std::sqrt(s.rr) / bn : std::sqrt(s.tr2) / bn;
        if (!res[k].converged) out = (res[k].flags & ST_BREAK) ? FL_ERR_BREAKDOWN : FL_ERR_NOCONV;
    }
    if ((e = hip_check(c0, hipStreamSynchronize(st), "sync"))) return e;
    return out;
}

}  // namespace

fl_status solve_schur_batch(SolveBatch &sb, const fl_solver_params &p, std::vector<SysResult> &res)
{
    Solver s(sb, p);
    return s.run(res);
}

fl_status schur_apply_batch(SolveBatch &sb, const fl_solver_params &p, bool dag)
{
    Solver s(sb, p);
    return s.apply(dag);
}

/*
 * floop.h -- C ABI of the MI355X (gfx950) library for disconnected fermion
 * loops L(x) = Tr[Gamma G(x;x)] (Alexandrou, Hadjiyiannakou, Koutsou,
 * O Cais, Strelchenko, arXiv:1108.2473, Eq. (loop)).
 *
 * The library evaluates the loops exactly (12 V_s point-source inversions
 * per timeslice, Sec. II) or stochastically (diluted noise, Eq. (loop
 * stochastic), and the truncated solver method, Sec. II and III), each
 * inversion an even-odd preconditioned BiCGStab or CGNR solve of the
 * Wilson-Dirac operator run by hand-written HIP kernels.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  lattice   extents dims = {Lx, Ly, Lz, Lt}, each even and >= 2; site
 *            index s = x + Lx*(y + Ly*(z + Lz*t)); V = Lx*Ly*Lz*Lt,
 *            Vs = Lx*Ly*Lz.  Direction mu = 0..3 is x, y, z, t.
 *  operator  (D psi)(x) = psi(x) - kappa sum_mu [ (1-g_mu) U_mu(x) psi(x+mu)
 *                                             + (1+g_mu) U_mu(x-mu)^+ psi(x-mu) ]
 *            (N_f=2 Wilson fermions at hopping parameter kappa, Sec. II;
 *            the paper does not write the form, this is the r=1 Wilson
 *            operator in hopping normalisation).  Space is periodic; a hop
 *            across the time boundary is multiplied by bc_t.  Links carry
 *            no boundary phase.
 *  gammas    Hermitian chiral basis: g_k = [[0,-i s_k],[i s_k,0]],
 *            g_4 = [[0,1],[1,0]], g_5 = g1 g2 g3 g4 = diag(1,1,-1,-1).
 *            A Gamma insertion is a 4-bit mask: Gamma = g1^b0 g2^b1 g3^b2 g4^b3
 *            (1 -> 0, g_mu -> 1 << (mu-1), g_5 -> 15).  The paper's set
 *            Gamma = 1, g_5, g_mu is {0, 15, 1, 2, 4, 8}.
 *  gauge     double U[4][V][3][3][2]: U_mu(s), row, column, (re, im).
 *            Must be SU(3) to 1e-10 when 12-real link storage is used.
 *  spinors   double psi[nrhs][V][4][3][2]: spin, colour, (re, im).
 *  loops     double L[ngamma][nt][Vs][2] (complex, per Gamma, timeslice,
 *            spatial site xs = x + Lx*(y + Ly*z)).
 *  where     FL_HOST: pointers are host memory; FL_DEVICE: device memory
 *            on the context's device, used in place on the context stream.
 *  ownership the caller allocates every input and output; the library
 *            copies what it needs and keeps no caller pointer past return.
 *  errors    every call returns an fl_status; the text of the last error
 *            of a context is fl_last_error(ctx).  Arguments are checked
 *            before any device work is launched.  FL_ERR_NOCONV is not
 *            fatal: outputs hold the best iterate and the stats are filled.
 *  threads   a context is not thread-safe; use one per host thread.
 */
#ifndef FLOOP_H
#define FLOOP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fl_ctx fl_ctx;

typedef enum {
    FL_OK = 0,
    FL_ERR_ARG = -1,       /* invalid argument (checked before any launch) */
    FL_ERR_STATE = -2,     /* missing set-up (gauge field, kappa) */
    FL_ERR_DEVICE = -3,    /* HIP runtime error */
    FL_ERR_NOMEM = -4,     /* device allocation failed */
    FL_ERR_NOCONV = -5,    /* a solve missed its tolerance within max_iter */
    FL_ERR_BREAKDOWN = -6  /* Krylov breakdown with no fallback left */
} fl_status;

typedef enum { FL_HOST = 0, FL_DEVICE = 1 } fl_where;

typedef enum { FL_PREC_F64 = 0, FL_PREC_F32 = 1, FL_PREC_BF16 = 2, FL_PREC_H16 = 3 } fl_prec;

typedef enum { FL_SOLVER_BICGSTAB = 0, FL_SOLVER_CGNR = 1 } fl_solver_kind;

typedef enum { FL_NOISE_Z4 = 0, FL_NOISE_CZ2 = 1, FL_NOISE_Z2 = 2 } fl_noise_kind;

/* dilution bits (Sec. II): time, spin (x4), colour (x3), even-odd space
 * (x2), cubic (x8, one class per vertex of the elementary 3-cube) */
enum { FL_DIL_TIME = 1, FL_DIL_SPIN = 2, FL_DIL_COLOUR = 4, FL_DIL_EVENODD = 8,
       FL_DIL_CUBIC = 16 };

/*
 * Solver parameters.  The stopping rule is the paper's (Sec. III): the
 * relative deviation |D x - b| / |b| of the full Wilson-Dirac operator.
 *  solver      BiCGStab (the paper's choice for its truncated-solver runs)
 *              or CG on the normal equations of the Schur operator.
 *  tol         target relative residual of the full operator (FP64).
 *  max_iter    Krylov iterations per right-hand side, all cycles included.
 *  inner_prec  precision of the Krylov iteration.  FL_PREC_F64 runs the
 *              whole solve in FP64; F32 runs FP32 vectors and links; BF16
 *              stores the links in bfloat16 (FP32 vectors and arithmetic);
 *              H16 stores the iteration vectors as 16-bit fixed point with
 *              one FP32 scale per site (52 bytes per site instead of 96) and
 *              the links as 16-bit fixed point (12 reals, 24 bytes), with
 *              FP32 arithmetic (the paper ran mixed-precision GPU solvers,
 *              Sec. II; this is the narrowest storage offered here).
 *              For F32/BF16/H16 the iteration residual is replaced by the
 *              FP64 residual whenever it has dropped by `delta` since the
 *              last replacement (reliable updates): F32 and H16 carry the
 *              FP64 residual, subtracting D applied in FP64 to the
 *              low-precision correction that they then add to the FP64
 *              solution; BF16 (and any restart after a breakdown)
 *              recomputes b - Dx from the FP64 solution.  Every solve's
 *              result is checked on the full operator in FP64.
 *  gauge_reals 18 (full links) or 12 (rows 0 and 1; row 2 rebuilt as
 *              conj(row0 x row1)) for the F32 inner operator; BF16 and H16
 *              need 12.
 *  delta       reliable-update trigger in (0, 1); 0 selects 0.1 (0.3 for
 *              H16).  At a replacement BiCGStab and CGNR keep their search
 *              directions (CGNR recomputes D^+ r for the replaced r); they
 *              restart only after a breakdown.
 *  truncated   1: low-precision (LP) solve of the truncated solver method:
 *              inner precision only, stops when the iteration's own
 *              residual reaches tol, no FP64 correction.  The LP map is a
 *              deterministic function of the source, independent of the
 *              batch it is solved in.
 *  batch       maximum right-hand sides per device batch (0: default).
 *  max_outer   FP64 residual replacements (outer cycles of the mixed-
 *              precision solve) per right-hand side; 0: no limit.  A
 *              right-hand side that reaches it without meeting tol stops
 *              with FL_ERR_NOCONV.
 * Every solve that is not truncated is accepted on the FP64 residual of the
 * FULL operator, |b - D x| / |b| with x = (x_e, x_o) and x_o = b_o +
 * kappa H_oe x_e, recomputed after the Schur solve (fl_solve and every
 * fl_loops_* call); a right-hand side above tol is reported as not
 * converged.  In the terms of a classic outer/inner mixed-precision solver:
 * delta is the inner (per-outer-cycle) reduction target, updates are the
 * outer cycles, and truncated = 1 is an inner-only (LP) solve.
 */
typedef struct {
    int solver;
    double tol;
    int max_iter;
    int inner_prec;
    int gauge_reals;
    double delta;
    int truncated;
    int batch;
    int max_outer;
} fl_solver_params;

/* per right-hand side */
typedef struct {
    int iters;          /* Krylov iterations */
    int updates;        /* FP64 residual replacements (outer cycles) */
    int converged;      /* 1 if true_resid <= tol (truncated: its own residual reached tol) */
    double true_resid;  /* |D x - b| / |b| recomputed in FP64 on the full operator
                           (truncated solves: the iteration's own estimate) */
    double seconds;     /* wall time of the device batch this right-hand side was solved in */
} fl_solver_stats;

/*
 * Stochastic estimator parameters (Eq. (loop stochastic), dilution and the
 * truncated solver method of Sec. II):
 *   Lhat = (1/n_lp) sum_{r in LP} sum_d eta_{r,d}^+ Gamma phi^LP_{r,d}
 *        + (1/n_hp) sum_{r in HP} sum_d eta_{r,d}^+ Gamma (phi^HP - phi^LP)
 * with LP noise indices r0 .. r0+n_lp-1 and HP indices following them,
 * eta_{r,d} = P_d xi_r the diluted noise and phi = D^{-1} eta.  n_hp = 0
 * gives the plain estimator over n_lp vectors solved with the LP params.
 * Noise: xi_r(site, spin, colour) from the k-th output of SplitMix64
 * (Steele, Lea, Flood 2014) started at `seed`, k = ((r V + site) 4 + spin) 3
 * + colour; with b63, b62 its top bits, Z4: i^(2 b63 + b62); complex Z2:
 * ((-1)^b63 + i (-1)^b62)/sqrt 2; real Z2: (-1)^b63.
 */
typedef struct {
    int noise;                 /* fl_noise_kind */
    unsigned long long seed;
    long long r0;              /* first noise index */
    int n_lp, n_hp;
    int dilution;              /* FL_DIL_* mask */
    int t_begin, t_end;        /* timeslices estimated: t_begin .. t_end-1 */
} fl_noise_params;

/* Fill p with defaults: BiCGStab, tol 1e-12, max_iter 20000, FP32 inner
 * with 12-real links, delta 0 (the solver's default for the inner
 * precision), not truncated, default batch, no limit on outer cycles. */
void fl_solver_params_default(fl_solver_params *p);

/* Library version string. */
const char *fl_version(void);

/* Create a context for one lattice on HIP device `device`.  dims: four
 * even extents >= 2; bc_t = +1 (periodic) or -1 (antiperiodic) in time. */
fl_status fl_create(fl_ctx **ctx, int device, const int dims[4], int bc_t);

/* Release every device buffer of the context and its page-locked host
 * staging block (grown on demand by the solving calls for the per-system
 * solver state, masks, norms and host results).  NULL is accepted. */
fl_status fl_destroy(fl_ctx *ctx);

/* Stream for all later device work of the context (hipStream_t passed as
 * void*, e.g. torch.cuda.current_stream().cuda_stream); NULL: the default
 * stream.  Calls are asynchronous with respect to the host only where
 * noted; every entry point below returns after its work is complete. */
fl_status fl_set_stream(fl_ctx *ctx, void *hip_stream);

/* Gauge field U (layout above), copied to the device and converted to the
 * per-precision link layouts.  The paper's input configurations (Sec. II). */
fl_status fl_set_gauge(fl_ctx *ctx, const double *U, fl_where where);

/* Hopping parameter kappa > 0 (Sec. II). */
fl_status fl_set_kappa(fl_ctx *ctx, double kappa);

/* out = D in (dagger = 0) or D^+ in = g5 D g5 in (dagger = 1) for nrhs
 * spinors in the canonical layout, FP64. */
fl_status fl_apply_D(fl_ctx *ctx, const double *in, double *out, int nrhs, int dagger,
                     fl_where where);

/* fl_apply_D for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): in
 * and out are DEVICE pointers (canonical layout, FP64, nrhs spinors), and
 * the even/odd work fields live in a fixed device array of the library
 * (64 MiB per GPU, held until the process ends), so nrhs * V * 384 bytes
 * may not exceed 64 MiB (16^3 x 32: one spinor); larger requests return
 * FL_ERR_ARG.  Calls no hipMalloc, hipFree or allocating routine and does
 * not synchronise: the work is enqueued on the context stream and the call
 * returns (synchronise the stream before reading out).  The array is shared
 * by every call on one GPU, so calls that overlap on one GPU (other streams,
 * other host threads) race; nothing in it needs to start at zero.
 * FL_ERR_STATE before fl_set_gauge / fl_set_kappa. */
fl_status fl_apply_D_noalloc(fl_ctx *ctx, const double *in, double *out, int nrhs, int dagger);

/* The even-odd Schur operator Dhat = 1 - kappa^2 H_eo H_oe (dagger = 1:
 * Dhat^+ = g5 Dhat g5) as the solvers apply it, in the iteration precision
 * and link storage of p (inner_prec, gauge_reals; p->batch bounds the
 * right-hand sides per launch, the other fields are not used): the even
 * sites of each of the nrhs canonical FP64 spinors in `in` are rounded to
 * that storage, the two hops and the vector update run in its arithmetic,
 * and the even sites of `out` (canonical FP64, nrhs spinors) receive the
 * result widened to FP64; odd sites of `out` are set to 0 and odd sites of
 * `in` are not read.  The hopping-kernel shape and LDS mode of
 * fl_set_tile() apply.  Operator of the Schur system solved in Sec. III. */
fl_status fl_apply_schur(fl_ctx *ctx, const double *in, double *out, int nrhs, int dagger,
                         const fl_solver_params *p, fl_where where);

/* Solve D x_k = b_k for nrhs right-hand sides (canonical spinor layout)
 * to the stopping rule of Sec. III, via the Schur system
 * x_e = (1 - k^2 H_eo H_oe)^{-1} (b_e + k H_eo b_o), x_o = b_o + k H_oe x_e.
 * stats: NULL or an array of nrhs entries (host memory). */
fl_status fl_solve(fl_ctx *ctx, const double *b, double *x, int nrhs,
                   const fl_solver_params *p, fl_solver_stats *stats, fl_where where);

/* Exact loops, Eq. (loop), on whole timeslices t0[0..nt-1]: 12 Vs point
 * sources per timeslice (Sec. II).  L: [ngamma][nt][Vs][2];
 * S: NULL or [nt][Vs][4][4][2], the colour-traced S(y)_{alpha beta} =
 * sum_a G(y;y)_{alpha a, beta a} with L_Gamma = sum Gamma_{beta alpha} S_{alpha beta}.
 * L and S are in `where` memory. */
fl_status fl_loops_exact(fl_ctx *ctx, const int *t0, int nt, const int *gammas, int ngamma,
                         const fl_solver_params *p, double *L, double *S, fl_where where);

/* Exact loops at an explicit host list of lexicographic sites:
 * L: [ngamma][nsites][2], S: NULL or [nsites][4][4][2]. */
fl_status fl_loops_exact_sites(fl_ctx *ctx, const long long *sites, long long nsites,
                               const int *gammas, int ngamma, const fl_solver_params *p,
                               double *L, double *S, fl_where where);

/* Stochastic / truncated-solver-method loops (fl_noise_params above).
 * lp: solver of the first ensemble; hp: solver of the correction ensemble
 * (ignored when n_hp = 0).  L: [ngamma][t_end-t_begin][Vs][2].
 * FL_ERR_NOCONV (or FL_ERR_BREAKDOWN) when any solve of either ensemble
 * missed its tolerance (truncated solves: their own residual within
 * max_iter); L then holds the estimate from the best iterates and
 * fl_last_stats names the solves. */
fl_status fl_loops_stochastic(fl_ctx *ctx, const fl_noise_params *np, const int *gammas,
                              int ngamma, const fl_solver_params *lp,
                              const fl_solver_params *hp, double *L, fl_where where);

/* Truncated-solver-method loops for several lattices of uneven size in one
 * batch: every Krylov stage of all lattices runs in the same kernel launch
 * (nctx <= 4 contexts on the same device and stream).  np[i], L[i] as in
 * fl_loops_stochastic for context i. */
fl_status fl_loops_stochastic_multi(fl_ctx **ctxs, int nctx, const fl_noise_params *np,
                                    const int *gammas, int ngamma,
                                    const fl_solver_params *lp, const fl_solver_params *hp,
                                    double **L, fl_where where);

/* Gradient of F = Re sum_{Gamma,t,xs} conj(w[Gamma][t][xs]) L_Gamma(xs,t) for the
 * exact loops of timeslices t0 with respect to kappa and every link.
 * w: [ngamma][nt][Vs][2]; sites whose weights are all zero are not solved.
 * The adjoint solutions come from gamma_5-hermiticity, D^{-+} = g5 D^{-1} g5,
 * so no solves beyond the forward point sources are needed.
 * dU: [4][V][3][3][2] with dU = dF/dRe U + i dF/dIm U; dkappa: host double. */
fl_status fl_loops_grad(fl_ctx *ctx, const int *t0, int nt, const int *gammas, int ngamma,
                        const double *w, const fl_solver_params *p, double *dU,
                        double *dkappa, fl_where where);

/* Kernel timing with HIP events recorded on the context stream around every
 * launch of the named kernel while enabled (kernel ids below).  Reset on
 * enable.  ms: summed event time; launches: count; bytes: summed
 * algorithmic bytes of those launches (links and spinors read once, outputs
 * written once, counted for the systems still iterating).
 *   FL_PROF_DSLASH: the first hop of every Krylov iteration, H_oe of the
 *     Schur operator applied to the search direction (no epilogue).
 *   FL_PROF_DSLASH_END: the hop with the fused epilogue that ends the
 *     operator work of an iteration: for CGNR the second hop of Dhat^+ q
 *     with z -= alpha (q + c H q') and |z|^2 (reads q and z at the site), for
 *     truncated CGNR the second hop of Dhat^+ r with |z|^2, for BiCGStab
 *     the second hop of Dhat s with <t, s> and |t|^2 (reads s at the site).
 *   FL_PROF_BLAS_UPDATE: the vector update of every iteration: for CGNR
 *     x += alpha p and p = z + beta p (5 field passes), for BiCGStab
 *     x += alpha p + omega s and r = s - omega t (7 field passes). */
enum { FL_PROF_DSLASH = 0, FL_PROF_DSLASH_END = 1, FL_PROF_BLAS_UPDATE = 2, FL_PROF_NKERNELS = 4 };
fl_status fl_profile_enable(fl_ctx *ctx, int kernel, int enable);
fl_status fl_profile_read(fl_ctx *ctx, int kernel, double *ms, long long *launches,
                          double *bytes);

/* Half-dslash micro-benchmark: nrep launches of the hopping kernel
 * out_e = H_eo in_o for nrhs right-hand sides at precision `prec` and
 * gauge_reals, cycling through `nsets` independent buffer sets (links and
 * spinors, to defeat on-chip caches), timed with HIP events on the context
 * stream.  rt, group, lds: workgroup shape and LDS staging (0, 0, -1: the
 * context's current choice).
 * ms_per_launch and bytes_per_launch (algorithmic) are returned. */
fl_status fl_bench_dslash(fl_ctx *ctx, int prec, int gauge_reals, int nrhs, int nrep,
                          int nsets, int rt, int group, int lds, double *ms_per_launch,
                          double *bytes_per_launch);

/* Workgroup shape of the batched kernels for one precision / link storage:
 * rt right-hand sides (wavefronts) per workgroup (power of two <= 16; FP64
 * uses at most 8), `group` right-hand-side blocks that sweep the site
 * blocks together (0: all), and lds, the LDS staging of the hopping kernel:
 * 0 none, 1 each wavefront's x/y neighbour window, 2 windows plus the
 * workgroup's links, 3 (FL_PREC_H16 only) as 2 with the hop computed on the
 * stored 16-bit integers (packed int16 spin projection, exact int16 dot
 * products for the colour product, links staged at half scale in the two
 * forms those products need), 4 the workgroup's links only, no neighbour
 * windows (for FL_PREC_H16 the packed hop of 3, every neighbour spinor
 * loaded two directions before its use), -1 the built-in choice (4; 1 for
 * FP64 workgroups of fewer than 4 right-hand sides; falling back to a
 * smaller mode when its LDS does not fit).  rt = 0 restores the built-in workgroup size.
 * FL_ERR_ARG for out-of-range values or lds 3 with another precision. */
fl_status fl_set_tile(fl_ctx *ctx, int prec, int gauge_reals, int rt, int group, int lds);

/* Autotuner: time the hopping kernel for nrhs right-hand sides over the
 * workgroup shapes and LDS modes above and keep the fastest for this
 * context (returned in rt, group, lds and its launch time in ms; any output
 * pointer may be NULL). */
fl_status fl_autotune(fl_ctx *ctx, int prec, int gauge_reals, int nrhs, int *rt, int *group,
                      int *lds, double *ms);

/* Momentum projection of loops (Sec. III, Eq. all_dis_corr):
 *   Lp[g][k][t] = sum_x exp(+i p_k . x) L[g][t][x],
 *   p_k = 2 pi (n_x / Lx, n_y / Ly, n_z / Lz)  for the integer vector
 *   n_k = (mom[3k], mom[3k+1], mom[3k+2]) (any sign).
 * L: [ngamma][nt][V_s][2] doubles (loops on any nt timeslices, e.g. the
 * output of fl_loops_exact or fl_loops_stochastic; site x = (x, y, z) with x
 * fastest), Lp: [ngamma][nmom][nt][2]; 1 <= ngamma <= 16.  L and Lp are
 * both on the host or both on the device (`where`); mom is a host array.
 * Needs no gauge field and Lx + Ly + Lz <= 1024 (FL_ERR_ARG otherwise).
 * FP64, summed in a fixed order (deterministic). */
fl_status fl_momentum_project(fl_ctx *ctx, const double *L, int ngamma, int nt, const int *mom,
                              int nmom, double *Lp, fl_where where);

/* Disconnected two-point function (Sec. III, Eq. all_dis_corr), averaged
 * over the source timeslice ti:
 *   D[j][k][t] = (1/V_s) (1/T) sum_ti Lp1[A_j][k][(ti + t) mod T] * Lp2[B_j][k][ti]
 * Lp1, Lp2: [ngamma][nmom][T][2], loops on all T timeslices projected with
 * +p_k (Lp1) and -p_k (Lp2) by fl_momentum_project; pairs: npair host pairs
 * (A_j, B_j) of Gamma indices; D: [npair][nmom][T][2].  For stochastic loops
 * Lp1 and Lp2 must come from independent noise vectors: the product of one
 * estimate with itself is biased.  Lp1, Lp2 and D follow `where`. */
fl_status fl_disconnected_corr(fl_ctx *ctx, const double *Lp1, const double *Lp2, int ngamma,
                               int nmom, const int *pairs, int npair, double *D, fl_where where);

/* Gaussian smearing of quark fields (Sec. III), in place:
 *   psi <- F psi,  F = ((1 + alpha H) / norm)^n,
 *   H(x, y) = sum_{i=1..3} [U_i(x) delta_{x,y-i} + U_i(x-i)^+ delta_{x,y+i}]
 * with the context's links (pass APE-smeared links to it for the paper's
 * setup), colour only, within each timeslice.  norm = 1 is the paper's F;
 * norm = 1 + 6 alpha keeps the field of order one over n = 50 steps.
 * psi: [nrhs][V][4][3][2] doubles on the host or the device (`where`).
 * FP64. */
fl_status fl_smear(fl_ctx *ctx, double *psi, int nrhs, double alpha, int n, double norm,
                   fl_where where);

/* APE smearing of the spatial links that enter the Gaussian smearing kernel
 * H (Sec. III applies it; the paper states neither its form nor its
 * parameters): n steps of, for i = 1..3,
 *   U'_i(x) = P[ U_i(x) + alpha sum_{j=1..3, j != i} ( U_j(x) U_i(x+j) U_j(x+i)^+
 *                                               + U_j(x-j)^+ U_i(x-j) U_j(x-j+i) ) ],
 * P(V) = W exp(-i arg(det W) / 3) with W the unitary factor of the polar
 * decomposition V = W (V^+ V)^{1/2} and arg in (-pi, pi] (an SU(3) matrix;
 * V must be nonsingular).  The time links are unchanged.  FP64.  The
 * smeared links stay in the context and are used by fl_smear and
 * fl_pion_corr (the Dirac operator keeps the unsmeared links) until the
 * next fl_set_gauge or a call with n = 0, which returns to the unsmeared
 * links.  Uout: NULL, or [4][V][3][3][2] in `where` memory receiving the
 * smeared field.  alpha >= 0 finite, n >= 0. */
fl_status fl_ape_smear(fl_ctx *ctx, double alpha, int n, double *Uout, fl_where where);

/* Connected pseudoscalar two-point function (Sec. III, Eq. all_corr with
 * Gamma_A = Gamma_B = g5) from a point source at lexicographic site y0,
 * smeared at the source and/or the sink with F of fl_smear:
 *   C[k][t] = sum_x exp(+i p_k.(x - y0)) sum_{b, beta} |phi_{b,beta}(x, t0 + t)|^2,
 *   phi = F_sink D^-1 F_source e_{y0, b, beta}  (g5-hermiticity),
 * t counted from the source timeslice t0 (mod T); mom: nmom integer vectors
 * (host); C: [nmom][T][2] on the host or the device (`where`).  The 12
 * solves use params p (stopping rule on the full operator).  Needs
 * Lx + Ly + Lz <= 1024, as fl_momentum_project.  With local
 * fields (no smearing) and the disconnected part D(t) of
 * fl_disconnected_corr at p = 0 and Gamma = g5, the flavour-singlet
 * correlator of two degenerate flavours is C_pi(t) - 2 D(t). */
fl_status fl_pion_corr(fl_ctx *ctx, long long y0, const fl_solver_params *p, double alpha, int n,
                       double norm, int smear_source, int smear_sink, const int *mom, int nmom,
                       double *C, fl_where where);

/* Per-solve statistics of the last call on ctx that solved (fl_solve,
 * fl_loops_exact, fl_loops_exact_sites, fl_loops_stochastic, its share of
 * fl_loops_stochastic_multi, fl_loops_grad, fl_pion_corr), one entry per
 * right-hand side in the order of that call: fl_solve its right-hand
 * sides; the exact loops and the gradient 12 per site (12 k + 3 spin +
 * colour for the k-th site solved); the stochastic loops one per dilution
 * component, for each LP noise vector (time, spin, colour, space class,
 * the slowest first), then for each HP noise vector its LP solves followed
 * by its HP solves; fl_pion_corr the 12 spin-colour sources.  *n receives
 * the count; at most cap entries are written to stats (host memory; NULL
 * with cap 0 asks for the count only).  A call that failed before solving
 * leaves the previous statistics in place. */
fl_status fl_last_stats(const fl_ctx *ctx, fl_solver_stats *stats, long long cap, long long *n);

/* Text of the last error of ctx (or of the last failed fl_create when ctx
 * is NULL). */
const char *fl_last_error(const fl_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* FLOOP_H */

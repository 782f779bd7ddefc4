// fl_host.h -- internal declarations shared by the host side of the loop
// library: kernel argument blocks, launchers, the context object and the
// batched Schur solver.  Not part of the public ABI (include/floop.h).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "fl_common.h"
#include "floop.h"

// ---------------------------------------------------------------------------
// kernel argument blocks
// ---------------------------------------------------------------------------
// Operator formats of the hopping kernel: link storage, and with it the
// storage of the spinor fields it reads and writes (FP64 for LINK_F64_R18,
// 16-bit fixed point for LINK_Q16_R12, FP32 otherwise)
enum LinkFormat { LINK_F64_R18 = 0, LINK_F32_R18 = 1, LINK_F32_R12 = 2, LINK_BF16_R12 = 3, LINK_Q16_R12 = 4,
                  LINK_NFMT = 5 };
enum VecFormat { VEC_F64 = 0, VEC_F32 = 1, VEC_H16 = 2 };

inline VecFormat vec_format(LinkFormat f)
{
    return f == LINK_F64_R18 ? VEC_F64 : (f == LINK_Q16_R12 ? VEC_H16 : VEC_F32);
}

// bytes of one site of one right-hand side of a spinor field / of one link
inline size_t vec_site_bytes(VecFormat v) { return v == VEC_F64 ? 192 : (v == VEC_F32 ? 96 : 52); }
inline size_t link_bytes(LinkFormat f)
{
    return f == LINK_F64_R18 ? 144 : (f == LINK_F32_R18 ? 72 : (f == LINK_F32_R12 ? 48 : 24));
}

enum {
    EPI_PLAIN = 0,      // out = cb * H in
    EPI_XPAY = 1,       // out = ca * x + cb * H in
    EPI_DOTY = 2,       // partial slots slot0, slot0+1: <y, out>
    EPI_DOTX_NORM = 4,  // slots slot0, slot0+1: <out, x>; slot0+2: |out|^2
    EPI_NORM = 8,       // slot0+2: |out|^2
    EPI_SUBY16 = 16,    // FP64 fields only: out -= y, y a 16-bit field (its decoded values)
    EPI_CGZ = 32,       // with EPI_XPAY: out = y - alpha (ca x + cb H in), alpha = st[sys].alpha[0]
    EPI_ACCX = 64,      // with EPI_SUBY16 or EPI_SUBY32: also w += y (FP64 += the values of y), then y = 0
                        // (CGNR: z -= alpha Dhat^+ q, y = z updated in place)
    EPI_SUBY32 = 128    // FP64 fields only: out -= y, y an FP32 field
};

struct SysState;

struct DslashArgs {
    BatchGeom B;
    int par;  // output parity
    int slot0;
    int nsys;
    const int *mask;  // per-system: skip the right-hand side when 0 (may be null)
    double *partial;
    const void *in[FL_MAXLAT];
    void *out[FL_MAXLAT];
    const void *x[FL_MAXLAT];
    const void *y[FL_MAXLAT];
    const void *gauge[FL_MAXLAT];
    double ca[FL_MAXLAT], cb[FL_MAXLAT];
    int lds;    // 0: neighbours from memory; 1: x/y neighbours from an LDS window;
                // 2: also the workgroup's links staged in LDS once
    int wsmax;  // LDS window length in sites (64 + 2 * max Lx/2), set by the launcher
    const SysState *st;  // per-system scalars (EPI_CGZ)
    void *w[FL_MAXLAT];  // the FP64 field of EPI_ACCX
};

bool dslash_epi_supported(int epi);
// A dispatcher asked for a kernel variant that is not built records it here
// instead of launching nothing silently; hip_check() turns it into
// FL_ERR_ARG at the caller's next check of the stream.
void launch_unsupported(const char *what);
const char *take_launch_error();
// LDS bytes the staged kernel needs for RT right-hand sides
size_t dslash_lds_bytes(LinkFormat fmt, int RT, int wsmax, int lds);
void launch_dslash(LinkFormat fmt, const DslashArgs &a, bool dag, int epi, hipStream_t s);
// out = H in in FP64 arithmetic with FP64 links on a 16-bit input field (its
// decoded values, widened exactly), FP64 output; RT <= 8
// hop of a 16-bit or FP32 field (yf: VEC_H16 or VEC_F32) with FP64 links
// into an FP64 field, in FP64 arithmetic, no epilogue
void launch_dslash_wide(const DslashArgs &a, VecFormat yf, bool dag, hipStream_t s);

// per-system Krylov state kept on the device
struct SysState {
    double rho[2], alpha[2], omega[2], beta[2];
    double rr;      // |r|^2 of the iteration residual
    double stop2;   // iteration stops when rr <= stop2
    double tstop2;  // true residual target^2
    double rmax2;   // largest rr since the last residual replacement
    double delta2;  // replacement trigger: rr < delta2 * rmax2
    double tr2;     // last FP64 true residual^2
    double zz;      // CGNR: |z|^2
    int iter, max_iter;
    int flags;
    int xstamp;  // CGNR: iteration stamp whose x update (x += alpha p) is still to be applied
};

enum {
    ST_CONV_ITER = 1,  // iteration residual reached stop2
    ST_BREAK = 2,      // Krylov breakdown
    ST_MAXIT = 4,      // iteration budget exhausted
    ST_WANT_UPD = 8    // residual dropped by delta since the last replacement
};

enum BlasOp {
    OP_BICG_S = 0,    // f0 r, f1 v, f2 s:            s = r - alpha v
    OP_BICG_XR,       // f0 x, f1 p, f2 s, f3 t, f4 r, f5 r0: x += a p + w s; r = s - w t; <r0,r>, |r|^2
    OP_BICG_P,        // f0 p, f1 r, f2 v:            p = r + beta (p - omega v)
    OP_HI_TO_LO,      // f0 lo (out), f1 hi (FP64), f2 r0, f3 p, f4 xlo; flag 1: init r0 = p = lo, xlo = 0
    OP_ACC_HI,        // f0 hi (FP64) += f1 lo; flag 1: lo = 0
    OP_SUB_HI,        // f0 out (FP64) = f1 - f2 (FP64)
    OP_NORM,          // |f0|^2 -> slot0+2
    OP_ZERO,          // f0 = 0
    OP_CG_R,          // CGNR (truncated solves): f0 r -= a q (f1 q), |r|^2; real a = zz/qq
    OP_CG_P,          // CGNR: f0 p = f1 z + beta p
    OP_CG_PX,         // CGNR: f2 x += a p where the state carries this launch's stamp, then
                      //       f0 p = f1 z + beta p for the masked (active) systems
    OP_DOT,           // <f0, f1> = sum conj(f0) f1 -> slots slot0, slot0 + 1
    OP_CG_FIXP        // CGNR after a residual replacement: f0 p += c f1 z, complex c = beta[0..1]
};

struct BlasArgs {
    BatchGeom B;
    int op;
    int flag;
    int slot0;
    int nsys;
    const int *mask;
    double *partial;
    SysState *st;
    int stamp;  // iteration stamp (OP_CG_PX)
    void *f[6][FL_MAXLAT];
};

// precision of the fields of a BLAS launch: FP64 (all fields) or FP32 (all
// fields except the FP64 "hi" operands named above)
void launch_blas(VecFormat vf, const BlasArgs &a, hipStream_t s);

enum ScalStep { SC_ALPHA = 0, SC_OMEGA, SC_BETA, SC_RESET, SC_INIT, SC_CG_INIT, SC_CG_ALPHA, SC_CG_BETA, SC_CG_REZ };

struct ScalArgs {
    BatchGeom B;
    int step;
    int nsys;
    int *active;
    const int *mask;  // systems to process (null: all active)
    const double *partial;
    SysState *st;
    int stamp;  // iteration stamp, recorded by SC_CG_BETA
    int carried_r;  // SC_CG_BETA: |r|^2 of a carried residual in slot 5 (else the scalar recurrence)
};
void launch_scalars(const ScalArgs &a, hipStream_t s);

// ---------------------------------------------------------------------------
// field kernels (layouts, sources, contractions, gradient)
// ---------------------------------------------------------------------------
// canonical double[n][V][4][3][2] <-> device (even, odd) FP64 fields
void launch_canon_to_eo(const double *canon, double2 *even, double2 *odd, const LatGeom &g,
                        int nrhs, hipStream_t s);
void launch_eo_to_canon(const double2 *even, const double2 *odd, double *canon,
                        const LatGeom &g, int nrhs, hipStream_t s);
// canonical links double[4][V][3][3][2] -> [mu][par][NC][Vh] in the format fmt
void launch_pack_links(const double *canon, void *dst, LinkFormat fmt, const LatGeom &g,
                       hipStream_t s);
// SU(3) deviation: max over links of |U U^+ - 1| and |det U - 1| -> dev[0]
void launch_su3_check(const double *canon, double *dev_max, long long nlinks, hipStream_t s);

// point sources: rhs j = 12*k + 3*spin + colour at lexicographic site sites[k]
// momentum projection Lp[g][k][t] = sum_x exp(i p_k.x) L[g][t][x] (device
// arrays; dmom: device [nmom][3]) on stream s
void launch_momproj(const double2 *L, double2 *Lp, const int *dmom, int ngamma, int nt, int nmom, const int L4[4],
                    hipStream_t s);
// the spatial extents the projection's per-axis phase tables hold (Lx + Ly + Lz <= 1024)
bool momproj_fits(const int L4[4]);
void launch_point_sources(double2 *even, double2 *odd, const long long *sites, int nsites,
                          const LatGeom &g, hipStream_t s);

// per right-hand side of a stochastic batch: dilution component and noise
// index, and where its contraction goes (JOB_INTS ints each)
enum { JOB_T = 0, JOB_SPIN, JOB_COL, JOB_CLASS, JOB_R, JOB_TARGET, JOB_SIGN, JOB_INTS = 8 };

struct NoiseBatch {
    int type;
    unsigned long long seed;
    int dil;             // FL_DIL_* mask
    int ncomp;           // right-hand sides in this batch
    const int *job;      // device: JOB_INTS ints per right-hand side (-1 = not diluted)
};
void launch_noise_sources(double2 *even, double2 *odd, const NoiseBatch &nb, const LatGeom &g,
                          hipStream_t s);

// exact-loop contraction for nsites point-source sites (12 rhs each)
struct ExactContractArgs {
    LatGeom g;
    int nsites;
    const long long *sites;   // device, lexicographic
    const double2 *xe;        // solutions, even parity, rhs-major
    const double2 *be, *bo;   // sources (even, odd)
    const double2 *gauge;     // FP64 links [mu][par][9][Vh]
    double kappa;
    int ngamma;
    const double *gam;        // device [ngamma][4][4][2]
    double2 *L;               // [ngamma][L_stride] complex
    long long L_stride;       // entries per Gamma in L
    long long L_off;          // first entry for this batch
    double2 *S;               // [L_stride][16] or null
};
void launch_exact_contract(const ExactContractArgs &a, hipStream_t s);

// stochastic contraction: acc[gamma][t - t_begin][xs] += w * eta^+ Gamma phi
struct StochContractArgs {
    LatGeom g;
    int nrhs;
    const double2 *pe, *po;   // phi (even, odd), rhs-major
    const double2 *ne, *no;   // eta (even, odd), rhs-major
    const int *job;           // JOB_INTS per rhs: dilution component, target accumulator, sign
    int dil;
    int t_begin, t_end;
    int ngamma;
    const double *gam;
    double2 *acc0, *acc1;     // accumulators [ngamma][nt][Vs] for targets 0 and 1
};
void launch_stoch_contract(const StochContractArgs &a, hipStream_t s);
void launch_tsm_combine(double *a0, const double *a1, double w0, double w1, long long n, hipStream_t s);

// gradient kernels
struct ChiArgs {
    LatGeom g;
    int nsites;
    const long long *sites;   // device lexicographic sites of the batch (12 rhs each)
    const double2 *M;         // device [nsites][4][4] complex: sum_Gamma w g5 Gamma^+
    const double2 *pe, *po;   // psi (even, odd)
    double2 *ce, *co;         // chi (even, odd)
};
void launch_chi(const ChiArgs &a, hipStream_t s);

struct ForceArgs {
    LatGeom g;
    int nrhs;
    const double2 *pe, *po, *ce, *co;
    double kappa;
    double2 *dU;              // canonical [4][V][3][3] complex, accumulated
};
void launch_force(const ForceArgs &a, hipStream_t s);

// dot products <a, b> over both parities for nrhs fields -> partial sums
void launch_dot64(const double2 *a, const double2 *b, long long n, double *out2, hipStream_t s);

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct ProfSlot {
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    double bytes = 0;
    long long launches = 0;
};

struct fl_ctx {
    int device = 0;
    int L[4] = {0, 0, 0, 0};
    int bc_t = -1;
    long long V = 0, Vh = 0, Vs = 0;
    hipStream_t stream = nullptr;
    double kappa = 0;
    bool have_kappa = false;
    bool have_gauge = false;
    bool su3 = false;  // links are SU(3) to 1e-10 (12-real storage allowed)
    void *gauge[LINK_NFMT] = {};     // per LinkFormat, built on demand
    bool gauge_ok[LINK_NFMT] = {};   // packed from the current links
    double *gauge_canon = nullptr;                          // device copy of the input links
    std::string err;
    std::vector<DevBuf> pool;  // named workspace buffers
    ProfSlot prof[FL_PROF_NKERNELS];
    int tune_rt[LINK_NFMT] = {};                   // per LinkFormat; 0: heuristic
    int tune_g[LINK_NFMT] = {};
    int tune_lds[LINK_NFMT] = {-1, -1, -1, -1, -1};  // LDS staging mode; -1: built-in choice
    size_t max_lds = 65536;              // LDS bytes a workgroup may use on this device
    std::vector<fl_solver_stats> last_stats;  // per-solve statistics of the last solving call
    void *smear_gauge = nullptr;  // APE-smeared FP64 links (LINK_F64_R18 layout) for Gaussian smearing
    bool smear_ok = false;        // smear_gauge holds the smearing of the current links
    void *pinned = nullptr;       // page-locked host staging of the solver's per-system state and masks
    size_t pinned_bytes = 0;
};

// page-locked host memory of at least `bytes` owned by the context (grown,
// contents not kept; the stream is synchronised before an old block is freed)
void *pinned_get(fl_ctx *c, size_t bytes);

// LDS staging mode and window length for a hopping launch over batch B
void dslash_config(const fl_ctx *c, LinkFormat fmt, DslashArgs &a);

fl_status set_err(fl_ctx *c, fl_status st, const std::string &msg);
fl_status hip_check(fl_ctx *c, hipError_t e, const char *what);
// workspace buffer `slot` of at least `bytes` (grown, contents not kept)
void *ws_get(fl_ctx *c, int slot, size_t bytes);
void *links(fl_ctx *c, LinkFormat fmt);  // device links in that format (built on first use)
LatGeom lat_geom(const fl_ctx *c, int nrhs);
BatchGeom batch_geom(fl_ctx *const *ctx, const int *nrhs, int nlat, int RT, int G = 1 << 20);
// workgroup shape of the batched kernels for link format fmt and nrhs
// right-hand sides: RT waves (right-hand sides) per workgroup and G
// right-hand-side blocks per site sweep (the autotuner's choice if any)
void tile_shape(const fl_ctx *c, int fmt, int nrhs, int *RT, int *G);
// single-lattice hopping launch on FP64 fields with the given FP64 links:
// out = ca x + cb H in (x may be null: out = cb H in); epi < 0: XPAY if x
void hop64_launch(fl_ctx *c, const void *gauge, int nrhs, int par, const void *in, void *out, const void *x,
                  double ca, double cb, bool dag, int epi = -1);
// size of the fixed device scratch array of fl_apply_D_noalloc (MiB)
#define FL_NOALLOC_SCRATCH_MB 64
// takes the device address of that array on `device` (once; call with the
// device current)
hipError_t noalloc_scratch_setup(int device);
// kernel profiling hooks (events on the context stream)
void prof_begin(fl_ctx *c, int kernel);
void prof_end(fl_ctx *c, int kernel, double bytes);

// workspace slots
enum {
    WS_CANON = 0, WS_BE, WS_BO, WS_XE, WS_XO, WS_BH, WS_RH, WS_T64, WS_R, WS_R0, WS_P, WS_V, WS_S,
    WS_T, WS_XL, WS_TMP, WS_PART, WS_STATE, WS_MASK, WS_SITES, WS_GAM, WS_ACC,
    WS_ACC2, WS_COMP, WS_M, WS_CE, WS_CO, WS_DU, WS_HE, WS_HO, WS_XE2, WS_XO2, WS_MISC,
    WS_CORR_A, WS_CORR_B, WS_CORR_OUT, WS_CORR_IDX, WS_SM_E0, WS_SM_O0, WS_SM_E1, WS_SM_O1, WS_PI_SRC,
    WS_PI_SOL, WS_PI_RHO, WS_APE0, WS_APE1,
    WS_NSLOTS
};

// ---------------------------------------------------------------------------
// batched Schur solve: Dhat x_e = bhat_e for every right-hand side of up to
// FL_MAXLAT lattices at once (bhat_e, x_e FP64 even fields, rhs-major)
// ---------------------------------------------------------------------------
struct SolveBatch {
    int nlat = 0;
    fl_ctx *ctx[FL_MAXLAT] = {nullptr, nullptr, nullptr, nullptr};
    int nrhs[FL_MAXLAT] = {0, 0, 0, 0};
    const double2 *bh[FL_MAXLAT] = {nullptr, nullptr, nullptr, nullptr};
    double2 *xh[FL_MAXLAT] = {nullptr, nullptr, nullptr, nullptr};
    std::vector<double> bnorm;  // |b| of the full source, per system (host)
};

struct SysResult {
    int iters = 0, updates = 0, converged = 0, flags = 0;
    double true_resid = 0;
};

fl_status solve_schur_batch(SolveBatch &sb, const fl_solver_params &p,
                            std::vector<SysResult> &res);
// xh = Dhat bh (dag: Dhat^+ bh) for every system of the batch, computed in
// the iteration precision and link storage of p
fl_status schur_apply_batch(SolveBatch &sb, const fl_solver_params &p, bool dag);

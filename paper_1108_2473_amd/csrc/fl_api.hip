// fl_api.hip -- the C ABI (include/floop.h): contexts, gauge ingest, and the
// drivers that turn the paper's loop estimators into batches of Schur
// solves on the device.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "fl_host.h"

void hop64_launch(fl_ctx *c, const void *gauge, int nrhs, int par, const void *in, void *out, const void *x,
                  double ca, double cb, bool dag, int epi)
{
    int RT, G;
    tile_shape(c, LINK_F64_R18, nrhs, &RT, &G);
    fl_ctx *cs[1] = {c};
    int nr[1] = {nrhs};
    DslashArgs a;
    std::memset(&a, 0, sizeof(a));
    a.B = batch_geom(cs, nr, 1, RT, G);
    a.par = par;
    a.nsys = nrhs;
    a.in[0] = in;
    a.out[0] = out;
    a.x[0] = x;
    a.gauge[0] = gauge;
    a.ca[0] = ca;
    a.cb[0] = cb;
    if (epi < 0) epi = x ? EPI_XPAY : EPI_PLAIN;
    dslash_config(c, LINK_F64_R18, a);
    launch_dslash(LINK_F64_R18, a, dag, epi, c->stream);
}

namespace {

thread_local std::string g_last_error;

#ifndef FL_SRC_HASH
#define FL_SRC_HASH "unknown"
#endif
// the hash names the kernel sources the library was built from
const char *kVersion = "floop 0.2 (gfx950) src " FL_SRC_HASH;

// Dirac matrices of the chiral basis, g_k = [[0, -i s_k], [i s_k, 0]],
// g_4 = [[0, 1], [1, 0]], and products Gamma(mask) = g1^b0 g2^b1 g3^b2 g4^b3
struct C {
    double re, im;
};
C cmul(C a, C b) { return C{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }

void gamma_mu(int mu, C G[4][4])
{
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) G[i][j] = C{0, 0};
    if (mu == 3) {
        G[0][2] = G[1][3] = G[2][0] = G[3][1] = C{1, 0};
        return;
    }
    // s_k entries
    C s[3][2][2] = {{{C{0, 0}, C{1, 0}}, {C{1, 0}, C{0, 0}}},
                    {{C{0, 0}, C{0, -1}}, {C{0, 1}, C{0, 0}}},
                    {{C{1, 0}, C{0, 0}}, {C{0, 0}, C{-1, 0}}}};
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            C v = s[mu][i][j];
            G[i][2 + j] = C{v.im, -v.re};   // -i s
            G[2 + i][j] = C{-v.im, v.re};   // +i s
        }
}

void gamma_of_mask(int mask, C out[4][4])
{
    C G[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) G[i][j] = C{i == j ? 1.0 : 0.0, 0};
    for (int mu = 0; mu < 4; ++mu) {
        if (!(mask & (1 << mu))) continue;
        C g[4][4], T[4][4];
        gamma_mu(mu, g);
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                C acc{0, 0};
                for (int k = 0; k < 4; ++k) {
                    C p = cmul(G[i][k], g[k][j]);
                    acc.re += p.re;
                    acc.im += p.im;
                }
                T[i][j] = acc;
            }
        std::memcpy(G, T, sizeof(G));
    }
    std::memcpy(out, G, sizeof(G));
}

std::vector<double> gamma_table(const int *gammas, int ngamma)
{
    std::vector<double> t(32 * (size_t)ngamma);
    for (int k = 0; k < ngamma; ++k) {
        C G[4][4];
        gamma_of_mask(gammas[k], G);
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                t[32 * k + 2 * (4 * i + j)] = G[i][j].re;
                t[32 * k + 2 * (4 * i + j) + 1] = G[i][j].im;
            }
    }
    return t;
}

bool valid_ctx(const fl_ctx *c) { return c != nullptr; }

fl_status check_ready(fl_ctx *c)
{
    if (!c->have_gauge) return set_err(c, FL_ERR_STATE, "gauge field not set (fl_set_gauge)");
    if (!c->have_kappa) return set_err(c, FL_ERR_STATE, "kappa not set (fl_set_kappa)");
    return FL_OK;
}

fl_status check_params(fl_ctx *c, const fl_solver_params *p)
{
    if (!p) return set_err(c, FL_ERR_ARG, "solver params are NULL");
    if (!(p->tol > 0) || !std::isfinite(p->tol)) return set_err(c, FL_ERR_ARG, "tol must be > 0");
    if (p->solver != FL_SOLVER_BICGSTAB && p->solver != FL_SOLVER_CGNR)
        return set_err(c, FL_ERR_ARG, "unknown solver");
    if (p->inner_prec < FL_PREC_F64 || p->inner_prec > FL_PREC_H16)
        return set_err(c, FL_ERR_ARG, "unknown inner precision");
    if (p->gauge_reals != 18 && p->gauge_reals != 12) return set_err(c, FL_ERR_ARG, "gauge_reals must be 12 or 18");
    if (p->max_iter < 0 || p->batch < 0 || p->max_outer < 0)
        return set_err(c, FL_ERR_ARG, "negative max_iter, batch or max_outer");
    if ((p->inner_prec == FL_PREC_BF16 || p->inner_prec == FL_PREC_H16) && p->gauge_reals != 12)
        return set_err(c, FL_ERR_ARG, "bfloat16 and 16-bit fixed-point links are stored with 12 reals");
    if (p->inner_prec != FL_PREC_F64 && p->gauge_reals == 12 && !c->su3)
        return set_err(c, FL_ERR_ARG, "12-real links need SU(3) links; use gauge_reals = 18");
    return FL_OK;
}

// single-lattice hopping launch on FP64 fields
void hop64(fl_ctx *c, int nrhs, int par, const void *in, void *out, const void *x, double ca, double cb, bool dag,
           int epi = -1)
{
    hop64_launch(c, links(c, LINK_F64_R18), nrhs, par, in, out, x, ca, cb, dag, epi);
}

// |f|^2 per right-hand side of FP64 (even, odd) fields, summed on the host in
// a fixed order
fl_status norms64(fl_ctx *c, int nrhs, const void *fe, const void *fo, std::vector<double> &out)
{
    int RT, G;
    tile_shape(c, LINK_F64_R18, nrhs, &RT, &G);
    fl_ctx *cs[1] = {c};
    int nr[1] = {nrhs};
    BatchGeom B = batch_geom(cs, nr, 1, RT, G);
    size_t np = 6 * (size_t)nrhs * B.nsb_max;
    double *part = (double *)ws_get(c, WS_MISC, np * sizeof(double));
    if (!part) return set_err(c, FL_ERR_NOMEM, "device allocation failed (norms)");
    fl_status e;
    if ((e = hip_check(c, hipMemsetAsync(part, 0, np * sizeof(double), c->stream), "memset"))) return e;
    BlasArgs a;
    std::memset(&a, 0, sizeof(a));
    a.B = B;
    a.op = OP_NORM;
    a.nsys = nrhs;
    a.partial = part;
    a.slot0 = 0;
    a.f[0][0] = (void *)fe;
    launch_blas(VEC_F64, a, c->stream);
    a.slot0 = 3;
    a.f[0][0] = (void *)fo;
    launch_blas(VEC_F64, a, c->stream);
    // the two slots written (2 and 5), through the page-locked block
    const size_t per = (size_t)nrhs * B.nsb_max;
    double *h = (double *)pinned_get(c, 2 * per * sizeof(double));
    if (!h) return set_err(c, FL_ERR_NOMEM, "page-locked host allocation failed");
    if ((e = hip_check(c, hipMemcpyAsync(h, part + 2 * per, per * sizeof(double), hipMemcpyDeviceToHost, c->stream),
                       "download norms")))
        return e;
    if ((e = hip_check(c, hipMemcpyAsync(h + per, part + 5 * per, per * sizeof(double), hipMemcpyDeviceToHost,
                                         c->stream),
                       "download norms")))
        return e;
    if ((e = hip_check(c, hipStreamSynchronize(c->stream), "sync"))) return e;
    out.assign(nrhs, 0.0);
    const int nsb = B.lat[0].nsb, nb = B.nsb_max;
    for (int k = 0; k < nrhs; ++k) {
        double s = 0;
        for (int sb = 0; sb < nsb; ++sb) s += h[(size_t)k * nb + sb] + h[per + (size_t)k * nb + sb];
        out[k] = s;
    }
    return FL_OK;
}

// |b - D x|^2 per right-hand side on the full operator in FP64 for n
// right-hand sides of even/odd FP64 fields (x_o included), into r2 (host);
// uses the workspace slots WS_HE and WS_HO
fl_status full_residual2(fl_ctx *c, int n, const void *be, const void *bo, const void *xe, const void *xo,
                         std::vector<double> &r2)
{
    const size_t fb = (size_t)n * c->Vh * 192;
    void *he = ws_get(c, WS_HE, fb), *ho = ws_get(c, WS_HO, fb);
    if (!he || !ho) return set_err(c, FL_ERR_NOMEM, "device allocation failed (residual check)");
    // (D x)_e = x_e - k H_eo x_o, (D x)_o = x_o - k H_oe x_e
    hop64(c, n, 0, xo, he, xe, 1.0, -c->kappa, false);
    hop64(c, n, 1, xe, ho, xo, 1.0, -c->kappa, false);
    fl_ctx *cs[1] = {c};
    int nr[1] = {n};
    BlasArgs a;
    std::memset(&a, 0, sizeof(a));
    int RT, G;
    tile_shape(c, LINK_F64_R18, n, &RT, &G);
    a.B = batch_geom(cs, nr, 1, RT, G);
    a.op = OP_SUB_HI;
    a.nsys = n;
    a.f[0][0] = he;
    a.f[1][0] = (void *)be;
    a.f[2][0] = he;
    launch_blas(VEC_F64, a, c->stream);
    a.f[0][0] = ho;
    a.f[1][0] = (void *)bo;
    a.f[2][0] = ho;
    launch_blas(VEC_F64, a, c->stream);
    return norms64(c, n, he, ho, r2);
}

// statistics of one solve, stored at index idx of the context's last-call list
void put_stats(fl_ctx *c, size_t idx, const SysResult &r, bool truncated, double bnorm2, double r2, double tol,
               double secs)
{
    if (c->last_stats.size() <= idx) c->last_stats.resize(idx + 1);
    fl_solver_stats &s = c->last_stats[idx];
    s.iters = r.iters;
    s.updates = r.updates;
    s.seconds = secs;
    if (truncated) {
        s.true_resid = r.true_resid;
        s.converged = r.converged;
    } else {
        s.true_resid = bnorm2 > 0 ? std::sqrt(r2 / bnorm2) : std::sqrt(r2);
        s.converged = s.true_resid <= tol ? 1 : 0;
    }
}

// status of one solve from its statistics
fl_status solve_status(const fl_solver_stats &s, const SysResult &r)
{
    if (s.converged) return FL_OK;
    return (r.flags & ST_BREAK) ? FL_ERR_BREAKDOWN : FL_ERR_NOCONV;
}

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// default right-hand sides per device batch: about `budget` bytes of vectors
int default_batch(const fl_ctx *c, int multiple)
{
    // per right-hand side and checkerboard site: up to 11 FP64 fields (sources,
    // solutions, residuals, gradient work) and 8 iteration vectors
    const double per_rhs = 3700.0 * c->Vh;
    const double budget = 64e9;
    int n = (int)std::min(1536.0, std::max(1.0, budget / per_rhs));
    n = std::max(multiple, n - n % multiple);
    return n;
}

fl_status copy_out(fl_ctx *c, void *dst, const void *src, size_t bytes, fl_where where)
{
    return hip_check(c, hipMemcpyAsync(dst, src, bytes, where == FL_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                       c->stream),
                     "copy out");
}

}  // namespace

// ---------------------------------------------------------------------------
// internal helpers declared in fl_host.h
// ---------------------------------------------------------------------------
fl_status set_err(fl_ctx *c, fl_status st, const std::string &msg)
{
    if (c) c->err = msg;
    g_last_error = msg;
    return st;
}

namespace {
thread_local const char *g_launch_error = nullptr;
}

void launch_unsupported(const char *what)
{
    if (!g_launch_error) g_launch_error = what;
}

const char *take_launch_error()
{
    const char *w = g_launch_error;
    g_launch_error = nullptr;
    return w;
}

fl_status hip_check(fl_ctx *c, hipError_t e, const char *what)
{
    if (const char *le = take_launch_error())
        return set_err(c, FL_ERR_ARG, std::string(what) + ": internal: kernel variant not built (" + le + ")");
    if (e == hipSuccess) return FL_OK;
    return set_err(c, e == hipErrorOutOfMemory ? FL_ERR_NOMEM : FL_ERR_DEVICE,
                   std::string(what) + ": " + hipGetErrorString(e));
}

void *pinned_get(fl_ctx *c, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    if (c->pinned_bytes >= bytes) return c->pinned;
    if (c->pinned) {
        hipStreamSynchronize(c->stream);
        hipHostFree(c->pinned);
        c->pinned = nullptr;
        c->pinned_bytes = 0;
    }
    if (hipHostMalloc(&c->pinned, bytes, hipHostMallocDefault) != hipSuccess) {
        c->pinned = nullptr;
        (void)hipGetLastError();
        return nullptr;
    }
    c->pinned_bytes = bytes;
    return c->pinned;
}

void *ws_get(fl_ctx *c, int slot, size_t bytes)
{
    if ((int)c->pool.size() < WS_NSLOTS) c->pool.resize(WS_NSLOTS);
    DevBuf &b = c->pool[slot];
    if (bytes == 0) bytes = 256;
    if (b.bytes >= bytes) return b.p;
    if (b.p) {
        hipStreamSynchronize(c->stream);
        hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
    }
    if (hipMalloc(&b.p, bytes) != hipSuccess) {
        b.p = nullptr;
        (void)hipGetLastError();
        return nullptr;
    }
    b.bytes = bytes;
    return b.p;
}

LatGeom lat_geom(const fl_ctx *c, int nrhs)
{
    LatGeom g;
    std::memset(&g, 0, sizeof(g));
    for (int mu = 0; mu < 4; ++mu) g.L[mu] = c->L[mu];
    g.Lh0 = c->L[0] / 2;
    g.Vh = (int)c->Vh;
    g.bc_t = c->bc_t;
    g.nsb = (g.Vh + FL_WAVE - 1) / FL_WAVE;
    g.nrhs = nrhs;
    g.fLh0 = make_fastdiv((unsigned)g.Lh0);
    g.fLy = make_fastdiv((unsigned)g.L[1]);
    g.fLz = make_fastdiv((unsigned)g.L[2]);
    g.fnsb = make_fastdiv((unsigned)g.nsb);
    return g;
}

BatchGeom batch_geom(fl_ctx *const *ctx, const int *nrhs, int nlat, int RT, int G)
{
    BatchGeom B;
    std::memset(&B, 0, sizeof(B));
    B.nlat = nlat;
    B.RT = RT;
    B.G = G > 0 ? G : 1;
    int tiles = 0, sys = 0;
    for (int l = 0; l < nlat; ++l) {
        LatGeom g = lat_geom(ctx[l], nrhs[l]);
        g.sys0 = sys;
        g.nrb = (nrhs[l] + RT - 1) / RT;
        g.tile0 = tiles;
        tiles += g.nsb * g.nrb;
        sys += nrhs[l];
        B.nsb_max = std::max(B.nsb_max, g.nsb);
        B.lat[l] = g;
    }
    B.ntiles = tiles;
    return B;
}

void tile_shape(const fl_ctx *c, int fmt, int nrhs, int *RT, int *G)
{
    const int maxrt = fmt == LINK_F64_R18 ? 8 : 16;
    // built-in choice (measured on the 16^3x32 hopping kernel with 384
    // right-hand sides): 8 right-hand sides per workgroup, swept
    // right-hand-side-block by block so that the stencil's neighbours are
    // still in L2 when reused (FP64 with staged links: 3483 us per launch,
    // against 4391 us for 2 right-hand sides per workgroup with windows)
    int rt = c->tune_rt[fmt] > 0 ? c->tune_rt[fmt] : 8;
    // no more waves per workgroup than right-hand sides (next power of two)
    int cap = 1;
    while (cap < nrhs && cap < maxrt) cap *= 2;
    *RT = std::max(1, std::min(std::min(rt, maxrt), cap));
    *G = c->tune_g[fmt] > 0 ? c->tune_g[fmt] : 1;
}

void dslash_config(const fl_ctx *c, LinkFormat fmt, DslashArgs &a)
{
    // LDS window: the (z, t) planes that the 64 sites of a block lie in
    int ws = 0;
    for (int l = 0; l < a.B.nlat; ++l) {
        const LatGeom &g = a.B.lat[l];
        const int plane = g.Lh0 * g.L[1];
        for (int i0 = 0; i0 < g.Vh; i0 += FL_WAVE) {
            int lo = (i0 / plane) * plane;
            int hi = std::min(g.Vh, (std::min(i0 + FL_WAVE, g.Vh) - 1) / plane * plane + plane);
            ws = std::max(ws, hi - lo);
            if (plane % FL_WAVE == 0 && i0 >= plane) break;  // every block alike
        }
    }
    a.wsmax = (ws + 3) & ~3;  // 16-byte aligned windows for every site format
    int mode = c->tune_lds[fmt];
    // built-in (measured at 16^3x32): staged links and no windows (16-bit
    // fields: the packed hop; FP32 and bf16: 1611 and 1567 us against 1708
    // and 1651 us with windows, whose LDS held a CU to one workgroup; FP64
    // with 8 right-hand sides per workgroup: 3483 against 4554 us without
    // staging, its windows do not fit), except FP64 workgroups of fewer than
    // 4 right-hand sides (single solves), which keep the windows; a mode
    // that does not fit the LDS falls back to a smaller one
    if (mode < 0) mode = (fmt == LINK_F64_R18 && a.B.RT < 4) ? 1 : 4;
    if (mode == 3 && fmt != LINK_Q16_R12) mode = 2;  // the packed integer hop with windows: 16-bit fields only
    // a mode whose staging does not fit falls back: 4 -> 2 -> 1 -> 0 (3 -> 2 -> ...)
    while (mode > 0 && dslash_lds_bytes(fmt, a.B.RT, a.wsmax, mode) > c->max_lds)
        mode = (mode == 4 && fmt != LINK_Q16_R12) ? 2 : mode - 1;
    a.lds = mode;
}

void *links(fl_ctx *c, LinkFormat fmt)
{
    if (!c->have_gauge) return nullptr;
    if (!c->gauge[fmt]) {
        if (hipMalloc(&c->gauge[fmt], link_bytes(fmt) * 4 * (size_t)c->V) != hipSuccess) {
            c->gauge[fmt] = nullptr;
            (void)hipGetLastError();
            return nullptr;
        }
        c->gauge_ok[fmt] = false;
    }
    if (!c->gauge_ok[fmt]) {
        launch_pack_links(c->gauge_canon, c->gauge[fmt], fmt, lat_geom(c, 0), c->stream);
        c->gauge_ok[fmt] = true;
    }
    return c->gauge[fmt];
}

void prof_begin(fl_ctx *c, int kernel)
{
    ProfSlot &p = c->prof[kernel];
    if (!p.on) return;
    hipEvent_t a, b;
    hipEventCreate(&a);
    hipEventCreate(&b);
    hipEventRecord(a, c->stream);
    p.ev.push_back({a, b});
}

void prof_end(fl_ctx *c, int kernel, double bytes)
{
    ProfSlot &p = c->prof[kernel];
    if (!p.on || p.ev.empty()) return;
    hipEventRecord(p.ev.back().second, c->stream);
    p.bytes += bytes;
    p.launches += 1;
}

static void prof_reset(ProfSlot &p)
{
    for (auto &e : p.ev) {
        hipEventDestroy(e.first);
        hipEventDestroy(e.second);
    }
    p.ev.clear();
    p.bytes = 0;
    p.launches = 0;
}

// ---------------------------------------------------------------------------
// public ABI
// ---------------------------------------------------------------------------
extern "C" {

void fl_solver_params_default(fl_solver_params *p)
{
    if (!p) return;
    p->solver = FL_SOLVER_BICGSTAB;
    p->tol = 1e-12;
    p->max_iter = 20000;
    p->inner_prec = FL_PREC_F32;
    p->gauge_reals = 12;
    p->delta = 0.0;  // the solver picks its default for the inner precision
    p->truncated = 0;
    p->batch = 0;
    p->max_outer = 0;
}

const char *fl_version(void) { return kVersion; }

const char *fl_last_error(const fl_ctx *ctx)
{
    if (ctx) return ctx->err.c_str();
    return g_last_error.c_str();
}

fl_status fl_create(fl_ctx **out, int device, const int dims[4], int bc_t)
{
    if (!out) return set_err(nullptr, FL_ERR_ARG, "ctx pointer is NULL");
    *out = nullptr;
    if (!dims) return set_err(nullptr, FL_ERR_ARG, "dims is NULL");
    for (int mu = 0; mu < 4; ++mu)
        if (dims[mu] < 2 || dims[mu] % 2) return set_err(nullptr, FL_ERR_ARG, "lattice extents must be even and >= 2");
    if (bc_t != 1 && bc_t != -1) return set_err(nullptr, FL_ERR_ARG, "bc_t must be +1 or -1");
    // kernels address a whole link array (8 x 144 bytes per site pair in
    // FP64) through 32-bit buffer offsets; the volume is formed factor by
    // factor so that no product of four extents can overflow
    long long V = 1;
    for (int mu = 0; mu < 4; ++mu) {
        V *= dims[mu];
        if ((V / 2) * 8 * 144 >= (1LL << 31))
            return set_err(nullptr, FL_ERR_ARG, "lattice too large (V <= 3.7M sites)");
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        return set_err(nullptr, FL_ERR_DEVICE, "no HIP device available");
    }
    if (device < 0 || device >= ndev) return set_err(nullptr, FL_ERR_ARG, "device index out of range");
    if (hipSetDevice(device) != hipSuccess) return set_err(nullptr, FL_ERR_DEVICE, "hipSetDevice failed");
    fl_ctx *c = new fl_ctx();
    c->device = device;
    for (int mu = 0; mu < 4; ++mu) c->L[mu] = dims[mu];
    c->bc_t = bc_t;
    c->V = V;
    c->Vh = V / 2;
    c->Vs = (long long)dims[0] * dims[1] * dims[2];
    c->pool.resize(WS_NSLOTS);
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lds > 0)
        c->max_lds = (size_t)lds;
    // device address of the fixed scratch array of fl_apply_D_noalloc on this
    // device (once per device; a failure is reported by that entry point)
    (void)noalloc_scratch_setup(device);
    *out = c;
    return FL_OK;
}

fl_status fl_destroy(fl_ctx *c)
{
    if (!c) return FL_OK;
    hipSetDevice(c->device);
    hipStreamSynchronize(c->stream);
    for (auto &b : c->pool)
        if (b.p) hipFree(b.p);
    if (c->pinned) hipHostFree(c->pinned);
    for (int k = 0; k < LINK_NFMT; ++k)
        if (c->gauge[k]) hipFree(c->gauge[k]);
    if (c->gauge_canon) hipFree(c->gauge_canon);
    if (c->smear_gauge) hipFree(c->smear_gauge);
    for (auto &p : c->prof) prof_reset(p);
    delete c;
    return FL_OK;
}

fl_status fl_set_stream(fl_ctx *c, void *stream)
{
    if (!valid_ctx(c)) return set_err(nullptr, FL_ERR_ARG, "ctx is NULL");
    hipSetDevice(c->device);
    hipStreamSynchronize(c->stream);
    c->stream = (hipStream_t)stream;
    return FL_OK;
}

fl_status fl_set_kappa(fl_ctx *c, double kappa)
{
    if (!valid_ctx(c)) return set_err(nullptr, FL_ERR_ARG, "ctx is NULL");
    if (!(kappa > 0) || !std::isfinite(kappa)) return set_err(c, FL_ERR_ARG, "kappa must be finite and > 0");
    c->kappa = kappa;
    c->have_kappa = true;
    return FL_OK;
}

fl_status fl_set_gauge(fl_ctx *c, const double *U, fl_where where)
{
    if (!valid_ctx(c)) return set_err(nullptr, FL_ERR_ARG, "ctx is NULL");
    if (!U) return set_err(c, FL_ERR_ARG, "gauge pointer is NULL");
    hipSetDevice(c->device);
    size_t bytes = (size_t)4 * c->V * 18 * sizeof(double);
    fl_status e;
    if (!c->gauge_canon) {
        if ((e = hip_check(c, hipMalloc(&c->gauge_canon, bytes), "alloc links"))) {
            c->gauge_canon = nullptr;
            return e;
        }
    }
    if ((e = hip_check(c, hipMemcpyAsync(c->gauge_canon, U, bytes,
                                         where == FL_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                         c->stream),
                       "upload links")))
        return e;
    long long nlinks = 4 * c->V;
    long long nblk = (nlinks + 255) / 256;
    double *bm = (double *)ws_get(c, WS_MISC, nblk * sizeof(double));
    if (!bm) return set_err(c, FL_ERR_NOMEM, "device allocation failed");
    launch_su3_check(c->gauge_canon, bm, nlinks, c->stream);
    std::vector<double> h(nblk);
    if ((e = hip_check(c, hipMemcpyAsync(h.data(), bm, nblk * sizeof(double), hipMemcpyDeviceToHost, c->stream),
                       "su3 check")))
        return e;
    if ((e = hip_check(c, hipStreamSynchronize(c->stream), "sync"))) return e;
    double dev = 0;
    for (double v : h) dev = std::max(dev, v);
    if (!std::isfinite(dev)) return set_err(c, FL_ERR_ARG, "gauge field holds non-finite values");
    c->su3 = dev <= 1e-10;
    for (int k = 0; k < LINK_NFMT; ++k) c->gauge_ok[k] = false;
    c->smear_ok = false;  // APE-smeared links belong to the previous field
    c->have_gauge = true;
    if (!links(c, LINK_F64_R18)) return set_err(c, FL_ERR_NOMEM, "device allocation failed (links)");
    return hip_check(c, hipStreamSynchronize(c->stream), "pack links");
}

fl_status fl_apply_D(fl_ctx *c, const double *in, double *out, int nrhs, int dagger, fl_where where)
{
    if (!valid_ctx(c)) return set_err(nullptr, FL_ERR_ARG, "ctx is NULL");
    if (nrhs < 0 || (nrhs > 0 && (!in || !out))) return set_err(c, FL_ERR_ARG, "bad spinor arguments");
    fl_status e;
    if ((e = check_ready(c))) return e;
    hipSetDevice(c->device);
    const int chunk = std::max(1, std::min(nrhs, default_batch(c, 1)));
    const size_t per = (size_t)c->V * 24 * sizeof(double);
    for (int k0 = 0; k0 < nrhs; k0 += chunk) {
        int n = std::min(chunk, nrhs - k0);
        const double *src = in + (size_t)k0 * c->V * 24;
        double *dst = out + (size_t)k0 * c->V * 24;
        double *cin = (double *)src, *cout = dst;
        if (where == FL_HOST) {
            cin = (double *)ws_get(c, WS_CANON, per * n);
            cout = cin;
            if (!cin) return set_err(c, FL_ERR_NOMEM, "device allocation failed");
            if ((e = hip_check(c, hipMemcpyAsync(cin, src, per * n, hipMemcpyHostToDevice, c->stream), "upload")))
                return e;
        }
        size_t fb = (size_t)n * c->Vh * 192;
        void *be = ws_get(c, WS_BE, fb), *bo = ws_get(c, WS_BO, fb);
        void *xe = ws_get(c, WS_XE, fb), *xo = ws_get(c, WS_XO, fb);
        if (!be || !bo || !xe || !xo) return set_err(c, FL_ERR_NOMEM, "device allocation failed");
        LatGeom g = lat_geom(c, n);
        launch_canon_to_eo(cin, (double2 *)be, (double2 *)bo, g, n, c->stream);
        // (D psi)_e = psi_e - k H_eo psi_o, (D psi)_o = psi_o - k H_oe psi_e
        hop64(c, n, 0, bo, xe, be, 1.0, -c->kappa, dagger != 0);
        hop64(c, n, 1, be, xo, bo, 1.0, -c->kappa, dagger != 0);
        launch_eo_to_canon((double2 *)xe, (double2 *)xo, cout, g, n, c->stream);
        if (where == FL_HOST)
            if ((e = hip_check(c, hipMemcpyAsync(dst, cout, per * n, hipMemcpyDeviceToHost, c->stream), "download")))
                return e;
        if ((e = hip_check(c, hipStreamSynchronize(c->stream), "apply D"))) return e;
    }
    return hip_check(c, hipGetLastError(), "apply D");
}

fl_status fl_apply_schur(fl_ctx *c, const double *in, double *out, int nrhs, int dagger,
                         const fl_solver_params *p, fl_where where)
{
    if (!valid_ctx(c)) return set_err(nullptr, FL_ERR_ARG, "ctx is NULL");
    if (nrhs < 0 || (nrhs > 0 && (!in || !out))) return set_err(c, FL_ERR_ARG, "bad spinor arguments");
    fl_status e;
    if ((e = check_ready(c))) return e;
    if ((e = check_params(c, p))) return e;
    hipSetDevice(c->device);
    const int chunk = std::max(1, std::min(nrhs, p->batch > 0 ? p->batch : default_batch(c, 1)));
    const size_t per = (size_t)c->V * 24 * sizeof(double);
    for (int k0 = 0; k0 < nrhs; k0 += chunk) {
        int n = std::min(chunk, nrhs - k0);
        const double *src = in + (size_t)k0 * c->V * 24;
        double *dst = out + (size_t)k0 * c->V * 24;
        double *cin = (double *)src, *cout = dst;
        if (where == FL_HOST) {
            cin = (double *)ws_get(c, WS_CANON, per * n);
            cout = cin;
            if (!cin) return set_err(c, FL_ERR_NOMEM, "device allocation failed");
            if ((e = hip_check(c, hipMemcpyAsync(cin, src, per * n, hipMemcpyHostToDevice, c->stream), "upload")))
                return e;
        }
        size_t fb = (size_t)n * c->Vh * 192;
        void *be = ws_get(c, WS_BE, fb), *bo = ws_get(c, WS_BO, fb);
        void *xe = ws_get(c, WS_XE, fb), *xo = ws_get(c, WS_XO, fb);
        if (!be || !bo || !xe || !xo) return set_err(c, FL_ERR_NOMEM, "device allocation failed");
        LatGeom g = lat_geom(c, n);
        launch_canon_to_eo(cin, (double2 *)be, (double2 *)bo, g, n, c->stream);
        SolveBatch sb;
        sb.nlat = 1;
        sb.ctx[0] = c;
        sb.nrhs[0] = n;
        sb.bh[0] = (const double2 *)be;
        sb.xh[0] = (double2 *)xe;
        sb.bnorm.assign(n, 1.0);
        if ((e = schur_apply_batch(sb, *p, dagger != 0))) return e;
        if ((e = hip_check(c, hipMemsetAsync(xo, 0, fb, c->stream), "memset"))) return e;
        launch_eo_to_canon((double2 *)xe, (double2 *)xo, cout, g, n, c->stream);
        if (where == FL_HOST)
            if ((e = hip_check(c, hipMemcpyAsync(dst, cout, per * n, hipMemcpyDeviceToHost, c->stream), "download")))
                return e;
        if ((e = hip_check(c, hipStreamSynchronize(c->stream), "apply Schur operator"))) return e;
    }
    return hip_check(c, hipGetLastError(), "apply Schur operator");
}

fl_status fl_solve(fl_ctx *c, const double *b, double *x, int nrhs, const fl_solver_params *p,
                   fl_solver_stats *stats, fl_where where)
{
    if (!valid_ctx(c)) return set_err(nullptr, FL_ERR_ARG, "ctx is NULL");
    if (nrhs < 0 || (nrhs > 0 && (!b || !x))) return set_err(c, FL_ERR_ARG, "bad spinor arguments");
    fl_status e;
    if ((e = check_ready(c))) return e;
    if ((e = check_params(c, p))) return e;
    hipSetDevice(c->device);
    const int chunk = std::max(1, std::min(nrhs, p->batch > 0 ? p->batch : default_batch(c, 1)));
    const size_t per = (size_t)c->V * 24 * sizeof(double);
    fl_status worst = FL_OK;
    c->last_stats.assign(nrhs, fl_solver_stats{});
    for (int k0 = 0; k0 < nrhs; k0 += chunk) {
        const double t_batch = now_s();
        int n = std::min(chunk, nrhs - k0);
        const double *src = b + (size_t)k0 * c->V * 24;
        double *dst = x + (size_t)k0 * c->V * 24;
        double *cin = (double *)src;
        double *cout = dst;
        if (where == FL_HOST) {
            cin = (double *)ws_get(c, WS_CANON, per * n);
            cout = cin;
            if (!cin) return set_err(c, FL_ERR_NOMEM, "device allocation failed");
            if ((e = hip_check(c, hipMemcpyAsync(cin, src, per * n, hipMemcpyHostToDevice, c->stream), "upload")))
                return e;
        }
        size_t fb = (size_t)n * c->Vh * 192;
        void *be = ws_get(c, WS_BE, fb), *bo = ws_get(c, WS_BO, fb), *bh = ws_get(c, WS_BH, fb);
        void *xe = ws_get(c, WS_XE, fb), *xo = ws_get(c, WS_XO, fb);
        if (!be || !bo || !bh || !xe || !xo) return set_err(c, FL_ERR_NOMEM, "device allocation failed");
        LatGeom g = lat_geom(c, n);
        launch_canon_to_eo(cin, (double2 *)be, (double2 *)bo, g, n, c->stream);
        std::vector<double> b2;
        if ((e = norms64(c, n, be, bo, b2))) return e;
        // bhat_e = b_e + k H_eo b_o
        hop64(c, n, 0, bo, bh, be, 1.0, c->kappa, false);
        SolveBatch sb;
        sb.nlat = 1;
        sb.ctx[0] = c;
        sb.nrhs[0] = n;
        sb.bh[0] = (const double2 *)bh;
        sb.xh[0] = (double2 *)xe;
        sb.bnorm.resize(n);
        for (int k = 0; k < n; ++k) sb.bnorm[k] = std::sqrt(b2[k]);
        std::vector<SysResult> res;
        fl_status se = solve_schur_batch(sb, *p, res);
        if (se != FL_OK && se != FL_ERR_NOCONV && se != FL_ERR_BREAKDOWN) return se;
        // x_o = b_o + k H_oe x_e
        hop64(c, n, 1, xe, xo, bo, 1.0, c->kappa, false);
        // stopping rule on the full operator: r = b - D x
        std::vector<double> r2;
        if ((e = full_residual2(c, n, be, bo, xe, xo, r2))) return e;
        launch_eo_to_canon((double2 *)xe, (double2 *)xo, cout, g, n, c->stream);
        if (where == FL_HOST)
            if ((e = hip_check(c, hipMemcpyAsync(dst, cout, per * n, hipMemcpyDeviceToHost, c->stream), "download")))
                return e;
        if ((e = hip_check(c, hipStreamSynchronize(c->stream), "solve"))) return e;
        const double secs = now_s() - t_batch;
        for (int k = 0; k < n; ++k) {
            // truncated solves report the iteration's own residual; a zero
            // source has the zero solution
            put_stats(c, k0 + k, res[k], p->truncated != 0, b2[k], b2[k] > 0 ? r2[k] : 0.0, p->tol, secs);
            const fl_solver_stats &s = c->last_stats[k0 + k];
            if (stats) stats[k0 + k] = s;
            fl_status q = solve_status(s, res[k]);
            if (q != FL_OK && worst == FL_OK) worst = q;
        }
    }
    if (worst != FL_OK) return set_err(c, worst, "some right-hand sides did not reach tol");
    return FL_OK;
}

fl_status fl_loops_exact_sites(fl_ctx *c, const long long *sites, long long nsites, const int *gammas, int ngamma,
                               const fl_solver_params *p, double *L, double *S, fl_where where)
{
    if (!valid_ctx(c)) return set_err(nullptr, FL_ERR_ARG, "ctx is NULL");
    if (nsites < 0 || (nsites > 0 && (!sites || !L))) return set_err(c, FL_ERR_ARG, "bad site list or output");
    if (ngamma < 1 || ngamma > 16 || !gammas) return set_err(c, FL_ERR_ARG, "ngamma must be in 1..16");
    for (int k = 0; k < ngamma; ++k)
        if (gammas[k] < 0 || gammas[k] > 15) return set_err(c, FL_ERR_ARG, "gamma masks are 4-bit");
    for (long long k = 0; k < nsites; ++k)
        if (sites[k] < 0 || sites[k] >= c->V) return set_err(c, FL_ERR_ARG, "site index out of range");
    fl_status e;
    if ((e = check_ready(c))) return e;
    if ((e = check_params(c, p))) return e;
    if (nsites == 0) return FL_OK;
    hipSetDevice(c->device);
    const int batch = std::max(12, (p->batch > 0 ? p->batch : default_batch(c, 12)) / 12 * 12);
    const int nsb = batch / 12;
    double2 *dL = (double2 *)ws_get(c, WS_ACC, sizeof(double2) * ngamma * (size_t)nsites);
    double2 *dS = S ? (double2 *)ws_get(c, WS_ACC2, sizeof(double2) * 16 * (size_t)nsites) : nullptr;
    long long *dsites = (long long *)ws_get(c, WS_SITES, sizeof(long long) * nsites);
    std::vector<double> gt = gamma_table(gammas, ngamma);
    double *dgam = (double *)ws_get(c, WS_GAM, gt.size() * sizeof(double));
    if (!dL || (S && !dS) || !dsites || !dgam) return set_err(c, FL_ERR_NOMEM, "device allocation failed");
    if ((e = hip_check(c, hipMemcpyAsync(dsites, sites, sizeof(long long) * nsites, hipMemcpyHostToDevice, c->stream),
                       "upload sites")))
        return e;
    if ((e = hip_check(c, hipMemcpyAsync(dgam, gt.data(), gt.size() * sizeof(double), hipMemcpyHostToDevice, c->stream),
                       "upload gammas")))
        return e;
    fl_status worst = FL_OK;
    c->last_stats.assign((size_t)12 * nsites, fl_solver_stats{});
    for (long long s0 = 0; s0 < nsites; s0 += nsb) {
        const double t_batch = now_s();
        int ns = (int)std::min<long long>(nsb, nsites - s0);
        int n = 12 * ns;
        size_t fb = (size_t)n * c->Vh * 192;
        void *be = ws_get(c, WS_BE, fb), *bo = ws_get(c, WS_BO, fb), *bh = ws_get(c, WS_BH, fb);
        void *xe = ws_get(c, WS_XE, fb), *xo = ws_get(c, WS_XO, fb);
        if (!be || !bo || !bh || !xe || !xo) return set_err(c, FL_ERR_NOMEM, "device allocation failed");
        LatGeom g = lat_geom(c, n);
        if ((e = hip_check(c, hipMemsetAsync(be, 0, fb, c->stream), "memset"))) return e;
        if ((e = hip_check(c, hipMemsetAsync(bo, 0, fb, c->stream), "memset"))) return e;
        launch_point_sources((double2 *)be, (double2 *)bo, dsites + s0, ns, g, c->stream);
        hop64(c, n, 0, bo, bh, be, 1.0, c->kappa, false);
        SolveBatch sb;
        sb.nlat = 1;
        sb.ctx[0] = c;
        sb.nrhs[0] = n;
        sb.bh[0] = (const double2 *)bh;
        sb.xh[0] = (double2 *)xe;
        sb.bnorm.assign(n, 1.0);
        std::vector<SysResult> res;
        fl_status se = solve_schur_batch(sb, *p, res);
        if (se != FL_OK && se != FL_ERR_NOCONV && se != FL_ERR_BREAKDOWN) return se;
        // acceptance on the full operator (point sources: |b| = 1)
        hop64(c, n, 1, xe, xo, bo, 1.0, c->kappa, false);  // x_o = b_o + k H_oe x_e
        std::vector<double> r2;
        if ((e = full_residual2(c, n, be, bo, xe, xo, r2))) return e;
        const double secs = now_s() - t_batch;
        for (int k = 0; k < n; ++k) {
            put_stats(c, (size_t)12 * s0 + k, res[k], p->truncated != 0, 1.0, r2[k], p->tol, secs);
            fl_status q = solve_status(c->last_stats[(size_t)12 * s0 + k], res[k]);
            if (q != FL_OK && worst == FL_OK) worst = q;
        }
        ExactContractArgs a;
        a.g = g;
        a.nsites = ns;
        a.sites = dsites + s0;
        a.xe = (const double2 *)xe;
        a.be = (const double2 *)be;
        a.bo = (const double2 *)bo;
        a.gauge = (const double2 *)links(c, LINK_F64_R18);
        a.kappa = c->kappa;
        a.ngamma = ngamma;
        a.gam = dgam;
        a.L = dL;
        a.L_stride = nsites;
        a.L_off = s0;
        a.S = dS;
        launch_exact_contract(a, c->stream);
    }
    if ((e = copy_out(c, L, dL, sizeof(double2) * ngamma * (size_t)nsites, where))) return e;
    if (S && (e = copy_out(c, S, dS, sizeof(double2) * 16 * (size_t)nsites, where))) return e;
    if ((e = hip_check(c, hipStreamSynchronize(c->stream), "exact loops"))) return e;
    if (worst != FL_OK) return set_err(c, worst, "some point-source solves did not reach tol");
    return FL_OK;
}

fl_status fl_loops_exact(fl_ctx *c, const int *t0, int nt, const int *gammas, int ngamma, const fl_solver_params *p,
                         double *L, double *S, fl_where where)
{
    if (!valid_ctx(c)) return set_err(nullptr, FL_ERR_ARG, "ctx is NULL");
    if (nt < 0 || (nt > 0 && !t0)) return set_err(c, FL_ERR_ARG, "bad timeslice list");
    std::vector<long long> sites;
    sites.reserve((size_t)nt * c->Vs);
    for (int i = 0; i < nt; ++i) {
        if (t0[i] < 0 || t0[i] >= c->L[3]) return set_err(c, FL_ERR_ARG, "timeslice out of range");
        for (long long xs = 0; xs < c->Vs; ++xs) sites.push_back(xs + c->Vs * t0[i]);
    }
    return fl_loops_exact_sites(c, sites.data(), (long long)sites.size(), gammas, ngamma, p, L, S, where);
}

// stochastic and truncated-solver estimates for up to FL_MAXLAT lattices
fl_status fl_loops_stochastic_multi(fl_ctx **ctxs, int nctx, const fl_noise_params *np, const int *gammas,
                                    int ngamma, const fl_solver_params *lp, const fl_solver_params *hp, double **Lout,
                                    fl_where where)
{
    if (!ctxs || nctx < 1 || nctx > FL_MAXLAT || !np || !Lout) return set_err(nullptr, FL_ERR_ARG, "bad lattice list");
    for (int l = 0; l < nctx; ++l) {
        if (!ctxs[l]) return set_err(nullptr, FL_ERR_ARG, "ctx is NULL");
        // a context holds one lattice's workspace: twice in one batch, the
        // sources and Krylov vectors of one entry would overwrite the other's
        for (int m = 0; m < l; ++m)
            if (ctxs[m] == ctxs[l]) return set_err(nullptr, FL_ERR_ARG, "the same context appears twice in the batch");
    }
    fl_ctx *c0 = ctxs[0];
    for (int l = 1; l < nctx; ++l)
        if (ctxs[l]->device != c0->device || ctxs[l]->stream != c0->stream)
            return set_err(c0, FL_ERR_ARG, "batched lattices must share device and stream");
    if (ngamma < 1 || ngamma > 16 || !gammas) return set_err(c0, FL_ERR_ARG, "ngamma must be in 1..16");
    for (int k = 0; k < ngamma; ++k)
        if (gammas[k] < 0 || gammas[k] > 15) return set_err(c0, FL_ERR_ARG, "gamma masks are 4-bit");
    fl_status e;
    bool any_hp = false;
    for (int l = 0; l < nctx; ++l) {
        fl_ctx *c = ctxs[l];
        const fl_noise_params &q = np[l];
        if ((e = check_ready(c))) return e;
        if ((e = check_params(c, lp))) return e;
        if (q.n_hp > 0) {
            any_hp = true;
            if ((e = check_params(c, hp))) return e;
        }
        if (q.noise < 0 || q.noise > 2) return set_err(c, FL_ERR_ARG, "unknown noise type");
        if (q.n_lp < 0 || q.n_hp < 0 || q.n_lp + q.n_hp == 0) return set_err(c, FL_ERR_ARG, "need n_lp + n_hp > 0");
        if (q.n_hp > 0 && q.n_lp == 0) return set_err(c, FL_ERR_ARG, "the correction ensemble needs n_lp > 0");
        if (q.t_begin < 0 || q.t_end > c->L[3] || q.t_begin >= q.t_end)
            return set_err(c, FL_ERR_ARG, "timeslice range out of bounds");
        if (q.dilution < 0 || q.dilution > 31 || ((q.dilution & FL_DIL_EVENODD) && (q.dilution & FL_DIL_CUBIC)))
            return set_err(c, FL_ERR_ARG, "bad dilution mask");
        if (q.r0 < 0 || q.r0 + q.n_lp + q.n_hp > (1LL << 31)) return set_err(c, FL_ERR_ARG, "noise index out of range");
        if (!Lout[l]) return set_err(c, FL_ERR_ARG, "output is NULL");
    }
    hipSetDevice(c0->device);
    hipStream_t st = c0->stream;
    std::vector<double> gt = gamma_table(gammas, ngamma);
    // per-lattice job lists: (component, noise index, target, sign, solver)
    struct Job {
        int v[JOB_INTS];
        int hp;  // solved with the high-precision parameters
    };
    std::vector<std::vector<Job>> jobs(nctx);
    for (int l = 0; l < nctx; ++l) {
        const fl_noise_params &q = np[l];
        const int dil = q.dilution;
        std::vector<int> ts;
        if (dil & FL_DIL_TIME)
            for (int t = q.t_begin; t < q.t_end; ++t) ts.push_back(t);
        else
            ts.push_back(-1);
        int nsp = (dil & FL_DIL_SPIN) ? 4 : 1, ncl = (dil & FL_DIL_COLOUR) ? 3 : 1;
        int nspace = (dil & FL_DIL_CUBIC) ? 8 : ((dil & FL_DIL_EVENODD) ? 2 : 1);
        auto add = [&](long long r, int target, int sign, int hpflag) {
            for (int t : ts)
                for (int s = 0; s < nsp; ++s)
                    for (int a = 0; a < ncl; ++a)
                        for (int k = 0; k < nspace; ++k) {
                            Job j;
                            j.v[JOB_T] = t;
                            j.v[JOB_SPIN] = (dil & FL_DIL_SPIN) ? s : -1;
                            j.v[JOB_COL] = (dil & FL_DIL_COLOUR) ? a : -1;
                            j.v[JOB_CLASS] = nspace > 1 ? k : -1;
                            j.v[JOB_R] = (int)r;
                            j.v[JOB_TARGET] = target;
                            j.v[JOB_SIGN] = sign;
                            j.v[7] = 0;
                            j.hp = hpflag;
                            jobs[l].push_back(j);
                        }
        };
        for (int r = 0; r < q.n_lp; ++r) add(q.r0 + r, 0, +1, 0);
        for (int r = 0; r < q.n_hp; ++r) {
            add(q.r0 + q.n_lp + r, 1, -1, 0);  // phi^LP of the correction ensemble
            add(q.r0 + q.n_lp + r, 1, +1, 1);  // phi^HP
        }
    }
    // accumulators per lattice
    std::vector<double2 *> acc0(nctx), acc1(nctx);
    std::vector<double *> dgam(nctx);
    std::vector<size_t> nacc(nctx);
    for (int l = 0; l < nctx; ++l) {
        fl_ctx *c = ctxs[l];
        nacc[l] = (size_t)ngamma * (np[l].t_end - np[l].t_begin) * c->Vs;
        acc0[l] = (double2 *)ws_get(c, WS_ACC, sizeof(double2) * nacc[l]);
        acc1[l] = (double2 *)ws_get(c, WS_ACC2, sizeof(double2) * nacc[l]);
        dgam[l] = (double *)ws_get(c, WS_GAM, gt.size() * sizeof(double));
        if (!acc0[l] || !acc1[l] || !dgam[l]) return set_err(c, FL_ERR_NOMEM, "device allocation failed");
        if ((e = hip_check(c, hipMemsetAsync(acc0[l], 0, sizeof(double2) * nacc[l], st), "memset"))) return e;
        if ((e = hip_check(c, hipMemsetAsync(acc1[l], 0, sizeof(double2) * nacc[l], st), "memset"))) return e;
        if ((e = hip_check(c, hipMemcpyAsync(dgam[l], gt.data(), gt.size() * sizeof(double), hipMemcpyHostToDevice, st),
                           "upload gammas")))
            return e;
    }
    // batches: all LP-type jobs, then all HP jobs; lattices advance together
    fl_status worst = FL_OK;
    for (int l = 0; l < nctx; ++l) ctxs[l]->last_stats.assign(jobs[l].size(), fl_solver_stats{});
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1 && !any_hp) break;
        const fl_solver_params &prm = pass ? *hp : *lp;
        std::vector<std::vector<int>> sel(nctx);
        int maxb = 1 << 30;
        for (int l = 0; l < nctx; ++l) {
            for (int k = 0; k < (int)jobs[l].size(); ++k)
                if (jobs[l][k].hp == pass) sel[l].push_back(k);
            int b = prm.batch > 0 ? prm.batch : default_batch(ctxs[l], 1);
            maxb = std::min(maxb, b);
        }
        std::vector<size_t> pos(nctx, 0);
        while (true) {
            int nr[FL_MAXLAT] = {0, 0, 0, 0};
            bool any = false;
            for (int l = 0; l < nctx; ++l) {
                nr[l] = (int)std::min<size_t>(maxb, sel[l].size() - pos[l]);
                any |= nr[l] > 0;
            }
            if (!any) break;
            const double t_batch = now_s();
            // every lattice takes part in the batch (possibly with no rhs)
            SolveBatch sb;
            sb.nlat = 0;
            std::vector<int> lat_of;
            for (int l = 0; l < nctx; ++l) {
                sb.ctx[sb.nlat] = ctxs[l];
                sb.nrhs[sb.nlat] = nr[l];
                lat_of.push_back(l);
                sb.nlat++;
            }
            std::vector<std::vector<double>> bn(nctx);
            for (int l = 0; l < nctx; ++l) {
                fl_ctx *c = ctxs[l];
                int n = nr[l];
                size_t fb = (size_t)std::max(n, 1) * c->Vh * 192;
                void *be = ws_get(c, WS_BE, fb), *bo = ws_get(c, WS_BO, fb), *bh = ws_get(c, WS_BH, fb);
                void *xe = ws_get(c, WS_XE, fb);
                int *djob = (int *)ws_get(c, WS_COMP, sizeof(int) * JOB_INTS * std::max(n, 1));
                if (!be || !bo || !bh || !xe || !djob) return set_err(c, FL_ERR_NOMEM, "device allocation failed");
                sb.bh[l] = (const double2 *)bh;
                sb.xh[l] = (double2 *)xe;
                if (n == 0) continue;
                // the job table through the page-locked block: the stream
                // is synchronised before the block is written again or freed
                int *hj = (int *)pinned_get(c, sizeof(int) * JOB_INTS * (size_t)n);
                if (!hj) return set_err(c, FL_ERR_NOMEM, "page-locked host allocation failed");
                for (int k = 0; k < n; ++k)
                    std::memcpy(hj + (size_t)JOB_INTS * k, jobs[l][sel[l][pos[l] + k]].v, sizeof(int) * JOB_INTS);
                if ((e = hip_check(c, hipMemcpyAsync(djob, hj, sizeof(int) * JOB_INTS * (size_t)n, hipMemcpyHostToDevice,
                                                     st),
                                   "upload jobs")))
                    return e;
                NoiseBatch nbt;
                nbt.type = np[l].noise;
                nbt.seed = np[l].seed;
                nbt.dil = np[l].dilution;
                nbt.ncomp = n;
                nbt.job = djob;
                LatGeom g = lat_geom(c, n);
                launch_noise_sources((double2 *)be, (double2 *)bo, nbt, g, st);
                if ((e = norms64(c, n, be, bo, bn[l]))) return e;
                hop64(c, n, 0, bo, bh, be, 1.0, c->kappa, false);
            }
            for (int l = 0; l < nctx; ++l)
                for (int k = 0; k < nr[l]; ++k) sb.bnorm.push_back(std::sqrt(bn[l][k]));
            std::vector<SysResult> res;
            fl_status se = solve_schur_batch(sb, prm, res);
            if (se != FL_OK && se != FL_ERR_NOCONV && se != FL_ERR_BREAKDOWN) return se;
            int sys0 = 0;
            for (int l = 0; l < nctx; ++l) {
                fl_ctx *c = ctxs[l];
                int n = nr[l];
                if (n == 0) continue;
                size_t fb = (size_t)n * c->Vh * 192;
                void *be = c->pool[WS_BE].p, *bo = c->pool[WS_BO].p, *xe = c->pool[WS_XE].p;
                void *xo = ws_get(c, WS_XO, fb);
                if (!xo) return set_err(c, FL_ERR_NOMEM, "device allocation failed");
                hop64(c, n, 1, xe, xo, bo, 1.0, c->kappa, false);  // x_o = eta_o + k H_oe x_e
                // statistics; solves that are not truncated are accepted on the
                // full operator
                std::vector<double> r2;
                if (!prm.truncated && (e = full_residual2(c, n, be, bo, xe, xo, r2))) return e;
                const double secs = now_s() - t_batch;
                for (int k = 0; k < n; ++k) {
                    const size_t job = (size_t)sel[l][pos[l] + k];
                    const SysResult &r = res[sys0 + k];
                    put_stats(c, job, r, prm.truncated != 0, bn[l][k], prm.truncated ? 0.0 : r2[k], prm.tol, secs);
                    fl_status q = solve_status(c->last_stats[job], r);
                    if (q != FL_OK && worst == FL_OK) worst = q;
                }
                sys0 += n;
                StochContractArgs a;
                a.g = lat_geom(c, n);
                a.nrhs = n;
                a.pe = (const double2 *)xe;
                a.po = (const double2 *)xo;
                a.ne = (const double2 *)be;
                a.no = (const double2 *)bo;
                a.job = (const int *)c->pool[WS_COMP].p;
                a.dil = np[l].dilution;
                a.t_begin = np[l].t_begin;
                a.t_end = np[l].t_end;
                a.ngamma = ngamma;
                a.gam = dgam[l];
                a.acc0 = acc0[l];
                a.acc1 = acc1[l];
                launch_stoch_contract(a, st);
                pos[l] += n;
            }
            if ((e = hip_check(c0, hipStreamSynchronize(st), "stochastic batch"))) return e;
        }
    }
    // L = acc0 / n_lp + acc1 / n_hp, formed on the device; host results
    // leave through the context's page-locked block (one DMA per lattice)
    size_t hbytes = 0;
    for (int l = 0; l < nctx; ++l) hbytes += sizeof(double2) * nacc[l];
    unsigned char *stage = nullptr;
    if (where != FL_DEVICE && hbytes) {
        stage = (unsigned char *)pinned_get(c0, hbytes);
        if (!stage) return set_err(c0, FL_ERR_NOMEM, "page-locked host allocation failed");
    }
    size_t off = 0;
    for (int l = 0; l < nctx; ++l) {
        fl_ctx *c = ctxs[l];
        const double w0 = np[l].n_lp > 0 ? 1.0 / np[l].n_lp : 0.0, w1 = np[l].n_hp > 0 ? 1.0 / np[l].n_hp : 0.0;
        launch_tsm_combine((double *)acc0[l], (const double *)acc1[l], w0, w1, 2LL * (long long)nacc[l], st);
        if ((e = hip_check(c, hipGetLastError(), "combine"))) return e;
        const size_t nb = sizeof(double2) * nacc[l];
        if ((e = hip_check(c, hipMemcpyAsync(stage ? (void *)(stage + off) : (void *)Lout[l], acc0[l], nb,
                                             stage ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, st),
                           "copy out")))
            return e;
        off += nb;
    }
    if ((e = hip_check(c0, hipStreamSynchronize(st), "sync"))) return e;
    if (stage) {
        off = 0;
        for (int l = 0; l < nctx; ++l) {
            const size_t nb = sizeof(double2) * nacc[l];
            std::memcpy(Lout[l], stage + off, nb);
            off += nb;
        }
    }
    if (worst != FL_OK) return set_err(c0, worst, "some solves did not reach their tolerance (fl_last_stats)");
    return FL_OK;
}

fl_status fl_loops_stochastic(fl_ctx *c, const fl_noise_params *np, const int *gammas, int ngamma,
                              const fl_solver_params *lp, const fl_solver_params *hp, double *L, fl_where where)
{
    if (!valid_ctx(c)) return set_err(nullptr, FL_ERR_ARG, "ctx is NULL");
    fl_ctx *cs[1] = {c};
    double *Ls[1] = {L};
    return fl_loops_stochastic_multi(cs, 1, np, gammas, ngamma, lp, hp, Ls, where);
}

fl_status fl_loops_grad(fl_ctx *c, const int *t0, int nt, const int *gammas, int ngamma, const double *w,
                        const fl_solver_params *p, double *dU, double *dkappa, fl_where where)
{
    if (!valid_ctx(c)) return set_err(nullptr, FL_ERR_ARG, "ctx is NULL");
    if (nt < 1 || !t0 || !w || !dU || !dkappa) return set_err(c, FL_ERR_ARG, "bad arguments");
    if (ngamma < 1 || ngamma > 16 || !gammas) return set_err(c, FL_ERR_ARG, "ngamma must be in 1..16");
    for (int k = 0; k < ngamma; ++k)
        if (gammas[k] < 0 || gammas[k] > 15) return set_err(c, FL_ERR_ARG, "gamma masks are 4-bit");
    for (int i = 0; i < nt; ++i)
        if (t0[i] < 0 || t0[i] >= c->L[3]) return set_err(c, FL_ERR_ARG, "timeslice out of range");
    fl_status e;
    if ((e = check_ready(c))) return e;
    if ((e = check_params(c, p))) return e;
    hipSetDevice(c->device);
    hipStream_t st = c->stream;
    const long long Vs = c->Vs;
    // weights on the host
    std::vector<double> hw((size_t)2 * ngamma * nt * Vs);
    if ((e = hip_check(c, hipMemcpyAsync(hw.data(), w, hw.size() * sizeof(double),
                                         where == FL_DEVICE ? hipMemcpyDeviceToHost : hipMemcpyHostToHost, st),
                       "weights")))
        return e;
    if ((e = hip_check(c, hipStreamSynchronize(st), "sync"))) return e;
    // sites with a nonzero weight, and M_y = sum_Gamma w_Gamma(y) g5 Gamma^+ for each
    C g5[4][4];
    gamma_of_mask(15, g5);
    std::vector<C> Gm((size_t)ngamma * 16);
    for (int k = 0; k < ngamma; ++k) gamma_of_mask(gammas[k], (C(*)[4]) & Gm[16 * k]);
    std::vector<long long> sites;
    std::vector<double> Mh;
    for (int i = 0; i < nt; ++i)
        for (long long xs = 0; xs < Vs; ++xs) {
            bool any = false;
            for (int k = 0; k < ngamma; ++k) {
                size_t o = 2 * (((size_t)k * nt + i) * Vs + xs);
                any |= hw[o] != 0 || hw[o + 1] != 0;
            }
            if (!any) continue;
            sites.push_back(xs + Vs * t0[i]);
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) {
                    C m{0, 0};
                    for (int k = 0; k < ngamma; ++k) {
                        size_t o = 2 * (((size_t)k * nt + i) * Vs + xs);
                        C wk{hw[o], hw[o + 1]};
                        C acc{0, 0};
                        for (int q = 0; q < 4; ++q) {
                            C gd = Gm[16 * k + 4 * b + q];  // Gamma^+_{q b} = conj(Gamma_{b q})
                            gd.im = -gd.im;
                            C pr = cmul(g5[a][q], gd);
                            acc.re += pr.re;
                            acc.im += pr.im;
                        }
                        C t = cmul(wk, acc);
                        m.re += t.re;
                        m.im += t.im;
                    }
                    Mh.push_back(m.re);
                    Mh.push_back(m.im);
                }
        }
    const size_t ub = (size_t)4 * c->V * 9 * sizeof(double2);
    double2 *ddU = (double2 *)ws_get(c, WS_DU, ub);
    if (!ddU) return set_err(c, FL_ERR_NOMEM, "device allocation failed");
    if ((e = hip_check(c, hipMemsetAsync(ddU, 0, ub, st), "memset"))) return e;
    double dk = 0;
    const long long nsites = (long long)sites.size();
    long long *dsites = (long long *)ws_get(c, WS_SITES, sizeof(long long) * std::max<long long>(1, nsites));
    double2 *dM = (double2 *)ws_get(c, WS_M, sizeof(double) * std::max<size_t>(2, Mh.size()));
    if (!dsites || !dM) return set_err(c, FL_ERR_NOMEM, "device allocation failed");
    if (nsites) {
        if ((e = hip_check(c, hipMemcpyAsync(dsites, sites.data(), sizeof(long long) * nsites, hipMemcpyHostToDevice, st),
                           "upload")))
            return e;
        if ((e = hip_check(c, hipMemcpyAsync(dM, Mh.data(), sizeof(double) * Mh.size(), hipMemcpyHostToDevice, st),
                           "upload")))
            return e;
    }
    const int batch = std::max(12, (p->batch > 0 ? p->batch : default_batch(c, 12)) / 12 * 12);
    const int nsb = batch / 12;
    fl_status worst = FL_OK;
    c->last_stats.assign((size_t)12 * nsites, fl_solver_stats{});
    for (long long s0 = 0; s0 < nsites; s0 += nsb) {
        const double t_batch = now_s();
        int ns = (int)std::min<long long>(nsb, nsites - s0);
        int n = 12 * ns;
        size_t fb = (size_t)n * c->Vh * 192;
        void *be = ws_get(c, WS_BE, fb), *bo = ws_get(c, WS_BO, fb), *bh = ws_get(c, WS_BH, fb);
        void *xe = ws_get(c, WS_XE, fb), *xo = ws_get(c, WS_XO, fb);
        void *ce = ws_get(c, WS_CE, fb), *co = ws_get(c, WS_CO, fb);
        void *he = ws_get(c, WS_HE, fb), *ho = ws_get(c, WS_HO, fb);
        double *dp = (double *)ws_get(c, WS_MISC, 1024 * sizeof(double));
        if (!be || !bo || !bh || !xe || !xo || !ce || !co || !he || !ho || !dp)
            return set_err(c, FL_ERR_NOMEM, "device allocation failed");
        LatGeom g = lat_geom(c, n);
        if ((e = hip_check(c, hipMemsetAsync(be, 0, fb, st), "memset"))) return e;
        if ((e = hip_check(c, hipMemsetAsync(bo, 0, fb, st), "memset"))) return e;
        launch_point_sources((double2 *)be, (double2 *)bo, dsites + s0, ns, g, st);
        hop64(c, n, 0, bo, bh, be, 1.0, c->kappa, false);
        SolveBatch sb;
        sb.nlat = 1;
        sb.ctx[0] = c;
        sb.nrhs[0] = n;
        sb.bh[0] = (const double2 *)bh;
        sb.xh[0] = (double2 *)xe;
        sb.bnorm.assign(n, 1.0);
        std::vector<SysResult> res;
        fl_status se = solve_schur_batch(sb, *p, res);
        if (se != FL_OK && se != FL_ERR_NOCONV && se != FL_ERR_BREAKDOWN) return se;
        hop64(c, n, 1, xe, xo, bo, 1.0, c->kappa, false);  // psi_o = b_o + k H_oe psi_e
        ChiArgs ca;
        ca.g = g;
        ca.nsites = ns;
        ca.sites = dsites + s0;
        ca.M = dM + (size_t)16 * s0;
        ca.pe = (const double2 *)xe;
        ca.po = (const double2 *)xo;
        ca.ce = (double2 *)ce;
        ca.co = (double2 *)co;
        launch_chi(ca, st);
        // dF/dkappa = Re sum_s chi_s^+ H psi_s
        hop64(c, n, 0, xo, he, nullptr, 0.0, 1.0, false);
        hop64(c, n, 1, xe, ho, nullptr, 0.0, 1.0, false);
        long long ne = (long long)n * 12 * c->Vh;
        launch_dot64((const double2 *)ce, (const double2 *)he, ne, dp, st);
        launch_dot64((const double2 *)co, (const double2 *)ho, ne, dp + 512, st);
        std::vector<double> hp(1024);
        if ((e = hip_check(c, hipMemcpyAsync(hp.data(), dp, 1024 * sizeof(double), hipMemcpyDeviceToHost, st),
                           "download")))
            return e;
        ForceArgs fa;
        fa.g = g;
        fa.nrhs = n;
        fa.pe = (const double2 *)xe;
        fa.po = (const double2 *)xo;
        fa.ce = (const double2 *)ce;
        fa.co = (const double2 *)co;
        fa.kappa = c->kappa;
        fa.dU = ddU;
        launch_force(fa, st);
        // acceptance of the forward solves on the full operator (|b| = 1);
        // the residual check reuses he, ho after the force kernel
        std::vector<double> r2;
        if ((e = full_residual2(c, n, be, bo, xe, xo, r2))) return e;
        if ((e = hip_check(c, hipStreamSynchronize(st), "gradient batch"))) return e;
        for (int k = 0; k < 256; ++k) dk += hp[2 * k] + hp[512 + 2 * k];
        const double secs = now_s() - t_batch;
        for (int k = 0; k < n; ++k) {
            put_stats(c, (size_t)12 * s0 + k, res[k], p->truncated != 0, 1.0, r2[k], p->tol, secs);
            fl_status q = solve_status(c->last_stats[(size_t)12 * s0 + k], res[k]);
            if (q != FL_OK && worst == FL_OK) worst = q;
        }
    }
    *dkappa = dk;
    if ((e = copy_out(c, dU, ddU, ub, where))) return e;
    if ((e = hip_check(c, hipStreamSynchronize(st), "gradient"))) return e;
    if (worst != FL_OK) return set_err(c, worst, "some point-source solves did not reach tol");
    return FL_OK;
}

fl_status fl_last_stats(const fl_ctx *c, fl_solver_stats *stats, long long cap, long long *n)
{
    if (!c) return set_err(nullptr, FL_ERR_ARG, "ctx is NULL");
    if (!n || cap < 0 || (cap > 0 && !stats)) return set_err(const_cast<fl_ctx *>(c), FL_ERR_ARG, "bad output");
    *n = (long long)c->last_stats.size();
    const long long m = std::min<long long>(cap, *n);
    for (long long k = 0; k < m; ++k) stats[k] = c->last_stats[(size_t)k];
    return FL_OK;
}

fl_status fl_profile_enable(fl_ctx *c, int kernel, int enable)
{
    if (!valid_ctx(c)) return set_err(nullptr, FL_ERR_ARG, "ctx is NULL");
    if (kernel < 0 || kernel >= FL_PROF_NKERNELS) return set_err(c, FL_ERR_ARG, "unknown kernel id");
    hipSetDevice(c->device);
    hipStreamSynchronize(c->stream);
    prof_reset(c->prof[kernel]);
    c->prof[kernel].on = enable != 0;
    return FL_OK;
}

fl_status fl_profile_read(fl_ctx *c, int kernel, double *ms, long long *launches, double *bytes)
{
    if (!valid_ctx(c)) return set_err(nullptr, FL_ERR_ARG, "ctx is NULL");
    if (kernel < 0 || kernel >= FL_PROF_NKERNELS) return set_err(c, FL_ERR_ARG, "unknown kernel id");
    hipSetDevice(c->device);
    fl_status e;
    if ((e = hip_check(c, hipStreamSynchronize(c->stream), "sync"))) return e;
    ProfSlot &p = c->prof[kernel];
    double tot = 0;
    for (auto &ev : p.ev) {
        float t = 0;
        if (hipEventElapsedTime(&t, ev.first, ev.second) == hipSuccess) tot += t;
    }
    if (ms) *ms = tot;
    if (launches) *launches = (long long)p.ev.size();
    if (bytes) *bytes = p.bytes;
    return FL_OK;
}

static fl_status fmt_of(fl_ctx *c, int prec, int gauge_reals, LinkFormat *fmt)
{
    if (prec == FL_PREC_F64 && gauge_reals == 18)
        *fmt = LINK_F64_R18;
    else if (prec == FL_PREC_F32)
        *fmt = gauge_reals == 18 ? LINK_F32_R18 : LINK_F32_R12;
    else if (prec == FL_PREC_BF16 && gauge_reals == 12)
        *fmt = LINK_BF16_R12;
    else if (prec == FL_PREC_H16 && gauge_reals == 12)
        *fmt = LINK_Q16_R12;
    else
        return set_err(c, FL_ERR_ARG, "unsupported precision / link storage");
    if (*fmt != LINK_F64_R18 && *fmt != LINK_F32_R18 && !c->su3)
        return set_err(c, FL_ERR_ARG, "12-real links need SU(3) links");
    return FL_OK;
}

static fl_status bench_impl(fl_ctx *c, LinkFormat fmt, int nrhs, int nrep, int nsets, int rt, int group, int lds,
                            double *ms_per_launch, double *bytes_per_launch)
{
    hipSetDevice(c->device);
    hipStream_t st = c->stream;
    const size_t sb = vec_site_bytes(vec_format(fmt));
    const size_t lb = link_bytes(fmt);
    const size_t fbytes = (size_t)nrhs * c->Vh * sb, gbytes = lb * 4 * (size_t)c->V;
    void *src = links(c, fmt);
    if (!src) return set_err(c, FL_ERR_NOMEM, "device allocation failed (links)");
    std::vector<void *> ins(nsets, nullptr), outs(nsets, nullptr), gs(nsets, nullptr);
    auto release = [&]() {
        for (int q = 0; q < nsets; ++q) {
            if (ins[q]) hipFree(ins[q]);
            if (outs[q]) hipFree(outs[q]);
            if (gs[q]) hipFree(gs[q]);
        }
    };
    for (int k = 0; k < nsets; ++k) {
        if (hipMalloc(&ins[k], fbytes) != hipSuccess || hipMalloc(&outs[k], fbytes) != hipSuccess ||
            hipMalloc(&gs[k], gbytes) != hipSuccess) {
            (void)hipGetLastError();
            release();
            return set_err(c, FL_ERR_NOMEM, "device allocation failed (benchmark buffers)");
        }
        hipMemsetAsync(ins[k], 0x3c, fbytes, st);
        hipMemcpyAsync(gs[k], src, gbytes, hipMemcpyDeviceToDevice, st);
    }
    int RT, G;
    tile_shape(c, fmt, nrhs, &RT, &G);
    const int maxrt = fmt == LINK_F64_R18 ? 8 : 16;
    if (rt > 0) RT = std::min(rt, maxrt);
    if (group > 0) G = group;
    fl_ctx *cs[1] = {c};
    int nr[1] = {nrhs};
    DslashArgs a;
    std::memset(&a, 0, sizeof(a));
    a.B = batch_geom(cs, nr, 1, RT, G);
    a.par = 0;
    a.nsys = nrhs;
    a.cb[0] = 1.0;
    {
        int saved = c->tune_lds[fmt];
        if (lds >= 0) c->tune_lds[fmt] = lds;
        dslash_config(c, fmt, a);
        c->tune_lds[fmt] = saved;
    }
    if (lds > a.lds) {
        release();
        return set_err(c, FL_ERR_ARG, "LDS staging does not fit this workgroup shape");
    }
    auto launch = [&](int k) {
        a.in[0] = ins[k];
        a.out[0] = outs[k];
        a.gauge[0] = gs[k];
        launch_dslash(fmt, a, false, EPI_PLAIN, st);
    };
    for (int k = 0; k < nsets; ++k) launch(k);
    hipEvent_t t0, t1;
    hipEventCreate(&t0);
    hipEventCreate(&t1);
    hipEventRecord(t0, st);
    for (int r = 0; r < nrep; ++r) launch(r % nsets);
    hipEventRecord(t1, st);
    fl_status e = hip_check(c, hipEventSynchronize(t1), "benchmark");
    float ms = 0;
    hipEventElapsedTime(&ms, t0, t1);
    hipEventDestroy(t0);
    hipEventDestroy(t1);
    release();
    if (e) return e;
    if (ms_per_launch) *ms_per_launch = ms / nrep;
    if (bytes_per_launch) *bytes_per_launch = (double)(8 * lb * c->Vh) + 2.0 * (double)fbytes;
    return FL_OK;
}

fl_status fl_bench_dslash(fl_ctx *c, int prec, int gauge_reals, int nrhs, int nrep, int nsets, int rt, int group,
                          int lds, double *ms_per_launch, double *bytes_per_launch)
{
    if (!valid_ctx(c)) return set_err(nullptr, FL_ERR_ARG, "ctx is NULL");
    if (nrhs < 1 || nrep < 1 || nsets < 1 || nsets > 64 || rt < 0 || rt > 16 || group < 0)
        return set_err(c, FL_ERR_ARG, "bad benchmark sizes");
    fl_status e;
    if ((e = check_ready(c))) return e;
    LinkFormat fmt;
    if ((e = fmt_of(c, prec, gauge_reals, &fmt))) return e;
    if (lds < -1 || lds > 4 || (lds == 3 && fmt != LINK_Q16_R12))
        return set_err(c, FL_ERR_ARG, "lds must be -1, 0, 1, 2 or 4 (3: 16-bit fields only)");
    return bench_impl(c, fmt, nrhs, nrep, nsets, rt, group, lds, ms_per_launch, bytes_per_launch);
}

fl_status fl_set_tile(fl_ctx *c, int prec, int gauge_reals, int rt, int group, int lds)
{
    if (!valid_ctx(c)) return set_err(nullptr, FL_ERR_ARG, "ctx is NULL");
    if (rt < 0 || rt > 16 || (rt & (rt - 1)) || group < 0 || lds < -1 || lds > 4)
        return set_err(c, FL_ERR_ARG, "rt must be 0 or a power of two <= 16, group >= 0, lds in -1..4");
    LinkFormat fmt;
    if (prec == FL_PREC_F64 && gauge_reals == 18)
        fmt = LINK_F64_R18;
    else if (prec == FL_PREC_F32)
        fmt = gauge_reals == 18 ? LINK_F32_R18 : LINK_F32_R12;
    else if (prec == FL_PREC_BF16 && gauge_reals == 12)
        fmt = LINK_BF16_R12;
    else if (prec == FL_PREC_H16 && gauge_reals == 12)
        fmt = LINK_Q16_R12;
    else
        return set_err(c, FL_ERR_ARG, "unsupported precision / link storage");
    if (lds == 3 && fmt != LINK_Q16_R12) return set_err(c, FL_ERR_ARG, "lds 3 needs 16-bit fields");
    c->tune_rt[fmt] = rt;
    c->tune_g[fmt] = group;
    c->tune_lds[fmt] = lds;
    return FL_OK;
}

fl_status fl_autotune(fl_ctx *c, int prec, int gauge_reals, int nrhs, int *rt_out, int *group_out, int *lds_out,
                      double *ms_out)
{
    if (!valid_ctx(c)) return set_err(nullptr, FL_ERR_ARG, "ctx is NULL");
    if (nrhs < 1) return set_err(c, FL_ERR_ARG, "nrhs must be >= 1");
    fl_status e;
    if ((e = check_ready(c))) return e;
    LinkFormat fmt;
    if ((e = fmt_of(c, prec, gauge_reals, &fmt))) return e;
    const int maxrt = fmt == LINK_F64_R18 ? 8 : 16;
    double best = 1e300;
    int brt = 0, bg = 0, bl = 0;
    for (int lds = 0; lds <= 4; ++lds)
        for (int rt = 1; rt <= maxrt; rt *= 2) {
            if (lds == 3 && fmt != LINK_Q16_R12) break;
            if (rt > 1 && rt / 2 >= nrhs) break;
            int nrb = (nrhs + rt - 1) / rt;
            for (int g = 1;; g *= 2) {
                int gg = std::min(g, nrb);
                double ms = 0;
                // two buffer sets larger than the on-chip caches, a few repetitions
                e = bench_impl(c, fmt, nrhs, 6, 2, rt, gg, lds, &ms, nullptr);
                if (e == FL_ERR_ARG) break;  // staging does not fit this shape
                if (e) return e;
                if (ms < best) {
                    best = ms;
                    brt = rt;
                    bg = gg;
                    bl = lds;
                }
                if (gg == nrb) break;
            }
        }
    c->err.clear();
    c->tune_rt[fmt] = brt;
    c->tune_g[fmt] = bg;
    c->tune_lds[fmt] = bl;
    if (rt_out) *rt_out = brt;
    if (group_out) *group_out = bg;
    if (lds_out) *lds_out = bl;
    if (ms_out) *ms_out = best;
    return FL_OK;
}

}  // extern "C"

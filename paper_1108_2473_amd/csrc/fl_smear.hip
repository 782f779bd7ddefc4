// fl_smear.hip -- Gaussian smearing of quark fields and the connected
// pseudoscalar two-point function (Sec. III):
//
//   q_smear = F q,  F = ((1 + alpha H) / norm)^n,
//   H(x, y) = sum_{i=1..3} [U_i(x) delta_{x, y-i} + U_i(x-i)^+ delta_{x, y+i}]
//
// H acts on colour within each timeslice (spin is a spectator); norm = 1 is
// the paper's F, any other value rescales F by norm^-n (without it
// (1 + 4H)^50 grows to ~25^50).  The connected function of Eq. (all_corr)
// with Gamma_A = Gamma_B = g5 and a point source at y0 is, by
// g5-hermiticity G(y0; x) = g5 G(x; y0)^+ g5,
//
//   C(p, t) = sum_x exp(+i p.(x - y0)) sum_{b, beta} |phi_{b, beta}(x, t0 + t)|^2,
//   phi = F_sink D^-1 F_source e_{y0, b, beta},
//
// which the momentum-projection kernel evaluates on the density.
#include <cmath>
#include <cstring>
#include <vector>

#include "fl_host.h"

namespace {

constexpr int BLK = 256;
constexpr int SM_RT = BLK / FL_WAVE;  // right-hand sides per smearing workgroup
constexpr double kPi = 3.14159265358979323846;

struct SmearArgs {
    const double2 *same;   // input field of the output parity  [nrhs][12][Vh]
    const double2 *other;  // input field of the other parity
    double2 *out;          // output field                      [nrhs][12][Vh]
    const double2 *gauge;  // FP64 18-real links [mu][par][9][Vh]
    LatGeom g;
    int nrhs, par;
    double alpha, inv_norm;
};

// acc += alpha * M psi (spin components independently), M = U or U^+
template <bool ADJ>
__device__ __forceinline__ void colour_hop(cx<double> acc[12], const cx<double> U[3][3], const cx<double> psi[12],
                                           double alpha)
{
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cx<double> v = ADJ ? cjmul(U[0][a], psi[3 * s]) : U[a][0] * psi[3 * s];
#pragma unroll
            for (int b = 1; b < 3; ++b) v = ADJ ? cjmad(v, U[b][a], psi[3 * s + b]) : cmad(v, U[a][b], psi[3 * s + b]);
            acc[3 * s + a] = cx<double>{fma(alpha, v.re, acc[3 * s + a].re), fma(alpha, v.im, acc[3 * s + a].im)};
        }
}

// one step of (1 + alpha H) / norm for the sites of parity `par`.  A
// workgroup is a tile of FL_WAVE sites x SM_RT right-hand sides (one wave
// each), tiles in XCD-contiguous order with the right-hand-side groups of a
// site block consecutive: the links of a site block are read by its waves
// within one CU and one XCD's L2 instead of once per right-hand side from
// HBM (in site-major order a site's right-hand sides were Vh / BLK
// workgroups apart, on different XCDs)
__global__ __launch_bounds__(BLK) void k_smear(SmearArgs a)
{
    const LatGeom &g = a.g;
    const int nrg = (a.nrhs + SM_RT - 1) / SM_RT;
    const int tile = xcd_tile(blockIdx.x, gridDim.x, 0);
    const int sb = tile / nrg, rg = tile - sb * nrg;
    const int rhs = rg * SM_RT + (int)threadIdx.x / FL_WAVE, i = sb * FL_WAVE + (int)threadIdx.x % FL_WAVE;
    if (rhs >= a.nrhs || i >= g.Vh) return;
    const size_t fs = (size_t)12 * g.Vh;
    const Coord c = cb_coords(g, a.par, i);
    cx<double> acc[12], psi[12], U[3][3];
    SpinorFmt<double>::load(a.same + rhs * fs, g.Vh, i, acc);
    const int Lh0 = g.Lh0, xh = c.x >> 1, Ly = g.L[1], Lz = g.L[2];
    for (int mu = 0; mu < 3; ++mu) {
        int nf, nb;
        if (mu == 0) {
            const int xf = (c.x + 1 == g.L[0]) ? 0 : c.x + 1, xb = (c.x == 0) ? g.L[0] - 1 : c.x - 1;
            nf = (xf >> 1) + Lh0 * c.rest;
            nb = (xb >> 1) + Lh0 * c.rest;
        } else if (mu == 1) {
            const int yf = (c.y + 1 == Ly) ? 0 : c.y + 1, yb = (c.y == 0) ? Ly - 1 : c.y - 1;
            const int zt = Ly * (c.z + Lz * c.t);
            nf = xh + Lh0 * (yf + zt);
            nb = xh + Lh0 * (yb + zt);
        } else {
            const int zf = (c.z + 1 == Lz) ? 0 : c.z + 1, zb = (c.z == 0) ? Lz - 1 : c.z - 1;
            const int base = xh + Lh0 * c.y, st = Lh0 * Ly;
            nf = base + st * (zf + Lz * c.t);
            nb = base + st * (zb + Lz * c.t);
        }
        // U_mu(x) psi(x + mu): link stored with the site's parity
        link_load<LinkF64R18>(a.gauge + (size_t)(mu * 2 + a.par) * 9 * g.Vh, g.Vh, i, U);
        SpinorFmt<double>::load(a.other + rhs * fs, g.Vh, nf, psi);
        colour_hop<false>(acc, U, psi, a.alpha);
        // U_mu(x - mu)^+ psi(x - mu): link stored at the neighbour
        link_load<LinkF64R18>(a.gauge + (size_t)(mu * 2 + 1 - a.par) * 9 * g.Vh, g.Vh, nb, U);
        SpinorFmt<double>::load(a.other + rhs * fs, g.Vh, nb, psi);
        colour_hop<true>(acc, U, psi, a.alpha);
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = cx<double>{acc[k].re * a.inv_norm, acc[k].im * a.inv_norm};
    SpinorFmt<double>::store(a.out + rhs * fs, g.Vh, i, acc);
}

// rho[s] = sum over right-hand sides and components of |phi|^2 at canonical site s
__global__ __launch_bounds__(BLK) void k_density(const double *__restrict__ phi, double2 *rho, long long V, int nrhs)
{
    const long long s = blockIdx.x * (long long)BLK + threadIdx.x;
    if (s >= V) return;
    double acc = 0.0;
    for (int r = 0; r < nrhs; ++r) {
        const double *p = phi + ((size_t)r * V + s) * 24;
        for (int k = 0; k < 24; ++k) acc = fma(p[k], p[k], acc);
    }
    rho[s] = make_double2(acc, 0.0);  // one store, ends the kernel
}

// the 12 spin-colour point sources at canonical site y0 (fields cleared before)
__global__ void k_canon_point(double *src, long long V, long long y0)
{
    const int k = threadIdx.x;
    if (k < 12) src[((size_t)k * V + y0) * 24 + 2 * k] = 1.0;  // one store, ends the kernel
}

unsigned blocks(long long n) { return (unsigned)((n + BLK - 1) / BLK); }

// ---------------------------------------------------------------------------
// APE smearing of the spatial links (the links of H; Sec. III)
// ---------------------------------------------------------------------------
typedef cx<double> M3[3][3];

__device__ __forceinline__ void m3_load(const double *U, long long V, int mu, long long s, M3 m)
{
    const double *p = U + ((size_t)mu * V + s) * 18;
#pragma unroll
    for (int e = 0; e < 9; ++e) m[e / 3][e % 3] = cx<double>{p[2 * e], p[2 * e + 1]};
}

// c = a b (ADJB: a b^+; ADJA: a^+ b)
template <bool ADJA, bool ADJB>
__device__ __forceinline__ void m3_mul(const M3 a, const M3 b, M3 c)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<double> acc{0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const cx<double> x = ADJA ? cj(a[k][i]) : a[i][k];
                const cx<double> y = ADJB ? cj(b[j][k]) : b[k][j];
                acc = cmad(acc, x, y);
            }
            c[i][j] = acc;
        }
}

__device__ __forceinline__ cx<double> m3_det(const M3 m)
{
    return m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
           m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
}

__device__ __forceinline__ double m3_norm2(const M3 m)
{
    double s = 0.0;
#pragma unroll
    for (int e = 0; e < 9; ++e) s += m[e / 3][e % 3].re * m[e / 3][e % 3].re + m[e / 3][e % 3].im * m[e / 3][e % 3].im;
    return s;
}

// the SU(3) matrix assigned to a nonsingular V: the unitary factor W of the
// polar decomposition V = W P, by the scaled Newton iteration
// W <- (g W + (g W)^{-+}) / 2 (Higham 1986; quadratic convergence, g the
// Frobenius-norm scaling), divided by exp(i arg(det W) / 3), arg in (-pi, pi]
__device__ void su3_project(M3 W)
{
    for (int it = 0; it < 40; ++it) {
        // inverse by the adjugate: inv[i][j] = cof[j][i] / det
        const cx<double> d = m3_det(W);
        const double dd = d.re * d.re + d.im * d.im;
        const cx<double> di{d.re / dd, -d.im / dd};
        M3 inv;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int r0 = (j + 1) % 3, r1 = (j + 2) % 3, c0 = (i + 1) % 3, c1 = (i + 2) % 3;
                inv[i][j] = (W[r0][c0] * W[r1][c1] - W[r0][c1] * W[r1][c0]) * di;
            }
        const double g = it < 6 ? sqrt(sqrt(m3_norm2(inv) / m3_norm2(W))) : 1.0;
        double delta = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                // (inv^+)[i][j] = conj(inv[j][i])
                const cx<double> n{0.5 * (g * W[i][j].re + inv[j][i].re / g), 0.5 * (g * W[i][j].im - inv[j][i].im / g)};
                delta += (n.re - W[i][j].re) * (n.re - W[i][j].re) + (n.im - W[i][j].im) * (n.im - W[i][j].im);
                W[i][j] = n;
            }
        if (g == 1.0 && delta < 1e-30) break;
    }
    const cx<double> d = m3_det(W);
    const double ph = -atan2(d.im, d.re) / 3.0;
    const cx<double> f{cos(ph), sin(ph)};
#pragma unroll
    for (int e = 0; e < 9; ++e) W[e / 3][e % 3] = W[e / 3][e % 3] * f;
}

struct ApeArgs {
    const double *in;  // canonical links [4][V][3][3][2]
    double *out;
    long long V;
    int L[4];
    double alpha;
};

// one APE step for the spatial link (i, s); the time links are copied
__global__ __launch_bounds__(BLK) void k_ape_step(ApeArgs a)
{
    const long long id = blockIdx.x * (long long)BLK + threadIdx.x;
    if (id >= 4 * a.V) return;
    const int i = (int)(id / a.V);
    const long long s = id - (long long)i * a.V;
    double *o = a.out + ((size_t)i * a.V + s) * 18;
    const double *p = a.in + ((size_t)i * a.V + s) * 18;
    if (i == 3) {
        double v[18];
#pragma unroll
        for (int k = 0; k < 18; ++k) v[k] = p[k];
        double *const q[18] = {o, o + 1, o + 2, o + 3, o + 4, o + 5, o + 6, o + 7, o + 8,
                               o + 9, o + 10, o + 11, o + 12, o + 13, o + 14, o + 15, o + 16, o + 17};
        ptr_store_group<18, double>(q, v);
        return;
    }
    int x[4];
    long long r = s;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        x[m] = (int)(r % a.L[m]);
        r /= a.L[m];
    }
    auto idx = [&](const int y[4]) -> long long {
        return y[0] + (long long)a.L[0] * (y[1] + (long long)a.L[1] * (y[2] + (long long)a.L[2] * y[3]));
    };
    M3 acc, A, B, C, T1, T2;
    m3_load(a.in, a.V, i, s, acc);
    int xi[4] = {x[0], x[1], x[2], x[3]};
    xi[i] = (x[i] + 1) % a.L[i];
    for (int j = 0; j < 3; ++j) {
        if (j == i) continue;
        int xj[4] = {x[0], x[1], x[2], x[3]}, xmj[4] = {x[0], x[1], x[2], x[3]};
        xj[j] = (x[j] + 1) % a.L[j];
        xmj[j] = (x[j] + a.L[j] - 1) % a.L[j];
        int xmji[4] = {xmj[0], xmj[1], xmj[2], xmj[3]};
        xmji[i] = (xmj[i] + 1) % a.L[i];
        // U_j(x) U_i(x + j) U_j(x + i)^+
        m3_load(a.in, a.V, j, s, A);
        m3_load(a.in, a.V, i, idx(xj), B);
        m3_load(a.in, a.V, j, idx(xi), C);
        m3_mul<false, false>(A, B, T1);
        m3_mul<false, true>(T1, C, T2);
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            acc[e / 3][e % 3].re = fma(a.alpha, T2[e / 3][e % 3].re, acc[e / 3][e % 3].re);
            acc[e / 3][e % 3].im = fma(a.alpha, T2[e / 3][e % 3].im, acc[e / 3][e % 3].im);
        }
        // U_j(x - j)^+ U_i(x - j) U_j(x - j + i)
        m3_load(a.in, a.V, j, idx(xmj), A);
        m3_load(a.in, a.V, i, idx(xmj), B);
        m3_load(a.in, a.V, j, idx(xmji), C);
        m3_mul<true, false>(A, B, T1);
        m3_mul<false, false>(T1, C, T2);
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            acc[e / 3][e % 3].re = fma(a.alpha, T2[e / 3][e % 3].re, acc[e / 3][e % 3].re);
            acc[e / 3][e % 3].im = fma(a.alpha, T2[e / 3][e % 3].im, acc[e / 3][e % 3].im);
        }
    }
    su3_project(acc);
    double v[18];
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        v[2 * e] = acc[e / 3][e % 3].re;
        v[2 * e + 1] = acc[e / 3][e % 3].im;
    }
    double *const q[18] = {o, o + 1, o + 2, o + 3, o + 4, o + 5, o + 6, o + 7, o + 8,
                           o + 9, o + 10, o + 11, o + 12, o + 13, o + 14, o + 15, o + 16, o + 17};
    ptr_store_group<18, double>(q, v);
}

// links of the smearing kernel H: APE-smeared when fl_ape_smear made them
const double2 *smear_links(fl_ctx *c)
{
    if (c->smear_ok && c->smear_gauge) return (const double2 *)c->smear_gauge;
    return (const double2 *)links(c, LINK_F64_R18);
}

// F^n on canonical fields in place (device), through checkerboard copies
fl_status smear_canon(fl_ctx *c, double *canon, int nrhs, double alpha, int n, double norm)
{
    const size_t fb = (size_t)nrhs * c->Vh * 192;
    double2 *e0 = (double2 *)ws_get(c, WS_SM_E0, fb), *o0 = (double2 *)ws_get(c, WS_SM_O0, fb);
    double2 *e1 = (double2 *)ws_get(c, WS_SM_E1, fb), *o1 = (double2 *)ws_get(c, WS_SM_O1, fb);
    const double2 *gauge = smear_links(c);
    if (!e0 || !o0 || !e1 || !o1 || !gauge) return set_err(c, FL_ERR_NOMEM, "device allocation failed (smearing)");
    LatGeom g = lat_geom(c, nrhs);
    launch_canon_to_eo(canon, e0, o0, g, nrhs, c->stream);
    // tiles of FL_WAVE sites x SM_RT right-hand sides
    const unsigned nb = (unsigned)(((c->Vh + FL_WAVE - 1) / FL_WAVE) * (long long)((nrhs + SM_RT - 1) / SM_RT));
    for (int k = 0; k < n; ++k) {
        SmearArgs a{e0, o0, e1, gauge, g, nrhs, 0, alpha, 1.0 / norm};
        hipLaunchKernelGGL(k_smear, dim3(nb), dim3(BLK), 0, c->stream, a);
        SmearArgs b{o0, e0, o1, gauge, g, nrhs, 1, alpha, 1.0 / norm};
        hipLaunchKernelGGL(k_smear, dim3(nb), dim3(BLK), 0, c->stream, b);
        std::swap(e0, e1);
        std::swap(o0, o1);
    }
    launch_eo_to_canon(e0, o0, canon, g, nrhs, c->stream);
    return hip_check(c, hipGetLastError(), "smearing");
}

}  // namespace

fl_status fl_smear(fl_ctx *c, double *psi, int nrhs, double alpha, int n, double norm, fl_where where)
{
    if (!c) return set_err(nullptr, FL_ERR_ARG, "ctx is NULL");
    if (nrhs < 0 || (nrhs > 0 && !psi) || n < 0 || !(norm > 0) || !std::isfinite(alpha) || !std::isfinite(norm))
        return set_err(c, FL_ERR_ARG, "bad smearing arguments (nrhs >= 0, n >= 0, norm > 0, finite alpha)");
    if (where != FL_HOST && where != FL_DEVICE) return set_err(c, FL_ERR_ARG, "bad `where`");
    if (!c->have_gauge) return set_err(c, FL_ERR_STATE, "gauge field not set (fl_set_gauge)");
    if (nrhs == 0 || n == 0) return FL_OK;
    hipSetDevice(c->device);
    const size_t per = (size_t)c->V * 24 * sizeof(double);
    fl_status e;
    for (int k0 = 0; k0 < nrhs; k0 += 12) {
        const int m = std::min(12, nrhs - k0);
        double *f = psi + (size_t)k0 * c->V * 24;
        if (where == FL_HOST) {
            double *d = (double *)ws_get(c, WS_PI_SRC, per * m);
            if (!d) return set_err(c, FL_ERR_NOMEM, "device allocation failed");
            if ((e = hip_check(c, hipMemcpyAsync(d, f, per * m, hipMemcpyHostToDevice, c->stream), "upload"))) return e;
            if ((e = smear_canon(c, d, m, alpha, n, norm))) return e;
            if ((e = hip_check(c, hipMemcpyAsync(f, d, per * m, hipMemcpyDeviceToHost, c->stream), "download")))
                return e;
        } else if ((e = smear_canon(c, f, m, alpha, n, norm))) {
            return e;
        }
    }
    return hip_check(c, hipStreamSynchronize(c->stream), "smearing");
}

fl_status fl_pion_corr(fl_ctx *c, long long y0, const fl_solver_params *p, double alpha, int n, double norm,
                       int smear_source, int smear_sink, const int *mom, int nmom, double *C, fl_where where)
{
    if (!c) return set_err(nullptr, FL_ERR_ARG, "ctx is NULL");
    if (y0 < 0 || y0 >= c->V) return set_err(c, FL_ERR_ARG, "source site outside the lattice");
    if (nmom < 1 || !mom || !C || !p) return set_err(c, FL_ERR_ARG, "need params, nmom >= 1, mom and C");
    if (!momproj_fits(c->L)) return set_err(c, FL_ERR_ARG, "momentum projection needs Lx + Ly + Lz <= 1024");
    if ((smear_source || smear_sink) && (n < 0 || !(norm > 0) || !std::isfinite(alpha)))
        return set_err(c, FL_ERR_ARG, "bad smearing arguments (n >= 0, norm > 0, finite alpha)");
    if (where != FL_HOST && where != FL_DEVICE) return set_err(c, FL_ERR_ARG, "bad `where`");
    if (!c->have_gauge || !c->have_kappa) return set_err(c, FL_ERR_STATE, "gauge field and kappa must be set");
    hipSetDevice(c->device);
    const long long V = c->V;
    const int Vs = c->L[0] * c->L[1] * c->L[2], T = c->L[3];
    const size_t per = (size_t)V * 24 * sizeof(double);
    double *src = (double *)ws_get(c, WS_PI_SRC, 12 * per), *sol = (double *)ws_get(c, WS_PI_SOL, 12 * per);
    double2 *rho = (double2 *)ws_get(c, WS_PI_RHO, (size_t)V * sizeof(double2));
    double2 *P = (double2 *)ws_get(c, WS_CORR_OUT, (size_t)nmom * T * sizeof(double2));
    int *dmom = (int *)ws_get(c, WS_CORR_IDX, sizeof(int) * 3 * (size_t)nmom);
    if (!src || !sol || !rho || !P || !dmom) return set_err(c, FL_ERR_NOMEM, "device allocation failed");
    fl_status e;
    // the 12 spin-colour point sources at y0 (canonical layout: spin, colour, re/im)
    if ((e = hip_check(c, hipMemsetAsync(src, 0, 12 * per, c->stream), "clear sources"))) return e;
    hipLaunchKernelGGL(k_canon_point, dim3(1), dim3(64), 0, c->stream, src, V, y0);
    if (smear_source && n > 0 && (e = smear_canon(c, src, 12, alpha, n, norm))) return e;
    std::vector<fl_solver_stats> st(12);
    // a solve that misses tol is not fatal: the correlator is built from the
    // best iterates and the status is returned at the end
    fl_status se = fl_solve(c, src, sol, 12, p, st.data(), FL_DEVICE);
    if (se != FL_OK && se != FL_ERR_NOCONV && se != FL_ERR_BREAKDOWN) return se;
    if (smear_sink && n > 0 && (e = smear_canon(c, sol, 12, alpha, n, norm))) return e;
    hipLaunchKernelGGL(k_density, dim3(blocks(V)), dim3(BLK), 0, c->stream, sol, rho, V, 12);
    if ((e = hip_check(c, hipMemcpyAsync(dmom, mom, sizeof(int) * 3 * (size_t)nmom, hipMemcpyHostToDevice,
                                         c->stream), "upload momenta")))
        return e;
    launch_momproj(rho, P, dmom, 1, T, nmom, c->L, c->stream);
    std::vector<double> hp((size_t)nmom * T * 2), out((size_t)nmom * T * 2);
    if ((e = hip_check(c, hipMemcpyAsync(hp.data(), P, hp.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream),
                       "download")) ||
        (e = hip_check(c, hipStreamSynchronize(c->stream), "pion correlator")))
        return e;
    // C[k][t] = exp(-i p_k.x0) P[k][(t0 + t) mod T]: phase of the source position, time from the source
    const long long t0 = y0 / Vs, xs0 = y0 % Vs;
    const int x0[3] = {(int)(xs0 % c->L[0]), (int)((xs0 / c->L[0]) % c->L[1]), (int)(xs0 / (c->L[0] * c->L[1]))};
    for (int k = 0; k < nmom; ++k) {
        double ph = 0.0;
        for (int d = 0; d < 3; ++d) ph += (double)mom[3 * k + d] * x0[d] / c->L[d];
        const double cs = std::cos(2.0 * kPi * ph), sn = -std::sin(2.0 * kPi * ph);
        for (int t = 0; t < T; ++t) {
            const size_t q = ((size_t)k * T + (size_t)((t0 + t) % T)) * 2;
            out[((size_t)k * T + t) * 2] = cs * hp[q] - sn * hp[q + 1];
            out[((size_t)k * T + t) * 2 + 1] = cs * hp[q + 1] + sn * hp[q];
        }
    }
    if (where == FL_HOST) {
        std::memcpy(C, out.data(), out.size() * sizeof(double));
        return se == FL_OK ? FL_OK : set_err(c, se, "some point-source solves did not reach tol (fl_last_stats)");
    }
    if ((e = hip_check(c, hipMemcpyAsync(C, out.data(), out.size() * sizeof(double), hipMemcpyHostToDevice,
                                         c->stream), "upload result")))
        return e;
    if ((e = hip_check(c, hipStreamSynchronize(c->stream), "pion correlator"))) return e;
    return se == FL_OK ? FL_OK : set_err(c, se, "some point-source solves did not reach tol (fl_last_stats)");
}

fl_status fl_ape_smear(fl_ctx *c, double alpha, int n, double *Uout, fl_where where)
{
    if (!c) return set_err(nullptr, FL_ERR_ARG, "ctx is NULL");
    if (!(alpha >= 0) || !std::isfinite(alpha) || n < 0)
        return set_err(c, FL_ERR_ARG, "APE smearing needs a finite alpha >= 0 and n >= 0");
    if (where != FL_HOST && where != FL_DEVICE) return set_err(c, FL_ERR_ARG, "bad `where`");
    if (!c->have_gauge) return set_err(c, FL_ERR_STATE, "gauge field not set (fl_set_gauge)");
    hipSetDevice(c->device);
    const size_t ub = (size_t)4 * c->V * 18 * sizeof(double);
    fl_status e;
    double *cur = c->gauge_canon;
    if (n > 0) {
        double *b0 = (double *)ws_get(c, WS_APE0, ub), *b1 = (double *)ws_get(c, WS_APE1, ub);
        if (!b0 || !b1) return set_err(c, FL_ERR_NOMEM, "device allocation failed (APE smearing)");
        if (!c->smear_gauge && hipMalloc(&c->smear_gauge, link_bytes(LINK_F64_R18) * 4 * (size_t)c->V) != hipSuccess) {
            c->smear_gauge = nullptr;
            (void)hipGetLastError();
            return set_err(c, FL_ERR_NOMEM, "device allocation failed (APE-smeared links)");
        }
        ApeArgs a;
        a.V = c->V;
        for (int m = 0; m < 4; ++m) a.L[m] = c->L[m];
        a.alpha = alpha;
        for (int k = 0; k < n; ++k) {
            a.in = cur;
            a.out = (k % 2 == 0) ? b0 : b1;
            hipLaunchKernelGGL(k_ape_step, dim3(blocks(4 * c->V)), dim3(BLK), 0, c->stream, a);
            cur = a.out;
        }
        launch_pack_links(cur, c->smear_gauge, LINK_F64_R18, lat_geom(c, 0), c->stream);
        c->smear_ok = true;
    } else {
        c->smear_ok = false;
    }
    if (Uout &&
        (e = hip_check(c, hipMemcpyAsync(Uout, cur, ub, where == FL_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                         c->stream), "copy APE-smeared links")))
        return e;
    return hip_check(c, hipStreamSynchronize(c->stream), "APE smearing");
}

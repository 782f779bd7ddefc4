// fl_fields.hip -- kernels around the solver: layout conversion between the
// canonical lexicographic arrays and the checkerboard device fields, link
// packing per precision, point and noise sources, the loop contractions of
// Eq. (loop) and Eq. (loop stochastic), and the gradient kernels.
#include "fl_host.h"
#include "fl_stencil.h"

namespace {

struct LexSite {
    int x, y, z, t, par, cb;
};

__device__ __forceinline__ LexSite lex_site(const LatGeom &g, long long s)
{
    LexSite r;
    r.x = (int)(s % g.L[0]);
    s /= g.L[0];
    r.y = (int)(s % g.L[1]);
    s /= g.L[1];
    r.z = (int)(s % g.L[2]);
    r.t = (int)(s / g.L[2]);
    r.par = (r.x + r.y + r.z + r.t) & 1;
    r.cb = cb_index(g, r.x, r.y, r.z, r.t);
    return r;
}

__device__ __forceinline__ long long lex_of(const LatGeom &g, int x, int y, int z, int t)
{
    return x + (long long)g.L[0] * (y + (long long)g.L[1] * (z + (long long)g.L[2] * t));
}

// --- layout conversion --------------------------------------------------
__global__ void k_canon_to_eo(const double *__restrict__ canon, double2 *even, double2 *odd,
                              LatGeom g, int nrhs)
{
    long long V = 2LL * g.Vh;
    long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (id >= V * nrhs) return;
    int rhs = (int)(id / V);
    long long s = id - (long long)rhs * V;
    LexSite ls = lex_site(g, s);
    double2 *f = (ls.par ? odd : even) + (size_t)rhs * 12 * g.Vh;
    const double *src = canon + (size_t)id * 24;
    double2 *p[12];
    double2 v[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        p[c] = f + (size_t)c * g.Vh + ls.cb;
        v[c] = make_double2(src[2 * c], src[2 * c + 1]);
    }
    ptr_store_group(p, v);
}

__global__ void k_eo_to_canon(const double2 *even, const double2 *odd, double *__restrict__ canon,
                              LatGeom g, int nrhs)
{
    long long V = 2LL * g.Vh;
    long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (id >= V * nrhs) return;
    int rhs = (int)(id / V);
    long long s = id - (long long)rhs * V;
    LexSite ls = lex_site(g, s);
    const double2 *f = (ls.par ? odd : even) + (size_t)rhs * 12 * g.Vh;
    double2 *dst = (double2 *)(canon + (size_t)id * 24);
    double2 *p[12];
    double2 v[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        v[c] = f[(size_t)c * g.Vh + ls.cb];
        p[c] = dst + c;
    }
    ptr_store_group(p, v);
}

// --- links --------------------------------------------------------------
__global__ void k_pack_links(const double *__restrict__ canon, void *dst, int fmt, LatGeom g)
{
    long long V = 2LL * g.Vh;
    long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (id >= 4 * V) return;
    int mu = (int)(id / V);
    long long s = id - (long long)mu * V;
    LexSite ls = lex_site(g, s);
    const double *u = canon + (size_t)id * 18;
    const size_t Vh = g.Vh;
    size_t base = (size_t)(mu * 2 + ls.par);
    if (fmt == LINK_F64_R18) {
        double2 *d = (double2 *)dst + base * 9 * Vh;
        double2 *p[9];
        double2 v[9];
        for (int c = 0; c < 9; ++c) {
            p[c] = d + c * Vh + ls.cb;
            v[c] = make_double2(u[2 * c], u[2 * c + 1]);
        }
        ptr_store_group(p, v);
    } else if (fmt == LINK_F32_R18) {
        float2 *d = (float2 *)dst + base * 9 * Vh;
        float2 *p[9];
        float2 v[9];
        for (int c = 0; c < 9; ++c) {
            p[c] = d + c * Vh + ls.cb;
            v[c] = make_float2((float)u[2 * c], (float)u[2 * c + 1]);
        }
        ptr_store_group(p, v);
    } else if (fmt == LINK_F32_R12) {
        float4 *d = (float4 *)dst + base * 3 * Vh;
        float4 *p[3];
        float4 v[3];
        for (int c = 0; c < 3; ++c) {
            p[c] = d + c * Vh + ls.cb;
            v[c] = make_float4((float)u[4 * c], (float)u[4 * c + 1], (float)u[4 * c + 2], (float)u[4 * c + 3]);
        }
        ptr_store_group(p, v);
    } else if (fmt == LINK_Q16_R12) {
        // round(32767 u) of each real of rows 0 and 1 (|u| <= 1 for SU(3))
        uint2 *d = (uint2 *)dst + base * 3 * Vh;
        uint2 *p[3];
        uint2 v[3];
        for (int c = 0; c < 3; ++c) {
            uint32_t q[4];
            for (int k = 0; k < 4; ++k) {
                double x = rint(32767.0 * u[4 * c + k]);
                x = x > 32767.0 ? 32767.0 : (x < -32767.0 ? -32767.0 : x);
                q[k] = (uint32_t)(uint16_t)(int16_t)(int)x;
            }
            p[c] = d + c * Vh + ls.cb;
            v[c] = make_uint2(q[0] | (q[1] << 16), q[2] | (q[3] << 16));
        }
        ptr_store_group(p, v);
    } else {
        uint2 *d = (uint2 *)dst + base * 3 * Vh;
        uint2 *p[3];
        uint2 v[3];
        for (int c = 0; c < 3; ++c) {
            // fp64 -> fp32 (nearest) -> bf16 (nearest even)
            uint32_t h0 = f32_to_bf16_rne((float)u[4 * c]), h1 = f32_to_bf16_rne((float)u[4 * c + 1]);
            uint32_t h2 = f32_to_bf16_rne((float)u[4 * c + 2]), h3 = f32_to_bf16_rne((float)u[4 * c + 3]);
            p[c] = d + c * Vh + ls.cb;
            v[c] = make_uint2(h0 | (h1 << 16), h2 | (h3 << 16));
        }
        ptr_store_group(p, v);
    }
}

__global__ void k_su3_check(const double *__restrict__ canon, double *blockmax, long long nlinks)
{
    __shared__ double red[256];
    long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    double dev = 0;
    if (id < nlinks) {
        const double *u = canon + (size_t)id * 18;
        cx<double> U[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) U[a][b] = cx<double>{u[2 * (3 * a + b)], u[2 * (3 * a + b) + 1]};
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                cx<double> acc{0, 0};
                for (int k = 0; k < 3; ++k) acc = acc + U[a][k] * cj(U[b][k]);
                double re = acc.re - (a == b ? 1.0 : 0.0);
                double m = sqrt(re * re + acc.im * acc.im);
                dev = m > dev ? m : dev;
            }
        cx<double> det = U[0][0] * (U[1][1] * U[2][2] - U[1][2] * U[2][1]) -
                         U[0][1] * (U[1][0] * U[2][2] - U[1][2] * U[2][0]) +
                         U[0][2] * (U[1][0] * U[2][1] - U[1][1] * U[2][0]);
        double m = sqrt((det.re - 1) * (det.re - 1) + det.im * det.im);
        dev = m > dev ? m : dev;
        if (!(dev == dev)) dev = 1e300;
    }
    red[threadIdx.x] = dev;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) blockmax[blockIdx.x] = red[0];
}

// --- sources --------------------------------------------------------------
__global__ void k_point_sources(double2 *even, double2 *odd, const long long *sites, int nsites, LatGeom g)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= 12 * nsites) return;
    int k = j / 12, c = j % 12;  // c = 3*spin + colour
    LexSite ls = lex_site(g, sites[k]);
    double2 *f = (ls.par ? odd : even) + (size_t)j * 12 * g.Vh;
    f[(size_t)c * g.Vh + ls.cb] = make_double2(1.0, 0.0);
}

// SplitMix64 (Steele, Lea, Flood 2014): output k of the generator whose state
// starts at `seed` is the 64-bit finaliser applied to seed + (k+1)*gamma with
// gamma = 0x9e3779b97f4a7c15.
__device__ __forceinline__ uint64_t splitmix_output(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1ULL) * 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double2 noise_value(int type, uint64_t h)
{
    int b63 = (int)(h >> 63), b62 = (int)((h >> 62) & 1ULL);
    if (type == FL_NOISE_Z4) {
        int q = 2 * b63 + b62;  // i^q
        const double re[4] = {1, 0, -1, 0}, im[4] = {0, 1, 0, -1};
        return make_double2(re[q], im[q]);
    } else if (type == FL_NOISE_CZ2) {
        const double r = 0.70710678118654752440;
        return make_double2(b63 ? -r : r, b62 ? -r : r);
    }
    return make_double2(b63 ? -1.0 : 1.0, 0.0);
}

__device__ __forceinline__ int space_class(int dil, int x, int y, int z)
{
    if (dil & FL_DIL_CUBIC) return (x & 1) + 2 * (y & 1) + 4 * (z & 1);
    if (dil & FL_DIL_EVENODD) return (x + y + z) & 1;
    return 0;
}

__device__ __forceinline__ bool in_support(int dil, const int *job, const LexSite &ls, int spin, int col)
{
    if ((dil & FL_DIL_TIME) && ls.t != job[JOB_T]) return false;
    if ((dil & FL_DIL_SPIN) && spin != job[JOB_SPIN]) return false;
    if ((dil & FL_DIL_COLOUR) && col != job[JOB_COL]) return false;
    if ((dil & (FL_DIL_CUBIC | FL_DIL_EVENODD)) && space_class(dil, ls.x, ls.y, ls.z) != job[JOB_CLASS])
        return false;
    return true;
}

__global__ void k_noise_sources(double2 *even, double2 *odd, NoiseBatch nb, LatGeom g)
{
    long long V = 2LL * g.Vh;
    long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (id >= V * nb.ncomp) return;
    int j = (int)(id / V);
    long long s = id - (long long)j * V;
    LexSite ls = lex_site(g, s);
    const int *job = nb.job + JOB_INTS * j;
    const uint64_t r = (uint64_t)(uint32_t)job[JOB_R];
    double2 *f = (ls.par ? odd : even) + (size_t)j * 12 * g.Vh;
    double2 *p[12];
    double2 v[12];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double2 x = make_double2(0.0, 0.0);
            if (in_support(nb.dil, job, ls, sp, a)) {
                uint64_t key = ((r * (uint64_t)V + (uint64_t)s) * 4 + (uint64_t)sp) * 3 + (uint64_t)a;
                x = noise_value(nb.type, splitmix_output(nb.seed, key));
            }
            v[3 * sp + a] = x;
            p[3 * sp + a] = f + (size_t)(3 * sp + a) * g.Vh + ls.cb;
        }
    ptr_store_group(p, v);
}

// --- contractions ---------------------------------------------------------
// one point-source site per thread: its 12 solutions at the site itself
__global__ void k_exact_contract(ExactContractArgs a)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.nsites) return;
    const LatGeom &g = a.g;
    LexSite ls = lex_site(g, a.sites[k]);
    const size_t fs = (size_t)12 * g.Vh;
    cx<double> S[4][4];
    for (int al = 0; al < 4; ++al)
        for (int be = 0; be < 4; ++be) S[al][be] = cx<double>{0, 0};
    for (int be = 0; be < 4; ++be)
        for (int col = 0; col < 3; ++col) {
            int j = 12 * k + 3 * be + col;
            cx<double> psi[12];
            if (ls.par == 0) {
                SpinorFmt<double>::load(a.xe + j * fs, g.Vh, ls.cb, psi);
            } else {
                // x_o = b_o + kappa (H_oe x_e) at this single site
                Coord c;
                c.x = ls.x;
                c.y = ls.y;
                c.z = ls.z;
                c.t = ls.t;
                c.rest = ls.y + g.L[1] * (ls.z + g.L[2] * ls.t);
                cx<double> h[12], b[12];
                PtrSrc<double, LinkF64R18> src{a.xe + j * fs, a.gauge, g.Vh};
                hop_site<false, double>(g, 1, ls.cb, c, src, h);
                SpinorFmt<double>::load(a.bo + j * fs, g.Vh, ls.cb, b);
                for (int q = 0; q < 12; ++q) psi[q] = b[q] + a.kappa * h[q];
            }
            for (int al = 0; al < 4; ++al) S[al][be] = S[al][be] + psi[3 * al + col];
        }
    for (int gi = 0; gi < a.ngamma; ++gi) {
        const double *G = a.gam + gi * 32;
        cx<double> acc{0, 0};
        for (int al = 0; al < 4; ++al)
            for (int be = 0; be < 4; ++be) {
                cx<double> gba{G[2 * (4 * be + al)], G[2 * (4 * be + al) + 1]};
                acc = acc + gba * S[al][be];
            }
        a.L[gi * a.L_stride + a.L_off + k] = make_double2(acc.re, acc.im);
        store_drain();  // one store per gamma (their number is a run-time value)
    }
    if (a.S) {
        double2 *p[16];
        double2 v[16];
        for (int al = 0; al < 4; ++al)
            for (int be = 0; be < 4; ++be) {
                p[4 * al + be] = a.S + (a.L_off + k) * 16 + 4 * al + be;
                v[4 * al + be] = make_double2(S[al][be].re, S[al][be].im);
            }
        ptr_store_group(p, v);
    }
}

// one estimated site (t, xs) per thread, summing over the batch's sources
// in order: acc[gamma] += sign * sum_{al, be, a} conj(eta_{al a}) Gamma_{al be} phi_{be a}
__global__ void k_stoch_contract(StochContractArgs a)
{
    const LatGeom &g = a.g;
    long long Vs = (long long)g.L[0] * g.L[1] * g.L[2];
    int nt = a.t_end - a.t_begin;
    long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (id >= Vs * nt) return;
    int tt = (int)(id / Vs);
    long long xs = id - tt * Vs;
    long long s = xs + Vs * (a.t_begin + tt);
    LexSite ls = lex_site(g, s);
    const size_t fs = (size_t)12 * g.Vh;
    const double2 *pf = ls.par ? a.po : a.pe;
    const double2 *nf = ls.par ? a.no : a.ne;
    cx<double> acc[2][16];
    for (int q = 0; q < 2; ++q)
        for (int gi = 0; gi < a.ngamma; ++gi) acc[q][gi] = cx<double>{0, 0};
    for (int j = 0; j < a.nrhs; ++j) {
        const int *job = a.job + JOB_INTS * j;
        if ((a.dil & FL_DIL_TIME) && job[JOB_T] != ls.t) continue;
        const int tgt = job[JOB_TARGET] ? 1 : 0;
        const double sg = (double)job[JOB_SIGN];
        cx<double> eta[12], phi[12];
        SpinorFmt<double>::load(nf + j * fs, g.Vh, ls.cb, eta);
        SpinorFmt<double>::load(pf + j * fs, g.Vh, ls.cb, phi);
        for (int gi = 0; gi < a.ngamma; ++gi) {
            const double *G = a.gam + gi * 32;
            cx<double> v{0, 0};
            for (int al = 0; al < 4; ++al)
                for (int be = 0; be < 4; ++be) {
                    cx<double> gab{G[2 * (4 * al + be)], G[2 * (4 * al + be) + 1]};
                    if (gab.re == 0 && gab.im == 0) continue;
                    for (int c = 0; c < 3; ++c) v = v + cjmul(eta[3 * al + c], gab * phi[3 * be + c]);
                }
            acc[tgt][gi] = acc[tgt][gi] + sg * v;
        }
    }
    for (int q = 0; q < 2; ++q) {
        double2 *base = q ? a.acc1 : a.acc0;
        if (!base) continue;
        for (int gi = 0; gi < a.ngamma; ++gi) {
            double2 *o = base + (gi * nt + tt) * Vs + xs;
            double2 cur = *o;
            *o = make_double2(cur.x + acc[q][gi].re, cur.y + acc[q][gi].im);
            store_drain();  // one store per gamma (their number is a run-time value)
        }
    }
}

// --- gradient ---------------------------------------------------------------
// chi_{y,be,b}(x) = g5 sum_al M_y[al][be] psi_{y,al,b}(x); thread per (site x, rhs)
__global__ void k_chi(ChiArgs a)
{
    const LatGeom &g = a.g;
    long long V = 2LL * g.Vh;
    int nrhs = 12 * a.nsites;
    long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (id >= V * nrhs) return;
    int j = (int)(id / V);
    long long rest = id - (long long)j * V;
    int par = (int)(rest / g.Vh);
    int cb = (int)(rest - (long long)par * g.Vh);
    int k = j / 12, be = (j % 12) / 3, col = j % 3;
    const size_t fs = (size_t)12 * g.Vh;
    const double2 *pf = par ? a.po : a.pe;
    double2 *cf = par ? a.co : a.ce;
    const double2 *M = a.M + (size_t)k * 16;
    cx<double> out[12];
    for (int q = 0; q < 12; ++q) out[q] = cx<double>{0, 0};
    for (int al = 0; al < 4; ++al) {
        double2 m = M[4 * al + be];
        cx<double> mm{m.x, m.y};
        if (m.x == 0 && m.y == 0) continue;
        cx<double> psi[12];
        SpinorFmt<double>::load(pf + (size_t)(12 * k + 3 * al + col) * fs, g.Vh, cb, psi);
        for (int q = 0; q < 12; ++q) out[q] = out[q] + mm * psi[q];
    }
    // g5 = diag(1, 1, -1, -1) in the chiral basis
    for (int q = 6; q < 12; ++q) out[q] = -out[q];
    SpinorFmt<double>::store(cf + (size_t)j * fs, g.Vh, cb, out);
}

// (1 + s g_mu) psi as a full 4-spinor, through the same projection as H
template <int MU, int S>
__device__ __forceinline__ void proj_full(const cx<double> psi[12], cx<double> out[12])
{
    cx<double> h[6];
    project<MU, S>(psi, h);
    for (int q = 0; q < 12; ++q) out[q] = cx<double>{0, 0};
    accumulate<MU, S>(out, h);
}

template <int MU>
__device__ void force_link(const ForceArgs &a, int par, int cb, int nf, double sgn, long long lex)
{
    const LatGeom &g = a.g;
    const size_t fs = (size_t)12 * g.Vh;
    const double2 *pe_x = par ? a.po : a.pe, *ce_x = par ? a.co : a.ce;
    const double2 *pe_f = par ? a.pe : a.po, *ce_f = par ? a.ce : a.co;
    cx<double> A[3][3], B[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) A[i][j] = B[i][j] = cx<double>{0, 0};
    for (int r = 0; r < a.nrhs; ++r) {
        cx<double> chi_x[12], psi_f[12], chi_f[12], psi_x[12], Pm[12], Pp[12];
        SpinorFmt<double>::load(ce_x + r * fs, g.Vh, cb, chi_x);
        SpinorFmt<double>::load(pe_f + r * fs, g.Vh, nf, psi_f);
        SpinorFmt<double>::load(ce_f + r * fs, g.Vh, nf, chi_f);
        SpinorFmt<double>::load(pe_x + r * fs, g.Vh, cb, psi_x);
        proj_full<MU, -1>(psi_f, Pm);  // (1 - g_mu) psi(x + mu)
        proj_full<MU, 1>(psi_x, Pp);   // (1 + g_mu) psi(x)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                for (int al = 0; al < 4; ++al) {
                    A[i][j] = A[i][j] + cjmul(chi_x[3 * al + i], Pm[3 * al + j]);
                    B[i][j] = B[i][j] + cjmul(chi_f[3 * al + i], Pp[3 * al + j]);
                }
    }
    double2 *o = a.dU + ((size_t)MU * 2 * g.Vh + lex) * 9;
    double f = a.kappa * sgn;
    double2 *p[9];
    double2 w[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            // entry (i, j): conj(A_ij) + B_ji
            cx<double> v = cj(A[i][j]) + B[j][i];
            double2 cur = o[3 * i + j];
            p[3 * i + j] = o + 3 * i + j;
            w[3 * i + j] = make_double2(cur.x + f * v.re, cur.y + f * v.im);
        }
    ptr_store_group(p, w);
}

__global__ void k_force(ForceArgs a)
{
    const LatGeom &g = a.g;
    long long V = 2LL * g.Vh;
    long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (id >= 4 * V) return;
    int mu = (int)(id / V);
    long long s = id - (long long)mu * V;
    LexSite ls = lex_site(g, s);
    int c[4] = {ls.x, ls.y, ls.z, ls.t};
    double sgn = 1.0;
    c[mu] += 1;
    if (c[mu] == g.L[mu]) {
        c[mu] = 0;
        if (mu == 3) sgn = (double)g.bc_t;
    }
    int nf = cb_index(g, c[0], c[1], c[2], c[3]);
    switch (mu) {
    case 0: force_link<0>(a, ls.par, ls.cb, nf, sgn, s); break;
    case 1: force_link<1>(a, ls.par, ls.cb, nf, sgn, s); break;
    case 2: force_link<2>(a, ls.par, ls.cb, nf, sgn, s); break;
    default: force_link<3>(a, ls.par, ls.cb, nf, sgn, s); break;
    }
}

// block partial sums of <a, b> over n complex entries
__global__ void k_dot64(const double2 *a, const double2 *b, long long n, double *out2)
{
    __shared__ double re[256], im[256];
    double sr = 0, si = 0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        double2 u = a[i], v = b[i];
        sr += u.x * v.x + u.y * v.y;
        si += u.x * v.y - u.y * v.x;
    }
    re[threadIdx.x] = sr;
    im[threadIdx.x] = si;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            re[threadIdx.x] += re[threadIdx.x + w];
            im[threadIdx.x] += im[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) ((double2 *)out2)[blockIdx.x] = make_double2(re[0], im[0]);  // one store, ends the kernel
}

// the two-estimator combination L = w0 a0 + w1 a1 (Sec. II, truncated
// solver method) in place of a0, reals of complex entries; each product is
// rounded before the sum (no fused multiply-add).  One element per thread,
// so the store ends the kernel.
__global__ void k_tsm_combine(double *a0, const double *a1, double w0, double w1, long long n)
{
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i < n) a0[i] = __dadd_rn(__dmul_rn(a0[i], w0), __dmul_rn(a1[i], w1));
}

inline unsigned nblk(long long n, int b = 256) { return (unsigned)((n + b - 1) / b); }

}  // namespace

void launch_canon_to_eo(const double *canon, double2 *even, double2 *odd, const LatGeom &g, int nrhs,
                        hipStream_t s)
{
    long long n = 2LL * g.Vh * nrhs;
    if (n) hipLaunchKernelGGL(k_canon_to_eo, dim3(nblk(n)), dim3(256), 0, s, canon, even, odd, g, nrhs);
}

void launch_eo_to_canon(const double2 *even, const double2 *odd, double *canon, const LatGeom &g,
                        int nrhs, hipStream_t s)
{
    long long n = 2LL * g.Vh * nrhs;
    if (n) hipLaunchKernelGGL(k_eo_to_canon, dim3(nblk(n)), dim3(256), 0, s, even, odd, canon, g, nrhs);
}

void launch_pack_links(const double *canon, void *dst, LinkFormat fmt, const LatGeom &g, hipStream_t s)
{
    long long n = 8LL * g.Vh;
    hipLaunchKernelGGL(k_pack_links, dim3(nblk(n)), dim3(256), 0, s, canon, dst, (int)fmt, g);
}

void launch_su3_check(const double *canon, double *blockmax, long long nlinks, hipStream_t s)
{
    hipLaunchKernelGGL(k_su3_check, dim3(nblk(nlinks)), dim3(256), 0, s, canon, blockmax, nlinks);
}

void launch_point_sources(double2 *even, double2 *odd, const long long *sites, int nsites,
                          const LatGeom &g, hipStream_t s)
{
    if (nsites)
        hipLaunchKernelGGL(k_point_sources, dim3(nblk(12LL * nsites)), dim3(256), 0, s, even, odd, sites,
                           nsites, g);
}

void launch_noise_sources(double2 *even, double2 *odd, const NoiseBatch &nb, const LatGeom &g, hipStream_t s)
{
    long long n = 2LL * g.Vh * nb.ncomp;
    if (n) hipLaunchKernelGGL(k_noise_sources, dim3(nblk(n)), dim3(256), 0, s, even, odd, nb, g);
}

void launch_exact_contract(const ExactContractArgs &a, hipStream_t s)
{
    if (a.nsites) hipLaunchKernelGGL(k_exact_contract, dim3(nblk(a.nsites, 64)), dim3(64), 0, s, a);
}

void launch_stoch_contract(const StochContractArgs &a, hipStream_t s)
{
    long long n = (long long)a.g.L[0] * a.g.L[1] * a.g.L[2] * (a.t_end - a.t_begin);
    if (n) hipLaunchKernelGGL(k_stoch_contract, dim3(nblk(n, 128)), dim3(128), 0, s, a);
}

void launch_chi(const ChiArgs &a, hipStream_t s)
{
    long long n = 2LL * a.g.Vh * 12 * a.nsites;
    if (n) hipLaunchKernelGGL(k_chi, dim3(nblk(n)), dim3(256), 0, s, a);
}

void launch_force(const ForceArgs &a, hipStream_t s)
{
    long long n = 8LL * a.g.Vh;
    if (a.nrhs) hipLaunchKernelGGL(k_force, dim3(nblk(n, 128)), dim3(128), 0, s, a);
}

void launch_tsm_combine(double *a0, const double *a1, double w0, double w1, long long n, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_tsm_combine, dim3(nblk(n)), dim3(256), 0, s, a0, a1, w0, w1, n);
}

void launch_dot64(const double2 *a, const double2 *b, long long n, double *out2, hipStream_t s)
{
    hipLaunchKernelGGL(k_dot64, dim3(256), dim3(256), 0, s, a, b, n, out2);
}

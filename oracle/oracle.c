/*
 * oracle.c -- plain, slow, FP64 CPU reference for disconnected fermion loops
 * (Alexandrou, Hadjiyiannakou, Koutsou, O Cais, Strelchenko, arXiv:1108.2473).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker, not the product: only
 * the test-suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no code, header, table or helper with the GPU
 * library; the two agree only through the published definitions below.
 *
 * Everything is written from the definitions, in double precision, with the
 * 4x4 Dirac matrices applied as full matrices (no spin projection, no
 * even-odd tricks beyond the Schur complement that the definition implies).
 *
 * Conventions (readings of points the paper leaves open):
 *  - site index s = x + Lx*(y + Ly*(z + Lz*t)); direction mu = 0..3 is x,y,z,t
 *    and gamma_{mu+1} is its Dirac matrix (gamma_4 is time, as the paper's
 *    nucleon projector Gamma_0 = (1+gamma_4)/4 in its Sec. IV implies).
 *  - gauge field U[mu][s][a][b] (complex, row a, column b); spinors
 *    psi[s][alpha][a] with alpha the spin and a the colour index.
 *  - Wilson operator in hopping normalisation (Sec. II: N_f=2 Wilson fermions
 *    at hopping parameter kappa; the form is not written in the paper):
 *      (D psi)(x) = psi(x) - kappa * sum_mu [ (1-g_mu) U_mu(x) psi(x+mu)
 *                                          + (1+g_mu) U_mu(x-mu)^+ psi(x-mu) ]
 *    periodic in space; a hop that crosses the time boundary is multiplied
 *    by bc_t (+1 periodic, -1 antiperiodic).  No phase is stored in links.
 *  - Dirac matrices: Hermitian, {g_mu, g_nu} = 2 delta, g_5 = g1 g2 g3 g4.
 *    basis 0 (chiral):  g_k = [[0,-i s_k],[i s_k,0]], g_4 = [[0,1],[1,0]]
 *    basis 1 (Dirac-Pauli): g_k as above, g_4 = [[1,0],[0,-1]].
 *  - Gamma insertion encoded as a 4-bit mask: Gamma = g1^b0 g2^b1 g3^b2 g4^b3
 *    (1 -> 0, g_mu -> 1<<(mu-1), g_5 -> 15).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* ------------------------------------------------------------------ */
/* geometry                                                           */
/* ------------------------------------------------------------------ */
typedef struct {
    int L[4];
    long V;
    int bc_t;
} geom;

static geom make_geom(const int *dims, int bc_t)
{
    geom g;
    for (int mu = 0; mu < 4; ++mu) g.L[mu] = dims[mu];
    g.V = (long)dims[0] * dims[1] * dims[2] * dims[3];
    g.bc_t = bc_t;
    return g;
}

static void coords(const geom *g, long s, int c[4])
{
    for (int mu = 0; mu < 4; ++mu) {
        c[mu] = (int)(s % g->L[mu]);
        s /= g->L[mu];
    }
}

static long index_of(const geom *g, const int c[4])
{
    return c[0] + (long)g->L[0] * (c[1] + (long)g->L[1] * (c[2] + (long)g->L[2] * c[3]));
}

/* neighbour of s in direction mu, step +1 or -1; *sign receives the
 * boundary factor of that hop (bc_t if it crosses the time boundary). */
static long neighbour(const geom *g, long s, int mu, int step, double *sign)
{
    int c[4];
    coords(g, s, c);
    *sign = 1.0;
    c[mu] += step;
    if (c[mu] == g->L[mu]) {
        c[mu] = 0;
        if (mu == 3) *sign = (double)g->bc_t;
    } else if (c[mu] < 0) {
        c[mu] = g->L[mu] - 1;
        if (mu == 3) *sign = (double)g->bc_t;
    }
    return index_of(g, c);
}

static int parity_of(const geom *g, long s)
{
    int c[4];
    coords(g, s, c);
    return (c[0] + c[1] + c[2] + c[3]) & 1;
}

/* ------------------------------------------------------------------ */
/* Dirac matrices                                                     */
/* ------------------------------------------------------------------ */
static void gamma_mu(int basis, int mu, cplx G[4][4])
{
    /* Pauli matrices s_1, s_2, s_3 */
    const cplx s[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -I}, {I, 0}},
        {{1, 0}, {0, -1}},
    };
    memset(G, 0, sizeof(cplx) * 16);
    if (mu < 3) {
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                G[i][2 + j] = -I * s[mu][i][j];
                G[2 + i][j] = I * s[mu][i][j];
            }
    } else if (basis == 0) {
        for (int i = 0; i < 2; ++i) {
            G[i][2 + i] = 1;
            G[2 + i][i] = 1;
        }
    } else {
        G[0][0] = G[1][1] = 1;
        G[2][2] = G[3][3] = -1;
    }
}

static void matmul4(const cplx A[4][4], const cplx B[4][4], cplx C[4][4])
{
    cplx T[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cplx acc = 0;
            for (int k = 0; k < 4; ++k) acc += A[i][k] * B[k][j];
            T[i][j] = acc;
        }
    memcpy(C, T, sizeof(T));
}

/* Gamma = g1^b0 g2^b1 g3^b2 g4^b3 for mask (b3 b2 b1 b0). */
static void gamma_mask(int basis, int mask, cplx G[4][4])
{
    memset(G, 0, sizeof(cplx) * 16);
    for (int i = 0; i < 4; ++i) G[i][i] = 1;
    for (int mu = 0; mu < 4; ++mu)
        if (mask & (1 << mu)) {
            cplx g[4][4];
            gamma_mu(basis, mu, g);
            matmul4(G, g, G);
        }
}

void or_gamma(int basis, int mask, double *out)
{
    cplx G[4][4];
    gamma_mask(basis, mask, G);
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            out[2 * (4 * i + j)] = creal(G[i][j]);
            out[2 * (4 * i + j) + 1] = cimag(G[i][j]);
        }
}

/* projectors (1 - g_mu) and (1 + g_mu) for the 4 directions */
typedef struct {
    cplx minus[4][4][4];
    cplx plus[4][4][4];
} projectors;

static void make_projectors(int basis, projectors *P)
{
    for (int mu = 0; mu < 4; ++mu) {
        cplx g[4][4];
        gamma_mu(basis, mu, g);
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                cplx id = (i == j) ? 1.0 : 0.0;
                P->minus[mu][i][j] = id - g[i][j];
                P->plus[mu][i][j] = id + g[i][j];
            }
    }
}

/* ------------------------------------------------------------------ */
/* hopping term                                                       */
/* ------------------------------------------------------------------ */
#define LINK(U, g, mu, s) ((U) + (((size_t)(mu) * (g)->V + (size_t)(s)) * 9))
#define SPIN(p, s) ((p) + (size_t)(s) * 12)

/*
 * out(x) = sum_mu [ Pf_mu U_mu(x) in(x+mu) + Pb_mu U_mu(x-mu)^+ in(x-mu) ]
 * for the sites x of parity out_parity (all sites if out_parity < 0);
 * other output sites are set to zero.  dagger = 0 uses Pf = 1-g, Pb = 1+g
 * (the hopping term of D); dagger = 1 uses Pf = 1+g, Pb = 1-g, which is the
 * adjoint of the former because each g_mu is Hermitian.
 */
static void hop(const geom *g, const projectors *P, const cplx *U, const cplx *in,
                cplx *out, int out_parity, int dagger)
{
#pragma omp parallel for schedule(static)
    for (long x = 0; x < g->V; ++x) {
        cplx *o = SPIN(out, x);
        for (int k = 0; k < 12; ++k) o[k] = 0;
        if (out_parity >= 0 && parity_of(g, x) != out_parity) continue;
        for (int mu = 0; mu < 4; ++mu) {
            const cplx(*Pf)[4] = dagger ? P->plus[mu] : P->minus[mu];
            const cplx(*Pb)[4] = dagger ? P->minus[mu] : P->plus[mu];
            double sf, sb;
            long xf = neighbour(g, x, mu, +1, &sf);
            long xb = neighbour(g, x, mu, -1, &sb);
            const cplx *Uf = LINK(U, g, mu, x);  /* U_mu(x) */
            const cplx *Ub = LINK(U, g, mu, xb); /* U_mu(x-mu) */
            const cplx *pf = SPIN(in, xf);
            const cplx *pb = SPIN(in, xb);
            cplx vf[4][3], vb[4][3];
            for (int al = 0; al < 4; ++al)
                for (int a = 0; a < 3; ++a) {
                    cplx af = 0, ab = 0;
                    for (int b = 0; b < 3; ++b) {
                        af += Uf[3 * a + b] * pf[3 * al + b];
                        ab += conj(Ub[3 * b + a]) * pb[3 * al + b];
                    }
                    vf[al][a] = sf * af;
                    vb[al][a] = sb * ab;
                }
            for (int al = 0; al < 4; ++al)
                for (int a = 0; a < 3; ++a) {
                    cplx acc = 0;
                    for (int be = 0; be < 4; ++be)
                        acc += Pf[al][be] * vf[be][a] + Pb[al][be] * vb[be][a];
                    o[3 * al + a] += acc;
                }
        }
    }
}

/* ------------------------------------------------------------------ */
/* vector helpers: fixed-chunk deterministic reductions               */
/* ------------------------------------------------------------------ */
#define NCHUNK 64

static cplx vdot(const cplx *a, const cplx *b, size_t n)
{
    cplx part[NCHUNK];
#pragma omp parallel for schedule(static)
    for (int c = 0; c < NCHUNK; ++c) {
        size_t lo = n * c / NCHUNK, hi = n * (c + 1) / NCHUNK;
        cplx acc = 0;
        for (size_t i = lo; i < hi; ++i) acc += conj(a[i]) * b[i];
        part[c] = acc;
    }
    cplx s = 0;
    for (int c = 0; c < NCHUNK; ++c) s += part[c];
    return s;
}

static double vnorm2(const cplx *a, size_t n)
{
    return creal(vdot(a, a, n));
}

/* ------------------------------------------------------------------ */
/* operator D and the even-odd Schur complement                       */
/* ------------------------------------------------------------------ */
typedef struct {
    geom g;
    projectors P;
    const cplx *U;
    double kappa;
    cplx *tmp; /* V*12 scratch */
    cplx *tmp2;
} opctx;

/* out = D in  (dagger: D^+) on the full lattice */
static void apply_D(opctx *c, const cplx *in, cplx *out, int dagger)
{
    hop(&c->g, &c->P, c->U, in, c->tmp, -1, dagger);
    size_t n = (size_t)c->g.V * 12;
#pragma omp parallel for schedule(static)
    for (size_t i = 0; i < n; ++i) out[i] = in[i] - c->kappa * c->tmp[i];
}

/*
 * Schur complement on even sites: with D = [[1, -k H_eo], [-k H_oe, 1]],
 *   Dhat x_e = x_e - k^2 H_eo H_oe x_e.
 * Vectors are full-lattice arrays whose odd sites are zero.
 * dagger applies Dhat^+ = 1 - k^2 (H_eo H_oe)^+ = 1 - k^2 H_eo^+' H_oe^+'
 * where the primed maps are the adjoint hopping restricted the same way.
 */
static void apply_Dhat(opctx *c, const cplx *in, cplx *out, int dagger)
{
    hop(&c->g, &c->P, c->U, in, c->tmp2, 1, dagger);
    hop(&c->g, &c->P, c->U, c->tmp2, c->tmp, 0, dagger);
    size_t n = (size_t)c->g.V * 12;
    double k2 = c->kappa * c->kappa;
#pragma omp parallel for schedule(static)
    for (size_t i = 0; i < n; ++i) out[i] = in[i] - k2 * c->tmp[i];
}

static void zero_parity(const geom *g, cplx *v, int parity)
{
#pragma omp parallel for schedule(static)
    for (long x = 0; x < g->V; ++x)
        if (parity_of(g, x) == parity)
            for (int k = 0; k < 12; ++k) v[12 * x + k] = 0;
}

/* ------------------------------------------------------------------ */
/* Krylov solvers                                                     */
/* ------------------------------------------------------------------ */
typedef void (*op_fn)(opctx *, const cplx *, cplx *, int);

/*
 * BiCGStab (van der Vorst 1992), the solver the paper names for its
 * truncated-solver runs (Sec. III).  Solves A x = b starting from x,
 * stopping when the recursive residual satisfies |r| <= stop_abs.
 * Returns iterations used, or -1 on breakdown (rho or omega vanishing).
 */
static int bicgstab(opctx *c, op_fn A, const cplx *b, cplx *x, size_t n,
                    double stop_abs, int max_iter, int *breakdown)
{
    cplx *r = malloc(n * sizeof(cplx)), *r0 = malloc(n * sizeof(cplx));
    cplx *p = malloc(n * sizeof(cplx)), *v = malloc(n * sizeof(cplx));
    cplx *s = malloc(n * sizeof(cplx)), *t = malloc(n * sizeof(cplx));
    *breakdown = 0;
    A(c, x, t, 0);
    for (size_t i = 0; i < n; ++i) {
        r[i] = b[i] - t[i];
        r0[i] = r[i];
        p[i] = 0;
        v[i] = 0;
    }
    cplx rho = 1, alpha = 1, omega = 1;
    int it = 0;
    double rr = vnorm2(r, n);
    while (sqrt(rr) > stop_abs && it < max_iter) {
        cplx rho_new = vdot(r0, r, n);
        if (cabs(rho_new) == 0.0 || !isfinite(creal(rho_new))) { *breakdown = 1; break; }
        cplx beta = (rho_new / rho) * (alpha / omega);
#pragma omp parallel for schedule(static)
        for (size_t i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        A(c, p, v, 0);
        cplx r0v = vdot(r0, v, n);
        if (cabs(r0v) == 0.0) { *breakdown = 1; break; }
        alpha = rho_new / r0v;
#pragma omp parallel for schedule(static)
        for (size_t i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
        ++it;
        double ss = vnorm2(s, n);
        if (sqrt(ss) <= stop_abs) {
            for (size_t i = 0; i < n; ++i) x[i] += alpha * p[i];
            for (size_t i = 0; i < n; ++i) r[i] = s[i];
            rr = ss;
            break;
        }
        A(c, s, t, 0);
        double tt = vnorm2(t, n);
        if (tt == 0.0) { *breakdown = 1; break; }
        omega = vdot(t, s, n) / tt;
        if (cabs(omega) == 0.0) { *breakdown = 1; break; }
#pragma omp parallel for schedule(static)
        for (size_t i = 0; i < n; ++i) {
            x[i] += alpha * p[i] + omega * s[i];
            r[i] = s[i] - omega * t[i];
        }
        rr = vnorm2(r, n);
        rho = rho_new;
        if (!isfinite(rr)) { *breakdown = 1; break; }
    }
    free(r); free(r0); free(p); free(v); free(s); free(t);
    return it;
}

/*
 * CG on the normal equations A^+ A x = A^+ b (the paper's other solver
 * family, Sec. II).  Stops when |b - A x| (tracked recursively) <= stop_abs.
 */
static int cgnr(opctx *c, op_fn A, const cplx *b, cplx *x, size_t n,
                double stop_abs, int max_iter)
{
    cplx *r = malloc(n * sizeof(cplx)), *z = malloc(n * sizeof(cplx));
    cplx *p = malloc(n * sizeof(cplx)), *q = malloc(n * sizeof(cplx));
    A(c, x, q, 0);
    for (size_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
    A(c, r, z, 1);
    for (size_t i = 0; i < n; ++i) p[i] = z[i];
    double zz = vnorm2(z, n);
    double rr = vnorm2(r, n);
    int it = 0;
    while (sqrt(rr) > stop_abs && it < max_iter && zz > 0) {
        A(c, p, q, 0);
        double qq = vnorm2(q, n);
        if (qq == 0.0) break;
        double a = zz / qq;
        for (size_t i = 0; i < n; ++i) {
            x[i] += a * p[i];
            r[i] -= a * q[i];
        }
        A(c, r, z, 1);
        double zz_new = vnorm2(z, n);
        double bta = zz_new / zz;
        for (size_t i = 0; i < n; ++i) p[i] = z[i] + bta * p[i];
        zz = zz_new;
        rr = vnorm2(r, n);
        ++it;
        if (!isfinite(rr)) break;
    }
    free(r); free(z); free(p); free(q);
    return it;
}

enum { OR_OK = 0, OR_NOCONV = 1 };

/*
 * Solve D x = b for one right-hand side, with the stopping rule of Sec. III:
 * the relative deviation |D x - b| / |b| of the full Wilson-Dirac operator.
 * method 0: even-odd (Schur) BiCGStab, falling back to CGNR on breakdown or
 *           non-convergence; method 1: BiCGStab on the full operator;
 *           method 2: even-odd CGNR.
 * The inner solver stops on the recursive residual; the true full-operator
 * residual is then recomputed and the solve restarted from the current
 * iterate while it is still above tol (a few restarts at most).
 */
static int solve_one(opctx *c, const cplx *b, cplx *x, double tol, int max_iter,
                     int method, int *iters, double *resid)
{
    const geom *g = &c->g;
    size_t n = (size_t)g->V * 12;
    cplx *bh = calloc(n, sizeof(cplx)), *r = malloc(n * sizeof(cplx));
    cplx *xe = calloc(n, sizeof(cplx));
    double bnorm = sqrt(vnorm2(b, n));
    int total = 0, status = OR_NOCONV;
    *resid = 0;
    if (bnorm == 0.0) {
        memset(x, 0, n * sizeof(cplx));
        free(bh); free(r); free(xe);
        *iters = 0;
        return OR_OK;
    }
    int use_cg = (method == 2);
    for (int attempt = 0; attempt < 8 && total < max_iter; ++attempt) {
        if (method == 1) {
            /* full operator: residual equation on the whole lattice */
            if (attempt == 0) memset(x, 0, n * sizeof(cplx));
            apply_D(c, x, r, 0);
            for (size_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
            cplx *e = calloc(n, sizeof(cplx));
            int bd = 0;
            total += bicgstab(c, apply_D, r, e, n, 0.5 * tol * bnorm, max_iter - total, &bd);
            for (size_t i = 0; i < n; ++i) x[i] += e[i];
            free(e);
        } else {
            /* b_hat_e = b_e + k H_eo b_o, residual of the Schur system */
            if (attempt == 0) {
                cplx *bo = malloc(n * sizeof(cplx));
                memcpy(bo, b, n * sizeof(cplx));
                zero_parity(g, bo, 0);
                hop(g, &c->P, c->U, bo, bh, 0, 0);
                for (size_t i = 0; i < n; ++i) bh[i] *= c->kappa;
                for (long s = 0; s < g->V; ++s)
                    if (parity_of(g, s) == 0)
                        for (int k = 0; k < 12; ++k) bh[12 * s + k] += b[12 * s + k];
                free(bo);
            }
            apply_Dhat(c, xe, r, 0);
            for (size_t i = 0; i < n; ++i) r[i] = bh[i] - r[i];
            cplx *e = calloc(n, sizeof(cplx));
            double stop = 0.5 * tol * bnorm;
            if (!use_cg) {
                int bd = 0;
                total += bicgstab(c, apply_Dhat, r, e, n, stop, max_iter - total, &bd);
                if (bd) use_cg = 1;
            } else {
                total += cgnr(c, apply_Dhat, r, e, n, stop, max_iter - total);
            }
            for (size_t i = 0; i < n; ++i) xe[i] += e[i];
            free(e);
            /* x_o = b_o + k H_oe x_e */
            hop(g, &c->P, c->U, xe, x, 1, 0);
            for (long s = 0; s < g->V; ++s) {
                int par = parity_of(g, s);
                for (int k = 0; k < 12; ++k) {
                    size_t i = 12 * s + k;
                    x[i] = par ? b[i] + c->kappa * x[i] : xe[i];
                }
            }
        }
        /* true residual of the full operator (stopping rule of Sec. III) */
        apply_D(c, x, r, 0);
        for (size_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
        *resid = sqrt(vnorm2(r, n)) / bnorm;
        if (*resid <= tol) { status = OR_OK; break; }
        if (!isfinite(*resid)) break;
        if (method == 0 && total >= max_iter / 2) use_cg = 1;
    }
    *iters = total;
    free(bh); free(r); free(xe);
    return status;
}

static void init_ctx(opctx *c, const int *dims, int bc_t, int basis, double kappa,
                     const double *U)
{
    c->g = make_geom(dims, bc_t);
    make_projectors(basis, &c->P);
    c->U = (const cplx *)U;
    c->kappa = kappa;
    c->tmp = malloc((size_t)c->g.V * 12 * sizeof(cplx));
    c->tmp2 = malloc((size_t)c->g.V * 12 * sizeof(cplx));
}

static void free_ctx(opctx *c)
{
    free(c->tmp);
    free(c->tmp2);
}

/* ------------------------------------------------------------------ */
/* public entry points (plain pointers, canonical layouts)            */
/* ------------------------------------------------------------------ */
int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads of the later parallel regions of the calling thread (n >= 1) */
void or_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* hopping term with parity restriction (out_parity -1: all sites) */
void or_hop(const int *dims, int bc_t, int basis, const double *U, const double *in,
            double *out, int out_parity, int dagger)
{
    geom g = make_geom(dims, bc_t);
    projectors P;
    make_projectors(basis, &P);
    hop(&g, &P, (const cplx *)U, (const cplx *)in, (cplx *)out, out_parity, dagger);
}

/* out = D in or D^+ in for nrhs spinors [nrhs][V][4][3] */
void or_apply_D(const int *dims, int bc_t, int basis, double kappa, const double *U,
                const double *in, double *out, int nrhs, int dagger)
{
    opctx c;
    init_ctx(&c, dims, bc_t, basis, kappa, U);
    size_t n = (size_t)c.g.V * 12;
    for (int k = 0; k < nrhs; ++k)
        apply_D(&c, (const cplx *)in + k * n, (cplx *)out + k * n, dagger);
    free_ctx(&c);
}

/* Schur operator on even-site vectors (full-lattice arrays, odd part 0) */
void or_apply_Dhat(const int *dims, int bc_t, int basis, double kappa, const double *U,
                   const double *in, double *out, int dagger)
{
    opctx c;
    init_ctx(&c, dims, bc_t, basis, kappa, U);
    apply_Dhat(&c, (const cplx *)in, (cplx *)out, dagger);
    free_ctx(&c);
}

/* Solve D x_k = b_k; iters[k], resid[k] receive per-RHS statistics.
 * Returns the number of right-hand sides that did not reach tol. */
int or_solve(const int *dims, int bc_t, int basis, double kappa, const double *U,
             const double *b, double *x, int nrhs, double tol, int max_iter,
             int method, int *iters, double *resid)
{
    opctx c;
    init_ctx(&c, dims, bc_t, basis, kappa, U);
    size_t n = (size_t)c.g.V * 12;
    int fails = 0;
    for (int k = 0; k < nrhs; ++k) {
        int it = 0;
        double rs = 0;
        int st = solve_one(&c, (const cplx *)b + k * n, (cplx *)x + k * n, tol, max_iter,
                           method, &it, &rs);
        if (iters) iters[k] = it;
        if (resid) resid[k] = rs;
        if (st != OR_OK) ++fails;
    }
    free_ctx(&c);
    return fails;
}

/*
 * Exact loops, Eq. (loop): L_Gamma(y) = Tr[Gamma G(y;y)], for an explicit
 * list of sites y (lexicographic indices).  For each site, spin beta and
 * colour b, D psi = e_{y,beta,b} is solved;
 * G(y;y)_{alpha a, beta b} = psi^{(y,beta,b)}(y)_{alpha a}.
 * S(y)_{alpha beta} = sum_a G(y;y)_{alpha a, beta a} is the colour-traced
 * block and L_Gamma(y) = sum_{alpha beta} Gamma_{beta alpha} S(y)_{alpha beta}.
 * Outputs: L [ngamma][nsites] complex, S (optional) [nsites][4][4] complex.
 * Returns the number of solves that missed tol.
 */
int or_loops_exact_sites(const int *dims, int bc_t, int basis, double kappa, const double *U,
                         const long *sites, long nsites, const int *gammas, int ngamma,
                         double tol, int max_iter, double *L, double *S)
{
    opctx c;
    init_ctx(&c, dims, bc_t, basis, kappa, U);
    const geom *g = &c.g;
    size_t n = (size_t)g->V * 12;
    cplx *b = calloc(n, sizeof(cplx)), *x = calloc(n, sizeof(cplx));
    cplx Gm[16][4][4];
    for (int k = 0; k < ngamma; ++k) gamma_mask(basis, gammas[k], Gm[k]);
    int fails = 0;
    for (long i = 0; i < nsites; ++i) {
        long y = sites[i];
        cplx Sy[4][4] = {{0}};
        for (int be = 0; be < 4; ++be)
            for (int bcol = 0; bcol < 3; ++bcol) {
                memset(b, 0, n * sizeof(cplx));
                b[12 * y + 3 * be + bcol] = 1.0;
                int its = 0;
                double rs = 0;
                if (solve_one(&c, b, x, tol, max_iter, 0, &its, &rs) != OR_OK) ++fails;
                for (int al = 0; al < 4; ++al) Sy[al][be] += x[12 * y + 3 * al + bcol];
            }
        for (int k = 0; k < ngamma; ++k) {
            cplx acc = 0;
            for (int al = 0; al < 4; ++al)
                for (int be = 0; be < 4; ++be) acc += Gm[k][be][al] * Sy[al][be];
            size_t o = (size_t)k * nsites + i;
            L[2 * o] = creal(acc);
            L[2 * o + 1] = cimag(acc);
        }
        if (S)
            for (int al = 0; al < 4; ++al)
                for (int be = 0; be < 4; ++be) {
                    size_t o = ((size_t)i * 4 + al) * 4 + be;
                    S[2 * o] = creal(Sy[al][be]);
                    S[2 * o + 1] = cimag(Sy[al][be]);
                }
    }
    free(b); free(x);
    free_ctx(&c);
    return fails;
}

/*
 * Exact loops on whole timeslices: 12 V_s inversions per timeslice, as
 * Sec. II counts them.  Outputs L [ngamma][nt][Vs], S [nt][Vs][4][4].
 */
int or_loops_exact(const int *dims, int bc_t, int basis, double kappa, const double *U,
                   const int *t0, int nt, const int *gammas, int ngamma, double tol,
                   int max_iter, double *L, double *S)
{
    long Vs = (long)dims[0] * dims[1] * dims[2];
    long ns = Vs * nt;
    long *sites = malloc(ns * sizeof(long));
    for (int it = 0; it < nt; ++it)
        for (long ys = 0; ys < Vs; ++ys) sites[it * Vs + ys] = ys + Vs * (long)t0[it];
    int fails = or_loops_exact_sites(dims, bc_t, basis, kappa, U, sites, ns, gammas, ngamma,
                                     tol, max_iter, L, S);
    free(sites);
    return fails;
}

/* ------------------------------------------------------------------ */
/* noise (Sec. II: complex Z2 noise; Eq. delta functions)             */
/* ------------------------------------------------------------------ */
/*
 * Counter-based generator: the k-th output of SplitMix64 (Steele, Lea,
 * Flood, OOPSLA 2014) started from state `seed`: the state advances by the
 * golden-ratio increment 0x9e3779b97f4a7c15 and is passed through the
 * published 64-bit finaliser.
 */
static uint64_t splitmix_finalise(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

uint64_t or_splitmix64(uint64_t seed, uint64_t k)
{
    return splitmix_finalise(seed + (k + 1) * 0x9e3779b97f4a7c15ULL);
}

/*
 * One unit-modulus noise value per (noise index r, site, spin, colour):
 * key k = ((r*V + site)*4 + spin)*3 + colour, h = splitmix64(seed, k);
 * with b63, b62 the two top bits of h:
 *   type 0 (Z4):          xi = i^(2*b63 + b62)
 *   type 1 (complex Z2):  xi = ((-1)^b63 + i (-1)^b62) / sqrt(2)
 *   type 2 (real Z2):     xi = (-1)^b63
 * All satisfy <xi> = 0 and <xi xi*> = 1 as the estimator requires.
 */
static cplx noise_value(int type, uint64_t seed, long r, long V, long site, int spin, int col)
{
    uint64_t k = (((uint64_t)r * (uint64_t)V + (uint64_t)site) * 4 + (uint64_t)spin) * 3 + (uint64_t)col;
    uint64_t h = or_splitmix64(seed, k);
    int b63 = (int)(h >> 63), b62 = (int)((h >> 62) & 1);
    if (type == 0) {
        const cplx z4[4] = {1, I, -1, -I};
        return z4[2 * b63 + b62];
    } else if (type == 1) {
        return ((b63 ? -1.0 : 1.0) + I * (b62 ? -1.0 : 1.0)) / sqrt(2.0);
    }
    return b63 ? -1.0 : 1.0;
}

void or_noise(int type, uint64_t seed, long r, const int *dims, double *out)
{
    geom g = make_geom(dims, 1);
    for (long s = 0; s < g.V; ++s)
        for (int al = 0; al < 4; ++al)
            for (int a = 0; a < 3; ++a) {
                cplx v = noise_value(type, seed, r, g.V, s, al, a);
                out[2 * (12 * s + 3 * al + a)] = creal(v);
                out[2 * (12 * s + 3 * al + a) + 1] = cimag(v);
            }
}

/*
 * Dilution (Sec. II): time dilution, spin (x4), colour (x3), even-odd space
 * (x2) and cubic (x8: one class per vertex of the elementary 3-cube).
 * A dilution component d fixes a value for every enabled kind; the diluted
 * source is eta_d = P_d xi with P_d the 0/1 projector onto the sites and
 * indices that carry that value.
 * mask bits: 1 time, 2 spin, 4 colour, 8 even-odd space, 16 cubic.
 */
typedef struct {
    int use_t, use_spin, use_col, nspace; /* nspace: 1, 2 (even-odd), 8 (cubic) */
    int space_kind;
} dilution;

static dilution make_dilution(int mask)
{
    dilution d;
    d.use_t = (mask & 1) != 0;
    d.use_spin = (mask & 2) != 0;
    d.use_col = (mask & 4) != 0;
    d.space_kind = (mask & 16) ? 2 : ((mask & 8) ? 1 : 0);
    d.nspace = d.space_kind == 2 ? 8 : (d.space_kind == 1 ? 2 : 1);
    return d;
}

static int space_class(const dilution *d, const int c[4])
{
    if (d->space_kind == 1) return (c[0] + c[1] + c[2]) & 1;
    if (d->space_kind == 2) return (c[0] & 1) + 2 * (c[1] & 1) + 4 * (c[2] & 1);
    return 0;
}

/* does site s (coords c), spin al, colour a belong to component
 * (t, spin be, colour bc, class sc)? (-1 = that kind is not diluted) */
static int in_support(const dilution *d, const int c[4], int al, int a, int t, int be,
                      int bc, int sc)
{
    if (d->use_t && c[3] != t) return 0;
    if (d->use_spin && al != be) return 0;
    if (d->use_col && a != bc) return 0;
    if (d->nspace > 1 && space_class(d, c) != sc) return 0;
    return 1;
}

/*
 * Estimator of Eq. (loop stochastic), generalised to dilution:
 *   Lhat_Gamma(x) = (1/N_r) sum_r sum_d eta_{r,d}(x)^+ Gamma phi_{r,d}(x),
 *   phi_{r,d} = D^{-1} eta_{r,d}.
 * It is an unbiased estimate of Tr[Gamma G(x;x)] because <phi xi*> = G
 * (Eq. propagator noise*result).
 *
 * Truncated solver method (Sec. II, following Bali et al.): with n_lp
 * low-precision noise vectors r = r0 .. r0+n_lp-1 and n_hp high-precision
 * ones r = r0+n_lp .. r0+n_lp+n_hp-1,
 *   Lhat = (1/n_lp) sum_{r in LP} sum_d eta^+ Gamma phi^LP
 *        + (1/n_hp) sum_{r in HP} sum_d eta^+ Gamma (phi^HP - phi^LP)
 * where phi^LP is the same truncated solve (stopped at relative residual
 * tol_lp) in both sums and phi^HP is solved to tol_hp.  With n_hp = 0 this
 * is the plain estimator over n_lp vectors solved to tol_lp.
 *
 * Output L[ngamma][t_end - t_begin][Vs] complex: the estimate at the sites
 * of timeslices t_begin .. t_end-1 (dilution components whose time lies
 * outside that range are not solved when time dilution is on).
 * Returns the number of HP solves that missed tol_hp.
 */
int or_loops_tsm(const int *dims, int bc_t, int basis, double kappa, const double *U,
                 int noise_type, uint64_t seed, long r0, int n_lp, int n_hp, double tol_lp,
                 double tol_hp, int dil_mask, int t_begin, int t_end, const int *gammas,
                 int ngamma, int max_iter, double *L)
{
    opctx c;
    init_ctx(&c, dims, bc_t, basis, kappa, U);
    const geom *g = &c.g;
    size_t n = (size_t)g->V * 12;
    long Vs = (long)g->L[0] * g->L[1] * g->L[2];
    int nt = t_end - t_begin;
    dilution d = make_dilution(dil_mask);
    cplx Gm[16][4][4];
    for (int k = 0; k < ngamma; ++k) gamma_mask(basis, gammas[k], Gm[k]);
    cplx *acc_lp = calloc((size_t)ngamma * nt * Vs, sizeof(cplx));
    cplx *acc_hp = calloc((size_t)ngamma * nt * Vs, sizeof(cplx));
    cplx *xi = malloc(n * sizeof(cplx)), *eta = malloc(n * sizeof(cplx));
    cplx *phi = calloc(n, sizeof(cplx)), *phi_hp = calloc(n, sizeof(cplx));
    int fails = 0;
    int tlist_lo = d.use_t ? t_begin : 0, tlist_hi = d.use_t ? t_end : 1;
    int nspin = d.use_spin ? 4 : 1, ncol = d.use_col ? 3 : 1;
    for (int rr = 0; rr < n_lp + n_hp; ++rr) {
        long r = r0 + rr;
        int is_hp = rr >= n_lp;
        for (long s = 0; s < g->V; ++s)
            for (int al = 0; al < 4; ++al)
                for (int a = 0; a < 3; ++a)
                    xi[12 * s + 3 * al + a] = noise_value(noise_type, seed, r, g->V, s, al, a);
        for (int t = tlist_lo; t < tlist_hi; ++t)
            for (int be = 0; be < nspin; ++be)
                for (int bc = 0; bc < ncol; ++bc)
                    for (int sc = 0; sc < d.nspace; ++sc) {
                        for (long s = 0; s < g->V; ++s) {
                            int cc[4];
                            coords(g, s, cc);
                            for (int al = 0; al < 4; ++al)
                                for (int a = 0; a < 3; ++a)
                                    eta[12 * s + 3 * al + a] =
                                        in_support(&d, cc, al, a, t, be, bc, sc) ? xi[12 * s + 3 * al + a] : 0;
                        }
                        int its;
                        double rs;
                        solve_one(&c, eta, phi, tol_lp, max_iter, 0, &its, &rs);
                        if (is_hp) {
                            if (solve_one(&c, eta, phi_hp, tol_hp, max_iter, 0, &its, &rs) != OR_OK)
                                ++fails;
                        }
                        /* contraction on the estimated timeslices */
                        for (int tt = 0; tt < nt; ++tt) {
                            int tx = t_begin + tt;
                            if (d.use_t && tx != t) continue;
                            for (long ys = 0; ys < Vs; ++ys) {
                                long x = ys + Vs * (long)tx;
                                const cplx *e = eta + 12 * x;
                                cplx dphi[12];
                                for (int k = 0; k < 12; ++k)
                                    dphi[k] = is_hp ? phi_hp[12 * x + k] - phi[12 * x + k] : phi[12 * x + k];
                                for (int k = 0; k < ngamma; ++k) {
                                    cplx v = 0;
                                    for (int al = 0; al < 4; ++al)
                                        for (int be2 = 0; be2 < 4; ++be2)
                                            for (int a = 0; a < 3; ++a)
                                                v += conj(e[3 * al + a]) * Gm[k][al][be2] * dphi[3 * be2 + a];
                                    size_t o = ((size_t)k * nt + tt) * Vs + ys;
                                    if (is_hp) acc_hp[o] += v; else acc_lp[o] += v;
                                }
                            }
                        }
                    }
    }
    size_t no = (size_t)ngamma * nt * Vs;
    for (size_t o = 0; o < no; ++o) {
        cplx v = (n_lp > 0 ? acc_lp[o] / n_lp : 0) + (n_hp > 0 ? acc_hp[o] / n_hp : 0);
        L[2 * o] = creal(v);
        L[2 * o + 1] = cimag(v);
    }
    free(acc_lp); free(acc_hp); free(xi); free(eta); free(phi); free(phi_hp);
    free_ctx(&c);
    return fails;
}

/* plain stochastic estimator: all n_noise vectors solved to tol */
int or_loops_stochastic(const int *dims, int bc_t, int basis, double kappa, const double *U,
                        int noise_type, uint64_t seed, long r0, int n_noise, int dil_mask,
                        int t_begin, int t_end, const int *gammas, int ngamma, double tol,
                        int max_iter, double *L)
{
    return or_loops_tsm(dims, bc_t, basis, kappa, U, noise_type, seed, r0, n_noise, 0, tol,
                        tol, dil_mask, t_begin, t_end, gammas, ngamma, max_iter, L);
}

/* ------------------------------------------------------------------ */
/* gradient of F = Re sum_{Gamma, y} conj(w_Gamma(y)) L_Gamma(y)      */
/* ------------------------------------------------------------------ */
/*
 * For the exact loops of a timeslice list, with weights w[ngamma][nt][Vs]:
 * writing L_Gamma(y) = sum_{beta b} e^+ Gamma D^{-1} e (e = e_{y,beta,b}) and
 * dD^{-1} = -D^{-1} dD D^{-1} gives dF = -Re sum_s chi_s^+ dD psi_s with
 *   psi_s = D^{-1} s,  chi_s = D^{-+} sum_Gamma w_Gamma(y) Gamma^+ s,
 * and D^{-+} = g5 D^{-1} g5 (gamma_5-hermiticity), so chi_s is a spin
 * recombination of the same-site solutions:
 *   chi_{y,beta,b} = g5 sum_alpha M_{alpha beta} psi_{y,alpha,b},
 *   M = sum_Gamma w_Gamma(y) g5 Gamma^+.
 * From dD/dkappa = -Hop:  dF/dkappa = Re sum_s chi_s^+ Hop psi_s.
 * From the U_mu(y) terms of D:
 *   dU_mu(y) = kappa * sgn * sum_s [ conj(A_s) + B_s^T ],
 *   A_s[i][j] = sum chi_s(y)^*_{al i} (1-g_mu)_{al be} psi_s(y+mu)_{be j},
 *   B_s[i][j] = sum chi_s(y+mu)^*_{al i} (1+g_mu)_{al be} psi_s(y)_{be j},
 * with sgn the boundary factor of the hop y -> y+mu and dU returned in the
 * convention dU = dF/dRe U + i dF/dIm U.
 * Sites whose weights are all zero are skipped (no solves).
 * Returns the number of solves that missed tol.
 */
int or_loops_grad(const int *dims, int bc_t, int basis, double kappa, const double *U,
                  const int *t0, int nt, const int *gammas, int ngamma, const double *w,
                  double tol, int max_iter, double *dU, double *dkappa)
{
    opctx c;
    init_ctx(&c, dims, bc_t, basis, kappa, U);
    const geom *g = &c.g;
    size_t n = (size_t)g->V * 12;
    long Vs = (long)g->L[0] * g->L[1] * g->L[2];
    cplx Gm[16][4][4], g5[4][4];
    for (int k = 0; k < ngamma; ++k) gamma_mask(basis, gammas[k], Gm[k]);
    gamma_mask(basis, 15, g5);
    const cplx *wc = (const cplx *)w;
    cplx *out = (cplx *)dU;
    memset(out, 0, (size_t)4 * g->V * 9 * sizeof(cplx));
    cplx dk = 0;
    cplx *psi = malloc(12 * n * sizeof(cplx)), *chi = malloc(12 * n * sizeof(cplx));
    cplx *b = calloc(n, sizeof(cplx)), *hp = malloc(n * sizeof(cplx));
    int fails = 0;
    for (int it = 0; it < nt; ++it)
        for (long ys = 0; ys < Vs; ++ys) {
            int any = 0;
            for (int k = 0; k < ngamma; ++k)
                if (wc[((size_t)k * nt + it) * Vs + ys] != 0) any = 1;
            if (!any) continue;
            long y = ys + Vs * (long)t0[it];
            for (int be = 0; be < 4; ++be)
                for (int bcol = 0; bcol < 3; ++bcol) {
                    memset(b, 0, n * sizeof(cplx));
                    b[12 * y + 3 * be + bcol] = 1.0;
                    int its;
                    double rs;
                    if (solve_one(&c, b, psi + (3 * be + bcol) * n, tol, max_iter, 0, &its, &rs) != OR_OK)
                        ++fails;
                }
            /* M = sum_Gamma w g5 Gamma^+ */
            cplx M[4][4] = {{0}};
            for (int k = 0; k < ngamma; ++k) {
                cplx wk = wc[((size_t)k * nt + it) * Vs + ys];
                for (int i = 0; i < 4; ++i)
                    for (int j = 0; j < 4; ++j) {
                        cplx acc = 0;
                        for (int l = 0; l < 4; ++l) acc += g5[i][l] * conj(Gm[k][j][l]);
                        M[i][j] += wk * acc;
                    }
            }
            /* chi_{beta b} = g5 sum_alpha M_{alpha beta} psi_{alpha b} */
            for (int be = 0; be < 4; ++be)
                for (int bcol = 0; bcol < 3; ++bcol) {
                    cplx *ch = chi + (3 * be + bcol) * n;
                    for (long s = 0; s < g->V; ++s)
                        for (int de = 0; de < 4; ++de)
                            for (int a = 0; a < 3; ++a) {
                                cplx acc = 0;
                                for (int ga = 0; ga < 4; ++ga) {
                                    cplx comb = 0;
                                    for (int al = 0; al < 4; ++al)
                                        comb += M[al][be] * psi[(3 * al + bcol) * n + 12 * s + 3 * ga + a];
                                    acc += g5[de][ga] * comb;
                                }
                                ch[12 * s + 3 * de + a] = acc;
                            }
                }
            /* accumulate dkappa and dU over the 12 sources of this site */
            for (int src = 0; src < 12; ++src) {
                const cplx *ps = psi + src * n, *ch = chi + src * n;
                hop(g, &c.P, c.U, ps, hp, -1, 0);
                dk += vdot(ch, hp, n);
                for (int mu = 0; mu < 4; ++mu) {
                    const cplx(*Pm)[4] = c.P.minus[mu];
                    const cplx(*Pp)[4] = c.P.plus[mu];
#pragma omp parallel for schedule(static)
                    for (long yy = 0; yy < g->V; ++yy) {
                        double sg;
                        long yf = neighbour(g, yy, mu, +1, &sg);
                        cplx *o = out + ((size_t)mu * g->V + yy) * 9;
                        for (int i = 0; i < 3; ++i)
                            for (int j = 0; j < 3; ++j) {
                                cplx A = 0, B = 0;
                                for (int al = 0; al < 4; ++al)
                                    for (int be = 0; be < 4; ++be) {
                                        A += conj(ch[12 * yy + 3 * al + i]) * Pm[al][be] * ps[12 * yf + 3 * be + j];
                                        B += conj(ch[12 * yf + 3 * al + i]) * Pp[al][be] * ps[12 * yy + 3 * be + j];
                                    }
                                /* conj(A) goes to entry (i,j), B to entry (j,i) */
                                o[3 * i + j] += kappa * sg * conj(A);
                                o[3 * j + i] += kappa * sg * B;
                            }
                    }
                }
            }
        }
    *dkappa = creal(dk);
    free(psi); free(chi); free(b); free(hp);
    free_ctx(&c);
    return fails;
}

/* Host driver that runs every entry point of the FP64 oracle once on a
 * 2^3x4 lattice; built with AddressSanitizer and UndefinedBehaviorSanitizer
 * by tests/test_oracle_sanitizers.py, which fails on any report. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void or_hop(const int *dims, int bc_t, int basis, const double *U, const double *in, double *out, int out_parity,
            int dagger);
void or_apply_D(const int *dims, int bc_t, int basis, double kappa, const double *U, const double *in, double *out,
                int nrhs, int dagger);
void or_apply_Dhat(const int *dims, int bc_t, int basis, double kappa, const double *U, const double *in,
                   double *out, int dagger);
int or_solve(const int *dims, int bc_t, int basis, double kappa, const double *U, const double *b, double *x,
             int nrhs, double tol, int max_iter, int method, int *iters, double *resid);
int or_loops_exact_sites(const int *dims, int bc_t, int basis, double kappa, const double *U, const long *sites,
                         long nsites, const int *gammas, int ngamma, double tol, int max_iter, double *L, double *S);
int or_loops_exact(const int *dims, int bc_t, int basis, double kappa, const double *U, const int *t0, int nt,
                   const int *gammas, int ngamma, double tol, int max_iter, double *L, double *S);
void or_noise(int type, uint64_t seed, long r, const int *dims, double *out);
int or_loops_tsm(const int *dims, int bc_t, int basis, double kappa, const double *U, int noise_type, uint64_t seed,
                 long r0, int n_lp, int n_hp, double tol_lp, double tol_hp, int dil_mask, int t_begin, int t_end,
                 const int *gammas, int ngamma, int max_iter, double *L);
int or_loops_grad(const int *dims, int bc_t, int basis, double kappa, const double *U, const int *t0, int nt,
                  const int *gammas, int ngamma, const double *w, double tol, int max_iter, double *dU,
                  double *dkappa);
void or_gamma(int basis, int mask, double *out);

static double urand(uint64_t *s)
{
    *s = *s * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(*s >> 11) / 9007199254740992.0;
}

int main(void)
{
    const int dims[4] = {2, 2, 2, 4};
    const long V = 32, Vs = 8;
    const double kappa = 0.11;
    uint64_t s = 12345;
    /* links near the identity (any complex 3x3 is a valid operator input) */
    double *U = malloc(sizeof(double) * 2 * 4 * V * 9);
    for (long k = 0; k < 4 * V * 9; ++k) {
        const int diag = (k % 9) % 4 == 0;
        U[2 * k] = (diag ? 1.0 : 0.0) + 0.2 * (urand(&s) - 0.5);
        U[2 * k + 1] = 0.2 * (urand(&s) - 0.5);
    }
    const size_t n = (size_t)V * 12 * 2;
    double *a = malloc(sizeof(double) * n * 2), *b = malloc(sizeof(double) * n * 2), *x = malloc(sizeof(double) * n * 2);
    for (size_t k = 0; k < 2 * n; ++k) a[k] = urand(&s) - 0.5;
    double G[32];
    for (int m = 0; m < 16; ++m) or_gamma(0, m, G);
    or_hop(dims, -1, 0, U, a, b, -1, 0);
    or_hop(dims, -1, 0, U, a, b, 0, 1);
    or_apply_D(dims, -1, 0, kappa, U, a, b, 2, 0);
    or_apply_D(dims, 1, 0, kappa, U, a, b, 2, 1);
    or_apply_Dhat(dims, -1, 0, kappa, U, a, b, 0);
    or_apply_Dhat(dims, -1, 0, kappa, U, a, b, 1);
    int it[2];
    double res[2];
    int fails = 0;
    for (int method = 0; method < 3; ++method) fails += or_solve(dims, -1, 0, kappa, U, a, x, 2, 1e-12, 500, method, it, res);
    const int gam[3] = {0, 15, 8};
    const long sites[3] = {0, 7, 31};
    double *L = malloc(sizeof(double) * 2 * 3 * V), *S = malloc(sizeof(double) * 2 * 16 * V);
    fails += or_loops_exact_sites(dims, -1, 0, kappa, U, sites, 3, gam, 3, 1e-12, 500, L, S);
    const int t0[2] = {0, 3};
    fails += or_loops_exact(dims, -1, 0, kappa, U, t0, 2, gam, 3, 1e-12, 500, L, S);
    for (int type = 0; type < 3; ++type) or_noise(type, 99, 5, dims, b);
    double *Lt = malloc(sizeof(double) * 2 * 3 * V);
    fails += or_loops_tsm(dims, -1, 0, kappa, U, 0, 7, 0, 3, 2, 1e-2, 1e-12, 1 | 2 | 4, 0, 4, gam, 3, 500, Lt);
    fails += or_loops_tsm(dims, -1, 0, kappa, U, 1, 7, 0, 2, 0, 1e-12, 1e-12, 8, 1, 3, gam, 3, 500, Lt);
    fails += or_loops_tsm(dims, -1, 0, kappa, U, 2, 7, 0, 2, 0, 1e-12, 1e-12, 16 | 1, 0, 4, gam, 3, 500, Lt);
    double *w = malloc(sizeof(double) * 2 * 3 * 1 * Vs), *dU = malloc(sizeof(double) * 2 * 4 * V * 9), dk[2];
    for (long k = 0; k < 2 * 3 * Vs; ++k) w[k] = urand(&s) - 0.5;
    fails += or_loops_grad(dims, -1, 0, kappa, U, t0, 1, gam, 3, w, 1e-12, 500, dU, dk);
    double chk = dk[0] + dk[1];
    for (long k = 0; k < 2 * 4 * V * 9; ++k) chk += dU[k];
    printf("fails %d checksum %.6e\n", fails, chk);
    free(U); free(a); free(b); free(x); free(L); free(S); free(Lt); free(w); free(dU);
    return (fails == 0 && isfinite(chk)) ? 0 : 3;
}

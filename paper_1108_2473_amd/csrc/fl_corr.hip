// fl_corr.hip -- momentum-projected loops and the disconnected two-point
// function built from them (Sec. III, Eq. all_dis_corr):
//
//   Lp_G(p, t) = sum_x exp(+i p.x) L_G(x, t),  p = 2 pi (n_x/Lx, n_y/Ly, n_z/Lz)
//   D_AB(p, t) = (1/V_s)(1/T) sum_ti Lp_A(p, ti + t) Lp_B(-p, ti)
//
// The phase of site x for the integer vector n is the product of the three
// per-axis factors exp(2 pi i r_mu / L_mu), r_mu = (n_mu x_mu) mod L_mu,
// each evaluated once per workgroup by sincospi on the exactly reduced
// argument 2 r_mu / L_mu and kept in LDS (two complex products per site
// instead of a sine and cosine).  Sums run in FP64 in a fixed order
// (per-thread partial sums over a strided site range, then a fixed tree in
// LDS), so results do not depend on the launch.
#include <cstring>
#include <vector>

#include "fl_host.h"

namespace {

constexpr int MAXG = 16;    // Gamma matrices per call
constexpr int BLK = 256;
constexpr int MAXAX = 1024;  // Lx + Ly + Lz: the per-axis phase tables in LDS (16 KB)
constexpr int GB = 4;        // Gamma matrices per workgroup of the projection

struct MomArgs {
    const double2 *L;  // [ngamma][nt][Vs]
    double2 *Lp;       // [ngamma][nmom][nt]
    const int *mom;    // [nmom][3]
    int ngamma, nt, nmom, Lx, Ly, Lz, Vs;
};

// one workgroup per (timeslice, momentum, group of up to GB Gammas), in
// XCD-contiguous order with the Gamma group innermost, then the momentum:
// each XCD takes a run of timeslices, so a timeslice's loops (ngamma x V_s
// values) come from HBM once and then from that XCD's L2 for every
// momentum.  The group's GB loads per site are unconditional (an index past
// the last Gamma repeats it; its sum is not stored), so they are all in
// flight together.
__global__ __launch_bounds__(BLK) void k_momproj(MomArgs a)
{
    const int ngr = (a.ngamma + GB - 1) / GB;
    const int tile = xcd_tile(blockIdx.x, gridDim.x, 0);
    const int g0 = (tile % ngr) * GB, k = (tile / ngr) % a.nmom, t = tile / (ngr * a.nmom);
    // exp(2 pi i n_mu x_mu / L_mu) for x_mu = 0..L_mu-1, the three axes in a row
    __shared__ double2 ph[MAXAX];
    const int nL = a.Lx + a.Ly + a.Lz;
    for (int i = threadIdx.x; i < nL; i += BLK) {
        const int mu = i < a.Lx ? 0 : (i < a.Lx + a.Ly ? 1 : 2);
        const int L = mu == 0 ? a.Lx : (mu == 1 ? a.Ly : a.Lz);
        const int x = i - (mu == 0 ? 0 : (mu == 1 ? a.Lx : a.Lx + a.Ly));
        long long r = ((long long)a.mom[3 * k + mu] * x) % L;
        if (r < 0) r += L;
        double sn, cs;
        sincospi(2.0 * (double)r / (double)L, &sn, &cs);
        ph[i] = make_double2(cs, sn);
    }
    __syncthreads();
    const double2 *src[GB];
#pragma unroll
    for (int j = 0; j < GB; ++j) src[j] = a.L + ((size_t)min(g0 + j, a.ngamma - 1) * a.nt + t) * a.Vs;
    double2 acc[GB];
#pragma unroll
    for (int j = 0; j < GB; ++j) acc[j] = make_double2(0.0, 0.0);
    for (int xs = threadIdx.x; xs < a.Vs; xs += BLK) {
        double2 v[GB];
#pragma unroll
        for (int j = 0; j < GB; ++j) v[j] = src[j][xs];
        const int xy = xs / a.Lx, x = xs - xy * a.Lx, z = xy / a.Ly, y = xy - z * a.Ly;
        const double2 px = ph[x], py = ph[a.Lx + y], pz = ph[a.Lx + a.Ly + z];
        const double ar = px.x * py.x - px.y * py.y, ai = px.x * py.y + px.y * py.x;
        const double cs = ar * pz.x - ai * pz.y, sn = ar * pz.y + ai * pz.x;
#pragma unroll
        for (int j = 0; j < GB; ++j) {
            acc[j].x += cs * v[j].x - sn * v[j].y;
            acc[j].y += cs * v[j].y + sn * v[j].x;
        }
    }
    __shared__ double2 red[BLK];
    __shared__ double2 res[GB];
#pragma unroll
    for (int j = 0; j < GB; ++j) {
        red[threadIdx.x] = acc[j];
        __syncthreads();
        for (int w = BLK / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) {
                red[threadIdx.x].x += red[threadIdx.x + w].x;
                red[threadIdx.x].y += red[threadIdx.x + w].y;
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) res[j] = red[0];
        __syncthreads();
    }
    // one store instruction (lane j writes Gamma g0 + j), which ends the kernel
    if ((int)threadIdx.x < GB && g0 + (int)threadIdx.x < a.ngamma)
        a.Lp[((size_t)(g0 + threadIdx.x) * a.nmom + k) * a.nt + t] = res[threadIdx.x];
}

struct CorrArgs {
    const double2 *Lp1, *Lp2;  // [ngamma][nmom][T]
    double2 *D;                // [npair][nmom][T]
    const int *pairs;          // [npair][2]
    int nmom, T, npair;
    double norm;  // 1 / (V_s T)
};

// one thread per (pair, momentum, separation), summing the source times in order
__global__ __launch_bounds__(BLK) void k_dcorr(CorrArgs a)
{
    const long long id = blockIdx.x * (long long)BLK + threadIdx.x;
    if (id >= (long long)a.npair * a.nmom * a.T) return;
    const int t = (int)(id % a.T), k = (int)((id / a.T) % a.nmom), j = (int)(id / ((long long)a.T * a.nmom));
    const double2 *f = a.Lp1 + ((size_t)a.pairs[2 * j] * a.nmom + k) * a.T;
    const double2 *h = a.Lp2 + ((size_t)a.pairs[2 * j + 1] * a.nmom + k) * a.T;
    double re = 0.0, im = 0.0;
    for (int ti = 0; ti < a.T; ++ti) {
        const double2 u = f[(ti + t) % a.T], v = h[ti];
        re += u.x * v.x - u.y * v.y;
        im += u.x * v.y + u.y * v.x;
    }
    a.D[id] = make_double2(re * a.norm, im * a.norm);
}

unsigned blocks(long long n) { return (unsigned)((n + BLK - 1) / BLK); }

}  // namespace

bool momproj_fits(const int L4[4]) { return L4[0] + L4[1] + L4[2] <= MAXAX; }

void launch_momproj(const double2 *L, double2 *Lp, const int *dmom, int ngamma, int nt, int nmom, const int L4[4],
                    hipStream_t s)
{
    MomArgs a{L, Lp, dmom, ngamma, nt, nmom, L4[0], L4[1], L4[2], L4[0] * L4[1] * L4[2]};
    const int ngr = (ngamma + GB - 1) / GB;
    hipLaunchKernelGGL(k_momproj, dim3((unsigned)(nt * nmom * ngr)), dim3(BLK), 0, s, a);
}

fl_status fl_momentum_project(fl_ctx *c, const double *L, int ngamma, int nt, const int *mom, int nmom, double *Lp,
                              fl_where where)
{
    if (!c) return set_err(nullptr, FL_ERR_ARG, "ctx is NULL");
    if (ngamma < 1 || ngamma > MAXG || nt < 1 || nmom < 1 || !L || !Lp || !mom)
        return set_err(c, FL_ERR_ARG, "need 1..16 Gammas, nt >= 1, nmom >= 1 and non-NULL arrays");
    if (!momproj_fits(c->L)) return set_err(c, FL_ERR_ARG, "momentum projection needs Lx + Ly + Lz <= 1024");
    if (where != FL_HOST && where != FL_DEVICE) return set_err(c, FL_ERR_ARG, "bad `where`");
    hipSetDevice(c->device);
    const int Vs = c->L[0] * c->L[1] * c->L[2];
    const size_t nin = (size_t)ngamma * nt * Vs * sizeof(double2), nout = (size_t)ngamma * nmom * nt * sizeof(double2);
    int *dmom = (int *)ws_get(c, WS_CORR_IDX, sizeof(int) * 3 * (size_t)nmom);
    if (!dmom) return set_err(c, FL_ERR_NOMEM, "device allocation failed");
    fl_status e;
    if ((e = hip_check(c, hipMemcpyAsync(dmom, mom, sizeof(int) * 3 * (size_t)nmom, hipMemcpyHostToDevice, c->stream),
                       "upload momenta")))
        return e;
    const double2 *din = (const double2 *)L;
    double2 *dout = (double2 *)Lp;
    if (where == FL_HOST) {
        double2 *bi = (double2 *)ws_get(c, WS_CORR_A, nin), *bo = (double2 *)ws_get(c, WS_CORR_OUT, nout);
        if (!bi || !bo) return set_err(c, FL_ERR_NOMEM, "device allocation failed");
        if ((e = hip_check(c, hipMemcpyAsync(bi, L, nin, hipMemcpyHostToDevice, c->stream), "upload loops"))) return e;
        din = bi;
        dout = bo;
    }
    launch_momproj(din, dout, dmom, ngamma, nt, nmom, c->L, c->stream);
    if ((e = hip_check(c, hipGetLastError(), "momentum projection"))) return e;
    if (where == FL_HOST &&
        (e = hip_check(c, hipMemcpyAsync(Lp, dout, nout, hipMemcpyDeviceToHost, c->stream), "download")))
        return e;
    return hip_check(c, hipStreamSynchronize(c->stream), "momentum projection");
}

fl_status fl_disconnected_corr(fl_ctx *c, const double *Lp1, const double *Lp2, int ngamma, int nmom,
                               const int *pairs, int npair, double *D, fl_where where)
{
    if (!c) return set_err(nullptr, FL_ERR_ARG, "ctx is NULL");
    if (ngamma < 1 || nmom < 1 || npair < 1 || !Lp1 || !Lp2 || !pairs || !D)
        return set_err(c, FL_ERR_ARG, "need ngamma, nmom, npair >= 1 and non-NULL arrays");
    for (int j = 0; j < 2 * npair; ++j)
        if (pairs[j] < 0 || pairs[j] >= ngamma) return set_err(c, FL_ERR_ARG, "pair index outside 0..ngamma-1");
    if (where != FL_HOST && where != FL_DEVICE) return set_err(c, FL_ERR_ARG, "bad `where`");
    hipSetDevice(c->device);
    const int T = c->L[3], Vs = c->L[0] * c->L[1] * c->L[2];
    const size_t nin = (size_t)ngamma * nmom * T * sizeof(double2), nout = (size_t)npair * nmom * T * sizeof(double2);
    int *dp = (int *)ws_get(c, WS_CORR_IDX, sizeof(int) * 2 * (size_t)npair);
    if (!dp) return set_err(c, FL_ERR_NOMEM, "device allocation failed");
    fl_status e;
    if ((e = hip_check(c, hipMemcpyAsync(dp, pairs, sizeof(int) * 2 * (size_t)npair, hipMemcpyHostToDevice,
                                         c->stream), "upload pairs")))
        return e;
    const double2 *a1 = (const double2 *)Lp1, *a2 = (const double2 *)Lp2;
    double2 *o = (double2 *)D;
    if (where == FL_HOST) {
        double2 *b1 = (double2 *)ws_get(c, WS_CORR_A, nin), *b2 = (double2 *)ws_get(c, WS_CORR_B, nin);
        double2 *bo = (double2 *)ws_get(c, WS_CORR_OUT, nout);
        if (!b1 || !b2 || !bo) return set_err(c, FL_ERR_NOMEM, "device allocation failed");
        if ((e = hip_check(c, hipMemcpyAsync(b1, Lp1, nin, hipMemcpyHostToDevice, c->stream), "upload")) ||
            (e = hip_check(c, hipMemcpyAsync(b2, Lp2, nin, hipMemcpyHostToDevice, c->stream), "upload")))
            return e;
        a1 = b1;
        a2 = b2;
        o = bo;
    }
    CorrArgs a{a1, a2, o, dp, nmom, T, npair, 1.0 / ((double)Vs * T)};
    hipLaunchKernelGGL(k_dcorr, dim3(blocks((long long)npair * nmom * T)), dim3(BLK), 0, c->stream, a);
    if ((e = hip_check(c, hipGetLastError(), "disconnected correlator"))) return e;
    if (where == FL_HOST &&
        (e = hip_check(c, hipMemcpyAsync(D, o, nout, hipMemcpyDeviceToHost, c->stream), "download")))
        return e;
    return hip_check(c, hipStreamSynchronize(c->stream), "disconnected correlator");
}

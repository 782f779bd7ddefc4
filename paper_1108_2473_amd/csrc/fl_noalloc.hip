// fl_noalloc.hip -- the entry point that allocates nothing: the Wilson-Dirac
// operator on device spinors with its even/odd work fields in a fixed
// device array of this library instead of allocated workspace.
//
// `scratch` is a file-scope device array; each GPU the library runs on holds
// its own copy until the process ends.  In host code its name is only a
// stand-in, never a device address: the address on a device comes from
// hipGetSymbolAddress, taken once per device with that device current (at
// fl_create) and kept in scratch_ptr[], which is what the launches receive.
#include <mutex>

#include "fl_host.h"

namespace {

constexpr size_t kScratchBytes = (size_t)FL_NOALLOC_SCRATCH_MB << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *scratch_ptr[kMaxDevices] = {};
bool scratch_tried[kMaxDevices] = {};
hipError_t scratch_err[kMaxDevices] = {};

}  // namespace

hipError_t noalloc_scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!scratch_tried[device]) {
        scratch_tried[device] = true;
        void *p = nullptr;
        scratch_err[device] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (scratch_err[device] == hipSuccess)
            scratch_ptr[device] = p;
        else
            (void)hipGetLastError();
    }
    return scratch_err[device];
}

static void *scratch_of(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return scratch_ptr[device];
}

extern "C" fl_status fl_apply_D_noalloc(fl_ctx *c, const double *in, double *out, int nrhs, int dagger)
{
    if (!c) return set_err(nullptr, FL_ERR_ARG, "ctx is NULL");
    if (nrhs < 0 || (nrhs > 0 && (!in || !out))) return set_err(c, FL_ERR_ARG, "bad spinor arguments");
    if (!c->have_gauge) return set_err(c, FL_ERR_STATE, "gauge field not set (fl_set_gauge)");
    if (!c->have_kappa) return set_err(c, FL_ERR_STATE, "kappa not set (fl_set_kappa)");
    // four FP64 half fields (even and odd of the input and of the result)
    const size_t half = (size_t)nrhs * c->Vh * 192;
    if (4 * half > kScratchBytes)
        return set_err(c, FL_ERR_ARG,
                       "fl_apply_D_noalloc: nrhs * V * 384 bytes exceed the " +
                           std::to_string(FL_NOALLOC_SCRATCH_MB) + " MiB scratch array");
    if (nrhs == 0) return FL_OK;
    unsigned char *base = (unsigned char *)scratch_of(c->device);
    if (!base) return set_err(c, FL_ERR_DEVICE, "fl_apply_D_noalloc: device scratch address not available");
    // the links of the FP64 operator were packed by fl_set_gauge
    const void *gauge = c->gauge_ok[LINK_F64_R18] ? c->gauge[LINK_F64_R18] : nullptr;
    if (!gauge) return set_err(c, FL_ERR_STATE, "FP64 links not packed (fl_set_gauge)");
    hipSetDevice(c->device);
    void *be = base, *bo = base + half, *xe = base + 2 * half, *xo = base + 3 * half;
    LatGeom g = lat_geom(c, nrhs);
    launch_canon_to_eo(in, (double2 *)be, (double2 *)bo, g, nrhs, c->stream);
    // (D psi)_e = psi_e - k H_eo psi_o, (D psi)_o = psi_o - k H_oe psi_e
    hop64_launch(c, gauge, nrhs, 0, bo, xe, be, 1.0, -c->kappa, dagger != 0);
    hop64_launch(c, gauge, nrhs, 1, be, xo, bo, 1.0, -c->kappa, dagger != 0);
    launch_eo_to_canon((const double2 *)xe, (const double2 *)xo, out, g, nrhs, c->stream);
    if (const char *le = take_launch_error())
        return set_err(c, FL_ERR_ARG, std::string("fl_apply_D_noalloc: kernel variant not built (") + le + ")");
    return hip_check(c, hipGetLastError(), "fl_apply_D_noalloc");
}

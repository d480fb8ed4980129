// hfr_residual_noalloc: the hybridized stage residuals of hfr_residual for
// callers that cannot allocate device memory (code under graph capture,
// serving loops).  It needs no solver: the element shares of the
// transmission residual, the kernels' only intermediate, live in a
// file-scope device array instead of a solver's workspace.
#include <mutex>
#include <string>

#include "mesh.h"

namespace hfr {
// Element shares g^(k) of the last call: [Nim][4][P][4] doubles.  Each GPU
// the library runs on holds one copy until the process ends; every call on
// that GPU uses it, so calls that overlap on one GPU race.
constexpr size_t kNoAllocScratchDoubles = size_t(1) << 20;   // 8 MiB
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];
}  // namespace hfr

using namespace hfr;

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's copy of `scratch`, looked up once per device
// with that device current (the array's name is a host-side stand-in).
fr_status scratch_address(double** out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(FR_E_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(FR_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                         hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<double*>(g_scratch_ptr[dev]);
    return FR_OK;
}

}  // namespace

extern "C" fr_status hfr_residual_noalloc(fr_mesh_t m, const double* u,
                                          const double* uhat, const double* ustar,
                                          double aii_dt, double* h, double* g,
                                          double* R_im, void* stream) {
    if (!m || !u || (!uhat && m->Ntp) || !ustar || (!h && m->Nim) || (!g && m->Ntp))
        return fail(FR_E_INVALID, "null argument");
    if (m->host_only) return fail(FR_E_INVALID, "host-only mesh");
    const size_t need = size_t(m->Nim) * 16 * m->P;
    if (need > kNoAllocScratchDoubles)
        return fail(FR_E_INVALID, "hfr_residual_noalloc: " + std::to_string(m->Nim) +
                                      " implicit elements need " + std::to_string(need) +
                                      " doubles of element shares, more than its " +
                                      std::to_string(kNoAllocScratchDoubles) +
                                      "-double scratch array");
    if (m->Nim == 0) return FR_OK;
    double* gk = nullptr;
    if (fr_status e = scratch_address(&gk)) return e;
    const hipStream_t st = hipStream_t(stream);
    ResidualLaunch a{};
    a.list = m->d_imp;
    a.nlist = m->Nim;
    a.u = u;
    a.Ne = m->Ne;
    a.verts = m->d_verts;
    a.finfo = m->d_finfo;
    a.fS = m->d_fS;
    a.uhat = uhat;
    a.phys = m->phys;
    a.efr_fnodes = m->efr ? m->d_efr_fnodes : nullptr;
    a.R = R_im;
    a.h = h;
    a.ustar = ustar;
    a.aii_dt = aii_dt;
    a.dtscale = m->d_dtscale;
    a.gk = gk;     // every entry is written by the residual kernel before the
                   // gather reads it, so nothing is cleared
    HIP_TRY(launch_residual(m->ops, a, st));
    if (m->Ntp == 0) return FR_OK;
    if (m->efr)
        HIP_TRY(launch_efr_gather_g(m->ops, m->Ntp, m->d_efr_inc_ptr, m->d_efr_inc, gk, g, st));
    else
        HIP_TRY(launch_trace_gather_g(m->Ntp, m->P, m->d_tpside, gk, g, st));
    return FR_OK;
}

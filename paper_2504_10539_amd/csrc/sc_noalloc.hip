// sc_noalloc.hip -- lbm_interface_metrics_noalloc (include/lbm.h): the
// interface metrics of a run (Sec. II-D Eqs. (9)-(13), Sec. IV-E Eqs.
// (14)-(16)) computed by the kernels of lbm_interface_metrics, with nothing
// allocated on the way.
//
// lbm_interface_metrics folds its per-block partials in the run's workspace
// and copies the result through a pinned host buffer that it allocates on
// first use.  This variant keeps the partials in `scratch`, a file-scope
// device array (one copy per GPU, held until the process ends), and writes the
// finished lbm_metrics record to caller device memory without waiting for the
// stream.  It calls no allocating routine, so code under HIP graph capture or
// a loop that must not allocate can use it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "sc_runtime.h"

namespace sclbm {
namespace {

// Partial records of the diagnostics pass (at most kMaxPartials blocks of
// kPartialStride doubles each), then the ten folded values.  Every block of a
// call writes the record it later reads, so nothing needs clearing between
// calls.
constexpr size_t kRawOffset = (size_t)kMaxPartials * kPartialStride;
constexpr size_t kScratchDoubles = kRawOffset + 32;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on device `dev`, looked up once per device with
// that device current.  Host code uses only this address: the array's own
// name is a host-side stand-in.
hipError_t scratch_on(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    const hipError_t back = cur != dev ? hipSetDevice(cur) : hipSuccess;
    if (e != hipSuccess) return e;
    if (back != hipSuccess) return back;
    g_scratch[dev] = static_cast<double*>(p);
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

// The metrics record from the ten folded values {mass, mom_x, mom_y, bad
// cells, cells above the threshold, G_max, sum |grad rho|, sum |grad rho|^2,
// rho_max, rho_min}, in the arithmetic of lbm_interface_metrics (Eqs. (9)-(13)
// with V_total = nx ny cells).
__global__ void k_metrics_record(const double* __restrict__ r, int nx, int ny, int64_t step,
                                 lbm_metrics* __restrict__ out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const double ncell = (double)nx * (double)ny;
  lbm_metrics m{};
  m.mass = r[0];
  m.mom_x = r[1];
  m.mom_y = r[2];
  m.finite = r[3] == 0.0 ? 1 : 0;
  m.n_above = (int64_t)r[4];
  m.Gmax = r[5];
  m.sum_grad = r[6];
  m.E_int = r[7];
  m.rho_max = r[8];
  m.rho_min = r[9];
  m.W = r[4] / ncell;
  m.drho = r[8] - r[9];
  m.W_eff = r[5] > 0.0 ? r[6] / (r[5] * ncell) : 0.0;
  m.step = step;
  *out = m;
}

}  // namespace
}  // namespace sclbm

using namespace sclbm;

extern "C" {

lbm_status lbm_interface_metrics_noalloc(lbm_ctx* c, lbm_metrics* out) {
  return guarded("lbm_interface_metrics_noalloc", [&]() -> lbm_status {
    if (!c || !out) return fail(LBM_EINVAL, "ctx or out is NULL");
    if ((uintptr_t)out & 7) return fail(LBM_EINVAL, "out must be 8-byte aligned device memory");
    const int blocks = diagnostics_blocks(c->p.nx, c->p.ny);
    if (blocks > kMaxPartials)
      return fail(LBM_ENOMEM, "the diagnostics need " + std::to_string(blocks) +
                                  " partial records; the static scratch holds " +
                                  std::to_string(kMaxPartials));
    // The stream's device (the current device for the null stream).
    int dev = 0;
    if (c->stream)
      SCLBM_HIP(hipStreamGetDevice(c->stream, &dev));
    else
      SCLBM_HIP(hipGetDevice(&dev));
    double* sp = nullptr;
    SCLBM_HIP(scratch_on(dev, &sp));
    double* raw = sp + kRawOffset;
    void* idle = c->pop[c->parity ^ 1];
    SCLBM_HIP(launch_diagnostics(c->p.storage, c->pop[c->parity], c->p.nx, c->p.ny,
                                 c->host_desc().rho0, reinterpret_cast<double*>(idle), sp, raw,
                                 c->stream));
    hipLaunchKernelGGL(k_metrics_record, dim3(1), dim3(64), 0, c->stream, (const double*)raw,
                       c->p.nx, c->p.ny, (int64_t)c->steps, out);
    SCLBM_HIP(hipGetLastError());
    return LBM_OK;
  });
}

}  // extern "C"

// The complex-step product for callers that cannot allocate device memory
// (code under stream capture, tight serving loops, harnesses that forbid
// allocation): dfr_jvp_complex_step_noalloc.  Its complex-FP32 form needs
// an FP32 copy of the linearisation state; dfr_jvp_complex_step keeps it in
// context memory allocated with the context, this variant in a file-scope
// device array, `scratch`, of fixed size.  The product's kernels, their tiles
// and their results are those of dfr_jvp_complex_step.
//
// The array exists once per device for the life of the process.  Its device
// address is looked up once per device, at context creation (with the
// context's device current), and kept in a table; host code never passes the
// array's name itself, which in host code is only a stand-in for the symbol.
#include "dfrsw_internal.h"

#include <mutex>
#include <string>
#include <vector>

namespace dfrsw {

constexpr size_t NOALLOC_SCRATCH_BYTES = DFR_NOALLOC_SCRATCH_BYTES;
static_assert(NOALLOC_SCRATCH_BYTES % 256 == 0, "whole 256-byte lines");

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

static std::mutex scratch_mu;
static std::vector<void *> scratch_addr;   // per device ordinal: the array's device address

int scratch_init(int device) {
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (device < 0) {
    set_error("scratch_init: no current device");
    return DFR_E_HIP;
  }
  if ((int)scratch_addr.size() <= device) scratch_addr.resize(device + 1, nullptr);
  if (scratch_addr[device]) return DFR_OK;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    set_error(std::string("device scratch array: hipGetSymbolAddress failed: ") + hipGetErrorString(e));
    return DFR_E_HIP;
  }
  scratch_addr[device] = p;
  return DFR_OK;
}

static void *scratch_ptr(int device) {
  std::lock_guard<std::mutex> lock(scratch_mu);
  return (device >= 0 && device < (int)scratch_addr.size()) ? scratch_addr[device] : nullptr;
}

}  // namespace dfrsw

using namespace dfrsw;

extern "C" {

int dfr_jvp_complex_step_noalloc(dfr_ctx *h, const double *q, const double *v, double eps, dfr_precision prec,
                                 double *jv) {
  if (h && h->c.ode_kind && prec != DFR_FP64) {
    set_error("dfr_jvp_complex_step_noalloc: test problems take the exact Jacobian in FP64 (DFR_FP64)");
    return DFR_E_INVAL;
  }
  if (!h || !q || !v || !jv || jv == q || jv == v || !eps_prec_ok(eps, prec)) {
    set_error("dfr_jvp_complex_step_noalloc: invalid argument (an FP32 form needs eps >= DFR_FP32_EPS_MIN)");
    return DFR_E_INVAL;
  }
  Ctx &c = h->c;
  // no event timing here: taking an event pair may create events
  struct NoTiming {
    KTimer &t;
    bool keep;
    explicit NoTiming(KTimer &tt) : t(tt), keep(tt.on) { t.on = false; }
    ~NoTiming() { t.on = keep; }
  } no_timing(c.tm);
  if (prec == DFR_FP64) return launch_dfr(&c, q, nullptr, v, nullptr, eps, true, false, jv, nullptr);
  const size_t need = sizeof(float) * (size_t)c.n3;
  if (need > NOALLOC_SCRATCH_BYTES) {
    set_error("dfr_jvp_complex_step_noalloc: the FP32 copy of q needs " + std::to_string(need) +
              " bytes, more than the " + std::to_string(NOALLOC_SCRATCH_BYTES) +
              "-byte device scratch array (at most " + std::to_string(NOALLOC_SCRATCH_BYTES / 12) + " nodes)");
    return DFR_E_INVAL;
  }
  float *q32 = static_cast<float *>(scratch_ptr(c.device));
  if (!q32) {
    set_error("dfr_jvp_complex_step_noalloc: no scratch address for the context's device");
    return DFR_E_HIP;
  }
  int rc = launch_copy_to_f32(&c, c.n3, q, q32);
  if (rc) return rc;
  return launch_dfr(&c, nullptr, q32, v, nullptr, eps, true, true, jv, nullptr);
}

}  // extern "C"

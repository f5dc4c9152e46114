// Handle-free entry point that allocates nothing: the misfit
// J = 1/2 (u - u_t)^T M_v (u - u_t) and its gradient, as eth_misfit computes
// them, for callers that cannot allocate device memory (code under HIP graph
// capture, serving loops, harnesses that forbid hipMalloc).
//
// The per-block partial sums of the reduction live in a fixed device array of
// this translation unit instead of a problem's workspace.  Every GPU that runs
// the library holds its own copy of the array until the process ends; its
// address on a device is looked up once, with that device current, and kept.
// Calls that overlap in time on one GPU share the array and race.
#include <mutex>

#include "../../include/eth.h"
#include "eth_kernels.h"

namespace {

// 2 MiB of FP64 partials: batch * 2 * ceil((2n+1)^2 / 256) must fit, i.e. one
// right-hand side up to n = 2048, eight at n = 1024
constexpr long long kScratchDoubles = 262144;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up once per device)
double* scratch_on(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) throw eth::HipError{e, "hipGetSymbolAddress(scratch)"};
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  return g_scratch_ptr[dev];
}

int fail(int code, const std::string& msg) {
  eth::g_setup_error = msg;
  return code;
}

}  // namespace

extern "C" {

int eth_misfit_noalloc(const eth_problem_desc* desc, const double* x, const double* x_target,
                       double* J, double* grad, int64_t batch, int64_t ld) {
  if (!desc || !x || !x_target || !J) return fail(ETH_EINVAL, "NULL argument");
  const int n = desc->n;
  if (n < 2) return fail(ETH_EINVAL, "n must be >= 2");
  if (!(desc->x1 > desc->x0) || !(desc->y1 > desc->y0)) return fail(ETH_EINVAL, "empty domain");
  if (std::fabs((desc->x1 - desc->x0) - (desc->y1 - desc->y0)) > 1e-12 * (desc->x1 - desc->x0))
    return fail(ETH_EINVAL, "square domain required");
  if (n > 8192) return fail(ETH_EINVAL, "n must be <= 8192");
  const eth::Geo g = eth::make_geo(n, (desc->x1 - desc->x0) / n);
  if (batch < 1 || batch > 65535) return fail(ETH_EINVAL, "batch must be in [1, 65535]");
  if (batch > 1 && ld < g.N) return fail(ETH_EINVAL, "ld must be >= the vector length");
  const long long need = (long long)batch * eth::adjoint_blocks(g);
  if (need > kScratchDoubles)
    return fail(ETH_EINVAL, "batch * 2 * ceil((2n+1)^2 / 256) = " + std::to_string(need) +
                                " partial sums exceed the fixed scratch of " +
                                std::to_string(kScratchDoubles));
  try {
    int dev = 0;
    ETH_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(ETH_EUNSUPPORTED, "device index beyond 63");
    double* partials = scratch_on(dev);
    hipStream_t st = static_cast<hipStream_t>(desc->stream);
    eth::RedCtx rc{};
    rc.partials = partials;
    rc.result = J;
    rc.nblocks = 0;  // set by the launcher from its grid
    rc.nvals = 1;
    rc.epi = eth::EPI_NONE;
    rc.epi_state = nullptr;
    if (grad) eth::launch_fill((long long)g.nk + g.n0, 0.0, grad + g.off_pk(), ld, (int)batch, st);
    eth::launch_velocity_mass(g, x, ld, x_target, ld, 0, grad, ld, &rc, (int)batch, st);
  } catch (const eth::HipError& e) {
    return fail(ETH_EDEVICE, e.where + ": " + hipGetErrorString(e.err));
  }
  return ETH_OK;
}

}  // extern "C"

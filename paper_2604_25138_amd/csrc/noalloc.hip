// laker_kernel_matvec_noalloc: the kernel product w = (lambda I + G) p for
// callers that cannot allocate device memory (code under HIP graph capture,
// serving loops, harnesses that forbid hipMalloc).  It runs the kernels of
// laker_kernel_matvec with their scratch (the prepared embedding copy and the
// product's partial sums) in a file-scope device array instead of a
// caller-provided workspace.
#include <math.h>

#include <mutex>

#include "pcg.hpp"

using namespace lk;

namespace {

// One copy per GPU that runs the library, held until the process ends.  Every
// call on a GPU uses that GPU's copy: calls that overlap on one GPU race.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

// Device address of `scratch` per GPU.  In host code the array's name is only a
// host-side stand-in for the symbol; kernels get this address.
void* g_scratch_dev[kMaxDevices];
std::mutex g_scratch_mu;

// Looks the address up on the GPU that runs `stream` (the current device for
// the null stream), with that device current, on the first call there.
laker_status scratch_address(hipStream_t stream, void** out) {
  int cur = 0;
  LK_TRY(hipGetDevice(&cur));
  int dev = cur;
  if (stream != nullptr) LK_TRY(hipStreamGetDevice(stream, &dev));
  if (dev < 0 || dev >= kMaxDevices) return LAKER_EHIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[dev] == nullptr) {
    if (dev != cur) LK_TRY(hipSetDevice(dev));
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (dev != cur) LK_TRY(hipSetDevice(cur));
    if (e != hipSuccess || ptr == nullptr) return LAKER_EHIP;
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return LAKER_OK;
}

// The scratch in the order the workspace of laker_kernel_matvec holds the same
// pieces: the prepared embeddings, then the partials.
struct MatvecScratch {
  void* emb;
  double* part;
  size_t total;
};

MatvecScratch plan_matvec_scratch(void* base, int64_t n, int dp, int prec) {
  WsCarver c(base);
  MatvecScratch m;
  m.emb = c.take<unsigned char>(embed_bytes(n, dp, prec));
  m.part = c.take<double>(kmv_part_elems(n, n));
  m.total = c.bytes();
  return m;
}

bool finite_pos(double x) { return isfinite(x) && x > 0.0; }

}  // namespace

extern "C" {

laker_status laker_kernel_matvec_noalloc(const laker_problem* prob, const double* p, double* w, int32_t precision,
                                         void* stream) {
  if (prob == nullptr || prob->E == nullptr || p == nullptr || w == nullptr) return LAKER_EINVAL;
  if (prob->n < 1 || prob->d < 1 || prob->d > kMaxD) return LAKER_EINVAL;
  if (!finite_pos(prob->lambda) || !finite_pos(prob->scale)) return LAKER_EINVAL;
  if (precision != LAKER_F64 && precision != LAKER_F32 && precision != LAKER_BF16) return LAKER_EINVAL;
  const int64_t n = prob->n;
  const int dp = pad_dim(prob->d);
  if (plan_matvec_scratch(nullptr, n, dp, precision).total > kNoAllocScratchBytes) return LAKER_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  void* base = nullptr;
  laker_status e = scratch_address(st, &base);
  if (e != LAKER_OK) return e;
  const MatvecScratch M = plan_matvec_scratch(base, n, dp, precision);
  LK_TRY(prep_embed(prob->E, n, prob->d, dp, prob->scale, precision, M.emb, st));
  // the arguments laker_kernel_matvec gives the same kernels (same plan, same
  // order of the partial sums: the results are bitwise equal)
  KmvArgs A{};
  A.Q = M.emb;
  A.m = n;
  A.K = M.emb;
  A.n = n;
  A.p = p;
  A.part = M.part;
  A.mode = 1;
  A.lam = prob->lambda;
  A.pself = p;
  A.out = w;
  LK_TRY(kmv_run(precision, dp, kmv_plan_square(n, dp, precision), A, st));
  return LAKER_OK;
}

}  // extern "C"

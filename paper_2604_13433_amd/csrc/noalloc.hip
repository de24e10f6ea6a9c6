// pksell_spmv_static: pksell_spmv for callers that cannot allocate device
// memory.  The products that need scratch (the chunk plan of CSR-packed
// matrices, split wide slices) take it from one array that the library
// holds per GPU, instead of the descriptor's ``partial``; every other
// product needs none and runs exactly as pksell_spmv.
#include <mutex>

#include "common.hpp"

namespace pksell {
int64_t spmv_partial_floats(const pksell_matrix *A, const float *x, int64_t k);
}

namespace {

// 16 MiB of float32 scratch per GPU, held until the process ends.
constexpr int64_t kScratchFloats = int64_t(1) << 22;
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) float scratch[kScratchFloats];

namespace {

// Device address of ``scratch`` on each GPU.  In host code the array's name
// is only a stand-in for the symbol, so kernels get these addresses, looked
// up once per device with that device current.
float *g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mutex;

int scratch_on(hipStream_t st, float **out) {
  int dev = 0;
  PKS_HIP(hipGetDevice(&dev));
  if (st) {
    hipDevice_t sdev = 0;
    PKS_HIP(hipStreamGetDevice(st, &sdev));
    PKS_CHECK((int)sdev == dev, PKSELL_EINVAL,
              "the stream belongs to device %d, but device %d is current", (int)sdev, dev);
  }
  PKS_CHECK(dev >= 0 && dev < kMaxDevices, PKSELL_ERANGE, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    PKS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    PKS_CHECK(p != nullptr, PKSELL_EHIP, "no device address for the scratch array");
    g_scratch[dev] = static_cast<float *>(p);
  }
  *out = g_scratch[dev];
  return PKSELL_OK;
}

}  // namespace

extern "C" int pksell_spmv_static(const pksell_matrix *A, const float *x, float *y, int64_t k,
                                  void *stream) {
  PKS_CHECK(A, PKSELL_EINVAL, "null matrix");
  const int64_t need = pksell::spmv_partial_floats(A, x, k);
  if (need == 0) return pksell_spmv(A, x, y, k, stream);
  PKS_CHECK(need <= kScratchFloats, PKSELL_ERANGE,
            "this product needs %lld scratch floats; the static scratch holds %lld",
            (long long)need, (long long)kScratchFloats);
  float *p = nullptr;
  const int rc = scratch_on(pksell::as_stream(stream), &p);
  if (rc) return rc;
  pksell_matrix local = *A;  // the same matrix with the library's scratch
  local.partial = p;
  return pksell_spmv(&local, x, y, k, stream);
}

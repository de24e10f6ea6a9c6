// A plain streaming read of a device buffer: the practical HBM read ceiling
// for a given transfer size on this GPU, measured the way the products are
// measured (one launch, nontemporal loads, eight in flight per lane).  Each
// wave reads ``chunks`` consecutive chunks of 64 lanes x ``width`` bytes.
// The loaded values are folded so the loads cannot be removed; nothing
// meaningful is stored.
#include "common.hpp"

namespace pksell {

namespace {

constexpr int kB = 256;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <typename T>
__device__ inline uint32_t fold(const T &v) {
  if constexpr (sizeof(T) == 4) return v;
  else return v.x ^ v.y ^ v.z ^ v.w;
}

template <typename T>
__global__ __launch_bounds__(kB) void k_stream_read(const T *__restrict__ src, uint64_t n,
                                                    uint32_t chunks, float *__restrict__ out) {
  const uint64_t wave = (uint64_t)xcd_remap(blockIdx.x, gridDim.x) * (kB / kWave) +
                        threadIdx.x / kWave;
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint64_t base = wave * chunks * kWave;
  uint32_t acc = 0;
  for (uint32_t c = 0; c < chunks; c += 8) {
    T v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const uint64_t i = base + (uint64_t)(c + q) * kWave + lane;
      v[q] = (c + q < chunks && i < n) ? __builtin_nontemporal_load(src + i) : T{};
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) acc ^= fold(v[q]);
  }
  if (acc == 0x9E3779B9u) out[0] = 1.0f;  // practically never; keeps the loads
}

}  // namespace
}  // namespace pksell

using namespace pksell;

extern "C" {

int pksell_stream_read(const void *src, size_t bytes, int32_t width, int32_t chunks, float *out,
                       void *stream) {
  PKS_CHECK(src && out, PKSELL_EINVAL, "null argument");
  PKS_CHECK(width == 4 || width == 16, PKSELL_EINVAL, "width must be 4 or 16");
  PKS_CHECK(chunks >= 1 && chunks <= 4096, PKSELL_EINVAL, "chunks must be in [1, 4096]");
  PKS_CHECK(bytes % 16 == 0 && bytes > 0, PKSELL_EINVAL, "bytes must be a positive multiple of 16");
  const uint64_t n = bytes / (uint64_t)width;
  const uint64_t waves = (n / kWave + (uint64_t)chunks - 1) / (uint64_t)chunks + 1;
  const int64_t blocks = cdiv((int64_t)waves, kB / kWave);
  PKS_CHECK(blocks < (int64_t(1) << 31), PKSELL_ERANGE, "too large");
  hipStream_t st = as_stream(stream);
  if (width == 4)
    k_stream_read<uint32_t><<<blocks, kB, 0, st>>>(static_cast<const uint32_t *>(src), n,
                                                   (uint32_t)chunks, out);
  else
    k_stream_read<u32x4><<<blocks, kB, 0, st>>>(static_cast<const u32x4 *>(src), n,
                                                (uint32_t)chunks, out);
  PKS_LAUNCHED();
  return PKSELL_OK;
}

}  // extern "C"

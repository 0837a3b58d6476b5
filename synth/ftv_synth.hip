// ftv_synth.hip -- device twin of the seeded input generator in synth/__init__.py.
//
// Same definitions, element for element: SplitMix64 output function over
// (seed, stream, index); U[-1,1) from 24 / 53 random bits; the Irwin-Hall
// stand-in for N(0,1) (12 draws of 24 bits, plus 24 extra low bits, exact in
// binary64, one round-to-nearest-even to fp32); magnitude-step ULP noise.
// Holds no part of the voter: it only writes inputs.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kSalt = 0x632BE59BD9B4E019ull;

__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__host__ __device__ inline uint64_t stream_key(uint64_t seed, uint64_t stream) {
  return mix64(seed ^ mix64(stream + kSalt));
}

__device__ inline uint64_t draw(uint64_t key, uint64_t idx) { return mix64(key + (idx + 1) * kGamma); }

// dtype: 0 f32, 1 f64, 2 i32, 3 i64.  dist: 0 uniform, 1 normal, 2 intfull.
__global__ void k_fill(void *dst, uint64_t n, int dtype, int dist, uint64_t key, uint64_t offset) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint64_t g = i + offset;
    if (dist == 2) {
      const uint64_t r = draw(key, g);
      if (dtype == 2) reinterpret_cast<uint32_t *>(dst)[i] = (uint32_t)(r >> 32);
      else reinterpret_cast<uint64_t *>(dst)[i] = r;
    } else if (dist == 0) {
      const uint64_t r = draw(key, g);
      if (dtype == 0) {
        const double m = (double)(r >> 40);
        reinterpret_cast<float *>(dst)[i] = (float)(m * 0x1p-23 - 1.0);
      } else {
        const double m = (double)(r >> 11);
        reinterpret_cast<double *>(dst)[i] = m * 0x1p-52 - 1.0;
      }
    } else {
      uint64_t acc = 0;
      for (int j = 0; j < 12; ++j) acc += draw(key, g * 13 + (uint64_t)j) >> 40;
      const uint64_t extra = draw(key, g * 13 + 12) >> 40;
      const uint64_t integer = (acc << 24) + extra;
      const double x = (double)integer * 0x1p-48 - 6.0;
      if (dtype == 0) reinterpret_cast<float *>(dst)[i] = (float)x;
      else reinterpret_cast<double *>(dst)[i] = x;
    }
  }
}

__global__ void k_ulp_noise(void *dst, uint64_t n, int dtype, uint64_t key, uint32_t thresh24,
                            uint32_t maxd) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint64_t r = draw(key, i);
    if ((r >> 40) >= thresh24) continue;
    const uint64_t d = 1 + ((r >> 1) % maxd);
    bool up = (r & 1) != 0;
    if (dtype == 0) {
      uint32_t *p = reinterpret_cast<uint32_t *>(dst) + i;
      const uint32_t u = *p, sign = u & 0x80000000u;
      uint64_t mag = u & 0x7fffffffu;
      up = up || mag < d;
      mag = up ? mag + d : mag - d;
      *p = sign | (uint32_t)mag;
    } else {
      uint64_t *p = reinterpret_cast<uint64_t *>(dst) + i;
      const uint64_t u = *p, sign = u & 0x8000000000000000ull;
      uint64_t mag = u & 0x7fffffffffffffffull;
      up = up || mag < d;
      mag = up ? mag + d : mag - d;
      *p = sign | mag;
    }
  }
}

unsigned grid_for(uint64_t n) {
  uint64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  return (unsigned)(g ? g : 1);
}

}  // namespace

extern "C" {

int ftvs_fill(void *dst, uint64_t n, int dtype, int dist, uint64_t seed, uint64_t stream,
              uint64_t offset, void *hip_stream) {
  if (!n) return 0;
  if (!dst || dtype < 0 || dtype > 3 || dist < 0 || dist > 2) return -1;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)hip_stream, dst, n, dtype,
                     dist, stream_key(seed, stream), offset);
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

int ftvs_ulp_noise(void *dst, uint64_t n, int dtype, uint64_t seed, uint64_t stream,
                   uint32_t thresh24, uint32_t maxd, void *hip_stream) {
  if (!n) return 0;
  if (!dst || (dtype != 0 && dtype != 1) || maxd == 0) return -1;
  hipLaunchKernelGGL(k_ulp_noise, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)hip_stream, dst, n,
                     dtype, stream_key(seed, stream), thresh24, maxd);
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

}  // extern "C"

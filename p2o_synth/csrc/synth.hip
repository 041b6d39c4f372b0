// Device-side seeded input generator.  Same definition as the host one in
// p2o_synth/__init__.py: SplitMix64 (Steele, Lea & Flood 2014) evaluated at a
// counter, then the cosine branch of Box-Muller.  Draws inputs only; nothing
// of the p2o method is computed here.
#include <hip/hip_runtime.h>
#include <cstdint>

namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ inline double normal_at(uint64_t key, uint64_t n) {
  const uint64_t a = mix64(key + (2 * n + 1) * kGolden);
  const uint64_t b = mix64(key + (2 * n + 2) * kGolden);
  const double u1 = (double)((a >> 11) + 1) * 0x1.0p-53;
  const double u2 = (double)(b >> 11) * 0x1.0p-53;
  return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

// out[k][s][p - p0] = z((k*Nd + s)*Nm + p) * env[k]
__global__ void blocks_kernel(double* __restrict__ out, int64_t Nt, int64_t Nd,
                              int64_t Nm, int64_t p0, int64_t pc, uint64_t key,
                              const double* __restrict__ env) {
  const int64_t total = Nt * Nd * pc;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t pl = i % pc;
    const int64_t ks = i / pc;  // k*Nd + s
    const int64_t k = ks / Nd;
    const uint64_t n = (uint64_t)(ks * Nm + p0 + pl);
    out[i] = normal_at(key, n) * env[k];
  }
}

__global__ void normals_kernel(double* __restrict__ out, int64_t n,
                               int64_t offset, uint64_t key, double scale) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    out[i] = normal_at(key, (uint64_t)(offset + i)) * scale;
  }
}

uint64_t stream_key(uint64_t seed, uint64_t array_id) {
  return mix64(seed * kGolden + array_id);
}

unsigned grid_for(int64_t total) {
  int64_t g = (total + 255) / 256;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (unsigned)g;
}

}  // namespace

extern "C" {

// Fills out[Nt][Nd][p1-p0] (device, float64) with block entries of columns
// p0..p1-1.  env: device array of Nt doubles.  Returns 0 or a hipError_t.
int synth_blocks_f64(double* out, int64_t Nt, int64_t Nd, int64_t Nm,
                     int64_t p0, int64_t p1, uint64_t seed, const double* env,
                     void* stream) {
  if (!out || !env || Nt < 1 || Nd < 1 || Nm < 1 || p0 < 0 || p1 <= p0 ||
      p1 > Nm)
    return (int)hipErrorInvalidValue;
  const int64_t pc = p1 - p0;
  const uint64_t key = stream_key(seed, 1);
  hipLaunchKernelGGL(blocks_kernel, dim3(grid_for(Nt * Nd * pc)), dim3(256), 0,
                     (hipStream_t)stream, out, Nt, Nd, Nm, p0, pc, key, env);
  return (int)hipGetLastError();
}

// out[i] = z(offset + i) * scale for i < n, stream (seed, array_id).
int synth_normals_f64(double* out, int64_t n, int64_t offset, uint64_t seed,
                      uint64_t array_id, double scale, void* stream) {
  if (!out || n < 0 || offset < 0) return (int)hipErrorInvalidValue;
  if (n == 0) return 0;
  const uint64_t key = stream_key(seed, array_id);
  hipLaunchKernelGGL(normals_kernel, dim3(grid_for(n)), dim3(256), 0,
                     (hipStream_t)stream, out, n, offset, key, scale);
  return (int)hipGetLastError();
}

}  // extern "C"

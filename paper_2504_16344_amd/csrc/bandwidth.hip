// Streaming-read ceiling of the device: a plain kernel that reads a buffer
// once with the same non-temporal 16-byte loads the block-product kernels
// stream their frequency blocks with, and does nothing else.  Its rate is
// the reference the block products' achieved bandwidth is compared with
// (section "Peak performance": the paper's own kernels are quoted at a
// fraction of the memory bandwidth).
#include "p2o_internal.h"

namespace p2o {
namespace {

typedef unsigned u4 __attribute__((ext_vector_type(4)));
constexpr int kReadThreads = 256;
constexpr int kReadUnroll = 4;

// Each thread owns entries i, i + 256, i + 512, i + 768 of a 1024-entry
// (16 KB) tile per step; the tiles are dealt to the work-groups round-robin.
// Full tiles are read with unconditional loads, the ragged tail after them
// entry by entry.  The loaded words are folded into one value whose only
// use is a store that never happens in practice (it keeps the loads alive).
__global__ void __launch_bounds__(kReadThreads)
read_stream(const u4* __restrict__ p, int64_t n16, double* __restrict__ sink) {
  constexpr int64_t kTile = (int64_t)kReadThreads * kReadUnroll;
  const int64_t full = n16 / kTile;
  unsigned acc = 0;
  for (int64_t t = blockIdx.x; t < full; t += gridDim.x) {
    const u4* q = p + t * kTile + threadIdx.x;
    u4 v[kReadUnroll];
#pragma unroll
    for (int u = 0; u < kReadUnroll; ++u) v[u] = __builtin_nontemporal_load(q + u * kReadThreads);
#pragma unroll
    for (int u = 0; u < kReadUnroll; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
  }
  for (int64_t i = full * kTile + (int64_t)blockIdx.x * kReadThreads + threadIdx.x; i < n16;
       i += (int64_t)gridDim.x * kReadThreads) {
    const u4 v = p[i];
    acc ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  if (acc == 0x8badf00du && threadIdx.x == 0 && blockIdx.x == 0) sink[0] = (double)acc;
}

}  // namespace

hipError_t launch_read_stream(const void* buf, int64_t bytes, double* sink, hipStream_t s) {
  const int64_t n16 = bytes / 16;
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const int64_t tiles = std::max<int64_t>(1, n16 / (kReadThreads * kReadUnroll));
  const unsigned grid = (unsigned)std::min<int64_t>(tiles, (int64_t)cus * 8);
  hipLaunchKernelGGL(read_stream, dim3(grid), dim3(kReadThreads), 0, s,
                     static_cast<const u4*>(buf), n16, sink);
  return hipGetLastError();
}

}  // namespace p2o

// Time-invariant spatial prior covariance: Gamma_prior = prior_var (I_Nt (x) C)
// (section "Real-time Bayesian inference and prediction framework", Phase 2:
// G* = Gamma_prior F* keeps the block Toeplitz structure when the prior acts
// on each time slice alike).  C is a synthetic smooth SPD covariance on an
// nx x ny grid of the spatial parameters (p = ix ny + iy):
//   C x = delta x + B (B x),   (B x)[ix, iy] = sum_{|a|,|b| <= r} w_a w_b x[ix + a, iy + b]
// with w_a = exp(-a^2 / (2 length^2)) and zero outside the grid, so B is
// symmetric and C is symmetric positive definite.  B is separable: B = Sy Sx
// with Sx, Sy the 1-D windows along each grid axis; C is applied as four
// 1-D passes, the last fused with the delta x term.
#include "p2o_internal.h"

namespace p2o {
namespace {

// out[s][ix][iy] = sum_a w[|a|] in[s][ix + a][iy] (AXIS 0) or in[s][ix][iy + a]
// (AXIS 1) over |a| <= r; with `base`, out = delta base + that sum (base may
// alias out: each element reads its own base entry before writing it).
template <int AXIS>
__global__ void __launch_bounds__(256)
window_pass(const double* __restrict__ in, double* out, const double* base, int64_t count,
            int64_t nx, int64_t ny, const double* __restrict__ w, int r, double delta) {
  const int64_t nm = nx * ny;
  const int64_t total = count * nm;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    const int64_t s = e / nm, p = e % nm;
    const int64_t ix = p / ny, iy = p % ny;
    const double* __restrict__ src = in + s * nm;
    double acc = 0.0;
    for (int a = -r; a <= r; ++a) {
      const int64_t jx = AXIS == 0 ? ix + a : ix, jy = AXIS == 0 ? iy : iy + a;
      if (jx >= 0 && jx < nx && jy >= 0 && jy < ny) acc += w[a < 0 ? -a : a] * src[jx * ny + jy];
    }
    out[e] = base ? delta * base[e] + acc : acc;
  }
}

unsigned grid_for(int64_t total) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 1 << 20));
}

}  // namespace

// x[count][nx * ny] <- C x in place; t1, t2 scratch of the same size.
hipError_t launch_apply_prior(double* x, double* t1, double* t2, int64_t count, int64_t nx,
                              int64_t ny, const double* w, int r, double delta, hipStream_t s) {
  const int64_t total = count * nx * ny;
  if (total <= 0) return hipSuccess;
  const unsigned g = grid_for(total);
  hipLaunchKernelGGL(window_pass<0>, dim3(g), dim3(256), 0, s, x, t1, nullptr, count, nx, ny, w,
                     r, 0.0);
  hipLaunchKernelGGL(window_pass<1>, dim3(g), dim3(256), 0, s, t1, t2, nullptr, count, nx, ny, w,
                     r, 0.0);
  hipLaunchKernelGGL(window_pass<0>, dim3(g), dim3(256), 0, s, t2, t1, nullptr, count, nx, ny, w,
                     r, 0.0);
  hipLaunchKernelGGL(window_pass<1>, dim3(g), dim3(256), 0, s, t1, x, x, count, nx, ny, w, r,
                     delta);
  return hipGetLastError();
}

}  // namespace p2o

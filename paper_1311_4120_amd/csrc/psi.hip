// Wave-function side of the energy: the density rho = |psi|^2 (the
// introduction, after eq. gpe2) and the derivative of E(rho) = (lambda/2) H
// sum rho u with respect to conj(psi).  With u = A rho and A symmetric,
// dE/drho = lambda H u, so dE/dpsi* = lambda H u psi.
#include "common.h"

namespace jgb {

namespace {

template <typename T>
struct alignas(2 * sizeof(T)) C2 {  // one 16-byte (fp64) or 8-byte (fp32) access
  T x, y;
};

template <typename T>
__global__ void k_abs2(const C2<T>* psi, T* rho, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) {
    const C2<T> v = psi[i];
    rho[i] = v.x * v.x + v.y * v.y;
  }
}

template <typename T>
__global__ void k_psi_grad(const C2<T>* psi, const T* u, const double* gscale, double scale, C2<T>* grad, int64_t n) {
  const double s = scale * (gscale ? *gscale : 1.0);
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) {
    const C2<T> v = psi[i];
    const double f = s * (double)u[i];
    grad[i] = C2<T>{(T)(f * (double)v.x), (T)(f * (double)v.y)};
  }
}

unsigned blocks_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

template <typename T>
hipError_t launch_density(const Plan& pl, const void* psi, void* rho, hipStream_t s) {
  const int64_t n = (int64_t)pl.n[0] * pl.n[1] * pl.n[2];
  hipLaunchKernelGGL(k_abs2<T>, dim3(blocks_for(n)), dim3(256), 0, s, (const C2<T>*)psi, (T*)rho, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_psi_gradient(const Plan& pl, const void* psi, const void* u, const double* gscale, double factor,
                               void* grad, hipStream_t s) {
  const int64_t n = (int64_t)pl.n[0] * pl.n[1] * pl.n[2];
  const double scale = factor * pl.p.lambda * pl.H;
  hipLaunchKernelGGL(k_psi_grad<T>, dim3(blocks_for(n)), dim3(256), 0, s, (const C2<T>*)psi, (const T*)u, gscale,
                     scale, (C2<T>*)grad, n);
  return hipGetLastError();
}

template hipError_t launch_density<double>(const Plan&, const void*, void*, hipStream_t);
template hipError_t launch_density<float>(const Plan&, const void*, void*, hipStream_t);
template hipError_t launch_psi_gradient<double>(const Plan&, const void*, const void*, const double*, double, void*,
                                                hipStream_t);
template hipError_t launch_psi_gradient<float>(const Plan&, const void*, const void*, const double*, double, void*,
                                               hipStream_t);

}  // namespace jgb

// Absorbing boundary term: coefficient rebuild, boundary records and the gradient
// term (see boundary.hpp).  Small launches over the boundary DOFs only.
#include "boundary.hpp"

namespace kmv {

namespace {
constexpr int kBlock = 256;

template <typename T>
__global__ void __launch_bounds__(kBlock) k_absorb_coef(const double* __restrict__ c, int nbd,
                                                        const int32_t* __restrict__ dof,
                                                        const double* __restrict__ coef, T* __restrict__ beta,
                                                        T* __restrict__ gamma, int nbr,
                                                        const int32_t* __restrict__ ref, T* __restrict__ beta_ref,
                                                        T* __restrict__ gamma_ref) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= nbd + nbr) return;
  const int t = i < nbd ? i : ref[2 * (i - nbd) + 1];
  const int32_t d = dof[t];
  const double a = coef[3 * t] + coef[3 * t + 1] * c[d];
  const T b = (T)((1.0 - a) / (1.0 + a)), g = (T)(coef[3 * t + 2] / (1.0 + a));
  if (i < nbd) {
    beta[d] = b;
    gamma[d] = g;
  } else {
    const int32_t r = ref[2 * (i - nbd)];
    beta_ref[r] = b;
    gamma_ref[r] = g;
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_gather_boundary(const T* __restrict__ lvl, int64_t ls, int ns, int nbd,
                                                            const int32_t* __restrict__ dof, T* __restrict__ out,
                                                            int64_t out_stride) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= (int64_t)ns * nbd) return;
  const int64_t sh = i / nbd, t = i - sh * nbd;
  out[sh * out_stride + t] = lvl[sh * ls + dof[t]];
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_gather_levels(const T* __restrict__ levels, int64_t level_stride,
                                                          int64_t ls, int ns, int64_t nlev, int nbd,
                                                          const int32_t* __restrict__ dof, T* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= (int64_t)ns * nlev * nbd) return;
  const int64_t t = i % nbd, r = i / nbd;  // r = sh*nlev + n
  const int64_t sh = r / nlev, n = r - sh * nlev;
  out[i] = levels[n * level_stride + sh * ls + dof[t]];
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_gather_ring(const T* __restrict__ ring, int K, int64_t slot_stride,
                                                        int64_t ls, int ns, int64_t n0, int cnt, int nbd,
                                                        const int32_t* __restrict__ dof, T* __restrict__ out,
                                                        int64_t out_stride) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= (int64_t)ns * cnt * nbd) return;
  const int64_t t = i % nbd, r = i / nbd;  // r = sh*cnt + j
  const int64_t sh = r / cnt, n = n0 + (r - sh * cnt);
  out[sh * out_stride + n * nbd + t] = ring[(n % K) * slot_stride + sh * ls + dof[t]];
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_absorb_part(const T* __restrict__ ub, const T* __restrict__ lb, int64_t nt,
                                                        int nbd, int ns, int nchunk, double* __restrict__ part) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const int k = blockIdx.y;
  if (t >= nbd) return;
  const int64_t len = (nt + nchunk - 1) / nchunk;
  const int64_t n0 = 1 + k * len, n1 = min(nt, (int64_t)(k + 1) * len);
  double acc = 0;
  for (int sh = 0; sh < ns; ++sh) {
    const T* u = ub + (int64_t)sh * (nt + 1) * nbd + t;
    const T* l = lb + (int64_t)sh * (nt + 1) * nbd + t;
    for (int64_t n = n0; n <= n1; ++n) {
      const double um2 = n >= 2 ? (double)u[(n - 2) * nbd] : 0.0;
      acc += (double)l[n * nbd] * ((double)u[n * nbd] - um2);
    }
  }
  part[(int64_t)k * nbd + t] = acc;
}

__global__ void __launch_bounds__(kBlock) k_absorb_add(const double* __restrict__ part, int nchunk, int nbd,
                                                       const int32_t* __restrict__ dof, const double* __restrict__ hb,
                                                       double* __restrict__ g) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= nbd) return;
  double acc = 0;
  for (int k = 0; k < nchunk; ++k) acc += part[(int64_t)k * nbd + t];
  g[dof[t]] += hb[t] * acc;
}

unsigned blocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }
}  // namespace

template <typename T>
hipError_t launch_absorb_coef(const double* c, int nbd, const int32_t* dof, const double* coef, T* beta,
                              T* gamma, int nbr, const int32_t* ref, T* beta_ref, T* gamma_ref, hipStream_t s) {
  if (nbd + nbr == 0) return hipSuccess;
  k_absorb_coef<T><<<blocks(nbd + nbr), kBlock, 0, s>>>(c, nbd, dof, coef, beta, gamma, nbr, ref, beta_ref,
                                                        gamma_ref);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gather_boundary(const T* lvl, int64_t ls, int ns, int nbd, const int32_t* dof, T* out,
                                  int64_t out_stride, hipStream_t s) {
  if (nbd == 0 || ns == 0) return hipSuccess;
  k_gather_boundary<T><<<blocks((int64_t)ns * nbd), kBlock, 0, s>>>(lvl, ls, ns, nbd, dof, out, out_stride);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gather_levels(const T* levels, int64_t level_stride, int64_t ls, int ns, int64_t nlev, int nbd,
                                const int32_t* dof, T* out, hipStream_t s) {
  if (nbd == 0 || ns == 0 || nlev == 0) return hipSuccess;
  k_gather_levels<T><<<blocks((int64_t)ns * nlev * nbd), kBlock, 0, s>>>(levels, level_stride, ls, ns, nlev, nbd,
                                                                         dof, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gather_ring(const T* ring, int K, int64_t slot_stride, int64_t ls, int ns, int64_t n0, int cnt,
                              int nbd, const int32_t* dof, T* out, int64_t out_stride, hipStream_t s) {
  if (nbd == 0 || ns == 0 || cnt <= 0) return hipSuccess;
  k_gather_ring<T><<<blocks((int64_t)ns * cnt * nbd), kBlock, 0, s>>>(ring, K, slot_stride, ls, ns, n0, cnt, nbd,
                                                                      dof, out, out_stride);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_absorb_grad(const T* ub, const T* lb, int64_t nt, int nbd, int ns, const int32_t* dof,
                              const double* hb, double* part, int nchunk, double* g, hipStream_t s) {
  if (nbd == 0 || nt < 1) return hipSuccess;
  k_absorb_part<T><<<dim3(blocks(nbd), (unsigned)nchunk), kBlock, 0, s>>>(ub, lb, nt, nbd, ns, nchunk, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_absorb_add<<<blocks(nbd), kBlock, 0, s>>>(part, nchunk, nbd, dof, hb, g);
  return hipGetLastError();
}

#define KMV_BOUNDARY_INST(T)                                                                                   \
  template hipError_t launch_absorb_coef<T>(const double*, int, const int32_t*, const double*, T*, T*, int,   \
                                            const int32_t*, T*, T*, hipStream_t);                              \
  template hipError_t launch_gather_boundary<T>(const T*, int64_t, int, int, const int32_t*, T*, int64_t,      \
                                                hipStream_t);                                                  \
  template hipError_t launch_gather_levels<T>(const T*, int64_t, int64_t, int, int64_t, int, const int32_t*, T*, \
                                              hipStream_t);                                                    \
  template hipError_t launch_gather_ring<T>(const T*, int, int64_t, int64_t, int, int64_t, int, int,          \
                                            const int32_t*, T*, int64_t, hipStream_t);                         \
  template hipError_t launch_absorb_grad<T>(const T*, const T*, int64_t, int, int, const int32_t*,            \
                                            const double*, double*, int, double*, hipStream_t);
KMV_BOUNDARY_INST(float)
KMV_BOUNDARY_INST(double)

}  // namespace kmv

// HIP kernels for gfx950 (CDNA4): matrix-free KMV stiffness apply fused with the
// leapfrog/sponge update, the reverse-time adjoint fused with the gradient
// accumulation, point injection/sampling, misfit and helpers.
//
// Work decomposition (one workgroup = one patch of cells, one thread = one cell):
//   1. coalesced loads of the patch-owned DOF values (a contiguous range) and
//      gathers of the DOFs the patch shares with neighbours, into LDS;
//   2. per cell, the reference-gradient contraction at the nodal quadrature
//      points, g_q = sum_b D[q][b] u_b, z_q = w_q c^2_q G_e g_q,
//      y_a = sum_q D[q][a] . z_q  (appendix, matrix K, with the KMV rule as
//      quadrature) -- the tables are kernel-uniform, so they live in scalar
//      registers, and the contraction runs on the VALU (fp32: 157 TF vector = the
//      fp32 MFMA rate on this part, so MFMA buys nothing at these shapes);
//   3. deterministic LDS scatter: cells are sorted by colour inside the patch and
//      colour c adds its y_a after colour c-1 (barrier in between), so every sum
//      has a fixed order and no atomics are needed;
//   4. leapfrog + sponge on the DOFs only this patch touches (eq. forward3 with a
//      diagonal leading matrix):  du <- beta du - gamma (K u - b),  u <- u + du;
//   5. partial sums of the shared DOFs to a buffer, finished by k_shared.
#include "kernels.hpp"

namespace kmv {

template <typename T, int DIM, int ND, bool ADJ>
__global__ void __launch_bounds__(512) k_patch(const PatchArgs<T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* su = reinterpret_cast<T*>(smem_raw);
  T* sc = su + A.nloc_max;
  T* sy = sc + A.nloc_max;
  T* sf = sy + A.nloc_max;   // ADJ only
  T* sr = sf + A.nloc_max;   // ADJ only
  const int p = blockIdx.x, tid = threadIdx.x, bs = blockDim.x;
  const int own0 = A.own_start[p], nown = A.own_start[p + 1] - own0;
  const int sh0 = A.sh_start[p], nsh = A.sh_start[p + 1] - sh0;

  for (int i = tid; i < nown; i += bs) {
    su[i] = A.u_in[own0 + i];
    sc[i] = A.c2[own0 + i];
    sy[i] = T(0);
    if (ADJ) {
      sf[i] = A.uf[own0 + i];
      sr[i] = T(0);
    }
  }
  for (int j = tid; j < nsh; j += bs) {
    const int g = A.sh_idx[sh0 + j];
    su[nown + j] = A.u_in[g];
    sc[nown + j] = A.c2[g];
    sy[nown + j] = T(0);
    if (ADJ) {
      sf[nown + j] = A.uf[g];
      sr[nown + j] = T(0);
    }
  }
  __syncthreads();

  const int c0 = A.cell_start[p], c1 = A.cell_start[p + 1];
  const int e = c0 + tid;
  const bool active = e < c1;
  int m[ND];
  T ye[ND];
  T re[ADJ ? ND : 1];
  if (active) {
    T ue[ND];
    T fe[ADJ ? ND : 1];
#pragma unroll
    for (int a = 0; a < ND; ++a) {
      m[a] = A.lmap[(int64_t)a * A.n_cells + e];
      ue[a] = su[m[a]];
      if (ADJ) fe[a] = sf[m[a]];
      ye[a] = T(0);
    }
    T G[DIM == 2 ? 3 : 6];
#pragma unroll
    for (int k = 0; k < (DIM == 2 ? 3 : 6); ++k) G[k] = A.geom[(int64_t)k * A.n_cells + e];
#pragma unroll
    for (int q = 0; q < ND; ++q) {
      T g[DIM];
#pragma unroll
      for (int r = 0; r < DIM; ++r) g[r] = T(0);
#pragma unroll
      for (int b = 0; b < ND; ++b)
#pragma unroll
        for (int r = 0; r < DIM; ++r) g[r] += A.D[(q * ND + b) * DIM + r] * ue[b];
      T v[DIM];
      if (DIM == 2) {
        v[0] = G[0] * g[0] + G[1] * g[1];
        v[1] = G[1] * g[0] + G[2] * g[1];
      } else {
        v[0] = G[0] * g[0] + G[1] * g[1] + G[2] * g[2];
        v[1] = G[1] * g[0] + G[3] * g[1] + G[4] * g[2];
        v[2] = G[2] * g[0] + G[4] * g[1] + G[5] * g[2];
      }
      const T wq = A.W[q];
      const T cw = wq * sc[m[q]];
      T z[DIM];
#pragma unroll
      for (int r = 0; r < DIM; ++r) z[r] = cw * v[r];
#pragma unroll
      for (int b = 0; b < ND; ++b)
#pragma unroll
        for (int r = 0; r < DIM; ++r) ye[b] += A.D[(q * ND + b) * DIM + r] * z[r];
      if (ADJ) {
        T gf[DIM];
#pragma unroll
        for (int r = 0; r < DIM; ++r) gf[r] = T(0);
#pragma unroll
        for (int b = 0; b < ND; ++b)
#pragma unroll
          for (int r = 0; r < DIM; ++r) gf[r] += A.D[(q * ND + b) * DIM + r] * fe[b];
        T s = T(0);
#pragma unroll
        for (int r = 0; r < DIM; ++r) s += gf[r] * v[r];
        re[ADJ ? q : 0] = wq * s;
      }
    }
  }

  // colour-ordered scatter into LDS
  const int ncol = A.ncol[p];
  int myc = -1;
  if (active) {
    const int32_t* cs = A.colour_start + (int64_t)p * kColStride;
    for (int c = 0; c < ncol; ++c)
      if (e >= cs[c] && e < cs[c + 1]) myc = c;
  }
  for (int c = 0; c < ncol; ++c) {
    if (myc == c) {
#pragma unroll
      for (int a = 0; a < ND; ++a) {
        sy[m[a]] += ye[a];
        if (ADJ) sr[m[a]] += re[ADJ ? a : 0];
      }
    }
    __syncthreads();
  }

  // point injection: one thread per target DOF, entries in a fixed order
  if (A.grp_ptr != nullptr) {
    for (int gi = A.grp_ptr[p] + tid; gi < A.grp_ptr[p + 1]; gi += bs) {
      T acc = T(0);
      for (int k = A.grp_eptr[gi]; k < A.grp_eptr[gi + 1]; ++k) acc += A.ent_w[k] * A.amp[A.ent_pt[k]];
      sy[A.grp_local[gi]] -= acc * A.amp_scale;
    }
    __syncthreads();
  }

  if (A.mode == 1) {
    for (int i = tid; i < nown; i += bs) A.y_out[own0 + i] = sy[i];
  } else {
    for (int i = tid; i < nown; i += bs) {
      const int gi = own0 + i;
      const T b = A.beta ? A.beta[gi] : T(1);
      const T dn = b * A.du[gi] - A.gamma[gi] * sy[i];
      A.du[gi] = dn;
      A.u_out[gi] = su[i] + dn;
      if (ADJ) A.gacc[gi] += (double)sr[i];
    }
  }
  for (int j = tid; j < nsh; j += bs) {
    A.partial[sh0 + j] = sy[nown + j];
    if (ADJ) A.partial_r[sh0 + j] = sr[nown + j];
  }
}

template <typename T, bool ADJ>
__global__ void __launch_bounds__(256) k_shared(const SharedArgs<T> A) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= A.n_shared) return;
  T y = T(0);
  const int k0 = A.shp_ptr[s], k1 = A.shp_ptr[s + 1];
  for (int k = k0; k < k1; ++k) y += A.partial[A.shp_slot[k]];
  const int64_t i = A.n_own + s;
  if (A.mode == 1) {
    A.y_out[i] = y;
    return;
  }
  const T b = A.beta ? A.beta[i] : T(1);
  const T dn = b * A.du[i] - A.gamma[i] * y;
  A.du[i] = dn;
  A.u_out[i] = A.u_in[i] + dn;
  if (ADJ) {
    T r = T(0);
    for (int k = k0; k < k1; ++k) r += A.partial_r[A.shp_slot[k]];
    A.gacc[i] += (double)r;
  }
}

template <typename T>
__global__ void k_sample(const T* __restrict__ u, const int32_t* __restrict__ dof,
                         const T* __restrict__ w, int npts, int nd, T* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= npts) return;
  T s = T(0);
  for (int a = 0; a < nd; ++a) s += w[j * nd + a] * u[dof[j * nd + a]];
  out[j] = s;
}

template <typename T>
__global__ void k_square(const double* __restrict__ c, T* __restrict__ c2, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) c2[i] = (T)(c[i] * c[i]);
}

template <typename T>
__global__ void k_fill(T* __restrict__ x, T v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

// Block-level float64 sum in a fixed tree order.
__device__ double block_sum(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (tid < off) sh[tid] += sh[tid + off];
    __syncthreads();
  }
  return sh[0];
}

template <typename T>
__global__ void __launch_bounds__(256) k_misfit(const T* __restrict__ d, const T* __restrict__ obs,
                                                T* __restrict__ resid, int64_t n,
                                                double* __restrict__ part) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double r = (double)obs[i] - (double)d[i];
    resid[i] = (T)r;
    acc += r * r;
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_reduce_parts(const double* __restrict__ part, int n,
                                                      double scale, double* __restrict__ out) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc += part[i];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) *out = scale * s;
}

__global__ void k_finalize_grad(const double* __restrict__ c, const double* __restrict__ gacc,
                                double scale, double* __restrict__ g, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) g[i] = scale * c[i] * gacc[i];
}

template <typename T>
__global__ void k_scale(const T* __restrict__ x, const T* __restrict__ s, T* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i] * s[i];
}

template <typename T>
__global__ void __launch_bounds__(256) k_dot(const T* __restrict__ x, const T* __restrict__ y, int64_t n,
                                             double* __restrict__ part) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    acc += (double)x[i] * (double)y[i];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

template <typename T>
__global__ void k_normalize(T* __restrict__ v, const T* __restrict__ w, const double* __restrict__ ww,
                            int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = (T)((double)w[i] / sqrt(*ww));
}

// ------------------------------------------------------------------ launchers
namespace {
inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <typename T, int DIM, int ND, bool ADJ>
hipError_t launch_patch_t(const PatchArgs<T>& a, int np, int block, hipStream_t s) {
  const int narr = ADJ ? 5 : 3;
  const size_t lds = (size_t)narr * a.nloc_max * sizeof(T);
  hipLaunchKernelGGL((k_patch<T, DIM, ND, ADJ>), dim3(np), dim3(block), lds, s, a);
  return hipGetLastError();
}

template <typename T, int DIM, int ND, bool ADJ>
hipError_t set_lds_t(int bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_patch<T, DIM, ND, ADJ>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

#define KMV_DISPATCH(FN, ...)                                                            \
  switch (dim * 100 + nd) {                                                              \
    case 203: return adjoint ? FN<T, 2, 3, true>(__VA_ARGS__) : FN<T, 2, 3, false>(__VA_ARGS__);     \
    case 207: return adjoint ? FN<T, 2, 7, true>(__VA_ARGS__) : FN<T, 2, 7, false>(__VA_ARGS__);     \
    case 212: return adjoint ? FN<T, 2, 12, true>(__VA_ARGS__) : FN<T, 2, 12, false>(__VA_ARGS__);   \
    case 218: return adjoint ? FN<T, 2, 18, true>(__VA_ARGS__) : FN<T, 2, 18, false>(__VA_ARGS__);   \
    case 230: return adjoint ? FN<T, 2, 30, true>(__VA_ARGS__) : FN<T, 2, 30, false>(__VA_ARGS__);   \
    case 304: return adjoint ? FN<T, 3, 4, true>(__VA_ARGS__) : FN<T, 3, 4, false>(__VA_ARGS__);     \
    case 315: return adjoint ? FN<T, 3, 15, true>(__VA_ARGS__) : FN<T, 3, 15, false>(__VA_ARGS__);   \
    case 332: return adjoint ? FN<T, 3, 32, true>(__VA_ARGS__) : FN<T, 3, 32, false>(__VA_ARGS__);   \
    default: return hipErrorInvalidValue;                                                \
  }
}  // namespace

template <typename T>
hipError_t launch_patch(int dim, int nd, bool adjoint, const PatchArgs<T>& a, int n_patches,
                        int block, hipStream_t s) {
  KMV_DISPATCH(launch_patch_t, a, n_patches, block, s)
}

template <typename T>
hipError_t set_patch_lds_limit(int dim, int nd, bool adjoint, int bytes) {
  KMV_DISPATCH(set_lds_t, bytes)
}

template <typename T>
hipError_t launch_shared(bool adjoint, const SharedArgs<T>& a, hipStream_t s) {
  if (a.n_shared == 0) return hipSuccess;
  const unsigned nb = blocks_for(a.n_shared, 256);
  if (adjoint)
    hipLaunchKernelGGL((k_shared<T, true>), dim3(nb), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_shared<T, false>), dim3(nb), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sample(const T* u, const int32_t* dof, const T* w, int npts, int nd, T* out,
                         hipStream_t s) {
  if (npts <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_sample<T>), dim3(blocks_for(npts, 256)), dim3(256), 0, s, u, dof, w, npts, nd, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_square(const double* c, T* c2, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_square<T>), dim3(blocks_for(n, 256)), dim3(256), 0, s, c, c2, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(T* x, T v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_fill<T>), dim3(blocks_for(n, 256)), dim3(256), 0, s, x, v, n);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* x, double v, int64_t n, hipStream_t s) { return launch_fill<double>(x, v, n, s); }

template <typename T>
hipError_t launch_misfit(const T* d, const T* obs, T* resid, int64_t n, double* scratch, int nblocks,
                         double* J_out, hipStream_t s) {
  hipLaunchKernelGGL((k_misfit<T>), dim3(nblocks), dim3(256), 0, s, d, obs, resid, n, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_parts, dim3(1), dim3(256), 0, s, scratch, nblocks, 0.5, J_out);
  return hipGetLastError();
}

hipError_t launch_finalize_grad(const double* c, const double* gacc, double scale, double* g, int64_t n,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_grad, dim3(blocks_for(n, 256)), dim3(256), 0, s, c, gacc, scale, g, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_scale(const T* x, const T* sc, T* y, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL((k_scale<T>), dim3(blocks_for(n, 256)), dim3(256), 0, st, x, sc, y, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dot(const T* x, const T* y, int64_t n, double* scratch, int nblocks, double* out,
                      hipStream_t s) {
  hipLaunchKernelGGL((k_dot<T>), dim3(nblocks), dim3(256), 0, s, x, y, n, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_parts, dim3(1), dim3(256), 0, s, scratch, nblocks, 1.0, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_axpby_norm(T* v, const T* w, const double* dot_ww, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_normalize<T>), dim3(blocks_for(n, 256)), dim3(256), 0, s, v, w, dot_ww, n);
  return hipGetLastError();
}

#define KMV_INST(T)                                                                                    \
  template hipError_t launch_patch<T>(int, int, bool, const PatchArgs<T>&, int, int, hipStream_t);     \
  template hipError_t set_patch_lds_limit<T>(int, int, bool, int);                                     \
  template hipError_t launch_shared<T>(bool, const SharedArgs<T>&, hipStream_t);                      \
  template hipError_t launch_sample<T>(const T*, const int32_t*, const T*, int, int, T*, hipStream_t); \
  template hipError_t launch_square<T>(const double*, T*, int64_t, hipStream_t);                      \
  template hipError_t launch_fill<T>(T*, T, int64_t, hipStream_t);                                    \
  template hipError_t launch_misfit<T>(const T*, const T*, T*, int64_t, double*, int, double*,         \
                                       hipStream_t);                                                  \
  template hipError_t launch_scale<T>(const T*, const T*, T*, int64_t, hipStream_t);                  \
  template hipError_t launch_dot<T>(const T*, const T*, int64_t, double*, int, double*, hipStream_t); \
  template hipError_t launch_axpby_norm<T>(T*, const T*, const double*, int64_t, hipStream_t);
KMV_INST(float)
KMV_INST(double)

}  // namespace kmv

// Absorbing boundary term: device kernels (host launchers).
//
// The first-order absorbing condition du/dt + c du/dn = 0 on the outer boundary
// puts the boundary integral of c phi_i phi_j in the damping matrix M_{u,1} (the
// appendix's matrices).  Lumped by rows with c at node i it is c_i b_i on the
// boundary DOFs, so their damping a_i = eta_i dt/2 + dt c_i b_i / (2 M_i) depends on
// the control c, and dJ/dc_i gains
//   (dt b_i / 2) sum_{n=1}^{N_t} lambda_i^n (u_i^n - u_i^{n-2}),   u^{-1} = u^0 = 0,
// the derivative of the discrete misfit through that damping.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace kmv {

// Ordered partial sums over time of the gradient term (one chunk of steps each).
constexpr int kBndChunks = 64;
// Adjoint levels kept in the ring while the term is on.
constexpr int kLamRing = 8;

// beta, gamma of the boundary DOFs (and their per-ref copies) from c:
// coef[3t..3t+2] = (eta_i dt/2, dt b_i/(2 M_i), dt^2/M_i) of boundary DOF t = dof[t];
// ref[2u], ref[2u+1] = (shared ref r, boundary DOF t) for the refs of boundary DOFs.
template <typename T>
hipError_t launch_absorb_coef(const double* c, int nbd, const int32_t* dof, const double* coef, T* beta,
                              T* gamma, int nbr, const int32_t* ref, T* beta_ref, T* gamma_ref, hipStream_t s);

// out[sh*out_stride + t] = lvl[sh*ls + dof[t]] for every shot sh < ns.
template <typename T>
hipError_t launch_gather_boundary(const T* lvl, int64_t ls, int ns, int nbd, const int32_t* dof, T* out,
                                  int64_t out_stride, hipStream_t s);

// The same for every level at once when all levels are kept:
// out[(sh*nlev + n)*nbd + t] = levels[n*level_stride + sh*ls + dof[t]], n < nlev.
template <typename T>
hipError_t launch_gather_levels(const T* levels, int64_t level_stride, int64_t ls, int ns, int64_t nlev, int nbd,
                                const int32_t* dof, T* out, hipStream_t s);

// Levels n0 .. n0+cnt-1 of a ring of K levels (level n in slot n % K, slots
// slot_stride apart, shots ls apart within a slot):
// out[sh*out_stride + n*nbd + t] = ring[(n % K)*slot_stride + sh*ls + dof[t]].
template <typename T>
hipError_t launch_gather_ring(const T* ring, int K, int64_t slot_stride, int64_t ls, int ns, int64_t n0, int cnt,
                              int nbd, const int32_t* dof, T* out, int64_t out_stride, hipStream_t s);

// g[dof[t]] += hb[t] * sum_sh sum_{n=1}^{nt} lb[sh][n][t] (ub[sh][n][t] - ub[sh][n-2][t])
// with rows [sh][n] of nbd values, n = 0..nt (ub row 0 = u^0 = 0; u^{-1} = 0); the sum
// over n is split in nchunk ordered partials (part: [nchunk*nbd] doubles), so the
// result does not depend on scheduling.
template <typename T>
hipError_t launch_absorb_grad(const T* ub, const T* lb, int64_t nt, int nbd, int ns, const int32_t* dof,
                              const double* hb, double* part, int nchunk, double* g, hipStream_t s);

}  // namespace kmv

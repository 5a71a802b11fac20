// HIP kernels for gfx950 (CDNA4): one fused launch per time step for the forward
// and for the reverse-time adjoint (fused with the float64 gradient accumulation),
// plus a small finisher, point sampling, misfit and helpers.
//
// Work decomposition of k_step (one workgroup = one patch of cells, one thread =
// one cell):
//   * every global load is issued up front.  A cell's interior DOFs (nodes inside
//     the cell: their DOF belongs to it alone) sit at own_start + j*nc + t, so the
//     thread of cell t loads them coalesced into registers and finishes them
//     itself.  The patch's other owned DOFs are one contiguous range, staged in
//     LDS; DOFs shared with neighbouring patches are finished from the previous
//     step's partial sums in a fixed order and staged too;
//   * per cell, the reference-gradient contraction at the nodal quadrature
//     points, g_q = sum_b D[q][b] u_b, z_q = w_q c^2_q G_e g_q,
//     y_a = sum_q D[q][a] . z_q (appendix, matrix K, with the KMV rule as the
//     quadrature).  The tables are compile-time constants (instruction literals,
//     zero entries dropped) and the contraction runs on the VALU; the point
//     sources of the cell enter the element vector;
//   * deterministic assembly of the non-interior DOFs: each cell writes its
//     contributions to its own LDS slots, then each DOF sums its slots in a fixed
//     (cell, node) order, read from one 32-bit gather word (one or two slots) or
//     a short list;
//   * leapfrog + sponge (eq. forward3 with a diagonal leading matrix):
//     du <- beta du - gamma (K u - b), u <- u + du.
#include <hip/hip_ext.h>

#include <algorithm>

#include "kernels.hpp"
#include "kmv_tables.inc"

namespace kmv {

__host__ __device__ constexpr size_t align16(size_t b) { return (b + 15) / 16 * 16; }

// LDS layout of k_step (element type first): su, sc [and sf] hold the level,
// c^2 [and the forward state] of the patch's non-interior DOFs; sx [and sr] the
// cell-node contributions, slot b*CS + t for node b of cell t plus a zero slot;
// then the gather lists (uint16).
// With ovl the slots start right after the level and overlay the c^2 [and u^m]
// staging, which is dead once every thread has read its element's values (3D:
// the slot arrays are the largest part, and LDS limits the resident workgroups).
// With gst (2D adjoints whose occupancy registers limit, not LDS) the float64
// gradient accumulators of the owned non-interior DOFs follow, at sg.
// With pml (2D) the auxiliary level, the two damping functions, and for the owned
// DOFs' update the previous auxiliary level, gamma and beta of the non-interior DOFs
// follow at sp (eight arrays of LB), then the two cell-node slot arrays of the
// gradient term t at st.
struct StepLds {
  size_t sx, gl, sg, sp, st, total;
  __host__ __device__ StepLds(int LB, int cs, int nb, int glmax, bool adj, size_t ts, bool ovl, bool gst,
                              bool pml = false) {
    const size_t nslot = (size_t)nb * cs + 1;
    const size_t stage = (size_t)(adj ? 3 : 2) * LB * ts, slots = (adj ? 2 : 1) * nslot * ts;
    if (ovl) {
      sx = align16((size_t)LB * ts);
      gl = align16(sx + slots > stage ? sx + slots : stage);
    } else {
      sx = align16(stage);
      gl = sx + align16(slots);
    }
    sg = gl + align16((size_t)glmax * 2);
    total = sg + (gst ? align16((size_t)LB * 8) : 0);
    sp = st = total;
    if (pml) {
      st = sp + align16((size_t)8 * LB * ts);
      total = st + align16((size_t)2 * nslot * ts);
    }
  }
};

// Owned non-interior gradient accumulators staged in LDS (see StepLds): FP32 2D
// adjoints of the elements where it costs no occupancy (KMV1, KMV2, and KMV4 with
// its register cap below; KMV3 would drop from four waves per SIMD to three, and
// the FP64 KMV4 adjoint from two workgroups per CU to one, by LDS).
constexpr bool stage_grad(bool adj, int dim, int nd, size_t ts) {
  return adj && dim == 2 && ts == 4 && (nd <= 7 || nd == 18);
}
template <typename T, bool ADJ, int DIM, int ND>
constexpr bool kStageGrad = stage_grad(ADJ, DIM, ND, sizeof(T));

// Shared refs per thread finished in the first batch of k_step (3D patches have
// several times more than 2D ones: a 256-cell KMV3 tetrahedron patch about five per
// thread); the rest go through the loop over the remaining refs, two per pass.
constexpr int first_batch_shared(int dim, int nd, bool adj) { return dim == 3 && !adj ? (nd == 32 ? 6 : 4) : 2; }

// Items per thread whose global loads are issued together (latency hiding).
template <typename T, bool ADJ = false, int ND = 18, int DIM = 2>
struct Batch {
  // owned non-interior DOFs in registers (fewer for the largest elements, whose
  // element vectors already fill the register file)
  static constexpr int kOwned = sizeof(T) == 4 ? (ND >= 30 ? 2 : 5) : 2;
  static constexpr int kWords = sizeof(T) == 4 ? 6 : 4;   // gather words in registers
  static constexpr int kShared = first_batch_shared(DIM, ND, ADJ);
  static constexpr int kList = 1;                         // 16-byte gather-list words
};

int step_first_batch_refs(int dim, int nd, bool adjoint, int block) {
  return first_batch_shared(dim, nd, adjoint) * block;
}

int step_block(int max_patch_cells) { return max_patch_cells <= 64 ? 64 : (max_patch_cells + 63) / 64 * 64; }

// Sum of the cell-node contributions of one local DOF, in its fixed slot order.
template <typename T>
__device__ __forceinline__ T gather_sum(uint32_t w, const T* x, const uint16_t* gl) {
  const uint32_t lo = w & 0xFFFFu, hi = w >> 16;
  if (hi != kGatherList) return x[lo] + x[hi];
  const int k = gl[lo];
  T y = x[gl[lo + 1]];
  for (int q = 1; q < k; ++q) y += x[gl[lo + 1 + q]];
  return y;
}

// Streaming accesses of data a step touches once (the level and increment it
// reads and writes, the forward state u^m, the gradient accumulators, the shared
// refs' copies and partial sums): in one-shot launches of the FP32 triangle kernels
// they carry the non-temporal hint, which keeps them from displacing the mesh tables
// and coefficients that every step re-reads from the caches (measured 662 -> 616 ms
// per C2 misfit + gradient).  With several shots per launch the hint measured
// slower (8 shots: 74 -> 91 us per forward launch), as did the FP64 kernels, and the
// tetrahedron kernels no faster; they keep plain accesses (NT = false).
template <typename T, int DIM>
constexpr bool kStream = sizeof(T) == 4 && DIM == 2;
// The hint is a template argument, never a run-time choice: two loads of one
// address under a run-time condition are merged by the compiler, hint dropped.
template <typename T, int DIM, bool NT, typename V>
__device__ __forceinline__ V ld_once(const V* p) {
  if constexpr (kStream<T, DIM> && NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <typename T, int DIM, bool NT, typename V>
__device__ __forceinline__ void st_once(V v, V* p) {
  if constexpr (kStream<T, DIM> && NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// Minimum waves per SIMD asked of the register allocator, for kernels whose
// natural allocation lands just above a step: FP32 KMV4 triangles and KMV2
// tetrahedra forward 4 (at most 128 VGPRs), so that four workgroups fit per CU
// when many are queued (several shots); FP64 KMV4 triangles forward and FP32 KMV4
// triangles adjoint (with its staged accumulators) 3 (at most 168 VGPRs).
// The PML instances run on the patches of the absorbing layer only and take no
// cap: their extra fields would spill under it.  Every instance is built for
// workgroups of at most 256 threads (patches of at most 256 cells), so one wave
// per SIMD is a legal occupancy: what does not fit in the 256 architectural VGPRs
// (the PML instances, the FP64 KMV5-triangle and KMV3-tetrahedron adjoints) is kept
// in AGPRs rather than in scratch memory.
template <typename T, int DIM, int ND, bool ADJ, bool PML = false>
struct StepWaves {
  static constexpr int kMin =
      PML ? 1
      : ADJ ? (sizeof(T) == 4 && DIM == 2 && ND == 18 ? 3 : 1)
            : sizeof(T) == 4 ? ((DIM == 2 && ND == 18) || (DIM == 3 && ND == 15) ? 4 : 1)
                             : (DIM == 2 && ND == 18 ? 3 : 1);
};

template <typename T, int DIM, int ND, bool ADJ, bool PML = false, bool NT = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(StepWaves<T, DIM, ND, ADJ, PML>::kMin)))
k_step(const StepArgs<T> A0) {
  static_assert(!PML || DIM == 2, "the PML instances are 2D");
  // XCD-aware work order: the dispatcher deals workgroups round-robin over the 8
  // XCDs (separate L2 caches), so workgroup b runs on XCD b % 8.  Each XCD gets a
  // contiguous run of work items, patch-major: neighbouring patches, which
  // exchange shared-DOF partials and read each other's levels, and the shots of
  // one patch, which read the same mesh tables and coefficients, mostly share one
  // L2.
  int p, shot;
  {
    const int b = blockIdx.x, nw = gridDim.x, x = b & 7, k = b >> 3;
    const int base = nw >> 3, rem = nw & 7;
    const int i = x * base + min(x, rem) + k;
    const int ns = A0.n_shots;
    p = ns == 1 ? i : i / ns;
    shot = i - p * ns;
    if (A0.patch_list != nullptr) p = A0.patch_list[p];
  }
  StepArgs<T> A = A0;
  if (shot != 0) {
    A.u_in += shot * A.ss_level;
    A.u_in_sh += shot * A.ss_level;
    A.u_prev += shot * A.ss_level;
    A.u_out += shot * A.ss_level;
    A.du += shot * A.ss_dof;
    A.dsh_prev += shot * A.ss_ref;
    A.dsh_cur += shot * A.ss_ref;
    A.part_prev += shot * A.ss_ref;
    A.part_cur += shot * A.ss_ref;
    if (A.amp != nullptr) A.amp += shot * A.ss_amp;
    if (A.trace_row != nullptr) A.trace_row += shot * A.ss_trace;
    if (A.inj_ptr != nullptr) A.inj_ptr += shot * A.ss_inj;
    if (ADJ) {
      A.uf += shot * A.ss_level;
      A.partr_prev += shot * A.ss_ref;
      A.partr_cur += shot * A.ss_ref;
      A.gacc += shot * A.ss_dof;
    }
    if (PML) {
      A.pp_in += shot * A.ss_pml;
      A.pp_in_sh += shot * A.ss_pml;
      A.pp_io += shot * A.ss_pml;
      A.pt_prev += shot * A.ss_pt;
      A.pt_cur += shot * A.ss_pt;
    }
  }
  using Tab = KmvTab<T, DIM, ND>;  // compile-time reference gradients, weights, node classes
  constexpr int NI = Tab::NI, NB = Tab::NB;
  constexpr int NIa = NI > 0 ? NI : 1, NBa = NB > 0 ? NB : 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int LB = A.nbl_max, CS = A.slot_stride;
  constexpr bool OVL = DIM == 3;  // slots overlay the c^2 [and u^m] staging
  constexpr bool GST = kStageGrad<T, ADJ, DIM, ND>;
  const StepLds lay(LB, CS, NB, A.glist_max, ADJ, sizeof(T), OVL, GST, PML);
  T* su = reinterpret_cast<T*>(smem_raw);  // level n of the non-interior DOFs
  T* sc = su + LB;                         // c^2
  T* sf = sc + LB;                         // forward state u^m (ADJ)
  T* sx = reinterpret_cast<T*>(smem_raw + lay.sx);  // K u - b per cell node
  T* sr = sx + (NB * CS + 1);                       // gradient pairing per cell node (ADJ)
  uint16_t* gl = reinterpret_cast<uint16_t*>(smem_raw + lay.gl);
  double* sg = reinterpret_cast<double*>(smem_raw + lay.sg);  // GST: owned accumulators
  // PML: auxiliary level (p^n, or mu^{m+1} in the adjoint) and sigma_x, sigma_z of the
  // non-interior DOFs; t slots per cell node
  T* sPx = reinterpret_cast<T*>(smem_raw + lay.sp);
  T* sPz = sPx + LB;
  T* sSx = sPz + LB;
  T* sSz = sSx + LB;
  T* sQx = sSz + LB;  // owned: the auxiliary level n-1 (adjoint: m+2), gamma, beta
  T* sQz = sQx + LB;
  T* sG = sQz + LB;
  T* sB = sG + LB;
  T* stx = reinterpret_cast<T*>(smem_raw + lay.st);
  T* stz = stx + (NB * CS + 1);
  const int tid = threadIdx.x, bs = blockDim.x;
  const int c0 = A.cell_start[p], nc = A.cell_start[p + 1] - c0;
  const int own0 = A.own_start[p], bo0 = own0 + NI * nc, nbo = A.own_start[p + 1] - bo0;
  const int sh0 = A.sh_start[p], nsh = A.sh_start[p + 1] - sh0;
  const int nbl = nbo + nsh;
  const bool step = A.mode == 0;

  // ---- every global load first, as one straight run: indices of idle lanes are
  // clamped into range instead of branched on (their values are never used), so
  // nothing forces a wait until the loads are all in flight.  What a shared ref
  // needs to finish its DOF is stored at the ref's own index (the level's copy, the
  // increment, c^2, gamma, beta), except the other patches' partial sums, whose
  // slots are loaded here and which are read after the bulk loads.
  constexpr int KH = Batch<T, ADJ, ND, DIM>::kShared;
  const int64_t N = A.n_dofs;
  const bool damped = A.beta != nullptr && A.damp_patch[p] != 0;
  const T* bsrc = damped ? A.beta : A.c2;          // undamped: a valid array already being read
  const T* bref = damped ? A.beta_ref : A.c2_ref;
  // shared-ref copies of level n-1 (or of level n without a previous level); the
  // apply mode's input has no copies and points u_prev at any level vector
  const T* uref = (step && !A.prev ? A.u_in : A.u_prev) + N;
  int jc[KH], gg[KH];
  int2 sl[KH];
  T up[KH], dp[KH], gm[KH], bt[KH], cc[KH], ff[KH];
#pragma unroll
  for (int t = 0; t < KH; ++t) {
    jc[t] = sh0 + min(tid + t * bs, max(nsh - 1, 0));  // padded: always in range
    gg[t] = A.sh_idx[jc[t]];
    sl[t] = reinterpret_cast<const int2*>(A.ref_slots)[jc[t]];
    cc[t] = A.c2_ref[jc[t]];
    if (ADJ) ff[t] = ld_once<T, DIM, NT>(A.uf + N + jc[t]);
    up[t] = ld_once<T, DIM, NT>(uref + jc[t]);
    dp[t] = ld_once<T, DIM, NT>(A.dsh_prev + jc[t]);
    gm[t] = A.gamma_ref[jc[t]];
    bt[t] = bref[jc[t]];
  }
  // gather lists of the DOFs with more than two contributions
  constexpr int KL = Batch<T>::kList;
  const int glo = A.glist_off[p], gln = (A.glist_off[p + 1] - glo) / 8;
  const uint4* glsrc = reinterpret_cast<const uint4*>(A.glist + glo);
  uint4 lw[KL];
#pragma unroll
  for (int k = 0; k < KL; ++k) lw[k] = glsrc[min(tid + k * bs, max(gln - 1, 0))];
  // cell data and the cell's interior DOFs
  const int tc = min(tid, nc - 1);
  const int e = c0 + tc;
  const bool active = tid < nc;
  constexpr int NG = DIM == 2 ? 3 : 6;
  constexpr int NB2 = (NB + 1) / 2;
  uint32_t mp[NB2 > 0 ? NB2 : 1];
  T G[NG];
#pragma unroll
  for (int q = 0; q < NB2; ++q) mp[q] = A.lmap[(int64_t)q * A.n_cells + e];
#pragma unroll
  for (int k = 0; k < NG; ++k) G[k] = A.geom[(int64_t)k * A.n_cells + e];
  const T gdet = A.gdet[e];  // dt^2 / |det J_e|: interior DOF i has M_i = w_a |det J_e|
  T ui[NIa], ci[NIa], di[NIa], gi[NIa], bi[NIa], fi[ADJ ? NIa : 1];
  double ga[ADJ ? NIa : 1];  // gradient accumulator of the interior DOFs (read early)
#pragma unroll
  for (int j = 0; j < NI; ++j) {
    const int gx = own0 + j * nc + tc;
    ui[j] = ld_once<T, DIM, NT>(A.u_in + gx);
    ci[j] = A.c2[gx];
    di[j] = ld_once<T, DIM, NT>(A.du + gx);
    bi[j] = bsrc[gx];
    if (ADJ) {
      fi[ADJ ? j : 0] = ld_once<T, DIM, NT>(A.uf + gx);
      ga[ADJ ? j : 0] = ld_once<T, DIM, NT>(A.gacc + gx);
    }
  }
  // gather words of the first local DOFs of this thread
  constexpr int KW = Batch<T>::kWords;
  const uint32_t* gwp = A.gword + A.gword_off[p];
  uint32_t gw[KW];
#pragma unroll
  for (int k = 0; k < KW; ++k) gw[k] = gwp[min(tid + k * bs, nbl - 1)];
  // owned non-interior DOFs: level, c^2 [, u^m] and the update operands
  constexpr int KO = Batch<T, ADJ, ND>::kOwned;
  T vu[KO], vc[KO], vf[ADJ ? KO : 1], pdu[KO], pg[KO], pb[KO];
  double pga[GST ? KO : 1];  // their gradient accumulators (staged in LDS below)
#pragma unroll
  for (int k = 0; k < KO; ++k) {
    const int gx = max(bo0 + min(tid + k * bs, nbo - 1), 0);
    vu[k] = ld_once<T, DIM, NT>(A.u_in + gx);
    vc[k] = A.c2[gx];
    if (ADJ) vf[ADJ ? k : 0] = ld_once<T, DIM, NT>(A.uf + gx);
    if (GST) pga[GST ? k : 0] = ld_once<T, DIM, NT>(A.gacc + gx);
    pdu[k] = ld_once<T, DIM, NT>(A.du + gx);
    pg[k] = A.gamma[gx];
    pb[k] = bsrc[gx];
  }
  // partial sums of the shared refs' DOFs, at the slots loaded first.  The empty
  // asm (no instruction) takes the slots as operands: the compiler cannot start
  // the address arithmetic before it nor move the loads above across it, so every
  // load above is in flight before these are issued, and waiting for the slots
  // costs nothing by then.
  // (adjoint: also the gradient accumulators of the refs' DOFs, which the first
  // touching patch updates while finishing them)
  T y0[KH], y1[KH], q0[ADJ ? KH : 1], q1[ADJ ? KH : 1];
  double gs[ADJ ? KH : 1];
#pragma unroll
  for (int t = 0; t < KH; ++t) {
    int sx = sl[t].x, sy = sl[t].y;
    asm volatile("" : "+v"(sx), "+v"(sy)::"memory");
    const int sy2 = sy >= 0 ? sy : sx;
    y0[t] = A.part_prev[sx];
    y1[t] = A.part_prev[sy2];
    if (ADJ) {
      q0[ADJ ? t : 0] = A.partr_prev[sx];
      q1[ADJ ? t : 0] = A.partr_prev[sy2];
      gs[ADJ ? t : 0] = ld_once<T, DIM, NT>(A.gacc + gg[t]);
    }
  }
  if (!damped) {
#pragma unroll
    for (int j = 0; j < NI; ++j) bi[j] = T(1);
#pragma unroll
    for (int k = 0; k < KO; ++k) pb[k] = T(1);
  }
  // interior gamma = dt^2 / (w_a |det J_e| (1+a)), with 1/(1+a) = (1+beta)/2
#pragma unroll
  for (int a = 0; a < ND; ++a) {
    if (!Tab::INT[a]) continue;
    const int j = Tab::IDX[a] < NI ? Tab::IDX[a] : 0;
    gi[j] = gdet * (T(1) / Tab::W[a]);
    if (damped) gi[j] = gi[j] * ((T(1) + bi[j]) * T(0.5));
  }
  int m[NBa];
#pragma unroll
  for (int b = 0; b < NB; ++b) m[b] = (int)((mp[b / 2] >> (16 * (b & 1))) & 0xFFFFu);

  // shared refs: finish the level from the previous step's partials
  if (!step) {  // apply mode: the input is a plain vector, read by global id
#pragma unroll
    for (int t = 0; t < KH; ++t) up[t] = A.u_in[gg[t]];
  }
  T uu[KH];
#pragma unroll
  for (int t = 0; t < KH; ++t) {
    uu[t] = up[t];
    const int j = tid + t * bs;
    if (!(step && A.prev) || j >= nsh) continue;
    const int r = jc[t], g = gg[t];
    const int64_t s = g - A.n_own;
    const bool pair = sl[t].y >= 0;  // else: three or more patches, CSR list
    T y = y0[t] + y1[t];
    if (!pair) {
      y = T(0);
      for (int k = A.shp_ptr[s]; k < A.shp_ptr[s + 1]; ++k) y += A.part_prev[A.shp_slot[k]];
    }
    const T dn = (damped ? bt[t] : T(1)) * dp[t] - gm[t] * y;
    uu[t] = up[t] + dn;
    st_once<T, DIM, NT>(uu[t], A.u_in_sh + N + r);  // every ref keeps its copy of the finished level
    st_once<T, DIM, NT>(dn, A.dsh_cur + r);
    if (sl[t].x == r) {  // the first touching patch stores the level itself
      A.u_in_sh[g] = uu[t];
      if (ADJ && A.pair_prev) {
        T rr = q0[ADJ ? t : 0] + q1[ADJ ? t : 0];
        if (!pair) {
          rr = T(0);
          for (int k = A.shp_ptr[s]; k < A.shp_ptr[s + 1]; ++k) rr += A.partr_prev[A.shp_slot[k]];
        }
        st_once<T, DIM, NT>(gs[ADJ ? t : 0] + (double)rr, A.gacc + g);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < KH; ++t) {
    const int j = tid + t * bs;
    if (j >= nsh) continue;
    su[nbo + j] = uu[t];
    sc[nbo + j] = cc[t];
    if (ADJ) sf[nbo + j] = ff[t];
  }
  // remaining shared refs (patches with more than KH * bs of them), two per pass
  // with every load of a pass issued before any is used
  for (int j0 = tid + KH * bs; j0 < nsh; j0 += 2 * bs) {
    int r2[2], g2[2];
    int2 s2[2];
    T u2[2], c2v[2], f2[2], d2[2], gm2[2], b2[2], p0[2], p1[2], pr0[2], pr1[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      r2[t] = sh0 + min(j0 + t * bs, nsh - 1);
      g2[t] = A.sh_idx[r2[t]];
      s2[t] = reinterpret_cast<const int2*>(A.ref_slots)[r2[t]];
      u2[t] = ld_once<T, DIM, NT>(uref + r2[t]);
      c2v[t] = A.c2_ref[r2[t]];
      if (ADJ) f2[t] = ld_once<T, DIM, NT>(A.uf + N + r2[t]);
      d2[t] = ld_once<T, DIM, NT>(A.dsh_prev + r2[t]);
      gm2[t] = A.gamma_ref[r2[t]];
      b2[t] = bref[r2[t]];
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int sy = s2[t].y >= 0 ? s2[t].y : s2[t].x;
      p0[t] = A.part_prev[s2[t].x];
      p1[t] = A.part_prev[sy];
      if (ADJ) {
        pr0[t] = A.partr_prev[s2[t].x];
        pr1[t] = A.partr_prev[sy];
      }
      if (!step) u2[t] = A.u_in[g2[t]];
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int j = j0 + t * bs;
      if (j >= nsh) continue;
      const int r = r2[t], g = g2[t];
      const int64_t s = g - A.n_own;
      const int2 sj = s2[t];
      const bool pair = sj.y >= 0;
      T u = u2[t];
      if (step && A.prev) {
        T y = p0[t] + p1[t];
        if (!pair) {
          y = T(0);
          for (int k = A.shp_ptr[s]; k < A.shp_ptr[s + 1]; ++k) y += A.part_prev[A.shp_slot[k]];
        }
        const T dn = (damped ? b2[t] : T(1)) * d2[t] - gm2[t] * y;
        u = u + dn;
        st_once<T, DIM, NT>(u, A.u_in_sh + N + r);
        st_once<T, DIM, NT>(dn, A.dsh_cur + r);
        if (sj.x == r) {
          A.u_in_sh[g] = u;
          if (ADJ && A.pair_prev) {
            T rr = pr0[t] + pr1[t];
            if (!pair) {
              rr = T(0);
              for (int k = A.shp_ptr[s]; k < A.shp_ptr[s + 1]; ++k) rr += A.partr_prev[A.shp_slot[k]];
            }
            A.gacc[g] += (double)rr;
          }
        }
      }
      su[nbo + j] = u;
      sc[nbo + j] = c2v[t];
      if (ADJ) sf[nbo + j] = f2[t];
    }
  }
  {
    uint4* gldst = reinterpret_cast<uint4*>(gl);
#pragma unroll
    for (int k = 0; k < KL; ++k) {
      const int v = tid + k * bs;
      if (v < gln) gldst[v] = lw[k];
    }
    for (int v = tid + KL * bs; v < gln; v += bs) gldst[v] = glsrc[v];
  }
  // ---- the staged stores
#pragma unroll
  for (int k = 0; k < KO; ++k) {
    const int i = tid + k * bs;
    if (i < nbo) {
      su[i] = vu[k];
      sc[i] = vc[k];
      if (ADJ) sf[i] = vf[ADJ ? k : 0];
      if (GST) sg[i] = pga[GST ? k : 0];
    }
  }
  for (int i = tid + KO * bs; i < nbo; i += bs) {
    su[i] = A.u_in[bo0 + i];
    sc[i] = A.c2[bo0 + i];
    if (ADJ) sf[i] = ld_once<T, DIM, NT>(A.uf + bo0 + i);
    if (GST) sg[i] = A.gacc[bo0 + i];
  }
  if (!OVL && tid == 0) {
    sx[NB * CS] = T(0);
    if (ADJ) sr[NB * CS] = T(0);
  }
  // ---- PML: the auxiliary level and the damping functions.  Forward: p^n, whose
  // shared DOFs are finished here (lagged, as u) from p^{n-2} at their ref copies and
  // the previous step's partial sums T of D_k u^{n-1}:
  //   (1 + b_k) p_k^n = (1 - b_k) p_k^{n-2} - (2 dt / M) c^2 Psi_2^kk T_k,
  // b_k = sigma_k dt, Psi_2^xx = sigma_x - sigma_z = -Psi_2^zz.  Adjoint (pml_trans,
  // with or without the gradient pairing): mu^{m+1} from mu^{m+3} and the partial
  // sums of D_k lambda^{m+2}, without the c^2 Psi_2 factor (it sits in the u row
  // there).  2 dt / M = 4 gamma / (dt (1 + beta)).
  T piX[NIa], piZ[NIa], Bm[4];
  if constexpr (PML) {
    const T* pin = A.pp_in;
    const int64_t ls = A.pml_ls, rs = A.pml_rs;
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      const int gx = own0 + j * nc + tc;
      piX[j] = pin[gx];
      piZ[j] = pin[ls + gx];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) Bm[k] = A.pml_b[(int64_t)k * A.n_cells + e];
    // owned non-interior DOFs, two per pass with every load issued first
    for (int i0 = tid; i0 < nbo; i0 += 2 * bs) {
      T v[2][8];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int gx = bo0 + min(i0 + k * bs, nbo - 1);
        v[k][0] = pin[gx];
        v[k][1] = pin[ls + gx];
        v[k][2] = A.sig[gx];
        v[k][3] = A.sig[N + gx];
        v[k][4] = A.pp_io[gx];
        v[k][5] = A.pp_io[ls + gx];
        v[k][6] = A.gamma[gx];
        v[k][7] = A.beta[gx];
      }
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int i = i0 + k * bs;
        if (i >= nbo) continue;
        sPx[i] = v[k][0];
        sPz[i] = v[k][1];
        sSx[i] = v[k][2];
        sSz[i] = v[k][3];
        sQx[i] = v[k][4];
        sQz[i] = v[k][5];
        sG[i] = v[k][6];
        sB[i] = v[k][7];
      }
    }
    // shared refs, two per pass: their copies, then the partial sums at their slots
    const int64_t nref = A.pml_rs;
    for (int j0 = tid; j0 < nsh; j0 += 2 * bs) {
      int r2[2];
      int2 sj[2];
      T px[2], pz[2], sxr[2], szr[2], c2r[2], gr[2], br[2], ta[2], tb[2], tc_[2], td[2];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int r = sh0 + min(j0 + k * bs, nsh - 1);
        r2[k] = r;
        px[k] = pin[N + r];
        pz[k] = pin[ls + N + r];
        sxr[k] = A.sig_ref[r];
        szr[k] = A.sig_ref[nref + r];
        sj[k] = reinterpret_cast<const int2*>(A.ref_slots)[r];
        c2r[k] = A.c2_ref[r];
        gr[k] = A.gamma_ref[r];
        br[k] = A.beta_ref[r];
      }
      if (step && A.prev) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const int sy = sj[k].y >= 0 ? sj[k].y : sj[k].x;
          ta[k] = A.pt_prev[sj[k].x];
          tb[k] = A.pt_prev[sy];
          tc_[k] = A.pt_prev[rs + sj[k].x];
          td[k] = A.pt_prev[rs + sy];
        }
      }
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int j = j0 + k * bs;
        if (j >= nsh) continue;
        const int r = r2[k];
        if (step && A.prev) {
          T tx = ta[k] + tb[k], tz = tc_[k] + td[k];
          if (sj[k].y < 0) {  // three or more patches: the CSR list, in patch order
            const int64_t sd = A.sh_idx[r] - A.n_own;
            tx = T(0);
            tz = T(0);
            for (int q = A.shp_ptr[sd]; q < A.shp_ptr[sd + 1]; ++q) {
              tx += A.pt_prev[A.shp_slot[q]];
              tz += A.pt_prev[rs + A.shp_slot[q]];
            }
          }
          const T m2 = T(4) * gr[k] * A.inv_dt / (T(1) + br[k]);
          if (!A.pml_trans) {
            const T cd = c2r[k] * (sxr[k] - szr[k]);
            tx = cd * tx;
            tz = -cd * tz;
          }
          const T bx = sxr[k] * A.pml_dt, bz = szr[k] * A.pml_dt;
          px[k] = ((T(1) - bx) * px[k] - m2 * tx) / (T(1) + bx);
          pz[k] = ((T(1) - bz) * pz[k] - m2 * tz) / (T(1) + bz);
          A.pp_in_sh[N + r] = px[k];
          A.pp_in_sh[ls + N + r] = pz[k];
        }
        sPx[nbo + j] = px[k];
        sPz[nbo + j] = pz[k];
        sSx[nbo + j] = sxr[k];
        sSz[nbo + j] = szr[k];
      }
    }
    if (tid == 0) {
      stx[NB * CS] = T(0);
      stz[NB * CS] = T(0);
    }
  }
  __syncthreads();

  // ---- per cell: receivers, element stiffness (and pairing), sources, interior DOFs
  T ue[ND], ce[ND], fe[ADJ ? ND : 1], ye[ND], re[ADJ ? ND : 1];
  if (active) {
#pragma unroll
    for (int a = 0; a < ND; ++a) {
      const int x = Tab::IDX[a];
      if (Tab::INT[a]) {
        ue[a] = ui[x < NI ? x : 0];
        ce[a] = ci[x < NI ? x : 0];
        if (ADJ) fe[ADJ ? a : 0] = fi[ADJ && x < NI ? x : 0];
      } else {
        const int l = m[x < NB ? x : 0];
        ue[a] = su[l];
        ce[a] = sc[l];
        if (ADJ) fe[ADJ ? a : 0] = sf[l];
      }
      ye[a] = T(0);
    }
  }
  if constexpr (OVL) {
    __syncthreads();  // the staged c^2 [and u^m] have been read: the slots may overwrite them
    if (tid == 0) {
      sx[NB * CS] = T(0);
      if (ADJ) sr[NB * CS] = T(0);
    }
  }
  if (active) {
    if (A.trace_row != nullptr) {
      for (int r = A.rec_ptr[p]; r < A.rec_ptr[p + 1]; ++r)
        if (A.rec_cell[r] == tid) {
          T s = T(0);
#pragma unroll
          for (int a = 0; a < ND; ++a) s += A.rec_w[(int64_t)r * ND + a] * ue[a];
          A.trace_row[A.rec_pt[r]] = s;
        }
    }
    T tiX[NIa], tiZ[NIa];  // PML: t at the interior nodes
    const T absJ = PML ? (T)fabs(Bm[0] * Bm[3] - Bm[1] * Bm[2]) : T(0);  // |det B_e| = |det J_e|
#pragma unroll
    for (int q = 0; q < ND; ++q) {
      T g[DIM];
#pragma unroll
      for (int r = 0; r < DIM; ++r) g[r] = T(0);
#pragma unroll
      for (int b = 0; b < ND; ++b)
#pragma unroll
        for (int r = 0; r < DIM; ++r) {
          const T dv = Tab::D[(q * ND + b) * DIM + r];
          if (dv != T(0)) g[r] += dv * ue[b];
        }
      T v[DIM];
      if constexpr (DIM == 2) {
        v[0] = G[0] * g[0] + G[1] * g[1];
        v[1] = G[1] * g[0] + G[2] * g[1];
      } else {
        v[0] = G[0] * g[0] + G[1] * g[1] + G[2] * g[2];
        v[1] = G[1] * g[0] + G[3] * g[1] + G[4] * g[2];
        v[2] = G[2] * g[0] + G[4] * g[1] + G[5] * g[2];
      }
      const T wq = Tab::W[q];
      const T cw = wq * ce[q];
      T z[DIM];
#pragma unroll
      for (int r = 0; r < DIM; ++r) z[r] = cw * v[r];
      // PML at node q: the u row's coupling sum_k D_k^T p_k (forward) or
      // sum_k D_k^T c^2 Psi_2^kk mu_k (adjoint) enters z as w_q B_e^T (.)_q; t_q =
      // w_q B_e ghat_q is node q's share of D_k u (of the level being stepped); and
      // the zeroth-order term M sigma_x sigma_z u enters the element vector
      T pxq = T(0), pzq = T(0), sxq = T(0), szq = T(0);
      if constexpr (PML) {
        const int x = Tab::IDX[q];
        if (Tab::INT[q]) {
          const int j = x < NI ? x : 0;
          pxq = piX[j];
          pzq = piZ[j];
          const int gx = own0 + j * nc + tid;
          sxq = A.sig[gx];
          szq = A.sig[N + gx];
        } else {
          const int l = m[x < NB ? x : 0];
          pxq = sPx[l];
          pzq = sPz[l];
          sxq = sSx[l];
          szq = sSz[l];
        }
        T qx = pxq, qz = pzq;
        if (A.pml_trans) {
          qx = ce[q] * (sxq - szq) * pxq;
          qz = ce[q] * (szq - sxq) * pzq;
        }
        z[0] += wq * (Bm[0] * qx + Bm[2] * qz);
        z[1] += wq * (Bm[1] * qx + Bm[3] * qz);
        const T tx = wq * (Bm[0] * g[0] + Bm[1] * g[1]), tz = wq * (Bm[2] * g[0] + Bm[3] * g[1]);
        if (Tab::INT[q]) {
          tiX[x < NI ? x : 0] = tx;
          tiZ[x < NI ? x : 0] = tz;
        } else {
          stx[x * CS + tid] = tx;
          stz[x * CS + tid] = tz;
        }
        ye[q] += wq * absJ * (sxq * szq) * ue[q];
      }
#pragma unroll
      for (int b = 0; b < ND; ++b)
#pragma unroll
        for (int r = 0; r < DIM; ++r) {
          const T dv = Tab::D[(q * ND + b) * DIM + r];
          if (dv != T(0)) ye[b] += dv * z[r];
        }
      if (ADJ) {
        T gf[DIM];
#pragma unroll
        for (int r = 0; r < DIM; ++r) gf[r] = T(0);
#pragma unroll
        for (int b = 0; b < ND; ++b)
#pragma unroll
          for (int r = 0; r < DIM; ++r) {
            const T dv = Tab::D[(q * ND + b) * DIM + r];
            if (dv != T(0)) gf[r] += dv * fe[ADJ ? b : 0];
          }
        T s = T(0);
#pragma unroll
        for (int r = 0; r < DIM; ++r) s += gf[r] * v[r];
        re[ADJ ? q : 0] = wq * s;
        if constexpr (PML) {  // gradient's PML term: sum_k Psi_2^kk mu_k (D_k u^m) at node q
          const T tfx = wq * (Bm[0] * gf[0] + Bm[1] * gf[1]), tfz = wq * (Bm[2] * gf[0] + Bm[3] * gf[1]);
          re[ADJ ? q : 0] += (sxq - szq) * (pxq * tfx - pzq * tfz);
        }
      }
    }
    // point sources in this cell: b enters the element vector as K u - b
    if (A.inj_ptr != nullptr) {
      for (int r = A.inj_ptr[p]; r < A.inj_ptr[p + 1]; ++r)
        if (A.inj_cell[r] == tid) {
          const T f = A.amp[(int64_t)A.inj_pt[r] * A.amp_stride] * A.amp_scale;
#pragma unroll
          for (int a = 0; a < ND; ++a) ye[a] -= f * A.inj_w[(int64_t)r * ND + a];
        }
    }
    // interior DOFs are complete: finish them here
#pragma unroll
    for (int a = 0; a < ND; ++a) {
      if (!Tab::INT[a]) continue;
      const int j = Tab::IDX[a] < NI ? Tab::IDX[a] : 0;
      const int gx = own0 + j * nc + tid;
      if (step) {
        const T dn = bi[j] * di[j] - gi[j] * ye[a];
        st_once<T, DIM, NT>(dn, A.du + gx);
        st_once<T, DIM, NT>(ui[j] + dn, A.u_out + gx);
        if (ADJ) st_once<T, DIM, NT>(ga[ADJ ? j : 0] + (double)re[ADJ ? a : 0], A.gacc + gx);
        if constexpr (PML) {  // the auxiliary level n+1 (adjoint: m) of the interior DOF
          const T sxj = A.sig[gx], szj = A.sig[N + gx];
          const T pmx = A.pp_io[gx], pmz = A.pp_io[A.pml_ls + gx];
          const T m2 = T(2) * A.pml_dt / (Tab::W[a] * absJ);
          T tx = tiX[j], tz = tiZ[j];
          if (!A.pml_trans) {
            const T cd = ce[a] * (sxj - szj);
            tx = cd * tx;
            tz = -cd * tz;
          }
          const T bx = sxj * A.pml_dt, bz = szj * A.pml_dt;
          A.pp_io[gx] = ((T(1) - bx) * pmx - m2 * tx) / (T(1) + bx);
          A.pp_io[A.pml_ls + gx] = ((T(1) - bz) * pmz - m2 * tz) / (T(1) + bz);
        }
      } else {
        A.y_out[gx] = ye[a];
      }
    }
#pragma unroll
    for (int a = 0; a < ND; ++a) {
      if (Tab::INT[a]) continue;
      const int b = Tab::IDX[a];
      sx[b * CS + tid] = ye[a];
      if (ADJ) sr[b * CS + tid] = re[ADJ ? a : 0];
    }
  }
  __syncthreads();

  // partial sums of the shared DOFs, at this ref's slot
  auto produce = [&](int j, T y, T r) {
    st_once<T, DIM, NT>(y, A.part_cur + sh0 + j);
    if (ADJ) st_once<T, DIM, NT>(r, A.partr_cur + sh0 + j);
  };
  // ---- non-interior DOFs: fixed-order sums of their slots
#pragma unroll
  for (int k = 0; k < KW; ++k) {
    const int l = tid + k * bs;
    if (l >= nbl) continue;
    const T y = gather_sum(gw[k], sx, gl);
    const T r = ADJ ? gather_sum(gw[k], sr, gl) : T(0);
    if (l < nbo) {
      const int gx = bo0 + l;
      if (!step) {
        A.y_out[gx] = y;
      } else {
        T dn, un;
        if (k < KO) {
          const int kk = k < KO ? k : 0;
          dn = pb[kk] * pdu[kk] - pg[kk] * y;
          un = vu[kk];
        } else {
          dn = (damped ? A.beta[gx] : T(1)) * A.du[gx] - A.gamma[gx] * y;
          un = su[l];
        }
        st_once<T, DIM, NT>(dn, A.du + gx);
        st_once<T, DIM, NT>(un + dn, A.u_out + gx);
        if (GST)
          st_once<T, DIM, NT>(sg[l] + (double)r, A.gacc + gx);  // staged: no dependent load here
        else if (ADJ)
          A.gacc[gx] += (double)r;
      }
    } else {
      produce(l - nbo, y, r);
    }
  }
  for (int l = tid + KW * bs; l < nbl; l += bs) {
    const uint32_t w = gwp[l];
    const T y = gather_sum(w, sx, gl);
    const T r = ADJ ? gather_sum(w, sr, gl) : T(0);
    if (l < nbo) {
      const int gx = bo0 + l;
      if (!step) {
        A.y_out[gx] = y;
      } else {
        const T dn = (damped ? A.beta[gx] : T(1)) * A.du[gx] - A.gamma[gx] * y;
        st_once<T, DIM, NT>(dn, A.du + gx);
        st_once<T, DIM, NT>(su[l] + dn, A.u_out + gx);
        if (GST)
          st_once<T, DIM, NT>(sg[l] + (double)r, A.gacc + gx);
        else if (ADJ)
          A.gacc[gx] += (double)r;
      }
    } else {
      produce(l - nbo, y, r);
    }
  }
  // ---- PML: t summed per non-interior DOF in the same fixed slot order; owned DOFs
  // take their auxiliary level n+1 (adjoint: m), shared ones write this patch's
  // partial sums
  if constexpr (PML) {
    const int64_t ls = A.pml_ls, rs = A.pml_rs;
    for (int l = tid; l < nbl; l += bs) {
      const uint32_t w = gwp[l];
      T tx = gather_sum(w, stx, gl), tz = gather_sum(w, stz, gl);
      if (l < nbo) {
        const int gx = bo0 + l;
        const T sxl = sSx[l], szl = sSz[l];
        const T m2 = T(4) * sG[l] * A.inv_dt / (T(1) + sB[l]);
        if (!A.pml_trans) {
          const T cd = sc[l] * (sxl - szl);
          tx = cd * tx;
          tz = -cd * tz;
        }
        const T bx = sxl * A.pml_dt, bz = szl * A.pml_dt;
        A.pp_io[gx] = ((T(1) - bx) * sQx[l] - m2 * tx) / (T(1) + bx);
        A.pp_io[ls + gx] = ((T(1) - bz) * sQz[l] - m2 * tz) / (T(1) + bz);
      } else {
        A.pt_cur[sh0 + (l - nbo)] = tx;
        A.pt_cur[rs + sh0 + (l - nbo)] = tz;
      }
    }
  }
}

template <typename T, bool ADJ>
__global__ void __launch_bounds__(256) k_finish(const FinishArgs<T> A0) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= A0.n_shared) return;
  FinishArgs<T> A = A0;
  const int shot = blockIdx.y;
  if (shot != 0) {
    A.part_prev += shot * A.ss_ref;
    A.u_prev += shot * A.ss_level;
    A.u_cur += shot * A.ss_level;
    A.dsh_prev += shot * A.ss_ref;
    A.dsh_cur += shot * A.ss_ref;
    if (ADJ) {
      A.partr_prev += shot * A.ss_ref;
      A.gacc += shot * A.ss_dof;
    }
  }
  const int64_t g = A.n_own + s;
  const int k0 = A.shp_ptr[s], k1 = A.shp_ptr[s + 1];
  if (ADJ && A.mode == 2) {  // pairing partials only
    T rr = A.partr_prev[A.shp_slot[k0]];
    for (int k = k0 + 1; k < k1; ++k) rr += A.partr_prev[A.shp_slot[k]];
    A.gacc[g] += (double)rr;
    return;
  }
  // the same fixed order as the step kernel (two patches: first + second)
  T y = A.part_prev[A.shp_slot[k0]];
  for (int k = k0 + 1; k < k1; ++k) y += A.part_prev[A.shp_slot[k]];
  if (A.mode == 1) {
    A.y_out[g] = y;
    return;
  }
  const int64_t r0 = A.shp_slot[k0];
  const T b = A.beta ? A.beta[g] : T(1);
  const T dn = b * A.dsh_prev[r0] - A.gamma[g] * y;
  const T u = A.u_prev[A.n_dofs + r0] + dn;
  A.u_cur[g] = u;
  for (int k = k0; k < k1; ++k) {  // every ref's copies
    const int64_t r = A.shp_slot[k];
    A.u_cur[A.n_dofs + r] = u;
    A.dsh_cur[r] = dn;
  }
  if (ADJ) {
    T rr = A.partr_prev[A.shp_slot[k0]];
    for (int k = k0 + 1; k < k1; ++k) rr += A.partr_prev[A.shp_slot[k]];
    A.gacc[g] += (double)rr;
  }
}

template <typename T>
__global__ void k_gather(const T* __restrict__ x, const int32_t* __restrict__ idx, T* __restrict__ out,
                         int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = x[idx[i]];
}

// One thread per (point, node) pair, then a fixed-order sum per point: the
// dependent index/value loads of a point are issued in parallel.
template <typename T>
__global__ void __launch_bounds__(256) k_sample(const T* __restrict__ u, const int32_t* __restrict__ dof,
                                                const T* __restrict__ w, int npts, int nd, T* __restrict__ out) {
  __shared__ T prod[256];
  const int per = 256 / nd;  // points per block
  const int j0 = blockIdx.x * per;
  const int t = threadIdx.x;
  const int jl = t / nd, a = t % nd;
  const int j = j0 + jl;
  T v = T(0);
  if (jl < per && j < npts) v = w[(int64_t)j * nd + a] * u[dof[(int64_t)j * nd + a]];
  prod[t] = v;
  __syncthreads();
  if (t < per && j0 + t < npts) {
    T s = T(0);
    for (int b = 0; b < nd; ++b) s += prod[t * nd + b];
    out[j0 + t] = s;
  }
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

__global__ void k_finalize_grad(const double* __restrict__ c, const double* __restrict__ gacc, int ns,
                                double scale, double* __restrict__ g, int64_t n, int accumulate) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a = gacc[i];
  for (int s = 1; s < ns; ++s) a += gacc[s * n + i];
  const double v = scale * c[i] * a;
  g[i] = accumulate ? g[i] + v : v;
}

// Sentinel for a solve that has left the floating-point range (an unstable step, or
// non-finite inputs): any NaN or infinity among the checked values raises the flag.
template <typename T>
__global__ void __launch_bounds__(256) k_check_finite(const T* __restrict__ x, int64_t n, int64_t stride,
                                                      int* __restrict__ flag) {
  const T* xv = x + (int64_t)blockIdx.y * stride;
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    bad |= !__builtin_isfinite(xv[i]);
  if (bad) *flag = 1;
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

// Launch with optional start/stop events recorded by the dispatch itself, so a
// sampled launch is timed without the event packets' own dispatch gaps.
template <typename K, typename... Args>
void launch_ev(K kernel, dim3 grid, dim3 block, uint32_t lds, hipStream_t s, hipEvent_t e0,
               hipEvent_t e1, Args... args) {
  if (e0)
    hipExtLaunchKernelGGL(kernel, grid, block, lds, s, e0, e1, 0u, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
}

template <typename T, int DIM, int ND, bool ADJ, bool PML = false>
hipError_t launch_step_t(const StepArgs<T>& a, int np, int block, hipStream_t s, hipEvent_t e0,
                         hipEvent_t e1) {
  const size_t lds = StepLds(a.nbl_max, a.slot_stride, KmvTab<T, DIM, ND>::NB, a.glist_max, ADJ, sizeof(T),
                             DIM == 3, kStageGrad<T, ADJ, DIM, ND>, PML)
                          .total;
  if constexpr (kStream<T, DIM>) {
    if (a.n_shots == 1) {  // the streaming-hint instance (see ld_once)
      launch_ev(k_step<T, DIM, ND, ADJ, PML, true>, dim3(np), dim3(block), (uint32_t)lds, s, e0, e1, a);
      return hipGetLastError();
    }
  }
  launch_ev(k_step<T, DIM, ND, ADJ, PML>, dim3(np * a.n_shots), dim3(block), (uint32_t)lds, s, e0, e1, a);
  return hipGetLastError();
}

template <typename T, int DIM, int ND, bool ADJ, bool PML = false>
hipError_t set_lds_t(int bytes) {
  if constexpr (kStream<T, DIM>) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_step<T, DIM, ND, ADJ, PML, true>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
  }
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_step<T, DIM, ND, ADJ, PML>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

#define KMV_DISPATCH(FN, ...)                                                                      \
  switch (dim * 100 + nd) {                                                                        \
    case 203: return adjoint ? FN<T, 2, 3, true>(__VA_ARGS__) : FN<T, 2, 3, false>(__VA_ARGS__);   \
    case 207: return adjoint ? FN<T, 2, 7, true>(__VA_ARGS__) : FN<T, 2, 7, false>(__VA_ARGS__);   \
    case 212: return adjoint ? FN<T, 2, 12, true>(__VA_ARGS__) : FN<T, 2, 12, false>(__VA_ARGS__); \
    case 218: return adjoint ? FN<T, 2, 18, true>(__VA_ARGS__) : FN<T, 2, 18, false>(__VA_ARGS__); \
    case 230: return adjoint ? FN<T, 2, 30, true>(__VA_ARGS__) : FN<T, 2, 30, false>(__VA_ARGS__); \
    case 304: return adjoint ? FN<T, 3, 4, true>(__VA_ARGS__) : FN<T, 3, 4, false>(__VA_ARGS__);   \
    case 315: return adjoint ? FN<T, 3, 15, true>(__VA_ARGS__) : FN<T, 3, 15, false>(__VA_ARGS__); \
    case 332: return adjoint ? FN<T, 3, 32, true>(__VA_ARGS__) : FN<T, 3, 32, false>(__VA_ARGS__); \
    default: return hipErrorInvalidValue;                                                          \
  }

// the PML instances (triangles)
#define KMV_DISPATCH_PML(FN, ...)                                                                              \
  switch (dim * 100 + nd) {                                                                                    \
    case 203: return adjoint ? FN<T, 2, 3, true, true>(__VA_ARGS__) : FN<T, 2, 3, false, true>(__VA_ARGS__);   \
    case 207: return adjoint ? FN<T, 2, 7, true, true>(__VA_ARGS__) : FN<T, 2, 7, false, true>(__VA_ARGS__);   \
    case 212: return adjoint ? FN<T, 2, 12, true, true>(__VA_ARGS__) : FN<T, 2, 12, false, true>(__VA_ARGS__); \
    case 218: return adjoint ? FN<T, 2, 18, true, true>(__VA_ARGS__) : FN<T, 2, 18, false, true>(__VA_ARGS__); \
    case 230: return adjoint ? FN<T, 2, 30, true, true>(__VA_ARGS__) : FN<T, 2, 30, false, true>(__VA_ARGS__); \
    default: return hipErrorInvalidValue;                                                                      \
  }
}  // namespace

size_t step_lds_bytes(int dim, int nd, int nbl_max, int slot_stride, int nb, int glist_max, bool adjoint,
                      size_t elem_size, bool pml) {
  const bool gst = stage_grad(adjoint, dim, nd, elem_size);
  return StepLds(nbl_max, slot_stride, nb, glist_max, adjoint, elem_size, dim == 3, gst, pml).total;
}

template <typename T>
hipError_t launch_step(int dim, int nd, bool adjoint, const StepArgs<T>& a, int n_items, int block,
                       hipStream_t s, hipEvent_t e0, hipEvent_t e1, bool pml) {
  if (n_items <= 0) return hipSuccess;
  if (pml) {
    KMV_DISPATCH_PML(launch_step_t, a, n_items, block, s, e0, e1)
  }
  KMV_DISPATCH(launch_step_t, a, n_items, block, s, e0, e1)
}

template <typename T>
hipError_t set_step_lds_limit(int dim, int nd, bool adjoint, int bytes, bool pml) {
  if (pml) {
    KMV_DISPATCH_PML(set_lds_t, bytes)
  }
  KMV_DISPATCH(set_lds_t, bytes)
}

template <typename T>
hipError_t launch_finish(bool adjoint, const FinishArgs<T>& a, hipStream_t s, hipEvent_t e0,
                         hipEvent_t e1) {
  if (a.n_shared == 0) return hipSuccess;
  const unsigned nb = blocks_for(a.n_shared, 256), ns = (unsigned)(a.n_shots > 0 ? a.n_shots : 1);
  if (adjoint)
    launch_ev(k_finish<T, true>, dim3(nb, ns), dim3(256), 0u, s, e0, e1, a);
  else
    launch_ev(k_finish<T, false>, dim3(nb, ns), dim3(256), 0u, s, e0, e1, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sample(const T* u, const int32_t* dof, const T* w, int npts, int nd, T* out,
                         hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (npts <= 0) return hipSuccess;
  if (nd > 256) return hipErrorInvalidValue;
  const int per = 256 / nd;
  launch_ev(k_sample<T>, dim3(blocks_for(npts, per)), dim3(256), 0u, s, e0, e1, u, dof, w, npts, nd,
            out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gather(const T* x, const int32_t* idx, T* out, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_gather<T>), dim3(blocks_for(n, 256)), dim3(256), 0, s, x, idx, out, n);
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
hipError_t launch_fill_i32(int* x, int v, int64_t n, hipStream_t s) { return launch_fill<int>(x, v, n, s); }

template <typename T>
hipError_t launch_misfit(const T* d, const T* obs, T* resid, int64_t n, double* scratch, int nblocks,
                         double* J_out, hipStream_t s) {
  hipLaunchKernelGGL((k_misfit<T>), dim3(nblocks), dim3(256), 0, s, d, obs, resid, n, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_parts, dim3(1), dim3(256), 0, s, scratch, nblocks, 0.5, J_out);
  return hipGetLastError();
}

hipError_t launch_finalize_grad(const double* c, const double* gacc, int n_shots, double scale, double* g,
                                int64_t n, hipStream_t s, bool accumulate) {
  hipLaunchKernelGGL(k_finalize_grad, dim3(blocks_for(n, 256)), dim3(256), 0, s, c, gacc, n_shots, scale, g,
                     n, accumulate ? 1 : 0);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_check_finite(const T* x, int64_t n, int64_t stride, int nvec, int* flag, hipStream_t s) {
  if (n <= 0 || nvec <= 0) return hipSuccess;
  const unsigned nb = (unsigned)std::min<int64_t>(blocks_for(n, 256), 512);
  hipLaunchKernelGGL((k_check_finite<T>), dim3(nb, (unsigned)nvec), dim3(256), 0, s, x, n, stride, flag);
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
hipError_t launch_normalize(T* v, const T* w, const double* dot_ww, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_normalize<T>), dim3(blocks_for(n, 256)), dim3(256), 0, s, v, w, dot_ww, n);
  return hipGetLastError();
}

#define KMV_INST(T)                                                                                    \
  template hipError_t launch_step<T>(int, int, bool, const StepArgs<T>&, int, int, hipStream_t,        \
                                     hipEvent_t, hipEvent_t, bool);                                   \
  template hipError_t set_step_lds_limit<T>(int, int, bool, int, bool);                                \
  template hipError_t launch_finish<T>(bool, const FinishArgs<T>&, hipStream_t, hipEvent_t,           \
                                       hipEvent_t);                                                   \
  template hipError_t launch_sample<T>(const T*, const int32_t*, const T*, int, int, T*, hipStream_t,  \
                                      hipEvent_t, hipEvent_t);                                       \
  template hipError_t launch_square<T>(const double*, T*, int64_t, hipStream_t);                      \
  template hipError_t launch_gather<T>(const T*, const int32_t*, T*, int64_t, hipStream_t);            \
  template hipError_t launch_fill<T>(T*, T, int64_t, hipStream_t);                                    \
  template hipError_t launch_misfit<T>(const T*, const T*, T*, int64_t, double*, int, double*,         \
                                       hipStream_t);                                                  \
  template hipError_t launch_scale<T>(const T*, const T*, T*, int64_t, hipStream_t);                  \
  template hipError_t launch_dot<T>(const T*, const T*, int64_t, double*, int, double*, hipStream_t); \
  template hipError_t launch_normalize<T>(T*, const T*, const double*, int64_t, hipStream_t);          \
  template hipError_t launch_check_finite<T>(const T*, int64_t, int64_t, int, int*, hipStream_t);
KMV_INST(float)
KMV_INST(double)

}  // namespace kmv

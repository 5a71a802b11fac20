/*
 * kmvwave — explicit mass-lumped KMV wave propagation (forward, adjoint, gradient)
 * on MI355X (gfx950).  C ABI.
 *
 * The method (Roberts et al., "Full waveform inversion using triangular waveform
 * adapted meshes"):
 *   - acoustic wave equation u_tt + eta u_t - div(c^2 grad u) = f   (section
 *     "Forward wave simulation", eq. acoustic_pml with only the tr(Psi_1) term
 *     kept as a quadratic sponge eta; homogeneous Neumann outer boundary);
 *   - continuous Galerkin on triangles/tetrahedra with mass-lumped KMV elements,
 *     degree 1..5 on triangles and 1..3 on tetrahedra (section "Higher-order mass
 *     lumping");
 *   - central differences in time, the diagonal leading matrix inverted pointwise
 *     (eqs. Leapfrog, forward3);
 *   - misfit J = 1/2 sum_n sum_j (d^n_j - dobs^n_j)^2 without a dt factor
 *     (eq. l2error and the remark after eq. gradient3);
 *   - discrete adjoint = transposed scheme, gradient dJ/dc_i from eq. gradient3
 *     (section "The adjoint-state and gradient problems discretized").
 *
 * Conventions
 *   - Every function returns an int status: KMV_OK (0) or a negative code; a
 *     message for the last failure on the calling thread is kmv_last_error().
 *     No C++ exception crosses this boundary.
 *   - Units: km, s, km/s.  Points are (x, z) in 2D, (x, y, z) in 3D.
 *   - "DOF order" is the library's own numbering of the global degrees of freedom
 *     (patch-contiguous); kmv_mesh_dof_coords gives the coordinates in that order.
 *   - Host pointers are read during the call and never retained.  Device pointers
 *     must be allocations on the current HIP device; work on them is enqueued on
 *     the given stream (a hipStream_t, NULL = the null stream) and is complete
 *     only when that stream is synchronised, except for calls that return a host
 *     scalar (they synchronise the stream before returning).
 *   - Precision: KMV_FP64 computes everything in float64.  KMV_FP32 keeps the
 *     wavefields, operators and traces in float32, accumulates the gradient over
 *     time steps and reduces the misfit in float64.  Trace and observed buffers
 *     have the problem's element type (float or double); wavespeed and gradient
 *     buffers are always double.
 */
#ifndef KMVWAVE_H
#define KMVWAVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  KMV_OK = 0,
  KMV_EINVAL = -1,   /* bad argument (null pointer, size, option) */
  KMV_ENOMEM = -2,   /* host or device allocation failed, or over the memory budget */
  KMV_EDEGREE = -3,  /* unsupported (dim, degree): tri 1..5, tet 1..3 */
  KMV_EMESH = -4,    /* invalid mesh: vertex index out of range, degenerate cell */
  KMV_EOUTSIDE = -5, /* a source or receiver lies outside every cell */
  KMV_ECFL = -6,     /* a solve left the floating-point range and dt exceeds the
                        Gershgorin step bound 2/sqrt(rho) of eq. spectral for its
                        wave speed (kmv_cfl_dt): the step is the likely cause.  The
                        bound is conservative, so a larger dt is not refused up
                        front; only a solve that blows up reports it */
  KMV_ENUMERIC = -7, /* a solve produced a NaN or infinity with dt within that bound
                        (non-finite inputs), or a result is not finite */
  KMV_EDEVICE = -8,  /* HIP runtime error */
  KMV_EBUSY = -9,    /* serving: result not ready yet (not a failure) */
  KMV_ESTATE = -10   /* call out of order (e.g. no sources set) */
};

enum { KMV_FP64 = 0, KMV_FP32 = 1 };

typedef struct kmv_mesh_s* kmv_mesh;       /* opaque, library-owned */
typedef struct kmv_problem_s* kmv_problem; /* opaque, library-owned */

/* Message describing the last failure on this thread ("" if none). */
const char* kmv_last_error(void);

/* ------------------------------------------------------------------ elements */

/* Reference KMV element tables (section "Higher-order mass lumping"; node
 * coordinates of figures fig:2dels/fig:3dels, weights = the nodal quadrature rule).
 * n_nodes: out, nodes per cell.  If nodes/weights/grads are non-NULL they receive
 * [n*dim] reference coordinates, [n] weights and [n*n*dim] basis gradients
 * grads[(q*n + a)*dim + r] = d phi_a / d xi_r at node q.  Host only.
 * Errors: KMV_EDEGREE. */
int kmv_element_tables(int dim, int degree, int* n_nodes, double* nodes, double* weights,
                       double* grads);

/* ---------------------------------------------------------------------- mesh */

/* Build the discretisation of a simplicial mesh (host only, no GPU needed):
 * global DOF numbering (one per distinct node; the local-to-global map g(j,k) of
 * section "Receivers and sources"), cell patches (interior DOFs of a cell numbered
 * together, the rest per patch), geometry, lumped mass M_i = sum w_q |det J_e|.
 *   coords [n_vertices*dim] (copied), cells [n_cells*(dim+1)] 0-based (copied).
 *   patch_cells: cells per patch, at most 256 (one GPU thread per cell; 0 = chosen
 *   from degree and dimension).
 * Errors: KMV_EINVAL (also 2^31 or more cells, vertices, DOFs or shared refs: the
 * device tables index them with 32-bit integers), KMV_EDEGREE, KMV_EMESH (index out
 * of range, zero volume). */
int kmv_mesh_create(int dim, int degree, const double* coords, int64_t n_vertices,
                    const int32_t* cells, int64_t n_cells, int patch_cells, kmv_mesh* out);
/* Sizes: any output pointer may be NULL. */
int kmv_mesh_info(kmv_mesh m, int64_t* n_dofs, int64_t* n_cells, int* n_nodes,
                  int64_t* n_patches, int64_t* n_shared_dofs);
/* DOF coordinates [n_dofs*dim], caller-owned host buffer. */
int kmv_mesh_dof_coords(kmv_mesh m, double* out);
/* Lumped mass [n_dofs] in DOF order (appendix, M_u with the KMV rule). */
int kmv_mesh_lumped_mass(kmv_mesh m, double* out);
/* Boundary mass [n_dofs] in DOF order: b_i = the integral over the mesh boundary
 * (facets of one cell only) of phi_i, the row sums of the boundary integral of
 * phi_i phi_j in the damping matrix M_{u,1} of the appendix; zero off the boundary.
 * The absorbing boundary term (kmv_set_absorbing_boundary) damps DOF i with c_i b_i.
 * Computed once per mesh and kept.  Host only.  Errors: KMV_EINVAL. */
int kmv_mesh_boundary_mass(kmv_mesh m, double* out);
/* Global DOF of every node of every input cell: out[cell*n_nodes + a], input cell
 * order, reference node order of kmv_element_tables. */
int kmv_mesh_cell_dofs(kmv_mesh m, int64_t* out);
/* Gershgorin estimate of the largest stable step, 2/sqrt(max_i sum_j |K_ij|/M_i)
 * (eq. spectral), for nodal wavespeed c_host [n_dofs] (host, DOF order).  Host
 * only.  Errors: KMV_EINVAL. */
int kmv_cfl_dt(kmv_mesh m, const double* c_host, double* dt_max);
/* Check the scheduling invariants the kernels rely on: interior DOFs sit at their
 * implicit positions, patch-local maps agree with the global DOF map, the gather
 * words of every patch collect each cell-node slot exactly once, every shared DOF
 * lists the partial slots of exactly the patches that touch it, in patch order,
 * and every lumped mass is positive.  Host only.
 * Returns KMV_OK or KMV_EMESH with the first violation in kmv_last_error(). */
int kmv_mesh_validate(kmv_mesh m);
/* Scheduling figures of the mesh's patches, for tests and tuning (host only):
 *   max_patch_cells   most cells in one patch (one GPU thread per cell, so the
 *                     step kernel's workgroup is this rounded up to whole
 *                     wavefronts of 64);
 *   max_shared_refs   most shared refs in one patch: DOFs the patch shares with
 *                     other patches, each finished in every touching patch from
 *                     the previous step's partial sums;
 *   first_batch_refs  shared refs a workgroup finishes in its first batch of
 *                     loads for the forward (adjoint = 0) or adjoint (1) step; a
 *                     patch with more finishes the rest in a second loop.
 * Any output may be NULL.  Errors: KMV_EINVAL. */
int kmv_mesh_patch_stats(kmv_mesh m, int adjoint, int64_t* max_patch_cells, int64_t* max_shared_refs,
                         int64_t* first_batch_refs);
int kmv_mesh_destroy(kmv_mesh m);

/* ------------------------------------------------------------------- problem */

typedef struct {
  int precision;            /* KMV_FP64 or KMV_FP32 */
  double dt;                /* time step (s) */
  int64_t n_steps;          /* N_t: steps n = 0..N_t-1 produce u^1..u^N_t */
  int64_t checkpoint_every; /* reverse sweep: 0 = store every state if it fits
                               mem_budget (else as < 0); > 0 = checkpoints every
                               this many steps; < 0 = checkpoints every
                               ceil(sqrt(2 N_t)) steps */
  size_t mem_budget;        /* bytes of device memory for stored states (0 = 8 GiB) */
  int n_shots;              /* shots stepped together (0 or 1 = one; at most 1024) */
  int64_t gradient_every;   /* r, gradient subsampling (section "Gradient subsampling"):
                               the reverse sweep pairs lambda^{n+1} with u^n only
                               for n % r == 0 and scales the sum by r, and with
                               checkpoint_every = 0 only every r-th forward state
                               is kept (floor(N_t/r) + 3 levels, no recompute) if
                               that fits mem_budget.  0 or 1 = every step (the
                               exact gradient of J). */
} kmv_options;

/* Allocate device state for n_shots shots on the current device.
 *
 * The shots of one problem share the mesh, the wave speed, the damping, dt, the
 * wavelet and the receivers, and differ in their source positions (the shots of
 * one acquisition, section "Parallelism": independent wave equations whose
 * misfits and gradients are summed, eq. gradient3).  Every step kernel launch
 * advances all shots; each shot's arithmetic is the same as in a one-shot
 * problem, so its traces are bitwise those of a one-shot problem with its
 * sources.  Per-shot inputs and outputs are shot-major: sources
 * [n_shots][n_src/n_shots][dim], traces, observed and adjoint-source data
 * [n_shots][n_steps][n_rec], source traces [n_shots][n_steps][n_src/n_shots].
 * J and grad are sums over the shots (float64, fixed order).
 * Errors: KMV_EINVAL (also when a patch's step kernel would need more than the
 * 160 KiB of LDS of a CU, e.g. FP64 KMV3 tetrahedra on a mesh whose patches have
 * unusually many non-interior DOFs: rebuild the mesh with a smaller patch_cells),
 * KMV_ENOMEM, KMV_EDEVICE. */
int kmv_problem_create(kmv_mesh m, const kmv_options* opt, kmv_problem* out);
/* Shots of a problem. */
int kmv_problem_num_shots(kmv_problem p, int* n_shots);
/* Spectral radius of M^-1 K(c) by a seeded power iteration on the GPU (the step
 * bound of eq. spectral without the Gershgorin over-estimate).  The start vector
 * is a normal deviate per DOF hashed from the seed and the DOF coordinates, so the
 * result does not depend on the internal DOF numbering.  Synchronises. */
int kmv_spectral_radius(kmv_problem p, const void* c_dev, int iters, uint64_t seed,
                        double* rho, void* stream);
/* Damping eta [n_dofs] in 1/s (host, DOF order; NULL = none).  The step uses
 * a = eta*dt/2 as the pointwise tr(Psi_1) term of eq. forward3.  Errors:
 * KMV_EINVAL (negative or non-finite), KMV_ESTATE (the PML is on). */
int kmv_set_damping(kmv_problem p, const double* eta);
/* Perfectly matched layer (section "Forward wave simulation in a PML truncated
 * medium": the PML system, its 2D form in eqs. forward2d_I / forward2d_II; the
 * appendix matrices).  sigma: [n_dofs*dim] host, DOF order, (sigma_x, sigma_z) per
 * DOF on triangles, (sigma_x, sigma_y, sigma_z) on tetrahedra: the damping
 * functions of the layer (zero in the physical domain), in 1/s; NULL turns it off.
 * With it on, each step also advances the auxiliary vector p (and on tetrahedra
 * omega, all in the same KMV space) and the u row gains the PML terms:
 *   u row: damping a = dt tr(Psi_1)/2 (in place of eta; kmv_set_damping is refused
 *          while the PML is on), the zeroth-order terms M tr(Psi_3) u + M det(Psi_1)
 *          omega (2D: M sigma_x sigma_z u), and sum_k D_k^T p_k, the divergence of p
 *          integrated by parts with n.p = 0, D_k = the integral of phi_i dphi_j/dx_k;
 *   p row: (1 + b_k) p_k^{n+1} = (1 - b_k) p_k^{n-1}
 *          - 2 dt M^-1 c^2 (Psi_2^kk D_k u^n - Psi_3^kk D_k omega^n), b_k = sigma_k dt
 *          (the damping term centred in time), Psi_2^kk = sigma_k - sum_{j!=k}
 *          sigma_j, Psi_3^kk = prod_{j!=k} sigma_j (zero in 2D);
 *   omega row (tetrahedra): omega^{n+1} = omega^n + dt (u^{n+1} + u^n)/2;
 * the adjoint is its exact transpose and dJ/dc gains
 * 2 c_i dt^2 sum_n sum_k mu_k,i^{n+1} (Psi_2^kk (D_k u^n)_i - Psi_3^kk (D_k omega^n)_i)
 * (zero outside the layer).  Triangles: the patches that touch the layer run a kernel
 * instance of their own; the gradient needs the forward states kept
 * (checkpoint_every = 0 with the states fitting mem_budget, or gradient_every > 1's
 * every r-th state), recomputing from checkpoints is refused with KMV_ENOMEM; device
 * memory 4 n_shots (n_dofs + R) elements per sweep for p or mu, 4 n_shots R for
 * their partial sums (R = the shared refs, at least 1).  Tetrahedra: per-cell and per-DOF passes beside
 * the stiffness apply; one shot per problem; the gradient keeps every forward level
 * of u and omega ((N_t + 1) (2 n_dofs + R) elements within mem_budget, else
 * KMV_ENOMEM); device memory 12 n_cells n_nodes elements of cell-node values and
 * 10 n_dofs of fields; not with the absorbing boundary term or kmv_forward_noalloc
 * (KMV_ESTATE).  Errors: KMV_EINVAL (negative or non-finite sigma, LDS on triangles,
 * several shots on tetrahedra), KMV_ESTATE (the absorbing boundary term is on, on
 * tetrahedra). */
int kmv_set_pml(kmv_problem p, const double* sigma);
/* First-order absorbing boundary (the condition du/dt + c du/dn = 0 on the outer
 * boundary of the forward problem; its weak form is the boundary integral of
 * c phi_i phi_j in the damping matrix M_{u,1} of the appendix).  enable = 1 turns
 * it on for every boundary facet of the mesh (facets of one cell only), 0 off (the
 * default: homogeneous Neumann).  Lumped by rows with c at node i it adds
 * dt c_i b_i / (2 M_i) to a_i, b_i = the boundary integral of phi_i, so the damping
 * of the boundary DOFs follows the c of each solve, and kmv_misfit_gradient adds
 * the matching term (dt b_i / 2) sum_n lambda_i^n (u_i^n - u_i^{n-2}) to dJ/dc_i
 * (at every step, also with gradient_every > 1).  The gradient keeps u^n and
 * lambda^n at the boundary DOFs of every level, 2 n_shots (n_steps+1) n_bnd
 * elements of device memory, and takes them from a ring of 8 adjoint levels
 * (8 n_shots level vectors) instead of 2; both are allocated on the first gradient
 * with the term on.  Errors: KMV_EINVAL. */
int kmv_set_absorbing_boundary(kmv_problem p, int enable);
/* Point sources x_s [n_src*dim] firing together with a Ricker wavelet
 * w(t) = amp (1 - 2 pi^2 f0^2 (t-t0)^2) exp(-pi^2 f0^2 (t-t0)^2) sampled at
 * t_n = n dt; injected as w(t_n) phi_a(x_s) (section "Receivers and sources").
 * With n_shots > 1 the points are shot-major and n_src is a multiple of
 * n_shots: shot s fires points s*n_src/n_shots .. (s+1)*n_src/n_shots - 1.
 * Errors: KMV_EOUTSIDE, KMV_EINVAL. */
int kmv_set_sources(kmv_problem p, const double* xs, int n_src, double f0, double t0,
                    double amp);
/* Replace the wavelet by w[n_steps] (host), the same for every shot.
 * Errors: KMV_EINVAL (NULL), KMV_ESTATE (no sources set yet). */
int kmv_set_source_wavelet(kmv_problem p, const double* w);
/* One wavelet per shot: w[n_shots*n_steps] (host, shot-major), shot s firing
 * w[s*n_steps + n] at t_n = n dt.  The paper fires every shot with the same Ricker
 * wavelet; this is for shots that differ in their signature (or polarity) within
 * one multi-shot problem.  kmv_set_sources or kmv_set_source_wavelet go back to one
 * shared wavelet.  Errors: KMV_EINVAL (NULL), KMV_ESTATE (no sources set yet). */
int kmv_set_source_wavelets(kmv_problem p, const double* w);
/* Receivers x_r [n_rec*dim]: d^n_j = sum_a phi_a(x_j) u^n_{g(e_j,a)}.
 * Errors: KMV_EOUTSIDE. */
int kmv_set_receivers(kmv_problem p, const double* xr, int n_rec);

/* Forward solve (eqs. Leapfrog/forward3).  c_dev: double [n_dofs] wavespeed (DOF
 * order).  traces_dev: [n_shots*n_steps*n_rec] of the problem's type, row n-1 of
 * a shot = d^n.  Asynchronous on stream; a blow-up is reported by
 * kmv_problem_status. */
int kmv_forward(kmv_problem p, const void* c_dev, void* traces_dev, void* stream);
/* As kmv_forward, but allocating nothing: for callers that cannot call hipMalloc
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * device allocation).  The two level buffers of the forward sweep live in the
 * library's static workspace of 64 MiB per device (held until the process ends)
 * instead of the problem's own, so the call needs 2 n_shots (n_dofs + R) elements of
 * workspace, R = the shared refs (at least 1); a larger problem is refused with
 * KMV_EINVAL before any work.  Everything else it uses was allocated when the problem was set up.  The
 * traces are bitwise those of kmv_forward.  Every call on one device shares that
 * workspace, so calls that overlap on one device (other streams, other threads)
 * race and must be serialised by the caller.  Launches are counted but not timed
 * by kmv_profile_enable.  Asynchronous on stream; a blow-up is reported by
 * kmv_problem_status.  Errors: KMV_EINVAL, KMV_ESTATE, KMV_EDEVICE. */
int kmv_forward_noalloc(kmv_problem p, const void* c_dev, void* traces_dev, void* stream);
/* Misfit and gradient: forward with stored or checkpointed states, J (eq.
 * l2error, no dt), adjoint sweep (eq. acoustic_pml_FEM_adj) fused with the
 * gradient accumulation (eq. gradient3).  observed_dev: [n_shots*n_steps*n_rec]
 * of the problem's type.  grad_dev: double [n_dofs] receives dJ/dc_i summed over
 * the shots (Euclidean; the mesh-independent gradient is grad/M).  traces_dev:
 * optional [n_shots*n_steps*n_rec] output of the forward traces (NULL = not
 * kept).  J_out (host) and the synchronisation: the stream is synchronised
 * before return. */
int kmv_misfit_gradient(kmv_problem p, const void* c_dev, const void* observed_dev,
                        double* J_out, double* grad_dev, void* traces_dev, void* stream);
/* As kmv_misfit_gradient, but adding to what the caller holds: *J_acc += J and
 * grad_acc[i] += dJ/dc_i, so that several problems (other shots, other
 * acquisitions on the same mesh and wave speed) are summed in place on the device,
 * in call order.  Synchronises.  Errors: as kmv_misfit_gradient. */
int kmv_misfit_gradient_accumulate(kmv_problem p, const void* c_dev, const void* observed_dev,
                                   double* J_acc, double* grad_acc, void* traces_dev, void* stream);
/* Misfit only (eq. l2error, no dt): the forward solve and the float64 reduction of
 * J, without stored states or the adjoint sweep (a line-search or finite-difference
 * probe).  J is bitwise the J of kmv_misfit_gradient for the same inputs.
 * traces_dev optional as there.  Synchronises.  Errors: as kmv_misfit_gradient. */
int kmv_misfit(kmv_problem p, const void* c_dev, const void* observed_dev, double* J_out, void* traces_dev,
               void* stream);
/* Non-finite sentinel of the most recent solve.  Every solve scans its wavefield
 * every 128 levels of each sweep, and its last level, for NaN or infinity.
 * kmv_misfit_gradient and kmv_misfit report a trip themselves; kmv_forward and
 * kmv_adjoint are asynchronous, so this call synchronises the stream and reports
 * theirs: KMV_ECFL or KMV_ENUMERIC (see the codes), else KMV_OK. */
int kmv_problem_status(kmv_problem p, void* stream);
/* Adjoint of the forward map for arbitrary receiver data y: lambda from the
 * transposed scheme, (1+a) lambda^m = 2 lambda^{m+1} - dt^2 M^-1 K lambda^{m+1}
 * - (1-a) lambda^{m+2} + M^-1 P^T y^m, m = N_t..1 (eq. acoustic_pml_FEM_adj).
 * adj_src_dev: [n_shots*n_steps*n_rec] of the problem's type, row m-1 of a shot
 * = y^m.  lambda_out_dev (optional, one-shot problems only):
 * [(n_steps+1)*n_dofs], row m-1 = lambda^m.
 * src_trace_dev (optional): [n_shots*n_steps*(n_src/n_shots)], row n of a shot =
 * lambda^{n+1} sampled at the shot's source points, so that for each shot
 * <y, P u> = dt^2 sum_n w(t_n) sum_s src_trace[n][s] (the dot-product identity
 * of the discrete adjoint). */
int kmv_adjoint(kmv_problem p, const void* c_dev, const void* adj_src_dev,
                void* lambda_out_dev, void* src_trace_dev, void* stream);
/* Matrix-free stiffness apply y = K(c) u (appendix, matrix K).  u_dev, y_dev of
 * the problem's type, [n_dofs], DOF order. */
int kmv_stiffness_apply(kmv_problem p, const void* c_dev, const void* u_dev, void* y_dev,
                        void* stream);
/* Kernel timing probe.  After kmv_profile_enable(p, every) (every >= 1; 0 turns it
 * off and clears the counters), every `every`-th launch of each kernel variant is
 * bracketed by HIP events recorded on the launch stream.  Variants:
 *   0 patch kernel, forward step      1 patch kernel, adjoint + gradient step
 *   2 shared-DOF finisher, forward    3 shared-DOF finisher, adjoint
 *   4 receiver sampling
 * kmv_profile_read synchronises the recorded events and returns the number of
 * launches, the number timed and their mean duration in milliseconds. */
int kmv_profile_enable(kmv_problem p, int every);
int kmv_profile_read(kmv_problem p, int variant, int64_t* n_launches, int64_t* n_timed,
                     double* mean_ms);
/* Sizes of a problem. */
int kmv_problem_info(kmv_problem p, int64_t* n_dofs, int64_t* n_steps, int* n_rec,
                     int* precision, int64_t* checkpoint_every);
int kmv_problem_destroy(kmv_problem p);

/* ------------------------------------------------------------------- serving */

/* A shot server keeps a queue of independent shot solves (the per-shot forward
 * and misfit-gradient evaluations of section "Parallelism", one shot per request)
 * and runs them on the current device.  Up to max_slots requests run at once,
 * each on its own stream and worker thread; a request is admitted, in arrival
 * order, when its device memory (states or checkpoints, traces, tables) fits in
 * what the running requests leave of mem_budget.  Requests admitted together
 * overlap on the GPU.  Every solve is deterministic and shares no buffer with
 * another, so a request's results are bitwise those it gets alone. */
typedef struct kmv_server_s* kmv_server;  /* opaque, library-owned */

typedef struct {
  kmv_mesh mesh;          /* must outlive the request; degree comes with it */
  int precision;          /* KMV_FP64 or KMV_FP32 */
  double dt;              /* time step (s) */
  int64_t n_steps;        /* N_t */
  const double* c;        /* [n_dofs] P-wave speed (host, DOF order) */
  const double* eta;      /* [n_dofs] damping in 1/s, or NULL */
  const double* xs;       /* [n_src*dim] source positions (Ricker, as kmv_set_sources;
                             shot-major when n_shots > 1) */
  int n_src;
  double f0, t0, amp;
  const double* xr;       /* [n_rec*dim] receiver positions */
  int n_rec;
  int forward_only;       /* 1: traces only; 0: misfit, traces and gradient */
  const void* observed;   /* [n_shots*n_steps*n_rec] host, element type of the precision */
  int n_shots;            /* shots in the request (0 or 1 = one): they share everything but
                             the sources, which are shot-major (n_src a multiple of
                             n_shots), and run as one multi-shot problem (one launch per
                             step for all of them, kmv_options.n_shots); J and grad are
                             sums over the shots */
  int absorbing;          /* 1: absorbing boundary term on (kmv_set_absorbing_boundary) */
  const double* wavelets; /* [n_shots*n_steps] host, shot-major: shot s fires its own
                             wavelet (as kmv_set_source_wavelets; f0, t0 and amp are then
                             unused), or NULL: the Ricker wavelet of f0, t0, amp for all */
} kmv_request;

typedef struct {
  int status;             /* KMV_OK or the solve's error code (text: kmv_last_error) */
  double J;               /* misfit (0 for forward-only requests) */
  const void* traces;     /* [n_shots*n_steps*n_rec] host, element type of the precision */
  const double* grad;     /* [n_dofs] host dJ/dc, or NULL for forward-only requests */
  int64_t n_steps, n_rec, n_dofs;
  double t_submit, t_admit, t_done;  /* seconds since the server was created */
  size_t device_bytes;    /* device memory reserved for the request while it ran */
  int64_t n_shots;        /* the request's n_shots (at least 1) */
} kmv_result;

/* mem_budget: device bytes for requests (0 = 80% of the free memory).  Each
 * request keeps all its states if they fit in min(mem_budget/2, 32 GiB), else it
 * checkpoints (as kmv_options.checkpoint_every = 0).
 * max_slots: requests that may run at once (1..64).
 * Errors: KMV_EINVAL, KMV_EDEVICE. */
int kmv_server_create(size_t mem_budget, int max_slots, kmv_server* out);
/* Copy the request's host inputs (the caller may free them on return) and queue
 * it.  Errors: KMV_EINVAL (missing inputs), KMV_ENOMEM (needs more than the whole
 * budget), KMV_ESTATE (server shutting down). */
int kmv_server_submit(kmv_server s, const kmv_request* req, uint64_t* ticket);
/* KMV_EBUSY while the request is pending, else KMV_OK with *out filled; the
 * result buffers stay valid until kmv_server_release.  Errors: KMV_EINVAL. */
int kmv_server_poll(kmv_server s, uint64_t ticket, kmv_result* out);
/* As kmv_server_poll, blocking up to timeout_s seconds (< 0: no limit). */
int kmv_server_wait(kmv_server s, uint64_t ticket, double timeout_s, kmv_result* out);
/* Free a finished request's results.  Errors: KMV_EBUSY, KMV_EINVAL. */
int kmv_server_release(kmv_server s, uint64_t ticket);
/* Requests running and queued, and device bytes reserved by the running ones. */
int kmv_server_stats(kmv_server s, int* running, int* queued, size_t* bytes_in_use);
/* Cancel queued requests, wait for the running ones, free everything. */
int kmv_server_destroy(kmv_server s);

#ifdef __cplusplus
}
#endif
#endif /* KMVWAVE_H */

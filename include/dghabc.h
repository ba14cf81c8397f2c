/* dghabc.h -- C ABI of the MI355X time stepper for nodal DG with high-order
 * absorbing boundary conditions (HABCs) and corner/edge compatibility.
 *
 * Method: A. Modave, A. Atle, J. Chan, T. Warburton, "A GPU-accelerated
 * nodal discontinuous Galerkin method with high-order absorbing boundary
 * conditions and corner/edge compatibility", arXiv:1610.05023.
 *
 * Every function returns dgh_status (0 = DGH_OK).  Nothing aborts, throws or
 * exits; on failure dgh_last_error() holds the reason.  One context per host
 * thread; contexts share no state apart from a process-wide, lock-protected
 * cache of per-device launch limits (LDS sizes, resident workgroups), so
 * contexts on different devices or threads may step at the same time.
 *
 * Call order: dgh_create -> dgh_upload_mesh -> dgh_set_order -> dgh_set_habc
 * -> dgh_set_material -> dgh_workspace_size -> dgh_bind_workspace ->
 * (dgh_set_state | dgh_set_source)* -> (dgh_step | dgh_read_fields |
 * dgh_energy)* -> dgh_destroy.  Calls out of order return DGH_ESTATE.
 * Calls before dgh_bind_workspace touch no GPU.
 *
 * Memory: all host pointers are caller-owned and only read/written during the
 * call.  Device memory is a single caller-owned workspace (e.g. a PyTorch
 * uint8 tensor) that the library never allocates or frees; every device
 * array of the method lives inside it.
 *
 * Canonical host layouts (row-major, FP64, leading shot index omitted when
 * n_shots = 1):
 *   q3, res3      [K][4][Np]          fields (p, u, v, w)
 *   q2, res2      [Ktri][P][3][Np2]   (p_i, two tangential velocity
 *                                      components in ascending axis order)
 *   qb3, q0_3     [Ktri][Np2]         incoming characteristic, r+ + r-
 *   q1, res1      [Klin][P*P][2][Np1] (p_ij, velocity along +axis); set
 *                                      index i*P + j, i on the earlier face
 *   qb2, q0_2     [Klin][2][P][Np1]   side 0 = earlier face (x-,x+,y-,...)
 *   qb1           [Kpnt][3][P*P]      slot a = the line along axis a
 * Node orders: tetrahedron lattice (i, j, k), i + j + k <= N, k slowest,
 * i fastest, Warp & Blend positions; triangle = tet nodes with k = 0;
 * line = GLL points.  Orderings of triangles, lines and corners are
 * documented in paper_1610_05023_amd/csrc/mesh.hpp.
 */
#ifndef DGHABC_H
#define DGHABC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dgh_ctx dgh_ctx;

typedef enum {
  DGH_OK = 0,
  DGH_EINVAL = -1,     /* bad argument, size or range */
  DGH_ESTATE = -2,     /* call out of order */
  DGH_EHIP = -3,       /* a HIP runtime call failed */
  DGH_ENOMEM = -4,     /* workspace too small */
  DGH_ENONFINITE = -5, /* non-finite value found by dgh_check */
  DGH_EUNSTABLE = -6   /* energy growth found by dgh_check */
} dgh_status;

/* Arithmetic of the 3D level (Section 3.2's volume, surface and update):
 * DGH_FP64; DGH_FP32_MFMA: FP32 3D state and residual with the volume and
 * LIFT contractions on the FP32 MFMA (FP32 accumulation); DGH_BF16_MFMA:
 * the same FP32 state, residual, fluxes and update, with the volume and
 * LIFT contractions on the BF16 MFMA (operators and the values entering
 * each contraction rounded to BF16, FP32 accumulation).  The face, edge and
 * corner levels, their RK accumulation and the energy stay FP64 in all.
 * The mixed forms differ from FP64 by rounding only; their errors are
 * reported by the tests, not bounded by the FP64 parity target. */
typedef enum { DGH_FP64 = 0, DGH_FP32_MFMA = 2, DGH_BF16_MFMA = 3 } dgh_precision;

/* Boundary condition of a face of the cuboid (faces x-, x+, y-, y+, z-, z+).
 * HABC: Pade HABC of order P (Section 2), with edge/corner compatibility where
 * two/three HABC faces meet; ABC: the basic ABC, incoming characteristic 0
 * (Section 3.2); DIRICHLET: p = 0 (Sections 2.4, 3.2); PERIODIC: both faces
 * of that axis are identified (used for plane-wave checks). */
typedef enum { DGH_BC_HABC = 0, DGH_BC_ABC = 1, DGH_BC_DIRICHLET = 2, DGH_BC_PERIODIC = 3 } dgh_bc;

/* Indices of the state arrays passed to dgh_set_state / dgh_read_fields. */
enum {
  DGH_Q3 = 0, DGH_RES3, DGH_Q2, DGH_RES2, DGH_QB3, DGH_Q03,
  DGH_Q1, DGH_RES1, DGH_QB2, DGH_Q02, DGH_QB1, DGH_NARRAYS
};

/* Counts reported by dgh_counts (indices into the int array). */
enum {
  DGH_C_K = 0, DGH_C_KTRI, DGH_C_KLIN, DGH_C_KPNT, DGH_C_NP, DGH_C_NP2, DGH_C_NP1,
  DGH_C_P, DGH_C_N, DGH_C_NSHOTS, DGH_NCOUNTS
};

/* Creates a context for HIP device `device`.  precision: DGH_FP64,
 * DGH_FP32_MFMA or DGH_BF16_MFMA (dgh_precision).
 * n_shots (1..4096): independent problems on the same mesh and medium,
 * each with its own state and point source, stepped together: every launch
 * covers all shots (the operators, geometry and maps are shared).  Each
 * state array is allocated per shot; a shot's 3D state must stay below
 * 4 GiB. */
dgh_status dgh_create(dgh_ctx** out, int device, int precision, int n_shots);

/* Tetrahedral mesh of the cuboid box = {lo[3], hi[3]} (Section 3.2: volume
 * mesh of K tetrahedra).  VX: Nv x 3 coordinates; EToV: K x 4 vertex ids,
 * each tetrahedron positively oriented.  periodic[3] (may be NULL): identify
 * the two faces of that axis.  The mesh must be conforming. */
dgh_status dgh_upload_mesh(dgh_ctx* ctx, int Nv, const double* VX, int K, const int* EToV,
                           const double* box /* lo[3], hi[3] */, const int* periodic);

/* Polynomial degree N of the nodal basis, 1 <= N <= 6 (Section 3.2). */
dgh_status dgh_set_order(dgh_ctx* ctx, int N);

/* HABC order P (0 <= P <= 12) and optional coefficients gamma[P] (NULL: the
 * Pade values tan^2(n pi/(2P+1)), Section 2.1); face_bc[6] per face
 * (NULL: HABC everywhere).  Builds the surface, line and corner meshes and
 * the edge/corner maps (Section 3.1). */
dgh_status dgh_set_habc(dgh_ctx* ctx, int P, const double* gamma, const int* face_bc);

/* Cellwise density rho[K] > 0 and wave speed c[K] > 0 (Section 2, the
 * pressure-velocity system; Section 3.2, cellwise constant materials). */
dgh_status dgh_set_material(dgh_ctx* ctx, const double* rho, const double* c);

/* Number of elements per level and sizes; out[DGH_NCOUNTS]. */
dgh_status dgh_counts(const dgh_ctx* ctx, int* out);

/* Physical coordinates of the tetrahedron nodes, K x Np x 3 (host). */
dgh_status dgh_node_coords(const dgh_ctx* ctx, double* out);

/* Bytes of device workspace the context needs. */
dgh_status dgh_workspace_size(dgh_ctx* ctx, size_t* bytes);

/* Binds the caller-owned device workspace (>= dgh_workspace_size bytes,
 * 256-byte aligned) and uploads operators, geometry, connectivity and HABC
 * maps; zeroes the state.  `stream` is a hipStream_t (NULL = default). */
dgh_status dgh_bind_workspace(dgh_ctx* ctx, void* device_ptr, size_t bytes, void* stream);

/* Sets the state of one shot (0 <= shot < n_shots) from host arrays in the
 * canonical layouts: the initial data of the problem statement (Section 2:
 * compactly supported initial pressure and velocity, and zero auxiliary
 * fields, which a NULL entry gives).  arrays[DGH_NARRAYS], a NULL entry
 * means zeros.  First waits for the work queued on the bound stream (a step
 * in flight), then copies on that stream and waits for the copies. */
dgh_status dgh_set_state(dgh_ctx* ctx, int shot, const double* const* arrays);

/* Copies the state of one shot to host arrays (NULL entries are skipped):
 * the pressure and velocity fields that Section 4.1 measures, and every
 * auxiliary and coupling array of the boundary levels.  Waits for the work
 * queued on the bound stream, then copies on it. */
dgh_status dgh_read_fields(dgh_ctx* ctx, int shot, double* const* arrays);

/* Point source delta(x - xs) S(t) in the pressure equation with
 * S(t) = amp (t - t0) exp(-pi^2 f0^2 (t - t0)^2), the integral of a Ricker
 * wavelet of peak frequency f0 (Section 4.1).  The source is projected on
 * the element that contains xs (the most interior one on ties).  amp = 0
 * removes the source of that shot.  Waits for the work queued on the bound
 * stream before it writes, then copies on that stream. */
dgh_status dgh_set_source(dgh_ctx* ctx, int shot, const double* xs, double f0, double t0,
                          double amp);

/* Advances all shots by n_steps steps of the five-stage low-storage RK
 * scheme (Section 3.2) with step dt, starting at time t_start; each stage
 * runs the volume, face, edge and corner levels in the order of Algorithm 1.
 * Asynchronous on the bound stream. */
dgh_status dgh_step(dgh_ctx* ctx, int n_steps, double dt, double t_start);

/* Group step (uneven batches): advances n (1..8) bound contexts -- meshes
 * of any size, with their own shots, materials and sources -- by n_steps
 * steps together; each stage runs the 3D level of all of them in one
 * persistent launch over a work list of their tiles, then the face, edge
 * and corner levels of each.  The members need the same precision (FP64,
 * FP32 or BF16 contractions), the same N <= 4, the tile-on-chip kernel (tuning
 * candidates 0-5), the same device and stream, and no closure; results
 * equal stepping each alone.  The member tables
 * live in ctxs[0]'s workspace.  Synchronises the stream once at the start.
 * DGH_EINVAL on a mismatch (reason in ctxs[0]'s dgh_last_error). */
dgh_status dgh_step_group(dgh_ctx* const* ctxs, int n, int n_steps, double dt, double t_start);

/* Replayed stepping: enable = 1 makes dgh_step capture one step (all its
 * launches, for each of the two parities of the double-buffered states) in
 * HIP graphs on a stream of the library's own, and replay one graph per
 * step on the bound stream; the stage times then come from a device clock
 * that dgh_step sets to t_start and every step advances, computed so that
 * results equal eager stepping bitwise.  The graphs are re-captured when dt,
 * the closure or the trace recording change, and dropped by enable = 0, a
 * new workspace or dgh_destroy.  Kernel timing (dgh_kernel_timing) uses
 * eager stepping. */
dgh_status dgh_set_graph(dgh_ctx* ctx, int enable);

/* Launch tuning of the 3D level (the counterpart of the paper's choice of
 * elements per block, Section 4.2).  Candidates (dgh_tuning_count: 18 for
 * FP64 with N <= 4 and the FP32 and BF16 variants with N <= 5, else 12)
 * are (kernel * 2 + order) * 3 + grid.  Where the tile fits on chip,
 * kernel 0 holds a whole tile of 16 elements per wave on chip (four waves
 * per workgroup), kernels 1 and 2 stream it through registers with 4 or 8
 * waves (64 or 128 elements) per workgroup; elsewhere kernels 0 and 1 are
 * the register-streaming kernel with its default and with the other
 * number of waves (the default is 8 for FP64 at N = 5 and for the FP32
 * and BF16 variants at N = 6, else 4).  Order 0
 * gives each of the 8 XCDs a contiguous range of tiles, order 1 deals tiles
 * round-robin over all workgroups; grid 0, 1, 2 launches 8, 6 or 4 eighths
 * of the workgroups that fit on the device at once, each walking more
 * tiles when there are fewer.  Every candidate computes the same step.
 * dgh_set_tuning forces a candidate; dgh_autotune times `launches`
 * launches (1..10000) of each on the bound workload -- they read the
 * current state and write only the other half of its double buffer, so the
 * state is unchanged -- keeps the fastest, returns its index in *best and,
 * if ms is not NULL, the milliseconds per launch of every candidate in
 * ms[0..count-1].  Both synchronise. */
dgh_status dgh_tuning_count(dgh_ctx* ctx, int* count);
dgh_status dgh_set_tuning(dgh_ctx* ctx, int candidate);
dgh_status dgh_autotune(dgh_ctx* ctx, int launches, int* best, double* ms);

/* FP64 energy sum_k J_k/2 (p^T M p/(rho c^2) + rho u^T M u) of the 3D fields
 * of one shot (the energy weights of Section 4.1).  Synchronises. */
dgh_status dgh_energy(dgh_ctx* ctx, int shot, double* e);

/* Failure check (the energy of Section 4.1 as a stability monitor): scans
 * every state array of every level of one shot for non-finite values and
 * computes the FP64 energy (written to *e_out when e_out is not NULL).
 * Returns DGH_ENONFINITE if any value (or the energy) is not finite, else
 * DGH_EUNSTABLE if e_ref > 0 and the energy exceeds e_ref (1 + rel_tol)
 * (rel_tol >= 0, else DGH_EINVAL), else DGH_OK.  The state is left as
 * computed, so the caller may restore its own checkpoint with
 * dgh_set_state.  Synchronises. */
dgh_status dgh_check(dgh_ctx* ctx, int shot, double e_ref, double rel_tol, double* e_out);

/* ---- Learned boundary closure (an extension beside the method: a small
 * MLP stands in for the order-P auxiliary recursion of Sections 2-3 on the
 * absorbing faces).  Network: 10 inputs (p and Z |u_t| of the 3D trace at a
 * face node, u_t the velocity tangential to the face, at the current step
 * end, then the root mean squares of p and of Z |u_t| over the recent past
 * at the four time scales of dgh_set_closure_memory -- exponential averages
 * of their squares updated at every step end; all divided by their root
 * mean square, times in_scale) -> 64 -> 64 -> 64 (tanh) -> y; r- = g_max tanh(y) r+ with r+ =
 * (p + Z n.u)/2 the current outgoing characteristic, so |r-| <= |g_max|
 * |r+| at every node and the closed loop cannot gain energy at the
 * boundary.  A sample row is the 10 raw inputs followed by r+.  Parameters (FP32,
 * flat, DGH_CLOSURE_PARAMS): in_scale, g_max (|g_max| <= 1), W1[64][10],
 * b1[64], W2[64][64], b2[64], W3[64][64], b3[64], W4[64], b4. */
#define DGH_CLOSURE_PARAMS 9091

/* Uses the closure for r- on every HABC face (host parameters, copied);
 * n_w = 0 returns to the plain method.  Needs P = 0 (no auxiliary fields)
 * and |g_max| <= 1 (DGH_EINVAL otherwise);
 * edges and corners then have no compatibility systems.  The network runs
 * once per step, at its end, on the inputs of that step end (those
 * dgh_closure_sample records); its r- then holds for every stage of the
 * next step.  dgh_set_state clears a shot's trace memory and its r- (qb3).
 * Waits for the work queued on the bound stream before it writes the
 * weights. */
dgh_status dgh_set_closure(dgh_ctx* ctx, const float* w, int n_w);

/* Time scales tau[DGH_CLOSURE_MEMORY] (> 0, time units of the problem) of
 * the closure's averaged inputs: at a step end of length dt each average
 * keeps exp(-dt/tau_k) of its value and takes the rest from the new
 * square.  NULL restores the default 1.25, 2.5, 5 and 10 times h / c_max,
 * h = (6 |Omega| / K)^(1/3) (the cell size of a Kuhn mesh).  Training data
 * and use must share them. */
#define DGH_CLOSURE_MEMORY 4
dgh_status dgh_set_closure_memory(dgh_ctx* ctx, const double* tau);

/* Keeps the per-node trace memory up to date at every step end (always on
 * while a closure is set), so that dgh_closure_sample can read it. */
dgh_status dgh_closure_record(dgh_ctx* ctx, int enable);

/* Training samples of one shot from the current state: x[Ktri*Np2][11]
 * (sample rows: the closure's raw inputs and r+) and y[Ktri*Np2] (the
 * current qb3, i.e. the r- the method produced at the last stage).  Host
 * arrays.
 * Synchronises. */
dgh_status dgh_closure_sample(dgh_ctx* ctx, int shot, float* x, float* y);

/* Training kernels of the closure, no context: every pointer is a device
 * pointer, stream a hipStream_t (NULL = default).  work: at least
 * dgh_mlp_work_size(batch) floats.  dgh_mlp_forward: Y[n] = r- for the sample rows X[n][11].
 * dgh_mlp_grad: G = gradient of the mean squared error (1/n) sum (r- - T)^2
 * over the batch (G[0] = G[1] = 0); loss (host, may be NULL: then no
 * synchronisation) receives the loss.  dgh_mlp_adam: one Adam step (beta
 * 0.9, 0.999, eps 1e-8) at step t >= 1 on every parameter but the scales. */
dgh_status dgh_mlp_work_size(int batch, size_t* floats);
dgh_status dgh_mlp_forward(const float* W, const float* X, int n, float* Y, void* stream);
dgh_status dgh_mlp_grad(const float* W, const float* X, const float* T, int n, float* G,
                        float* work, double* loss, void* stream);
dgh_status dgh_mlp_adam(float* W, const float* G, float* M, float* V, int t, float lr,
                        void* stream);

/* dgh_mlp_grad in BF16 on the matrix cores (the closure's BF16 training
 * with FP32 master weights): the weights and the activations and their
 * gradients are rounded to BF16 as they enter each product, every sum is
 * FP32; 64 samples per workgroup, the workgroups' partial gradients summed
 * in a fixed order, so two calls on the same inputs give the same bits.
 * The same arguments as dgh_mlp_grad: device pointers, work of at least
 * dgh_mlp_work_size(n) floats, loss on the host (may be NULL: no
 * synchronisation).  Results differ from dgh_mlp_grad by that rounding
 * (0.3-0.7% of the gradient in relative l2).  DGH_EINVAL for a NULL
 * pointer or n <= 0, DGH_EHIP when a launch or the loss copy fails. */
dgh_status dgh_mlp_grad_bf16(const float* W, const float* X, const float* T, int n, float* G,
                             float* work, double* loss, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving or training loops, harnesses that forbid
 * hipMalloc): dgh_mlp_grad without the work argument.  Same kernels and
 * results; the work buffer is a fixed array inside the library, one per
 * GPU (6.4 MB, held until the process ends), so 1 <= n <=
 * DGH_MLP_STATIC_BATCH (DGH_EINVAL otherwise).  Calls no allocating
 * routine.  Every call on a GPU shares that GPU's array: calls that overlap
 * on one GPU (other streams or host threads) race; the array needs no
 * clearing (every value is written before it is read).  Runs on the
 * device of `stream` (the current device for NULL). */
#define DGH_MLP_STATIC_BATCH 4096
dgh_status dgh_mlp_grad_static(const float* W, const float* X, const float* T, int n, float* G,
                               double* loss, void* stream);

/* Per-kernel timing with HIP events on the bound stream: enable = 1 starts
 * recording around every 3D-level launch, 0 stops.  dgh_kernel_time returns
 * the accumulated milliseconds and launch count of level `level` (3, 2, 1,
 * 0) since the last enable. Synchronises. */
dgh_status dgh_kernel_timing(dgh_ctx* ctx, int enable);
dgh_status dgh_kernel_time(dgh_ctx* ctx, int level, double* total_ms, long long* launches);

/* Reason of the last failure (never NULL). */
const char* dgh_last_error(const dgh_ctx* ctx);

void dgh_destroy(dgh_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* DGHABC_H */

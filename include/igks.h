/*
 * igks.h - C ABI of the MI355X (gfx950) implicit gas-kinetic scheme
 * library, libigks.so.
 *
 * What it computes (Pan, Zhong & Zhuo, "An Implicit Gas-Kinetic Scheme for
 * Turbulent Flow on Unstructured Hybrid Mesh"):
 *   - per face, the BGK gas-kinetic flux of Sec. 2.1 (least-squares
 *     reconstruction Eq.6-7 with the Eq.9-10 limiter, Maxwellian moments,
 *     the interface distribution Eq.13 and its flux Eq.14), with the
 *     Spalart-Allmaras working variable carried alongside (Sec. 2.3,
 *     Eq.26-34);
 *   - per iteration, the residual of Eq.16, the implicit CFL law Eq.24-25
 *     and the matrix-free LU-SGS forward/backward sweeps of Eq.18-22 and
 *     Eq.31-32, with the ghost-cell boundary conditions of Sec. 2.5;
 *   on a 2D hybrid mesh (triangles, quadrilaterals and polygons of up to
 *   eight vertices, such as the pentagons and hexagons that hanging nodes
 *   of an adaptive quadtree make, Sec. 2.4 and Sec. 3.1) given in the
 *   node / per-cell vertex list form of Sec. 2.4, on one GPU.
 *
 * Conventions
 *   - Every call returns an int status: IGKS_OK (0) or a negative error
 *     code; igks_last_error() gives a message.  A context is used by one
 *     host thread at a time; there is no global state.
 *   - Host pointers are read or written during the call only (copied); the
 *     caller keeps ownership.  Device memory comes from the caller: the
 *     library asks for a workspace size and works inside that one buffer,
 *     and never allocates or frees device memory itself.
 *   - All work is queued on the HIP stream given at creation (or, for a
 *     NULL stream, on a stream the library creates at default priority).
 *     Calls that return host data synchronise that stream.
 *   - Cells are numbered as uploaded.  The Gauss-Seidel sweeps visit them
 *     in increasing (forward) and decreasing (backward) index: the
 *     "j < i" and "j > i" of Eq.20.  The library runs each sweep as
 *     wavefronts of mutually independent cells, which gives the same result
 *     as the sequential sweep; fewer wavefronts = more parallel work per
 *     launch, so callers that want speed number cells by a colouring.
 *   - Non-dimensionalisation: rho_inf = 1, |V_inf| = 1, reference length 1,
 *     p_inf = 1/(gamma Ma^2), mu_inf = 1/Re; gamma = 1.4 (K = 3, Sec. 2.1).
 */
#ifndef IGKS_H
#define IGKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define IGKS_OK 0
#define IGKS_EINVAL (-1)   /* bad argument or call order */
#define IGKS_EMESH (-2)    /* invalid mesh (see igks_mesh_upload) */
#define IGKS_ENOMEM (-3)   /* workspace too small */
#define IGKS_ENONPHYS (-4) /* an update produced rho <= 0, p <= 0 or a non-finite value */
#define IGKS_EHIP (-5)     /* a HIP runtime call failed */

/* boundary tags of boundary edges (Sec. 2.5) */
#define IGKS_BC_FREESTREAM 1 /* ghost = free stream, ghost increment 0 */
#define IGKS_BC_SYMMETRY 2   /* normal momentum mirrored */
#define IGKS_BC_WALL 3       /* no-slip: momentum and nu-tilde negated */
#define IGKS_BC_OUTFLOW 4    /* Riemann-invariant outflow, ghost increment 0 */
#define IGKS_BC_FARFIELD 5   /* FREESTREAM where V_inf . n < 0, else OUTFLOW */
#define IGKS_BC_MOVING_WALL 6 /* no-slip wall moving with the tangential part of V_inf (a lid) */

/* precision of the implicit sweeps */
#define IGKS_FP64 0  /* everything in FP64 */
#define IGKS_MIXED 1 /* LU-SGS sweeps and Jacobian products in FP32; residual, update, SA source FP64 */

typedef struct igks_options {
    int precision;      /* IGKS_FP64 or IGKS_MIXED */
    int limiter;        /* 0: off, 1: the limiter of Eq.9-10 */
    double cfl_init;    /* implicit CFL of the first iteration (Eq.25 start) */
    double cfl_min;     /* clamp of the Eq.25 CFL */
    double cfl_max;
    int cfl_mode;       /* 0: Eq.25 (residual-ratio law), 1: fixed cfl_init */
    double cfl_flux;    /* delta_CFL0 of Eq.23 (time step inside the flux) */
    int visc_sr;        /* 1: add 2 nu_eff / |r.n| to the LU-SGS spectral radius */
    int mu_law;         /* 0: Sutherland, 1: constant viscosity */
    int chunk;          /* iterations per captured HIP graph launch; 0 = no graph */
    int block;          /* threads per block of the cell/face kernels; 0 = 256 */
    int sweep;          /* LU-SGS sweep schedule: 0 auto, 1 one launch per wavefront,
                           2 all wavefronts in one workgroup (barrier between wavefronts),
                           3 one wave per sweep block (igks_set_sweep_blocks), all blocks at once */
    int flux_lanes;     /* lanes per face of the flux kernel: 0 auto (2 below 32768 faces),
                           1 or 2; the two agree to rounding */
    int scheme;         /* 0: implicit LU-SGS (Eq.18-22); 1: explicit Eq.15 with local time
                           steps dt_i = CFL Omega_i / (Lambda_c)_i, CFL = cfl_init fixed
                           (the paper's explicit GKS baseline) */
    double wall_temp;   /* 0: adiabatic no-slip walls (the Sec. 2.5 ghost rule); > 0: WALL and
                           MOVING_WALL faces held at wall_temp x the free-stream temperature:
                           the same ghost plus the Navier-Stokes heat flux of the BGK model,
                           mu c_p (T_c - T_w) / d (Pr = 1, mu at the cell-centre temperature,
                           d the centroid-face distance), treated explicitly */
    double limiter_freeze; /* with the limiter on: once an instance's density residual has dropped
                              to this fraction of its first value, its Eq.9 limiter factors are held
                              at the values of that iteration (near convergence they otherwise
                              chatter and hold the residual up); 0 = never; in [0, 1).  The hold
                              ends with igks_set_freestream / igks_set_state. */
    int tau_jump;       /* 1: add dt |p_l - p_r| / (p_l + p_r) (reconstructed face pressures) to the
                           collision time of Eq.34, the usual gas-kinetic extra dissipation at
                           discontinuities (not in the paper); 0 (default): Eq.34 as printed */
    int block_passes;   /* with sweep blocks (igks_set_sweep_blocks): 1 (default; 0 means 1) one
                           block LU-SGS pass, the coupling across blocks left out of L and U;
                           2: a second pass solves the same block system again with the cross-block
                           terms of the first pass's increments moved to its right-hand side (one
                           block-Jacobi correction of the coupling the blocks leave out; not in the
                           paper).  Two passes run on the wave-per-block schedule (sweep 0 or 3;
                           1 or 2 with block_passes 2 is IGKS_EINVAL) and take a second increment
                           array in the workspace. */
    int lusgs_op;       /* dissipation of the LU-SGS operator (Eq.18-22): 0 (default) the scalar
                           spectral radius lambda_ij I of Eq.20; 1 the first-order Roe matrix
                           |A_ij| = R |Lambda| L of the Euler flux Jacobian at the Roe average of the
                           two cell-centre states (eigenvalue magnitudes held at least at 0.1 c) plus
                           the viscous part of lambda_ij times I, so that D becomes a 4x4 block per
                           cell (inverted once per iteration, 16 values per cell in the workspace).
                           The steady answer is the same; the implicit iteration converges in fewer
                           steps.  The SA equation keeps its scalar form, and faces between sweep
                           blocks keep lambda_ij I (with |A| there the block iteration stalls).
                           2: the same matrix with each eigenvalue magnitude |s| replaced by the
                           mean of |u| for normal velocities u spread as a Maxwellian of temperature
                           c^2 / gamma about s, s erf(s / sqrt(2RT)) + sqrt(2RT / pi) exp(-s^2 / 2RT)
                           (at least 0.67 c): slower than 1 where 1 converges, but it also converges
                           the SA plate and the flows where 1 stalls.
                           Ignored by the explicit scheme.  Other values: IGKS_EINVAL. */
} igks_options;

typedef struct igks_residual {
    int32_t iteration;  /* iterations committed so far */
    double res_l2;      /* ||M_rho||_2 of the last residual evaluation (Eq.16) */
    double res_drop;    /* res_l2 / the largest res_l2 so far */
    double res_inf;     /* max over cells and the 4 flow components of |M| */
    double eq40;        /* max_i ||W_i^{n+1} - W_i^n||_2 / ||W_i^n||_2 (Eq.40) */
    double cfl;         /* implicit CFL used by the last update (Eq.25) */
    double dt_flux;     /* Eq.23 time step used inside the flux */
    double sa_l2;       /* ||R_SA||_2 (Eq.27 right-hand side) */
} igks_residual;

/* iteration scalars for checkpoint / resume */
typedef struct igks_scalars {
    int32_t iteration;
    double cfl;          /* CFL of the last committed iteration */
    double res_inf_prev; /* ||M||_inf of the last committed iteration */
    double res0;         /* the largest ||M_rho||_2 so far (the drop's reference) */
} igks_scalars;

typedef struct igks_ctx igks_ctx;

/* Fill *opt with the defaults: FP64, limiter off, cfl_init 1000 (Sec. 3.1),
 * cfl_min 1, cfl_max 1e6, Eq.25 law, cfl_flux 1, visc_sr on, Sutherland,
 * chunk 20, block 256, sweep auto (a wave per sweep block when an instance has
 * sweep blocks, else one workgroup when the wavefronts are many and narrow:
 * more than 16 of them averaging under 1024 cells), flux_lanes auto. */
void igks_default_options(igks_options *opt);

/* Create a context.  opt may be NULL (defaults).  hip_stream is a
 * hipStream_t (NULL: the library creates its own).  *out owns the
 * context until igks_destroy. */
int igks_create(igks_ctx **out, const igks_options *opt, void *hip_stream);
void igks_destroy(igks_ctx *ctx);
const char *igks_last_error(const igks_ctx *ctx);

/* Mesh in the form of Sec. 2.4: n_nodes coordinates xy[2*n_nodes]
 * (x0,y0,x1,y1,...); cells as CSR: vertices of cell i are
 * cell_nodes[cell_ptr[i] .. cell_ptr[i+1]-1], 3 to 8 of them, either
 * orientation (a polygon may have collinear vertices: every edge is a
 * face); n_bfaces boundary edges bface_nodes[2*b], [2*b+1] with tags
 * bface_tag[b] (IGKS_BC_*).  All host memory, copied.
 * IGKS_EMESH: a cell with fewer than 3 or more than 8 nodes, a degenerate
 * (zero-area) cell, a non-convex cell (a vertex where the boundary turns
 * back by more than asin(0.1), about 5.7 degrees: the slight reflex turn of
 * a hanging node on a curved edge is accepted) or one whose centroid is not
 * strictly inside the half plane of each of its faces (the centroid-face
 * distances of Eq.5 divide), an edge shared by more than two cells, a cell edge on
 * the boundary without a tag, a tagged edge that is not on the boundary, a
 * bad tag, or a node index out of range.  Replaces any previous mesh and
 * unbinds the workspace. */
int igks_mesh_upload(igks_ctx *ctx, int32_t n_nodes, const double *xy, int32_t n_cells,
                     const int32_t *cell_ptr, const int32_t *cell_nodes, int32_t n_bfaces,
                     const int32_t *bface_nodes, const int32_t *bface_tag);

/* Sweep blocks of instance inst (0 for a single-instance context):
 * block_of_cell[i] >= 0 is the block of cell i (upload order, host array,
 * copied); NULL restores one block.  The LU-SGS sweeps of Eq.22 and Eq.31-32
 * then couple only cells of one block, each block swept in increasing
 * (forward) and decreasing (backward) cell index, with the neighbours in
 * other blocks left out of the lower and upper parts (their increments taken
 * as zero), as the sweeps of a partitioned mesh do; the diagonal keeps every
 * face and the residual is unchanged, so only the path to the steady state
 * changes.  Blocks cut the number of wavefronts (within a block of the
 * mesh's own order a few tens) while each block keeps the ordered
 * Gauss-Seidel coupling that carries information along the flow; a
 * colouring of the whole mesh, by contrast, leaves 3 wavefronts but a
 * sweep that converges poorly.  Call after the instance's mesh upload;
 * like an upload it unbinds the workspace (bind again, then set the free
 * streams).  IGKS_EINVAL for a negative block or an instance without a
 * mesh. */
int igks_set_sweep_blocks(igks_ctx *ctx, int32_t inst, const int32_t *block_of_cell);

/* Sizes of the uploaded mesh: cells, faces, wall faces, sweep wavefronts. */
int igks_mesh_info(const igks_ctx *ctx, int32_t *n_cells, int32_t *n_faces, int32_t *n_wall_faces,
                   int32_t *n_levels);

/* Cells in each sweep wavefront (Sec. 2.2, Eq.22: the cells of a wavefront
 * depend only on cells of earlier ones), over all instances.  sizes: host
 * array of cap entries; min(cap, n_levels) are written, in sweep order.
 * IGKS_EINVAL for a null pointer, cap < 1 or an instance without a mesh. */
int igks_wavefront_sizes(const igks_ctx *ctx, int32_t *sizes, int32_t cap);

/* Device bytes the library needs for the uploaded mesh and options. */
int igks_workspace_size(const igks_ctx *ctx, size_t *bytes);

/* Bind caller-owned device memory (at least igks_workspace_size bytes,
 * 256-byte aligned), upload the mesh data into it and compute the wall
 * distance on the GPU.  The caller keeps the buffer alive until the
 * context is destroyed or rebound.  IGKS_ENOMEM if too small. */
int igks_bind_workspace(igks_ctx *ctx, void *dptr, size_t bytes);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): bind the
 * library's own workspace, a static device array of 64 MiB (67108864 bytes)
 * on the current device, which must be the device of the context's stream,
 * in place of a caller's buffer.  Otherwise as igks_bind_workspace (mesh
 * data uploaded, wall distance computed, state to be set by
 * igks_set_freestream); no device memory is allocated or freed.
 * IGKS_ENOMEM (nothing bound) if igks_workspace_size exceeds 64 MiB (about
 * 70 000 cells; fewer with lusgs_op 1, whose blocks take 128 bytes per cell in
 * FP64).  The array is one per GPU and shared: binding it to a
 * context overwrites what it held for an earlier context on that GPU, which
 * then gets IGKS_EINVAL from every call that needs its workspace until it
 * binds one again; calls of different contexts on the same GPU that
 * overlap in time race on it.  IGKS_EHIP if its device address cannot be
 * obtained. */
int igks_bind_static_workspace(igks_ctx *ctx);

/* Free stream (Mach, angle of attack in degrees, Reynolds number per unit
 * reference length, nu-tilde_inf / nu_inf): the state W_inf of the
 * free-stream boundary condition (Sec. 2.5) and of the impulsive start, in
 * the non-dimensionalisation above; nu-tilde_inf is the SA inflow value
 * (Sec. 2.3, Sec. 3.3).  nut_ratio < 0 runs laminar
 * (no SA equation).  Sets every cell to the free stream (impulsive start),
 * the iteration counter to 0 and the CFL to cfl_init.  IGKS_EINVAL if
 * Ma <= 0 or Re <= 0 or no workspace is bound. */
int igks_set_freestream(igks_ctx *ctx, double mach, double alpha_deg, double reynolds, double nut_ratio);

/* Run n nonlinear iterations of Sec. 2.2: the residual of Eq.16 (GKS face
 * fluxes Eq.4-14 with the Eq.23 time step, SA right-hand side Eq.27-30),
 * the CFL law Eq.24-25, the LU-SGS sweeps Eq.18-22 and Eq.31-32 and the
 * update Eq.17, plus the Eq.40 convergence measure.
 * Work is queued in chunks of opt.chunk iterations (one HIP graph launch
 * each) and the stream is synchronised at each chunk end.  *n_done (may be
 * NULL) = iterations committed (instance 0).  IGKS_ENONPHYS: an update
 * of some instance was rejected during this call (that instance is frozen
 * at its last committed iterate; the others went on), or every instance was
 * already frozen.  A frozen instance runs again after igks_set_state or
 * igks_set_freestream. */
int igks_iterate(igks_ctx *ctx, int32_t n, int32_t *n_done);

/* Scalars of the last iteration. */
int igks_get_residual(igks_ctx *ctx, igks_residual *out);

/* Per-iteration history of the last igks_iterate call: up to max entries
 * of 6 doubles each (res_l2, res_inf, cfl, dt_flux, eq40, sa_l2), oldest
 * first.  *n_out = entries written. */
int igks_get_history(igks_ctx *ctx, double *out, int32_t max, int32_t *n_out);

/* State, SoA host array W[k * n_cells + i], k = rho, rho U, rho V, rho E,
 * nu-tilde, in upload cell order. */
int igks_get_state(igks_ctx *ctx, double *W);
/* Set the state (same layout).  sc may be NULL (iteration 0, CFL =
 * cfl_init) or the scalars of a checkpoint.  IGKS_ENONPHYS (state left
 * unchanged) if a cell has rho <= 0, p <= 0 or a non-finite value. */
int igks_set_state(igks_ctx *ctx, const double *W, const igks_scalars *sc);
int igks_get_scalars(igks_ctx *ctx, igks_scalars *out);

/* Residual of the current state, SoA host array M[k * n_cells + i]:
 * k = 0..3 the flow residual M of Eq.16 (minus the sum of the outgoing
 * face fluxes times face length), k = 4 the SA right-hand side
 * Omega Sr + R of Eq.27.  Does not advance the iteration. */
int igks_compute_residual(igks_ctx *ctx, double *M);

/* Wall loads of the current state from the face fluxes through WALL
 * faces: lift and drag coefficients per unit span (reference
 * 0.5 rho_inf |V_inf|^2 times length 1) and, per wall face in the order the
 * WALL edges appear in the uploaded boundary list, Cp, Cf and the x of the
 * face midpoint.  Every pointer may be NULL; arrays hold n_wall_faces. */
int igks_get_wall_loads(igks_ctx *ctx, double *cl, double *cd, double *cf, double *cp, double *xw);

/* ---------------------------------------------------------------------
 * Batches: many independent instances (mesh + flow condition, uneven
 * sizes) iterated together, every kernel launch and every captured graph
 * covering all of them.  The single-instance calls above act on instance
 * 0 of a one-instance context; the calls below take an instance index.
 * Order: igks_batch_create -> igks_batch_mesh_upload for every instance ->
 * igks_workspace_size / igks_bind_workspace -> igks_batch_set_freestream
 * for every instance -> igks_iterate (all instances) -> getters.
 * An instance whose update is rejected (IGKS_ENONPHYS) is frozen at its
 * last good state while the others go on; igks_iterate then returns
 * IGKS_ENONPHYS and igks_batch_status tells which.  Residual and wall-load
 * calls on a frozen instance return IGKS_ENONPHYS.  igks_mesh_info reports
 * the totals over all instances (wavefronts: the largest count of any
 * instance, since wavefronts of different instances run together).
 * ------------------------------------------------------------------- */
int igks_batch_create(igks_ctx **out, const igks_options *opt, void *hip_stream, int32_t n_inst);
int igks_batch_mesh_upload(igks_ctx *ctx, int32_t inst, int32_t n_nodes, const double *xy, int32_t n_cells,
                           const int32_t *cell_ptr, const int32_t *cell_nodes, int32_t n_bfaces,
                           const int32_t *bface_nodes, const int32_t *bface_tag);
int igks_batch_mesh_info(const igks_ctx *ctx, int32_t inst, int32_t *n_cells, int32_t *n_faces,
                         int32_t *n_wall_faces);
int igks_batch_set_freestream(igks_ctx *ctx, int32_t inst, double mach, double alpha_deg, double reynolds,
                              double nut_ratio);
int igks_batch_get_residual(igks_ctx *ctx, int32_t inst, igks_residual *out);
int igks_batch_get_history(igks_ctx *ctx, int32_t inst, double *out, int32_t max, int32_t *n_out);
int igks_batch_get_state(igks_ctx *ctx, int32_t inst, double *W);
int igks_batch_set_state(igks_ctx *ctx, int32_t inst, const double *W, const igks_scalars *sc);
int igks_batch_get_scalars(igks_ctx *ctx, int32_t inst, igks_scalars *out);
int igks_batch_compute_residual(igks_ctx *ctx, int32_t inst, double *M);
int igks_batch_get_wall_loads(igks_ctx *ctx, int32_t inst, double *cl, double *cd, double *cf, double *cp,
                              double *xw);
/* *halted = 1 if the instance was frozen by a rejected update. */
int igks_batch_status(igks_ctx *ctx, int32_t inst, int32_t *halted);

/* Autotuner: runs `iters` iterations under each candidate launch schedule
 * (threads per block 64/128/256 for the prep, flux, gather and sweep
 * kernels, the face flux on one or two lanes per face; for the sweeps also
 * one workgroup for all wavefronts, tried while wavefronts average under
 * 16384 cells, and a wave per sweep block when there are sweep blocks),
 * keeps the fastest per kernel class, and then restores both
 * state buffers, the scalars and the history bitwise.  Block sizes and the
 * sweep schedule never change results; the one- and two-lane flux kernels
 * agree to rounding (the compiler fuses a few multiply-adds differently).
 * schedule6 (may be NULL) receives the
 * block sizes of the four classes, the sweep schedule (1: one launch per
 * wavefront, 2: one workgroup, 3: a wave per sweep block) and the lanes per
 * face of the flux (1 or 2;
 * before any tuning 2 below 32768 faces).  IGKS_EINVAL unless
 * 1 <= iters <= 1000; IGKS_ENONPHYS if an instance is frozen. */
int igks_autotune(igks_ctx *ctx, int32_t iters, int32_t *schedule6);
int igks_get_schedule(const igks_ctx *ctx, int32_t *schedule6);
/* Apply a schedule in the layout igks_get_schedule reports (for example one
 * an earlier igks_autotune found for the same mesh): block sizes 64, 128 or
 * 256 for the four classes, sweep 1, 2 or 3, lanes per face 1 or 2.  Needs a
 * bound workspace (binding picks the automatic schedule again).  Block
 * sizes and the sweep schedule never change results; the two flux kernels
 * agree to rounding.  IGKS_EINVAL for a value outside those sets, and for a
 * sweep schedule other than 3 in a context with two block passes and sweep
 * blocks. */
int igks_set_schedule(igks_ctx *ctx, const int32_t *schedule6);

/* Iterations per captured HIP graph and kernel launches per iteration of the
 * current schedule (before binding: of the schedule binding will pick).  A
 * graph holds at most 8192 launches: with one launch per wavefront and sweep
 * direction an iteration of a many-wavefront batch is thousands of launches
 * long, and the chunk is cut to fit; 0 iterations: no graphs (chunk 0).
 * Works without a GPU once every instance has a mesh. */
int igks_graph_chunk(const igks_ctx *ctx, int32_t *iters_per_graph, int32_t *launches_per_iteration);

/* With profiling on (igks_set_profiling(ctx, 1)) igks_iterate launches
 * directly, not through graphs, and times each kernel class with HIP events
 * on the context's stream; igks_get_kernel_times then gives the average ms
 * per iteration of: prep (with the Eq.23 time step), flux, gather, norms
 * (with the Eq.25 CFL), sweep_fwd (the forward steps of the wavefronts
 * after the first, and the last one's backward step), sweep_bwd (the other
 * backward steps, with the Eq.17 update; the commit belongs to no class).
 * 0 when profiling was off.  Each interval includes the cost of its two
 * events (a few microseconds). */
int igks_set_profiling(igks_ctx *ctx, int on);
int igks_get_kernel_times(igks_ctx *ctx, double *ms6);

/* Average ms per launch of one residual-phase kernel class (klass 0 prep
 * with the Eq.23 time step, 1 flux (Eq.4-14), 2 gather (Eq.16)), from reps
 * back-to-back launches between two HIP events on the context's stream,
 * preceded by the launches that produce its inputs from the current state.
 * These kernels write only derived arrays, so the state, the iteration
 * count and the next iteration are unchanged.  Synchronises the stream.
 * IGKS_EINVAL for a null pointer, klass outside 0..2, reps outside
 * 1..10000, or before the workspace and every free stream are set;
 * IGKS_ENONPHYS when an instance is frozen; IGKS_EHIP when a HIP call
 * fails. */
int igks_time_kernel(igks_ctx *ctx, int32_t klass, int32_t reps, double *ms);

#ifdef __cplusplus
}
#endif
#endif /* IGKS_H */

/*
 * slimdg.h -- C ABI of the MI355X (gfx950) nodal-P1 DG tracer operator on
 * extruded prism meshes.
 *
 * The operator (paper, section 1.1 tracer equation; section 2.2 stage
 * equations and their explicit variant; section 2.4 column systems):
 *
 *   dT/dt + div_h(u T) + d(w T)/dz = d/dz(kappa dT/dz)
 *
 * on a triangle mesh extruded into columns of linear prisms.  Per field and
 * prism there are six nodal values: the three top-face nodes then the three
 * bottom-face nodes (the node split of Algorithm 1).
 *
 *   rhs_3d                   L(T) = M^-1 R(T): volume quadrature plus upwind
 *                            lateral and horizontal interface fluxes, then the
 *                            element-local inverse of the block-diagonal mass
 *                            matrix (explicit variant of the stage equation).
 *   rk_stage                 one SSP-RK3 stage, Tout = a Tn + b (Ts + dt L(Ts)),
 *                            (a, b) = (0, 1), (3/4, 1/4), (1/3, 2/3).
 *   vertical_implicit_solve  (M - dt A) Tout = M T* per column, A the interior-
 *                            penalty vertical diffusion operator; block
 *                            tridiagonal with 6x6 blocks whose off-diagonal
 *                            blocks have the half-block sparsity of section 2.4;
 *                            computed in FP64 (in FP32 only in SDG_FP32 contexts).
 *   step                     three rk_stage calls then one vertical solve, or the
 *                            two-step split-IMEX step of sections 2 and 3 (vertically
 *                            implicit over dt/2, then explicit over dt).
 *   mass                     m_f = sum_K 1^T M_K T_K, FP64, per member and field.
 *   column_dv_solve          the matrix-free column solves of section 2.3 (D_vu of
 *                            the horizontal pressure gradient, D_vd of w).
 * Optional horizontal diffusion (section 1.1, Okubo diffusivity) joins the
 * explicit operator when sdg_params.okubo_scale > 0.
 *
 * Storage layout ("cell layout", the paper's section 2.1.1 grouping of
 * columns, here with 64 columns per cell -- one wavefront): columns keep the
 * caller's triangle order and are grouped in cells of 64 consecutive
 * columns; cell k is as deep as its deepest column, D_k.  The prism of column
 * c, layer l (0 = surface) lives in slot
 *
 *     cell_base[c / 64] + l * 64 + (c % 64),   cell_base[k] = 64 * sum_{j<k} D_j,
 *
 * and every nodal array is [component][node 0..5][slot] with n_slots slots
 * (sdg_layout.n_slots).  Slots of padding (l >= nlayers[c], or columns past
 * the last triangle) of caller arrays are never written, and their values
 * never reach a result (the column walk copies whole 64-slot rows of a cell,
 * padding included, and discards the padding lanes).  sdg_prism_slots()
 * returns the slot of every prism in natural order (column by column, layers
 * top to bottom) so callers can scatter and gather.
 *
 * Ownership: the library never allocates device memory.  The caller provides
 * one workspace buffer (sdg_layout.workspace_bytes) at mesh upload; state,
 * velocity, diffusivity and outputs are caller-owned device buffers.  Device
 * pointers given to sdg_set_velocity / sdg_set_diffusivity / sdg_set_fields
 * are borrowed until replaced; the caller keeps them alive.
 *
 * Execution: every call enqueues on the stream given to sdg_create (NULL =
 * the default stream) and returns without synchronising, except
 * sdg_mesh_upload, sdg_mass and sdg_sync.  Argument, mesh and workspace
 * errors are reported synchronously; asynchronous kernel errors surface at
 * sdg_sync or sdg_mass.  No C++ exception crosses the ABI.  A context is used
 * by one host thread at a time.
 *
 * Precision (the paper's section 4.1 weighs FP64 against FP32 throughput):
 *   SDG_FP64                  state, velocity, geometry, fluxes and the
 *                             column solve in double;
 *   SDG_FP32_STATE_FP64_SOLVE state, velocity, geometry and fluxes in float,
 *                             the column solve in double (the precision form);
 *   SDG_FP32                  everything in float, the column solve included.
 * kappa, dt and the mass sums are double in every form.
 */
#ifndef SLIMDG_H
#define SLIMDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SDG_ABI_VERSION 8
#define SDG_CELL_COLUMNS 64
#define SDG_MAX_FIELDS 4

typedef enum {
  SDG_OK = 0,
  SDG_E_ARG = -1,         /* bad argument (null pointer, out-of-range value) */
  SDG_E_MESH = -2,        /* mesh description fails validation */
  SDG_E_HIP = -3,         /* HIP runtime error (message has the HIP string) */
  SDG_E_STATE = -4,       /* call made before the state it needs was set */
  SDG_E_UNSUPPORTED = -5, /* valid request the library does not support */
  SDG_E_NUMERIC = -6,     /* non-finite values found (check_finite) */
  SDG_E_WORKSPACE = -7    /* workspace too small or misaligned */
} sdg_status;

typedef enum {
  SDG_FP64 = 0,
  SDG_FP32 = 1,
  SDG_FP32_STATE_FP64_SOLVE = 2
} sdg_precision;

/* The two column systems of the matrix-free solvers (sdg_column_dv_solve). */
typedef enum {
  SDG_DV_VU = 0,   /* D_vu: horizontal pressure gradient system, solved from the surface down */
  SDG_DV_VD = 1    /* D_vd: vertical velocity system, solved from the seabed up */
} sdg_dv_kind;
#define SDG_DV_MAX_COMP 4

/* Time step of sdg_step (and of a captured step). */
typedef enum {
  SDG_SCHEME_SSPRK3_LIE = 0,  /* three SSP-RK3 stages of the explicit operator, then
                                 one backward-Euler vertical solve over dt */
  SDG_SCHEME_SPLIT_IMEX = 1   /* the two-step split-IMEX step of sections 2 and 3:
                                 vertically implicit over dt/2, then explicit over dt */
} sdg_time_scheme;

typedef struct sdg_ctx sdg_ctx; /* opaque */

/* Mesh description.  All pointers are HOST pointers, read during the call
 * (query, slots, upload) and not retained. */
typedef struct {
  int32_t n_members;              /* >= 1; members are disjoint meshes */
  int32_t n_tri;                  /* columns, all members concatenated */
  int32_t n_vert;
  const int32_t* member_tri_off;  /* [n_members+1] column offsets; NULL = one member */
  const double* vxy;              /* [n_vert][2] vertex coordinates [m] */
  const int32_t* tri;             /* [n_tri][3] vertex ids, counter-clockwise */
  const int32_t* nbr;             /* [n_tri][3]; edge k = (tri[k] -> tri[(k+1)%3]);
                                     neighbour column or -1 (open boundary) */
  const int32_t* nlayers;         /* [n_tri], >= 1 */
  const double* zlev;             /* per column (nlayers+1) levels x 3 vertex heights,
                                     top level first, columns concatenated [m] */
  int32_t n_fields;               /* 1 .. SDG_MAX_FIELDS */
  int32_t precision;              /* sdg_precision */
} sdg_mesh_desc;

typedef struct {
  int64_t n_prisms;        /* live prisms = sum(nlayers) */
  int64_t n_slots;         /* slots per nodal array (>= n_prisms) */
  int32_t n_cells;
  int32_t max_layers;
  int32_t n_fields;
  int32_t state_elem_bytes;   /* 8 (FP64) or 4 */
  size_t state_bytes;         /* bytes of one [n_fields][6][n_slots] state array */
  size_t velocity_bytes;      /* bytes of one [3][6][n_slots] velocity array */
  size_t workspace_bytes;     /* device workspace for sdg_mesh_upload */
} sdg_layout;

typedef struct {
  double dt;               /* time step [s], > 0 */
  double penalty_eta;      /* interior-penalty factor (4 if <= 0 is given) */
  const double* t_ext;     /* HOST [n_fields] exterior values on open boundaries; NULL = 0 */
  int32_t w_is_zero;       /* 1: the vertical velocity component is not read */
  int32_t check_finite;    /* 1: sdg_step checks the state after its last step */
  int32_t time_scheme;     /* sdg_time_scheme of sdg_step (0 = SDG_SCHEME_SSPRK3_LIE) */
  double okubo_scale;      /* >= 0; 0 = no horizontal diffusion.  Otherwise the explicit
                              operator also holds the horizontal diffusion of section 1.1
                              (Okubo diffusivity): along the layers, symmetric interior
                              penalty on the lateral faces (penalty_eta), zero flux at open
                              boundaries and walls, per column
                              kh = okubo_scale * 2.055e-4 * sqrt(J_h)^1.15 m^2/s */
} sdg_params;

int sdg_abi_version(void);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char* sdg_last_error(void);

/* Validate a mesh description and report sizes: columns grouped in cells of
 * 64, each as deep as its deepest column (the paper's section 2.1.1 cell
 * structure).  Host only; no GPU needed.  SDG_E_ARG / SDG_E_MESH with a
 * message on failure.  Limits: 1 to 65,535 layers per column (SDG_E_MESH
 * beyond); at most 89,478,485 slots, since the kernels address one field's
 * six node rows with 32-bit byte offsets (SDG_E_UNSUPPORTED beyond). */
sdg_status sdg_query_layout(const sdg_mesh_desc* mesh, sdg_layout* out);

/* Slot of each prism in natural order: host_slots[off[c] + l] for column c,
 * layer l, where off is the prefix sum of nlayers.  host_slots has
 * n_prisms entries.  Host only. */
sdg_status sdg_prism_slots(const sdg_mesh_desc* mesh, int64_t* host_slots);

/* Create a context on HIP device `device`; `hip_stream` (a hipStream_t) is
 * borrowed, NULL = default stream. */
sdg_status sdg_create(sdg_ctx** out, int device, void* hip_stream);
sdg_status sdg_destroy(sdg_ctx* ctx);

/* Validate, lay out and copy the mesh into the caller's device workspace
 * (>= workspace_bytes, 256-byte aligned), then compute the per-column
 * geometry on the device (the extruded triangle mesh of section 1; J_h of
 * the 2D mass matrix of section 2.3).  Synchronises the stream.  Any
 * previously set params / velocity / diffusivity / fields are forgotten
 * (params hold per-field exterior values and, with okubo_scale > 0, a
 * per-column diffusivity of the old mesh): set them again. */
sdg_status sdg_mesh_upload(sdg_ctx* ctx, const sdg_mesh_desc* mesh, void* dev_workspace,
                           size_t workspace_bytes);

/* Time step, interior-penalty factor of the vertical diffusion (section 2.4
 * system) and exterior values of the open boundaries.  Host struct, copied. */
sdg_status sdg_set_params(sdg_ctx* ctx, const sdg_params* params);

/* Nodal velocity [3][6][n_slots] (u, v, w) in the state precision: the
 * transport velocity of the section 1.1 tracer equation. */
sdg_status sdg_set_velocity(sdg_ctx* ctx, const void* dev_uvw);

/* Vertical diffusivity per layer index, [max_layers] doubles [m^2/s] (the
 * kappa of the section 1.1 tracer equation, constant in each layer). */
sdg_status sdg_set_diffusivity(sdg_ctx* ctx, const double* dev_kappa);

/* State advanced in place by sdg_step, [n_fields][6][n_slots]: nodal tracer
 * values, top three nodes then bottom three (the Algorithm 1 node split). */
sdg_status sdg_set_fields(sdg_ctx* ctx, void* dev_state);

/* dev_L = M^-1 R(dev_T): the horizontal flux operator of section 2.2 in its
 * explicit form (volume term plus upwind lateral and horizontal interface
 * fluxes, block-diagonal mass matrix), plus the horizontal diffusion when
 * okubo_scale > 0.  Needs velocity and params.  dev_L must not alias dev_T. */
sdg_status sdg_rhs_3d(sdg_ctx* ctx, const void* dev_T, void* dev_L);

/* dev_Tout = a dev_Tn + b (dev_Ts + dt L(dev_Ts)) for stage 0, 1, 2 of
 * SSP-RK3 in Shu-Osher form, (a, b) = (0, 1), (3/4, 1/4), (1/3, 2/3): the
 * explicit stage update of section 2.2.  Stage 0 does not read dev_Tn.
 * dev_Tout must not alias dev_Ts or dev_Tn. */
sdg_status sdg_rk_stage(sdg_ctx* ctx, int stage, const void* dev_Tn, const void* dev_Ts,
                        void* dev_Tout);

/* (M - dt A) dev_Tout = M dev_Tstar per column: the implicit vertical
 * diffusion system of sections 1.2 and 2.2, block tridiagonal with the
 * sparsity of section 2.4, solved in FP64 (FP32 in SDG_FP32) by block
 * Thomas.  Needs diffusivity and params.  dev_Tout may alias dev_Tstar. */
sdg_status sdg_vertical_implicit_solve(sdg_ctx* ctx, const void* dev_Tstar, void* dev_Tout);

/* n_steps time steps of the set fields, in place, using two stage buffers
 * inside the workspace.  The scheme is sdg_params.time_scheme:
 *   SDG_SCHEME_SSPRK3_LIE: 3 rk_stage + vertical_implicit_solve, the
 *     horizontally explicit, vertically implicit splitting of section 1.2
 *     taken as Lie splitting (three explicit stages, then one implicit
 *     vertical step over dt);
 *   SDG_SCHEME_SPLIT_IMEX: the two-step split-IMEX step (sections 2 and 3,
 *     step equation of section 3.2 with M_0 = M_1 = M):
 *       M x_h = M x_0 + dt/2 (R(x_0) + A x_h)   (vertically implicit, dt/2)
 *       M x_1 = M x_0 + dt (R(x_h) + A x_h)     (explicit, dt)
 *     with R the advective residual and A the vertical diffusion operator.
 *     The second step takes dt M^-1 A x_h = 2 (x_h - y), y the explicit
 *     half step x_0 + dt/2 M^-1 R(x_0), from the first step's own system.
 * Deterministic: the same inputs and launch shape give bitwise equal states. */
sdg_status sdg_step(sdg_ctx* ctx, int n_steps);

/* host_mass[m * n_fields + f] = sum over member m's prisms of 1^T M T_f, in
 * FP64 with a fixed summation order (the conserved quantity of the section
 * 1.1 tracer equation).  Synchronises the stream. */
sdg_status sdg_mass(sdg_ctx* ctx, const void* dev_T, double* host_mass);

/* For callers that cannot allocate device memory at the call (code under
 * stream capture, tight serving loops, harnesses that forbid it): sdg_mass
 * with its partial sums kept in a static device array of the library instead
 * of the mesh workspace.  Same arguments, results (bitwise: the same kernels
 * in the same order) and synchronisation as sdg_mass; it calls no device or
 * host allocator.  Limit: n_fields x (column slots + members) <= 8,388,608
 * doubles (64 MiB; column slots = 64 x cells), else SDG_E_WORKSPACE.  Each
 * device holds one such array from the first sdg_create on it until the
 * process ends, shared by every context on that device: calls that overlap
 * on one device (two streams, two threads) race on it. */
sdg_status sdg_mass_noalloc(sdg_ctx* ctx, const void* dev_T, double* host_mass);

/* Launch shape of the fused stage kernel (the paper's section 4.1 shows
 * throughput depending on the column block shape; section 2.1.2 sizes a
 * cell's block by its deepest column; here the library measures it).
 * Results do not depend on it (bitwise).
 * tile_layers: 1, 2 or 4 = layers per workgroup of 64 columns, one thread per
 *   prism (default 2); 8, 12, 16 or 32 = one wavefront walks that many layers of
 *   a cell, prefetching the next layer into LDS while computing the current;
 *   0 = a column walk whose segmentation depends on the cell's depth D, by
 *   bucket b = 0..5 for D in 1-8, 9-16, 17-24, 25-32, 33-48, > 48:
 *   walk_layers[b] = L in 8..64 cuts the cell into walks of L layers (the last
 *   one shorter), L in -64..-8 into ceil(D / |L|) walks of balanced lengths
 *   (e.g. D = 30, L = -12: 10 + 10 + 10);
 * xcd_remap: 1 = give each XCD one contiguous range of tiles (default);
 * persistent: 1 = launch only as many workgroups as the device holds at once,
 *   each walking tiles with a stride (default 0: one workgroup per tile).
 * walk_layers is read only with tile_layers = 0 and reported as zeros
 * otherwise; setting it needs an uploaded mesh (the table is built for it and
 * synchronises the stream), and a mesh upload returns to 2-layer tiles.
 * The adjoint stages use tile_layers and xcd_remap of a one-thread shape;
 * under a walk shape they use 2-layer tiles with the XCD remap.  They ignore
 * persistent. */
#define SDG_DEPTH_BUCKETS 6
typedef struct {
  int32_t tile_layers;
  int32_t xcd_remap;
  int32_t persistent;
  int32_t walk_layers[SDG_DEPTH_BUCKETS];
} sdg_tuning;

sdg_status sdg_get_tuning(sdg_ctx* ctx, sdg_tuning* out);
sdg_status sdg_set_tuning(sdg_ctx* ctx, const sdg_tuning* tuning);

/* Time every stage-kernel launch shape (7 tile heights x XCD remap off/on x
 * persistent off/on), each over reps repetitions of the three stages of a
 * step on the set fields and velocity (the fields are only read; the stages
 * write the workspace stage buffers), and keep the fastest.  When a column
 * walk wins, also choose a segmentation per depth bucket (walk_layers, fixed
 * 8/12/16/32/64 or balanced 8/12/16/24/32), timing each bucket's tiles alone
 * with that walk's XCD remap and persistent setting, and keep the per-bucket
 * table (tile_layers = 0) if all of it is faster than the uniform walk.
 * Synchronises the stream.  `chosen` may be NULL. */
sdg_status sdg_autotune(sdg_ctx* ctx, int reps, sdg_tuning* chosen);

/* Capture one sdg_step (three stages and the column solve, on the set fields)
 * into a HIP graph (section 3.3 of the paper discusses launch latency of
 * short kernels); replaces any previous capture.  Waits for the context
 * stream first.  Any later set_* / set_tuning / mesh_upload call invalidates
 * the capture (sdg_graph_launch then returns SDG_E_STATE). */
sdg_status sdg_graph_capture_step(sdg_ctx* ctx);

/* Replay the captured step n_steps times on the context stream. */
sdg_status sdg_graph_launch(sdg_ctx* ctx, int n_steps);

/* Y = M X (inverse = 0) or Y = M^-1 X (inverse != 0), prism by prism (the
 * block-diagonal DG mass matrix of section 2.2), for a [n_fields][6][n_slots]
 * array in the state precision.  Y may alias X. */
sdg_status sdg_apply_mass(sdg_ctx* ctx, const void* dev_X, void* dev_Y, int inverse);

/* host_out[m * n_fields + f] = sum over member m's prisms of X_f^T M Y_f
 * (FP64, fixed summation order; the M inner product the adjoint uses).
 * Synchronises the stream. */
sdg_status sdg_m_dot(sdg_ctx* ctx, const void* dev_X, const void* dev_Y, double* host_out);

/* Reverse of one sdg_step (FP64 contexts with SDG_SCHEME_SSPRK3_LIE only,
 * SDG_E_UNSUPPORTED otherwise): not in the paper; it is the
 * exact transpose of the section 2.2 stage equations and of the section 2.4
 * column system, in the variable Z = M^-1 lambda where lambda = dJ/dx is the
 * adjoint state:
 *   mu     = (M - dt A^T)^-1 M Z^{n+1}                     (transposed column solve)
 *   dkappa[l] += dt mu^T (dA/dkappa_l) x^{n+1}              (if dev_dkappa != NULL)
 *   Z^n    = reverse SSP-RK3 stages with M^-1 R_lin^T       (R_lin: the advective
 *            residual without the exterior inflow values, plus the
 *            horizontal diffusion D when okubo_scale > 0, D^T = D)
 * so that lambda^n = M Z^n.  dev_z_next, dev_z_out: [n_fields][6][n_slots]
 * doubles (may alias); dev_x_next: the state after the forward step being
 * reversed, which with dev_dkappa must not be dev_z_out (SDG_E_ARG);
 * dev_dkappa: [max_layers] doubles, accumulated.  Uses the workspace stage
 * buffers. */
sdg_status sdg_step_adjoint(sdg_ctx* ctx, const void* dev_z_next, void* dev_z_out, const void* dev_x_next,
                            double* dev_dkappa);

/* Matrix-free column solve of section 2.3 ("Matrix-free solvers"): in every
 * column, D x = F with D the block matrix the paper prints for a 3-layer
 * column, continued to the column's depth -- 1/2 times 3x3 blocks that are
 * multiples of M_h = J_h/24 [2 1 1; 1 2 1; 1 1 2]:
 *   SDG_DV_VU (D_vu): per layer l, top rows  2M x_bot(l-1) - M x_top(l) - M x_bot(l),
 *                                  bottom rows M x_top(l) - M x_bot(l);
 *             the discrete dx/dz = f with x = 0 at the surface, solved top-down;
 *   SDG_DV_VD (D_vd): per layer l, top rows    M x_top(l) - M x_bot(l),
 *                                  bottom rows M x_top(l) + M x_bot(l) - 2M x_top(l+1);
 *             the discrete dx/dz = f with x = 0 at the seabed, solved bottom-up.
 * dev_F, dev_x: [n_comp][6][n_slots] in the state precision (cell layout; per
 * prism the three top-face nodes, then the three bottom-face nodes), device
 * pointers owned by the caller; dev_x may equal dev_F (in place).  n_comp in
 * 1..SDG_DV_MAX_COMP (e.g. 2 for the horizontal pressure gradient, 1 for w).
 * Arithmetic in double except in SDG_FP32 contexts.  Padding slots are
 * neither read nor written.  Needs an uploaded mesh (SDG_E_STATE otherwise);
 * an unknown kind, n_comp out of range or a NULL pointer gives SDG_E_ARG.
 * Enqueued on the context stream; does not synchronise. */
sdg_status sdg_column_dv_solve(sdg_ctx* ctx, int kind, int n_comp, const void* dev_F, void* dev_x);

/* Reverse of one split-IMEX sdg_step (FP64 contexts with
 * SDG_SCHEME_SPLIT_IMEX only, SDG_E_UNSUPPORTED otherwise): not in the paper;
 * the exact transpose of the two-step scheme of sections 2 and 3 in the same
 * variable Z = M^-1 lambda as sdg_step_adjoint, with h = dt/2 and
 * L~ = M^-1 (R_lin + D)^T:
 *   w      = 2 (Z^{n+1} + h L~ Z^{n+1})
 *   mu'    = (M - h A^T)^-1 M w                      (transposed column solve)
 *   Z^n    = mu' + h L~ mu' + Z^{n+1} - w
 *   dkappa[l] += h mu'^T (dA/dkappa_l) x_h           (if dev_dkappa != NULL)
 * with x_h the vertically implicit half step from dev_x_prev, the state
 * BEFORE the forward step being reversed (rebuilt here when dkappa is asked
 * for).  dev_z_next, dev_z_out, dev_x_prev: [n_fields][6][n_slots] doubles;
 * dev_z_out must not alias dev_z_next or dev_x_prev; dev_dkappa: [max_layers]
 * doubles, accumulated.  Uses the workspace stage buffers. */
sdg_status sdg_step_adjoint_imex(sdg_ctx* ctx, const void* dev_z_next, void* dev_z_out, const void* dev_x_prev,
                                 double* dev_dkappa);

/* One split-IMEX step of the set fields, as sdg_step(ctx, 1) (contexts with
 * SDG_SCHEME_SPLIT_IMEX only, SDG_E_UNSUPPORTED otherwise), whose vertically
 * implicit half-step state x_h (the section 3 two-step scheme's first step)
 * is left in dev_x_half ([n_fields][6][n_slots] in the state precision)
 * rather than in the workspace: the state the reverse step pairs with the
 * kappa gradient.  dev_x_half must not be the set fields (SDG_E_ARG).
 * Enqueued on the context stream; does not synchronise (and, unlike
 * sdg_step, never runs the check_finite test). */
sdg_status sdg_step_keep_half(sdg_ctx* ctx, void* dev_x_half);

/* sdg_step_adjoint_imex given the reversed step's x_h (as left by
 * sdg_step_keep_half) instead of the state before it, so that x_h is not
 * rebuilt: the same result with one explicit half step and one column solve
 * fewer.  dev_z_out must not alias dev_z_next or dev_x_half. */
sdg_status sdg_step_adjoint_imex_half(sdg_ctx* ctx, const void* dev_z_next, void* dev_z_out, const void* dev_x_half,
                                      double* dev_dkappa);

/* Wait for the context's stream and report any asynchronous HIP error. */
sdg_status sdg_sync(sdg_ctx* ctx);

/* Measurement aid, not part of the method: the device's streaming bandwidth
 * with 16-byte accesses per lane, the ceiling against which the kernels'
 * algorithmic bandwidth is read besides the HBM peak.
 *   SDG_PROBE_READ:  sums dev_src (bytes), one double per workgroup to dev_dst;
 *   SDG_PROBE_WRITE: fills dev_dst (bytes) with 1.0;
 *   SDG_PROBE_COPY:  copies dev_src to dev_dst (bytes each).
 * Device pointers owned by the caller, 16-byte aligned; bytes a positive
 * multiple of 16; workgroups (256 threads each) >= 1 (for READ, dev_dst holds
 * at least that many doubles).  Enqueued on hip_stream (NULL: the default
 * stream), no synchronisation, no context needed; SDG_E_ARG on a bad
 * argument, SDG_E_HIP if the launch fails. */
typedef enum { SDG_PROBE_READ = 0, SDG_PROBE_WRITE = 1, SDG_PROBE_COPY = 2 } sdg_probe_kind;
sdg_status sdg_stream_probe(int kind, const void* dev_src, void* dev_dst, size_t bytes, int workgroups,
                            void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* SLIMDG_H */

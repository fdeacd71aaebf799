/*
 * lbm_ib.h - C interface of the MI355X (gfx950) immersed-boundary lattice
 * Boltzmann library.
 *
 * One call advances a D3Q27 lattice Boltzmann fluid, in a local frame that may
 * accelerate and rotate, coupled two-way to a skinned surface by the immersed
 * boundary method. This is the fluid-structure interaction module of the
 * paper (Sec. III-B, "GPU-accelerated localized fluid-structure
 * interaction"): Eq. (2) solved by a lattice Boltzmann method, the
 * fictitious frame force of Eq. (3), open domain faces by non-equilibrium
 * extrapolation (Sec. III-B, Simulation), a uniformly sampled surface
 * (Sec. III-B, Simulation) skinned by linear blend skinning (Sec. III-A) and
 * the fluid's force on the body, which enters Eq. (1) as the external
 * generalized force.
 *
 * Method as implemented (the paper leaves these details open):
 *   lattice      D3Q27, c_i in {-1,0,1}^3, i = (cx+1) + 3(cy+1) + 9(cz+1)
 *   collision    BGK, relaxation time tau > 1/2, second-order equilibrium;
 *                or two-relaxation-time (LBM_COLLIDE_TRT)
 *   forcing      Guo: velocity u = (m + F/2)/rho; F = g + rho a_ni(x, u),
 *                a_ni from Eq. (3), solved exactly for the Coriolis term
 *   streaming    pull; each axis periodic or open
 *   open faces   non-equilibrium extrapolation from the inward neighbour
 *   IB           Peskin 4-point kernel, explicit direct forcing
 *                F_k = alpha 2 rho_k (U_k - U*_k), optional multi-direct
 *                forcing passes, spreading g(x) = sum_k F_k dV_k delta(x - X_k);
 *                or the implicit velocity correction (LBM_IB_IMPLICIT)
 *
 * Conventions shared by every entry point:
 *   - Every pointer is a DEVICE pointer allocated and owned by the caller,
 *     unless its comment says [host]. The library never allocates or frees
 *     device memory and keeps no pointer after lbm_destroy.
 *   - Grids are x-fastest: cell (x, y, z) has index x + nx (y + ny z). A field
 *     with components is component-major: [comp][nz][ny][nx].
 *   - Populations in the caller's canonical layout are pre-collision values
 *     f_i(x, n), float32, [27][nz][ny][nx].
 *   - All device work is enqueued on the context's HIP stream. A call returns
 *     after enqueueing; it synchronizes only where it says so.
 *   - Every call returns an lbm_status; nothing is thrown across the boundary.
 *     Arguments are validated on the host before any device work is queued;
 *     on an error nothing is queued.
 */
#ifndef LBM_IB_H
#define LBM_IB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBM_OK = 0,
  LBM_ERR_ARG = -1,          /* bad argument: null pointer, size, tau <= 1/2, ... */
  LBM_ERR_DEVICE = -2,       /* a HIP runtime call or kernel launch failed */
  LBM_ERR_UNSTABLE = -3,     /* device guard: non-finite value or |u| >= 0.4 seen */
  LBM_ERR_MARKER_RANGE = -4, /* a marker came within 2 cells (3 on the high side) of an open face */
  LBM_ERR_CAPACITY = -5,     /* more markers than max_markers or active tiles than capacity */
  LBM_ERR_UNSUPPORTED = -6   /* valid request this build does not implement */
} lbm_status;

/* Face conditions. Each axis is periodic on both faces, or open on both (each
 * face VELOCITY or OUTFLOW): x by bc_lo (x = 0) and bc_hi (x = nx-1), y and z
 * by bc_y[2] and bc_z[2] (low, high). An open face takes the non-equilibrium
 * extrapolation of Sec. III-B from the node one step inward along every open
 * axis the boundary node lies on (a diagonal neighbour on edges and corners);
 * a node's velocity comes from its first velocity face in the order x low,
 * x high, y low, y high, z low, z high (u_lo of the frame, u_hi for x high),
 * or from its inward neighbour when it lies on outflow faces only. */
enum { LBM_BC_PERIODIC = 0, LBM_BC_VELOCITY = 1, LBM_BC_OUTFLOW = 2 };

/* Population storage. Every format stores h_i = f_i - w_i, the offset from
 * the rest equilibrium: F32 as float, F16 and BF16 rounded to nearest even.
 * The collision works on h (rho - 1 = sum h, momentum = sum h c), so the
 * rounding of stored values scales with |h|, not with w_i; all arithmetic
 * and all immersed-boundary sums stay in float32. The stored layout of a
 * state (lbm_state_save) holds, at cell x, h_i(x + c_i) of the post-collision
 * populations, arranged as lbm_params.layout says (LBM_LAYOUT_*). */
enum { LBM_STORE_F32 = 0, LBM_STORE_F16 = 1, LBM_STORE_BF16 = 2 };

/* Immersed-boundary schemes (lbm_params.ib_scheme).
 * DIRECT: explicit direct forcing F_k = alpha 2 rho_k (U_k - U*_k), then
 *   mdf_iters - 1 multi-direct-forcing passes, each adding
 *   alpha 2 rho_k (U_k - U_k^interp) with U_k^interp the velocity including
 *   the force so far.
 * IMPLICIT: the implicit velocity correction (the implicit immersed boundary
 *   the paper cites in its Introduction: Wu and Shu's velocity correction). The
 *   marker forces G_k = F_k dV_k make the velocity with their spread force,
 *   interpolated back, equal the body velocity at every marker:
 *     S G = (I + [omega]x) (U - U*),  S = interp . 1/(2 rho) . spread,
 *   (omega x: the Coriolis term of Eq. (3), which the fluid velocity solves
 *   for exactly), one symmetric positive semidefinite system per component,
 *   taken by mdf_iters steps of conjugate gradients from G = 0 with the
 *   diagonal preconditioner 2 rho_k; alpha = 0 once p.Sp is not positive,
 *   beta = 0 once r.z is 0. Each step costs one spread and one
 *   interpolation, like a multi-direct-forcing pass; ib_alpha is not used.
 *   Supported by lbm_ib_step and by the batched per-phase driver when every
 *   environment of the batch uses it; the persistent driver and the adjoint
 *   entry points return LBM_ERR_UNSUPPORTED. */
enum { LBM_IB_DIRECT = 0, LBM_IB_IMPLICIT = 1 };

/* Collisions (lbm_params.collision).
 * BGK: f*_i = f_i - (f_i - f^eq_i)/tau + (1 - 1/(2 tau)) S_i, S_i = Guo's
 *   source w_i [3 (c_i - u) + 9 (c_i.u) c_i].F.
 * TRT: the two-relaxation-time collision, the smallest member of the
 *   multiple-relaxation-time family the paper's solver family admits: with
 *   x+_i and x-_i the parts of x even and odd in c ((x_i +- x_opp(i))/2),
 *     f*_i = f_i - w+ (f+_i - f^eq+_i) - w- (f-_i - f^eq-_i)
 *            + (1 - w+/2) S+_i + (1 - w-/2) S-_i,
 *   w+ = 1/tau (the viscosity stays (tau - 1/2)/3) and w- = 1/tau- with
 *   (tau - 1/2)(tau- - 1/2) = trt_lambda (> 0; 3/16 is the usual choice).
 *   Open faces extrapolate as before, the non-equilibrium part's even and
 *   odd halves relaxing at w+ and w-. Supported by lbm_ib_step and the
 *   batched entry points; the adjoint entry points return
 *   LBM_ERR_UNSUPPORTED. */
enum { LBM_COLLIDE_BGK = 0, LBM_COLLIDE_TRT = 1 };

/* Immersed-wall condition (lbm_params.wall_mode).
 * NO_SLIP: direct forcing drives the marker velocity to the body's,
 *   F_k = alpha 2 rho_k (U_k - U*_k).
 * SLIP: the Neumann (slipping) condition the paper applies on the immersed
 *   solid (Sec. III-B, Formulation): only flow through the wall is stopped,
 *   F_k = alpha 2 rho_k ((U_k - U*_k).n_k) n_k, with n_k the marker's rest
 *   normal (lbm_markers.nrest) turned by its bones' blended rotations and
 *   scaled to unit length; multi-direct-forcing passes project the same way.
 *   With LBM_IB_IMPLICIT the unknown is one normal force gamma_k n_k per
 *   marker, (N^T S N) gamma = N^T (U - U*), in frames that do not rotate (a
 *   rotating frame returns LBM_ERR_UNSUPPORTED: the Coriolis solve makes
 *   that system unsymmetric). Needs nrest; the adjoint returns
 *   LBM_ERR_UNSUPPORTED. */
enum { LBM_WALL_NO_SLIP = 0, LBM_WALL_SLIP = 1 };

/* Stored population layout (lbm_params.layout). Population i of cell
 * (x, y, z) sits at element (z ny + y) rs + i ps + x of a population buffer;
 * lbm_population_strides gives ps and rs.
 * PLANES: [27][nz][ny][nx], each population a plane of its own
 *   (ps = plane stride, rs = nx).
 * ROWS: [nz][ny][27][nx], the 27 populations of one (y, z) row side by side
 *   (ps = nx, rs = 27 nx). A step then touches 9 source rows and 1 target
 *   row per cell instead of 27 + 27 planes, which streams faster from HBM.
 * AUTO: ROWS when nx is a multiple of 32 (every row starts on a 128-byte
 *   line), else PLANES. */
enum { LBM_LAYOUT_AUTO = 0, LBM_LAYOUT_PLANES = 1, LBM_LAYOUT_ROWS = 2 };

typedef struct lbm_ctx lbm_ctx;

/* [host] Problem description. */
typedef struct {
  int32_t nx, ny, nz;        /* lattice size, each >= 4 */
  int32_t bc_lo, bc_hi;      /* LBM_BC_* for the two x faces */
  int32_t storage;           /* LBM_STORE_* */
  int32_t max_markers;       /* capacity of the marker arrays, >= 0 */
  int32_t max_bones;         /* capacity of a pose array, >= 1 */
  int32_t mdf_iters;         /* IB passes, 1..16: direct-forcing passes (1 = explicit), or CG steps */
  int32_t max_active_tiles;  /* 8x8x8 tiles that may carry IB force; 0 = automatic */
  int32_t block_x, block_y;  /* collide block: block_x (a multiple of 64) by block_y cells, or block_x
                                consecutive cells of the x-fastest order when block_y = -1;
                                0, 0 = default (256 consecutive cells with LBM_LAYOUT_ROWS,
                                else 128 x 4 or 64 x 8) */
  int32_t with_adjoint;      /* nonzero: workspace also holds the adjoint buffers */
  double tau;                /* BGK relaxation time, > 1/2 (nu = (tau - 1/2)/3) */
  double ib_alpha;           /* direct-forcing gain, > 0 (1 = full correction) */
  int32_t bc_y[2], bc_z[2];  /* LBM_BC_* for the y and z faces; zeros = periodic */
  int32_t ib_scheme;         /* LBM_IB_*; 0 = direct forcing */
  int32_t collision;         /* LBM_COLLIDE_*; 0 = BGK */
  double trt_lambda;         /* TRT: (tau - 1/2)(tau- - 1/2) > 0; unused by BGK */
  int32_t wall_mode;         /* LBM_WALL_*; 0 = no-slip */
  int32_t layout;            /* LBM_LAYOUT_*; 0 = automatic */
  int32_t ib_workgroups;     /* direct forcing: > 0 runs the immersed-boundary phases in that many
                                workgroups beside the collide, one launch per step (see lbm_ib_step),
                                held to what the device runs at once (about two per compute unit);
                                0 or -1 runs them before the collide in launches of their own */
} lbm_params;

/* [host] Frame of one step (Eq. (3)). acc = linear acceleration of the frame
 * origin, omega = angular velocity, alpha = angular acceleration (vectors in
 * frame coordinates); x' = x - origin. u_lo / u_hi = velocity prescribed on
 * the x = 0 / x = nx-1 face when that face is LBM_BC_VELOCITY; y and z
 * velocity faces take u_lo (the far field of the local moving domain). */
typedef struct {
  double acc[3], omega[3], alpha[3], origin[3], u_lo[3], u_hi[3];
} lbm_frame;

/* Surface markers (Sec. III-B: uniformly sampled surface; Sec. III-A: linear
 * blend skinning). Structure-of-arrays, n entries each.
 *   xrest  [3][n] rest-pose position          (in)
 *   bone   [2][n] the two bones of each marker (in; 0 <= bone < nbones)
 *   weight [2][n] their blend weights          (in)
 *   dv     [n]    marker volume dV_k           (in)
 *   X, U   [3][n] position and velocity        (out, written by each step)
 *   F      [3][n] direct-forcing force density of the last step (out)
 *   nrest  [3][n] rest-pose outward unit normals (in; slip walls only, may be
 *                 NULL otherwise)
 * A bone pose is 24 float32: R (3x3 row-major), t, dR/dt (3x3 row-major), dt/dt;
 * X_k = sum_b w_kb (R_b xrest_k + t_b), U_k = sum_b w_kb (dR_b xrest_k + dt_b). */
typedef struct {
  int32_t n;
  int32_t nbones;
  const float *xrest;
  const int32_t *bone;
  const float *weight;
  const float *dv;
  float *X;
  float *U;
  float *F;
  const float *nrest;
} lbm_markers;

/* Bytes of one population buffer (two are needed) and of the workspace for
 * these parameters. 0 if the parameters are invalid. */
size_t lbm_population_bytes(const lbm_params *p);
size_t lbm_workspace_bytes(const lbm_params *p);

/* [host] strides[0] = ps, strides[1] = rs (elements) of the stored layout
 * these parameters select (see LBM_LAYOUT_*); strides[2] = 1 for ROWS, 0 for
 * PLANES. LBM_ERR_ARG if the parameters are invalid or strides is NULL. */
lbm_status lbm_population_strides(const lbm_params *p, int64_t *strides);

/* Create a context bound to caller buffers f_a, f_b (lbm_population_bytes
 * each), workspace (lbm_workspace_bytes, 256-byte aligned) and a HIP stream
 * (hipStream_t, NULL = default stream), and set the initial state to the
 * equilibrium f_i = f^eq_i(rho0, u0). This sets up the paper's local fluid
 * domain (Sec. III-B, Simulation: a grid of given resolution around the
 * body, fluid density and viscosity as the relaxation time tau) for the
 * lattice Boltzmann solution of Eq. (2).
 *   rho0 [nz][ny][nx] or NULL (rho = 1);  u0 [3][nz][ny][nx] or NULL (u = 0).
 * *out receives the context (host memory owned by the library; release with
 * lbm_destroy). Queues device work; does not synchronize. */
lbm_status lbm_init(lbm_ctx **out, const lbm_params *p, void *f_a, void *f_b, void *workspace,
                    const float *rho0, const float *u0, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): lbm_init
 * without a caller workspace. The context's workspace is a fixed array of
 * LBM_STATIC_WORKSPACE_BYTES (64 MiB) that the library holds on each device
 * it runs on until the process ends; the context itself is a per-device slot
 * of the library, so this call allocates no memory of any kind. Arguments as
 * lbm_init (f_a, f_b, rho0, u0, hip_stream) on the current device.
 * Errors: LBM_ERR_CAPACITY if lbm_workspace_bytes(p) exceeds
 * LBM_STATIC_WORKSPACE_BYTES (lower max_markers or max_active_tiles);
 * LBM_ERR_ARG as lbm_init; LBM_ERR_DEVICE if the runtime cannot resolve the
 * array on this device.
 * Sharing: every context created this way on one device is the same slot and
 * uses the same workspace. A second call on a device re-initialises that slot
 * for its own problem (the earlier handle then refers to the new one), and
 * calls that overlap in time on one device race. The workspace keeps the
 * last call's contents; this call clears every part of it that must start
 * cleared. lbm_destroy on such a context frees nothing. All other entry
 * points accept it as any context. */
#define LBM_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
lbm_status lbm_init_static(lbm_ctx **out, const lbm_params *p, void *f_a, void *f_b, const float *rho0,
                           const float *u0, void *hip_stream);

/* Replace the state with caller populations f [27][nz][ny][nx] (canonical
 * pre-collision layout). */
lbm_status lbm_load_populations(lbm_ctx *c, const float *f);

/* Write the current pre-collision populations to f [27][nz][ny][nx]. Values of
 * populations that would stream into an open-face node from outside the
 * domain are the face node's own post-collision values (never used). */
lbm_status lbm_read_populations(lbm_ctx *c, float *f);

/* Density rho [nz][ny][nx] and fluid velocity u [3][nz][ny][nx] of the
 * current pre-collision state (the macroscopic fields of Eq. (2)): u solves
 * u = (m + a0/2 - omega x u)/rho with a0 the frame force of Eq. (3) at that
 * node, i.e. the velocity with the frame force but without immersed-boundary
 * force. Either output may be NULL. frame [host] may be NULL (inertial
 * frame). */
lbm_status lbm_macros(lbm_ctx *c, const lbm_frame *frame, float *rho, float *u);

/* Advance nsteps time steps of the paper's coupled fluid-structure step
 * (Sec. III-B: the lattice Boltzmann solution of Eq. (2) in the local frame,
 * with the fictitious body force of Eq. (3), the immersed boundary of the
 * skinned surface of Sec. III-A, and the open-domain faces of Sec. III-B,
 * Simulation). For step s (global step n = current + s):
 *   skin the markers with poses[s] -> X, U; interpolate the unforced velocity
 *   and density to the markers; direct forcing -> F; spread -> g; collide
 *   (BGK + Guo with g and the frame force of frames[s]) and stream; open
 *   faces by non-equilibrium extrapolation; fluid wrench into wrench[s].
 *   m       markers (NULL or m->n == 0: no immersed body)
 *   poses   [nsteps][m->nbones][24] (may be NULL when m is NULL)
 *   frames  [host] [nsteps]
 *   wrench  [nsteps][8] or NULL: fluid force on the body (3), its torque about
 *           the frame origin (3), power delivered by the body to the fluid
 *           sum F_k . U_k dV_k (1), 0. All float32.
 * Markers leaving the allowed region, and unstable states, are detected on the
 * device and reported by lbm_check.
 * Scheduling (lbm_params.ib_workgroups > 0): with direct forcing and a body
 * present, each step is one launch: ib_workgroups workgroups run the band
 * macros, interpolation and spreading, collide the cells whose source node
 * lies in an active tile (the only cells with an immersed force), then skin
 * and bin the next step's markers, while the others collide every other cell
 * without waiting, so the collide's streaming overlaps them; the first
 * step's skinning and binning run in launches of their own. By default every
 * phase runs in a launch of its own before the collide. The results are the
 * same bits either way. */
lbm_status lbm_ib_step(lbm_ctx *c, const lbm_markers *m, const float *poses, const lbm_frame *frames,
                       int32_t nsteps, float *wrench);

/* Copy the current population state (the library's stored layout,
 * lbm_population_bytes) to dst, or replace it with src (device buffers).
 * Used for checkpoints. restore resets the step counter to step. */
lbm_status lbm_state_save(lbm_ctx *c, void *dst);
lbm_status lbm_state_restore(lbm_ctx *c, const void *src, int64_t step);

/* Rebind the two population buffers: the next step reads f_cur and writes
 * f_next, the step after that reads f_next and writes f_cur, and so on (the
 * roles lbm_init gives f_a and f_b). Both are caller-owned, distinct, of
 * lbm_population_bytes, in the stored layout; nothing is copied and the step
 * count is unchanged. This lets a reverse sweep recompute a segment of steps
 * straight into a ring of saved states (state n is the buffer step n reads),
 * with no copies. A context whose buffers are rebound must not belong to a
 * live batch (the batch keeps the pointers it was created with). */
lbm_status lbm_bind_populations(lbm_ctx *c, void *f_cur, void *f_next);

/* Discrete adjoint of one step: the reverse mode, in float32, of
 * lbm_ib_step for the step that starts from `state` (stored layout) with
 * markers m, bone poses `pose` ([m->nbones][24]) and `frame` [host]. It
 * linearises the collision around f = w + h of the stored deviations h (the
 * forward collide works on h; the two agree to float32 rounding). The step's own objective term is
 *   J_n = w[0..2] . (fluid force on the body) + w[3] * (power),
 * w [host] 4 doubles, as reported in the step's wrench. Given
 * lam_next = dJ/d(state after the step) it writes lam_prev = dJ/d(state
 * before the step) (both stored layout, F32) and adds the step's
 * dJ/d(bone pose) into pose_bar [m->nbones][24] (same layout as a pose).
 * Supported: F32 storage, BGK, direct forcing with mdf_iters = 1 on a
 * no-slip wall, omega = alpha = 0, with_adjoint set (else
 * LBM_ERR_UNSUPPORTED). The context's own state is left unchanged; m's
 * X, U, F are overwritten with the step's values. This is the differentiation
 * form: gradients of time-averaged thrust and power with respect to body
 * kinematics, through skinning (Sec. III-A) and the coupled step (Sec. III-B). */
lbm_status lbm_adjoint_step(lbm_ctx *c, const void *state, const lbm_markers *m, const float *pose,
                            const lbm_frame *frame, const double *w, const void *lam_next, void *lam_prev,
                            float *pose_bar);

/* Bytes of the immersed-boundary ring lbm_adjoint_segment needs for nseg
 * steps: per step, the marker state, tile map and band data of the forward
 * IB phases (sized by max_markers and the active-tile capacity). 0 on
 * invalid parameters. */
size_t lbm_adjoint_ring_bytes(const lbm_params *p, int32_t nseg);

/* Reverse sweep over one checkpointed segment of nseg steps, natively: from
 * ckpt (the state before the segment's first step, stored layout) the
 * segment is recomputed into ring[0..nseg-2] (caller-owned state buffers:
 * ring[t] receives the state after step t), keeping each step's forward IB
 * data in ib_ring (lbm_adjoint_ring_bytes(p, nseg) bytes, 256-byte aligned);
 * then lbm_adjoint_step's passes run for steps nseg-1 .. 0 without
 * recomputing the IB phases. poses [nseg][nbones][24], frames [host, nseg],
 * w [host] 4 doubles (the same weights each step), pose_bar [nseg][nbones][24]
 * (added into). lam holds dJ/d(state after the segment) on entry and
 * dJ/d(ckpt) on return; lam_tmp is scratch of the same size. ckpt, the ring
 * entries, lam and lam_tmp must be distinct. The context's own state and step
 * count are not touched. Same support as lbm_adjoint_step. The gradient is
 * the same as that of nseg lbm_adjoint_step calls on the recomputed states
 * (Sec. III-A skinning and Sec. III-B coupled step, differentiated). */
lbm_status lbm_adjoint_segment(lbm_ctx *c, const void *ckpt, void *const *ring, int32_t nseg, const lbm_markers *m,
                               const float *poses, const lbm_frame *frames, const double *w, void *lam,
                               void *lam_tmp, float *pose_bar, void *ib_ring);

/* The forward half of lbm_adjoint_segment, for callers that keep every state
 * of a horizon (the HBM of one device holds hundreds of states of a
 * 128x64x64 lattice): from ckpt, nseg steps are run with ring[t] receiving
 * the state after step t (t = 0 .. nseg-1; ring[nseg-1] may be NULL, which
 * skips the last collide), each step's forward IB data kept in ib_ring
 * (lbm_adjoint_ring_bytes(p, nseg) bytes, 256-byte aligned), and each step's
 * wrench row (force, torque, power, 0; as lbm_ib_step writes it) in wrench
 * [nseg][8] (device, or NULL). The states, IB data and wrench are those of
 * nseg lbm_ib_step calls from ckpt, bit for bit. Then lbm_adjoint_sweep with
 * the same ckpt, ring, ib_ring, markers, poses and frames gives the gradient
 * with no recompute. ckpt and the ring entries must be distinct. The
 * context's own state and step count are not touched. Same support as
 * lbm_adjoint_step. */
lbm_status lbm_adjoint_record(lbm_ctx *c, const void *ckpt, void *const *ring, int32_t nseg, const lbm_markers *m,
                              const float *poses, const lbm_frame *frames, void *ib_ring, float *wrench);

/* The reverse half of lbm_adjoint_segment: its reverse passes over a segment
 * that lbm_adjoint_record (or lbm_adjoint_segment) has left in ring (entries
 * 0 .. nseg-2 are read) and ib_ring, with the same ckpt, markers, poses and
 * frames. Arguments, errors and results as lbm_adjoint_segment. */
lbm_status lbm_adjoint_sweep(lbm_ctx *c, const void *ckpt, void *const *ring, int32_t nseg, const lbm_markers *m,
                             const float *poses, const lbm_frame *frames, const double *w, void *lam, void *lam_tmp,
                             float *pose_bar, void *ib_ring);

/* ------------------------------------------------------------------------
 * Free swimming (host functions, no device work): the articulated body of
 * Sec. III-A with the fluid's force as the external generalized force of
 * Eq. (1), for a planar chain of rigid links whose joint motion is prescribed.
 * Every joint being prescribed, articulated-body dynamics leaves the floating
 * base free, and its equations are the whole-body momentum balance
 * M dV/dt = F (mass centre), d/dt(I_c theta' + L_s) = T (about the mass centre),
 * I_c the chain's moment of inertia about its mass centre and L_s the angular
 * momentum of its shape change. The local domain follows the mass centre
 * (Sec. III-B), so the frame's velocity is the body's and its acceleration
 * enters the fluid by Eq. (3). Unit time steps, with k = added_mass:
 *   (1 + k) a(n+1) = F(n)/M + (r + k) a(n),  V(n+1) = V(n) + a(n)     (translation)
 *   (1 + k) I_c(n+1) theta'(n+1) = L(n) + T(n) + (r I_c(n) + k I_c(n+1)) theta''(n)
 *                                  - L_s(n+1) + k I_c(n+1) theta'(n),
 *   L(n+1) = I_c(n+1) theta'(n+1) + L_s(n+1),  theta(n+1) = theta(n) + theta'(n+1),
 *   theta''(n) = theta'(n) - theta'(n-1)
 * with r = rho_fluid / rho_body: the direct-forcing force includes the
 * reaction of the enclosed fluid, carried along with the body, and the r terms
 * add it back (rigid enclosed fluid). The frame acceleration of a step is
 * needed before its force is known, hence a(n+1) from F(n). k = 0 is plain
 * explicit coupling: if the fluid's force holds a reaction -m_a a(n) to the
 * body's acceleration (added mass m_a, plus the enclosed fluid), a(n+1)
 * carries -(m_a / M) a(n), which grows when m_a > M: bodies near neutral
 * buoyancy diverge (measured: explicit coupling needs rho_body / rho_fluid >=
 * 1.5 on the swimmer tests). k > 0 adds an artificial added mass k M (and
 * inertia k I_c) to both sides: the factor becomes (k M - m_a) / (M + k M),
 * of modulus below one whenever k > (m_a / M - 1) / 2, and a steady
 * acceleration is unchanged ((M + m_a) a = F_ext). The shape of a step is the
 * body-frame heading psi_j of every link and its rate (the chain of lbm_skin:
 * joint j+1 = joint j + h (cos psi_j, sin psi_j)). */
typedef struct {
  int32_t nbones;             /* links, 1 .. 64 */
  int32_t free_yaw;           /* 1: the body turns under the fluid's torque; 0: its heading is held */
  double link_length;         /* h */
  const double *mass;         /* [nbones] link masses, > 0 */
  const double *com;          /* [nbones] distance of a link's mass centre from its proximal joint, along it */
  const double *inertia;      /* [nbones] moment of inertia about z through the link's mass centre, > 0 */
  const double *joints_rest;  /* [nbones][3] rest joint positions of the skin (lbm_markers' rest pose) */
  double fluid_ratio;         /* r = rho_fluid / rho_body, >= 0 (0: no enclosed fluid) */
  double origin[3];           /* where the mass centre sits in the local domain (the frame origin) */
  double added_mass;          /* k >= 0: artificial added mass k M and inertia k I_c (0: explicit coupling) */
} lbm_swimmer;

typedef struct {
  double vel[2];     /* mass-centre velocity in the lab = the local frame's velocity (x, y) */
  double acc[2];     /* the frame acceleration of the coming step */
  double heading;    /* theta: rotation of the body frame about z */
  double spin;       /* theta' of the coming step */
  double spin_prev;  /* theta' of the step before */
  double ang_mom;    /* angular momentum about the mass centre (z) */
  double inertia;    /* I_c of the coming step */
  double pos[2];     /* mass-centre displacement in the lab since the start */
} lbm_swimmer_state;

/* Start at mass-centre velocity vel0 [host, 2] (NULL: rest) and heading,
 * not spinning, with the shape psi, psidot [host, nbones] of step 0. */
lbm_status lbm_swimmer_init(const lbm_swimmer *s, lbm_swimmer_state *st, const double *vel0, double heading,
                            const double *psi, const double *psidot);

/* Bone poses [host, nbones][24] (the lbm_ib_step pose layout) and the frame
 * [host] of the coming step from the state and that step's shape: the mass
 * centre at s->origin, link j at heading theta + psi_j, velocities relative
 * to the frame; the frame has the state's acceleration, no rotation, origin
 * s->origin, and far-field face velocities -vel. */
lbm_status lbm_swimmer_prepare(const lbm_swimmer *s, const lbm_swimmer_state *st, const double *psi,
                               const double *psidot, float *poses, lbm_frame *frame);

/* Advance the state over a step whose wrench [host, 8] (lbm_ib_step's: force
 * (3), torque about the frame origin (3), power, 0) is known, given the shape
 * psi, psidot of the next step. */
lbm_status lbm_swimmer_advance(const lbm_swimmer *s, lbm_swimmer_state *st, const float *wrench,
                               const double *psi_next, const double *psidot_next);

/* Fluid force on the body from the markers' last forces F (the external
 * generalized force of Eq. (1)). out [(1 + m->nbones)][8]: row 0 is the whole
 * body, row 1 + b the share of bone b (each marker's force split by its blend
 * weights); each row is force (3), torque about center (3), power (1), 0.
 * center [host] 3 doubles. */
lbm_status lbm_body_forces(lbm_ctx *c, const lbm_markers *m, const double *center, float *out);

/* Synchronize the stream and report device-side guards: LBM_ERR_UNSTABLE,
 * LBM_ERR_MARKER_RANGE, LBM_ERR_CAPACITY, LBM_ERR_ARG (a bone index out of
 * range), LBM_ERR_DEVICE (a barrier of the one-launch step waited past its
 * limit, which only a device shared with work that never yields can cause;
 * the steps since the last check are then void), or LBM_OK. Clears the
 * guards. */
lbm_status lbm_check(lbm_ctx *c);

/* Measurement hook. enable != 0: every later step brackets its two phases
 * (immersed-boundary kernels; fused collide-stream kernel) with HIP events on
 * the context stream (event pool of 4096 steps; later steps are not timed).
 * lbm_profile_collect synchronizes, returns the summed durations in
 * milliseconds and the number of timed steps, and empties the pool. Either
 * output may be NULL. */
lbm_status lbm_profile_enable(lbm_ctx *c, int enable);
lbm_status lbm_profile_collect(lbm_ctx *c, double *ib_ms, double *collide_ms, int64_t *steps);

/* Use another HIP stream for subsequent work. */
lbm_status lbm_set_stream(lbm_ctx *c, void *hip_stream);

/* Number of steps taken since lbm_init / lbm_load_populations. */
int64_t lbm_step_count(const lbm_ctx *c);

const char *lbm_strerror(lbm_status s);
void lbm_destroy(lbm_ctx *c);

/* ---------------------------------------------------------------------------
 * Batched environments: many lattices of different sizes, each with its own
 * body (the many-environment setting the simulator serves for learning,
 * Sec. III-C), advanced together by one work list per phase. Each
 * environment is an lbm_ctx created by lbm_init with F32 storage and a
 * collide block of block_x * block_y = 512 threads. Per-step inputs live in
 * device arrays so that a whole run can be one launch.
 * ------------------------------------------------------------------------- */
typedef struct lbm_batch lbm_batch;

/* [host] One environment of a batch. All pointers are device pointers valid
 * for the lifetime of the batch; poses/frames/wrench are indexed by the step
 * of a run (0 .. nsteps-1) and are re-read by every run. */
typedef struct {
  lbm_ctx *ctx;             /* initialized context (any storage, 512-thread collide block) */
  lbm_markers m;            /* n >= 1 markers, nbones <= the context's max_bones */
  const float *poses;       /* [nsteps][m.nbones][24] */
  const lbm_frame *frames;  /* [nsteps] device copy of the frames */
  float *wrench;            /* [nsteps][8] or NULL */
  int32_t rotating;         /* 0: every frame has omega = alpha = 0 (cheaper arithmetic); 1: general */
} lbm_env;

enum { LBM_BATCH_PHASES = 0,     /* one launch per phase per step */
       LBM_BATCH_PERSISTENT = 1  /* one launch for all steps, device-wide barriers between phases */
};

/* Bytes of the device buffer a batch of nenv environments needs (descriptors,
 * work-list prefixes, barrier state). 0 if nenv is outside [1, 512]. */
size_t lbm_batch_bytes(int32_t nenv);

/* Create a batch over envs [host, nenv entries] using the caller's device
 * buffer dev (lbm_batch_bytes(nenv), 256-byte aligned) and HIP stream
 * (must not be the null stream if graphs are used). All environments must
 * use the same mdf_iters and the same ib_scheme (else LBM_ERR_UNSUPPORTED;
 * also for the implicit correction on a slip wall in a rotating frame, as
 * lbm_ib_step). Each environment keeps its own collision (BGK or TRT),
 * storage, wall mode and faces. Uploads the descriptors and synchronizes. */
lbm_status lbm_batch_create(lbm_batch **out, const lbm_env *envs, int32_t nenv, void *dev, void *hip_stream);

/* Advance every environment by nsteps steps with the given driver. graph != 0:
 * the launches are captured once into a HIP graph (per (nsteps, mode)) and the
 * graph is replayed; nsteps must then be even, so that every replay starts
 * from the same population buffer. The persistent driver takes F32 storage
 * and direct forcing only: with an FP16 or BF16 environment or the implicit
 * correction it returns LBM_ERR_UNSUPPORTED (the per-phase driver takes
 * both, one collide launch per kind and format). Does not synchronize. */
lbm_status lbm_batch_run(lbm_batch *b, int32_t nsteps, int32_t mode, int32_t graph);

/* Tile-shape autotuner: for every environment time the collide kernel with
 * each 512-thread shape over reps launches and keep the fastest. Shapes
 * (block_x, block_y): 64x8, 128x4, 256x2 and 512x1 are 2-D blocks over
 * (x, y) rows; (512, 0) is the linear shape, 512 consecutive cells of the
 * x-fastest order per block with rows wrapped (no idle lanes at ragged row
 * ends). The state is not advanced. shapes_out [host, nenv][2] or NULL.
 * Sets the shapes the next run uses. */
lbm_status lbm_batch_autotune(lbm_batch *b, int32_t reps, int32_t *shapes_out);

/* Apply shapes [host, nenv][2] (e.g. a cached autotuning result); any of the
 * five autotuner shapes, else LBM_ERR_ARG. */
lbm_status lbm_batch_set_shapes(lbm_batch *b, const int32_t *shapes);

/* Concurrent groups for the per-phase driver, which otherwise leaves the
 * device part idle at every phase boundary of every step (each phase is a
 * launch that waits for the previous one). ngroups in [2, LBM_BATCH_MAX_GROUPS]
 * and at most nenv: the environments are split into ngroups groups of about
 * equal cell count (largest lattice first, each to the group with the fewest
 * cells; each group keeps the batch's order), and each group becomes a batch
 * of its own on streams[g] [host array of ngroups distinct HIP streams, owned
 * by the caller and alive while the groups are set]. A per-phase run then
 * waits for the work queued on the batch's stream, runs the groups
 * concurrently (one graph per group when graph != 0), and makes the batch's
 * stream wait for all of them; lbm_batch_check covers the groups. Each
 * environment's arithmetic is independent of the others, so the populations
 * and wrenches are bit for bit those of the ungrouped run. The persistent
 * driver always runs the whole batch in one launch. dev: device buffer of
 * lbm_batch_group_bytes(nenv, ngroups) bytes, 256-byte aligned, owned by the
 * caller and alive while the groups are set. ngroups = 1 drops the groups
 * (streams and dev may be NULL). Synchronizes the batch's stream. Returns
 * LBM_ERR_ARG for a count outside the range, a NULL or repeated stream or a
 * misaligned buffer. lbm_batch_group_bytes is 0 if nenv is outside
 * [1, 512] or ngroups outside [2, min(nenv, LBM_BATCH_MAX_GROUPS)]. */
enum { LBM_BATCH_MAX_GROUPS = 8 };
size_t lbm_batch_group_bytes(int32_t nenv, int32_t ngroups);
lbm_status lbm_batch_set_groups(lbm_batch *b, int32_t ngroups, void *const *streams, void *dev);

/* Synchronize; LBM_ERR_DEVICE if a persistent run's barrier timed out (its
 * steps stopped early, the populations are not those of a completed run; the
 * barrier is reset so later runs can proceed), otherwise the first non-OK
 * lbm_check of the environments. A persistent launch assumes its whole grid
 * (sized from the occupancy of one device with nothing else running) is
 * co-resident; every barrier wait is bounded (about a second), so a grid that
 * is not co-resident ends with this error instead of hanging. */
lbm_status lbm_batch_check(lbm_batch *b);

void lbm_batch_destroy(lbm_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* LBM_IB_H */

/*
 * stencil.h -- C ABI of libstencil.so, an MI355X (gfx950) implementation of
 * the time-iterated star-stencil sweep of "A shared compilation stack for
 * distributed-memory parallelism in stencil DSLs" (ASPLOS'24, arXiv 2404.02218).
 *
 * Semantics follow the paper's stencil dialect (Section 4.1):
 *   - a field is a memory buffer whose bounds include the halo (stencil.field);
 *   - one sweep loads the field (stencil.load), evaluates the update at every
 *     interior point reading neighbours at constant offsets (stencil.apply /
 *     stencil.access / stencil.return) and stores the result on a bounded range
 *     (stencil.store); a sweep never reads what it writes at an offset;
 *   - the halo is at least as wide as the largest access offset (Section 4.1,
 *     minimal-halo inference; Figure "stencil_intro": halo points are read-only).
 * Halo exchanges follow the dmp dialect's declarative exchange (Section 4.2).
 *
 * The update bodies (weights c_0..c_r of a centred star of radius r, D axes):
 *   (L u)_i = D c_0 u_i + sum_d sum_{k=1..r} c_k (u_{i+k e_d} + u_{i-k e_d})
 *   heat  (Section 5.1, Devito heat listing):  u^{n+1} = u^n + L u^n
 *         (the caller folds a dt / h^2 into the weights)
 *   wave  (Section 6.1, second order in time):
 *         u^{n+1} = 2 u^n - u^{n-1} + beta .* L u^n,  beta = (dt v / h)^2
 *
 * Conventions for every entry point:
 *   - Return value: STENCIL_OK (0) or a negative stencil_status.  On error no
 *     device work has been enqueued and no caller memory has been touched;
 *     stencil_last_error() returns a message (thread-local, valid until the
 *     next call on the same thread).  No C++ exception crosses the ABI.
 *   - All device pointers are HIP device allocations owned by the caller.
 *     The library only enqueues work on the caller's stream (a hipStream_t
 *     passed as void*; NULL = the legacy default stream); STENCIL_OK means
 *     "enqueued", not "finished".
 *   - The library uses whichever HIP runtime (libamdhip64) the process has
 *     loaded when it is loaded, and pointers and streams must come from that
 *     same runtime.  A host program that brings its own copy of the runtime
 *     (PyTorch does) loads that copy first; a second runtime in one process
 *     reports no device.
 *   - Arrays of shapes, coordinates and exchange declarations are host
 *     memory, C order (slowest axis first), and only the first ndim slots of
 *     a [3] array are read.
 *   - Compute is FP32 for every storage dtype; 16-bit storage is rounded to
 *     nearest even.  Source injection and receiver sampling are FP64.
 */
#ifndef STENCIL_H
#define STENCIL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    STENCIL_OK = 0,
    STENCIL_E_INVALID = -1,     /* bad argument (shape, radius, pointer, box, position) */
    STENCIL_E_UNSUPPORTED = -2, /* valid but not implemented (e.g. ndim 4) */
    STENCIL_E_NOMEM = -3,       /* host or device allocation failed, or size overflow */
    STENCIL_E_DEVICE = -4,      /* a HIP call failed; message holds hipGetErrorString */
    STENCIL_E_STATE = -5        /* call not valid for this plan (kind, dtype, workspace) */
} stencil_status;

typedef enum { STENCIL_HEAT = 0, STENCIL_WAVE2 = 1 } stencil_kind;
typedef enum { STENCIL_F32 = 0, STENCIL_BF16 = 1, STENCIL_F16 = 2 } stencil_dtype;
typedef enum { STENCIL_BC_DIRICHLET0 = 0, STENCIL_BC_PERIODIC = 1 } stencil_bc;

typedef struct stencil_plan_s* stencil_plan;

/* One dmp.exchange declaration (Section 4.2, listing "halo-swap-op" and figure
 * "exchange_decl"): receive into buffer box [at, at+size); the box sent to the
 * rank at relative offset `to` is [at+src_offset, at+src_offset+size).
 * Coordinates are buffer coordinates (halo included). */
typedef struct {
    int64_t at[3];
    int64_t size[3];
    int64_t src_offset[3];
    int32_t to[3];
    int32_t reserved;
} stencil_exchange;

/* Point sources (Devito's sparse source operation, Section 5.1): after the
 * sweep of step t, u^{t+1} at pos[s] becomes round_T(fl64(u^{t+1}) + q) with
 * q = amp[t*n + s], or q = fl64(amp[t*n + s] * scale[s]) when scale is not
 * NULL.  For the acoustic wave in m-form the amount is dt^2 v_s^2 w(t): pass
 * the wavelet samples w as amp and dt^2 v_s^2 as scale
 * (stencil_wave_point_scale forms it from m).  pos: host, [n][3] interior
 * coordinates.  amp: device FP64, [nsteps][n].  scale: device FP64 [n] or
 * NULL. */
typedef struct {
    int64_t n;
    const int64_t* pos;
    const double* amp;
    const double* scale;
} stencil_source;

/* Receivers (Devito's sparse interpolation of the wavefield, Section 5.1):
 * trace[t*n + r] = fl64(u^{t+1} at pos[r]) for t = 0..nsteps-1.
 * pos: host [n][3] interior coordinates.  trace: device FP64 [nsteps][n]. */
typedef struct {
    int64_t n;
    const int64_t* pos;
    double* trace;
} stencil_receivers;

/* Interpolated (off-grid) sources and receivers: Devito's sparse functions
 * (Section 5.1), at real positions instead of grid points.  pos: host,
 * [n][3] doubles, the first ndim entries used, each a real interior
 * coordinate in [0, extent - 1] (grid units).  A position spreads over the
 * 2^ndim corners of its cell with multilinear weights (stencil_interp_weights).
 * amp: device FP64 [nsteps][n]; trace: device FP64 [nsteps][n]. */
typedef struct {
    int64_t n;
    const double* pos;
    const double* amp;
} stencil_source_interp;

typedef struct {
    int64_t n;
    const double* pos;
    double* trace;
} stencil_receivers_interp;

/* ---------------------------------------------------------------- plans */

/* Create a plan for fields of interior `shape` (ndim 1..3) with a halo of
 * `halo` >= `radius` cells on every side of every axis (Section 4.1: the halo
 * must cover the largest stencil.access offset).  radius 1..4; `coeffs` holds
 * radius+1 host doubles c_0..c_r (heat: already scaled by a dt/h^2).  The plan
 * owns small device tables only (positions, coefficients, a captured graph);
 * every field-sized buffer, including the temporally blocked variants'
 * second level pair, is caller memory (stencil_set_workspace).
 * Errors: E_INVALID for ndim/radius/halo/shape out of range or NULL pointers;
 * E_NOMEM if a field would exceed 2^40 elements. */
stencil_status stencil_create(stencil_plan* out, stencil_kind kind, int ndim, const int64_t* shape,
                              int radius, const double* coeffs, int halo, stencil_dtype dtype,
                              stencil_bc bc);

/* Release a plan and the device tables it owns (no passage of the paper:
 * plan lifetime).  Caller memory (fields, workspaces) is untouched; work
 * enqueued with the plan must have finished. */
stencil_status stencil_destroy(stencil_plan plan);

/* Field layout (the stencil.field bounds, Section 4.1), identical for every
 * field of the plan (u, u_prev, beta).  extents[ndim] = shape + 2*halo;
 * strides[ndim] in elements; the element at buffer coordinate b is at
 * base + offset + sum_d b_d * strides[d].  Rows are padded so that the first
 * interior element of every row is 128-byte aligned.  bytes = allocation size.
 * Field pointers passed to the library are `base` and must be 256-byte
 * aligned.  The halo is never written by sweeps (Dirichlet-zero when the
 * caller zeroes it); with STENCIL_BC_PERIODIC the library refreshes it. */
stencil_status stencil_layout(stencil_plan plan, int64_t* extents, int64_t* strides,
                              int64_t* offset, int64_t* bytes);

/* One load/apply/store (Section 4.1) on the interior box [lo, hi) (interior
 * coordinates, host arrays).  heat: in = {u};  wave: in = {u_n, u_prev, beta}.
 * `out` must not alias in[0]; for the wave it may alias in[1] (only the
 * centre of u_prev is read).  Points of `out` outside the box are untouched.
 * No halo refresh. */
stencil_status stencil_apply(stencil_plan plan, void* out, const void* const* in,
                             const int64_t* lo, const int64_t* hi, void* stream);

/* nsteps sweeps of the time loop (Section 5.1: time buffering).
 *   heat:  fields = {u, u_next}: ping-pong buffers;
 *   wave:  fields = {u_n, u_prev, beta}: u^{n+1} overwrites u^{n-1} in place.
 * On return the pointer array is permuted so that fields[0] holds the newest
 * level (and, for the wave, fields[1] the one before).  With periodic
 * boundaries the halo of the current level is refreshed before each sweep by
 * a self-exchange (the dmp.swap of a one-rank periodic grid, Section 4.2).
 * src/rec may be NULL.  The launches of a run of two or more steps are
 * captured into one HIP graph per (pointers, nsteps, variant, tables) and
 * replayed; with the environment variable STENCIL_NO_GRAPH set to a value
 * other than 0 they are enqueued directly instead (the same kernels and
 * bits).  The temporally blocked wave variants need a caller workspace
 * (stencil_run_workspace / stencil_set_workspace); without one the call
 * fails with STENCIL_E_STATE.  The plan keeps small device tables of
 * positions and, for sources with scales, their formed amounts; it never
 * allocates field memory. */
stencil_status stencil_run(stencil_plan plan, void** fields, int64_t nsteps, const stencil_source* src,
                           const stencil_receivers* rec, void* stream);

/* stencil_run for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * Same arguments, results (bit for bit) and kernels as stencil_run, but it
 * calls no hipMalloc, hipFree or other allocating routine and captures no
 * graph of its own (it enqueues the sweeps directly).  The position tables
 * of the sources and receivers, and the formed amounts of sources with
 * scales, go into a static device array of 8 MiB that each GPU holds for
 * the life of the process; host data reaches it through the arguments of
 * small copy kernels, so a caller's own capture keeps a copy of it.  A run
 * needing more than 8 MiB there (about 9 bytes per step per scaled source,
 * plus about 40 bytes per source and receiver and 4 per xy tile) fails with
 * STENCIL_E_NOMEM before any device work.  The temporally blocked variants
 * still take the workspace attached with stencil_set_workspace (caller
 * memory).  Every call on one GPU shares that array: calls that may overlap
 * in time on one GPU (different streams, or host threads) race and must
 * not be issued; calls in order on one stream are safe.  Host memory is
 * used to build the tables. */
stencil_status stencil_run_noalloc(stencil_plan plan, void** fields, int64_t nsteps, const stencil_source* src,
                                   const stencil_receivers* rec, void* stream);

/* Absorbing layer for a wave plan (the boundary conditions Devito's
 * front end provides, Section 5.1): the sweep becomes the damped leapfrog
 *     u^{t+1} = (2u^t - (1 - g) u^{t-1} + beta .* L u^t) / (1 + g)
 * (m u_tt + eta u_t = laplace(u)/h^2 with centred u_t and g = eta dt / (2m)),
 * evaluated in FP32 as ((2u - u_prev) + g u_prev + beta L u) / (1 + g); where
 * g = 0 the update is the undamped one bit for bit.  g is separable: profile
 * is a host array of extent_0 + ... + extent_{ndim-1} doubles (the per-axis
 * profiles one after another in axis order), g at a point = the sum of its
 * coordinates' entries (added first axis first, in FP32).  Sources are added
 * after the damped update as before.  NULL removes the layer.  Every variant
 * of the plan takes the layer (the temporally blocked one in both of its
 * stages) and they agree bit for bit; the adjoint path refuses a damped
 * plan.  Errors: STENCIL_E_STATE for heat plans,
 * STENCIL_E_UNSUPPORTED for 16-bit storage, STENCIL_E_INVALID for negative
 * or non-finite entries. */
stencil_status stencil_wave_damping(stencil_plan plan, const double* profile);

/* Corners and weights of n interpolated positions (Devito's sparse
 * operations off the grid, Section 5.1; pos as in stencil_source_interp): corners [n][2^ndim][3] (first ndim entries set)
 * and weights [n][2^ndim], host arrays.  Per axis with extent e:
 * base = min(floor(x), e - 2) (0 when e < 2) and f = x - base (0 when
 * e < 2); corner bit 0 is (base, weight 1 - f), bit 1 is
 * (min(base + 1, e - 1), weight f).  Corner c has bit (c >> (ndim-1-j)) & 1
 * on axis j, and its weight is the product of the axes' weights in axis
 * order.  Host only; errors: STENCIL_E_INVALID for a position outside
 * [0, e - 1] or not finite. */
stencil_status stencil_interp_weights(stencil_plan plan, int64_t n, const double* pos, int64_t* corners,
                                      double* weights);

/* stencil_run with interpolated sources and receivers (Devito's sparse
 * source and receiver operations at real positions, Section 5.1).  After the sweep of
 * step t, source s adds w_c * amp[t*n + s] at each corner c, as a point
 * source of that amount.  Entries at a shared grid point are applied in
 * (source, corner) order.  Receiver r records trace[t*n + r], the sum over
 * its corners c in order of w_c * fl64(u^{t+1} at c), as FP64 fused
 * multiply-adds.  The plan keeps the weights and a corner trace of
 * nsteps * n * 2^ndim doubles, allocated on first use and reused.  Sweep
 * plans only (not batched); the temporally blocked variants take the
 * workspace as stencil_run does; errors as stencil_run, plus the position
 * errors of stencil_interp_weights. */
stencil_status stencil_run_interp(stencil_plan plan, void** fields, int64_t nsteps,
                                  const stencil_source_interp* src, const stencil_receivers_interp* rec,
                                  void* stream);

/* ------------------------------------------------------------ exchanges */

/* Exchange declarations of the rank at `coord` of a Cartesian rank grid
 * `grid` (the decomposition strategy's exchange generator, Section 4.2):
 * per axis and side with a neighbour, receive the radius-thick halo slab and
 * send the interior slab next to the same face.  Faces only, no corners (the
 * star stencil needs none).  A missing neighbour (non-periodic outer face)
 * produces no exchange, as the paper's lowering uses a null request for it
 * (Section 4.3).  *n: in = capacity of `out`, out = count (<= 2*ndim). */
stencil_status stencil_exchanges(stencil_plan plan, const int32_t* grid, const int32_t* coord,
                                 int periodic, stencil_exchange* out, int* n);

/* Exchange declarations including edges and corners: one per neighbour
 * direction d in {-1, 0, 1}^ndim other than 0 (3^ndim - 1 in all; 26 in 3D),
 * in C order of d with -1 before 0 before +1.  Per axis, d = -1 receives
 * [h - r, h) from the neighbour below (send box shifted by +r), d = +1
 * receives [h + n, h + n + r) (send box shifted by -r), d = 0 spans the
 * interior.  Needed by stencils that read diagonal offsets (a stencil
 * program's terms can; Section 4.2 declares exchanges as boxes, so an edge or
 * corner is one more box).  A direction exists when every axis with d != 0
 * has that neighbour, or `periodic`.  For a program plan r is its largest
 * offset.  *n: in = capacity of `out`, out = count. */
stencil_status stencil_exchanges_box(stencil_plan plan, const int32_t* grid, const int32_t* coord,
                                     int periodic, stencil_exchange* out, int* n);

/* Pack the send boxes of n exchanges (host array) from `field` into `buf`
 * (device): the send half of a dmp.swap as lowered to MPI (Section 4.3,
 * the send buffer filled from the box [at + src_offset, + size) of
 * Section 4.2), each box in C order, concatenated in declaration order.  The
 * number of elements is the sum of the box volumes; buf has the field's
 * storage dtype.  One launch for all boxes. */
stencil_status stencil_halo_pack(stencil_plan plan, const void* field, const stencil_exchange* ex,
                                 int n, void* buf, void* stream);

/* Unpack `buf` (as produced by a partner's pack) into the receive boxes
 * [at, at + size): the receive half of the lowered dmp.swap (Sections 4.2,
 * 4.3).  Same layout and error behaviour as stencil_halo_pack. */
stencil_status stencil_halo_unpack(stencil_plan plan, void* field, const stencil_exchange* ex, int n,
                                   const void* buf, void* stream);

/* ---------------------------------------------------------- batched shots */

/* A batch of independent wave problems (3D only) of uneven interior shapes
 * shapes[nshots][3], sharing radius, weights, halo and dtype.  Each shot
 * has its own fields (layout from stencil_batch_layout).  The paper has no
 * batched form: each shot is the Section 6.1 wave sweep (the operations of
 * stencil_run), and the batch only changes how the shots' tiles are
 * launched, to amortise the per-launch overhead the paper measured on its
 * GPU (Section 6.1) over many small problems. */
stencil_status stencil_batch_create(stencil_plan* out, int nshots, const int64_t* shapes, int radius,
                                    const double* coeffs, int halo, stencil_dtype dtype);
/* Field layout of shot `shot` of a batch (the stencil.field bounds of
 * Section 4.1, as stencil_layout). */
stencil_status stencil_batch_layout(stencil_plan batch, int shot, int64_t* extents, int64_t* strides,
                                    int64_t* offset, int64_t* bytes);

/* nsteps sweeps of every shot (Section 6.1 wave sweep per shot, as in
 * stencil_run), captured into one HIP graph.  By variant:
 *   - fused (zmarch_*, tb2_*): one launch per step (two steps for the
 *     temporally blocked form) covers the tiles of all shots;
 *   - persistent_zmarch_*: one launch runs every step over per-XCD queues of
 *     the shots' tiles, with a grid barrier between steps.  Its grid is as
 *     many workgroups as the GPU holds at once; a barrier wait is bounded
 *     (STENCIL_BARRIER_POLLS polls if set, else 2^20), and a wait that gives
 *     up (the grid was not all resident, e.g. beside other work on the GPU)
 *     fails the call with STENCIL_E_DEVICE and leaves the fields invalid.
 *     This variant synchronises `stream` before it returns, to read that
 *     flag;
 *   - shots_concurrent_4: every shot's own tuned run, on four branches of the
 *     graph.
 * fields[3*s + {0,1,2}] = shot s's {u_n, u_prev, beta}, permuted per shot as
 * in stencil_run.  src / rec: arrays of nshots entries, or NULL.  The
 * temporally blocked variant needs a workspace as stencil_run does (one
 * field pair per shot). */
stencil_status stencil_batch_run(stencil_plan batch, void** fields, int64_t nsteps,
                                 const stencil_source* src, const stencil_receivers* rec, void* stream);

/* ------------------------------------------------------------- adjoint */

/* The adjoint path (Section 5.1: Devito derives adjoint operators for
 * seismic inversion; the paper gives no derivation, so the discrete adjoint
 * of the wave recurrence is derived here).  Forward step n in m-form, with
 * m = 1/v^2 and beta = dt^2/(h^2 m):
 *   m (u^{n+1} - 2u^n + u^{n-1}) - (dt^2/h^2) L u^n - dt^2 q^n = 0,
 * u^0 = u^{-1} = 0.  For J = 1/2 sum_n |P u^n - d^n_obs|^2 the adjoint state
 * solves the same sweep backwards in time driven by the residuals,
 *   lam^{k-1} = 2 lam^k - lam^{k+1} + beta .* L lam^k + dt^2/m_r (d^k - d^k_obs)_r,
 * lam^N = lam^{N+1} = 0 (L is symmetric for the star with a zero halo), and
 *   dJ/dm = -(1/dt^2) sum_{n=0..N-1} lam^n .* (u^{n+1} - 2u^n + u^{n-1}).
 * Forward levels are recomputed segment by segment from checkpoints
 * (u^c, u^{c-1}) stored every checkpoint_every steps.  3D wave plans with
 * FP32 storage and the zero halo only. */

/* Workspace bytes of the adjoint path (Section 5.1 adjoint operators; the
 * checkpointing is this library's) for stencil_forward_ckpt /
 * stencil_adjoint / stencil_gradient: the checkpoints (u^c, u^{c-1}) every checkpoint_every
 * steps, one segment of second differences, two recompute levels, two
 * adjoint levels and an FP32 imaging partial (caller memory). */
stencil_status stencil_adjoint_workspace(stencil_plan plan, int64_t nsteps, int64_t checkpoint_every,
                                         size_t* bytes);

/* Forward run of the adjoint path (the Section 6.1 wave sweep as
 * stencil_run, fields = {u_n, u_prev, beta}), also storing (u^c, u^{c-1})
 * for c = 0, k, 2k, ... into the workspace (the sweeps write them there
 * directly) and the last segment's second differences, which the plan
 * notes for the next stencil_adjoint on the same workspace, nsteps and
 * checkpoint_every. */
stencil_status stencil_forward_ckpt(stencil_plan plan, void** fields, int64_t nsteps,
                                    int64_t checkpoint_every, const stencil_source* src,
                                    const stencil_receivers* rec, void* workspace,
                                    size_t workspace_bytes, void* stream);

/* Gradient of the data misfit with respect to m by the discrete adjoint
 * above (Section 5.1, adjoint operators):
 *   lam^{k-1} = 2 lam^k - lam^{k+1} + beta .* L lam^k
 *               + rec_scale[r] * resid[(k-1)*nrec + r] at receiver r,
 *   grad += -(1/dt^2) sum_n lam^n .* (u^{n+1} - 2u^n + u^{n-1}).
 * The forward levels are recomputed segment by segment from the checkpoints
 * left in `workspace` by stencil_forward_ckpt with the same nsteps,
 * checkpoint_every, beta and sources (the last segment's second
 * differences are taken from that forward when this plan's last
 * checkpointed forward used this workspace and no adjoint has recomputed
 * since).  The checkpoints are left intact: a second call on the same
 * workspace gives the same result.  For J = 1/2 |d - d_obs|^2:
 * resid = d - d_obs and rec_scale = dt^2 / m_r (stencil_wave_point_scale).
 * The forward and this backward are separate calls so that a caller can
 * drive the backward with any trace gradient (torch.autograd); see
 * stencil_gradient for the misfit and its gradient in one call.
 * beta: field layout.  resid, rec_scale: device FP64.  grad: device FP64,
 * dense interior [nz][ny][nx], accumulated into (not cleared). */
stencil_status stencil_adjoint(stencil_plan plan, const void* beta, int64_t nsteps,
                               int64_t checkpoint_every, const stencil_source* src,
                               const stencil_receivers* rec, const double* resid,
                               const double* rec_scale, double dt, double* grad,
                               void* workspace, size_t workspace_bytes, void* stream);

/* The misfit J = 1/2 sum |d - d_obs|^2 and its gradient dJ/dm in one call
 * (Section 5.1, adjoint operators; the recurrences above): writes
 * beta = dt^2/(h^2 m) into fields[2], zeroes fields[0] and fields[1]
 * (u^0 = u^{-1} = 0), runs the checkpointed forward with source amounts
 * dt^2/m_s * amp[t][s] (src->scale must be NULL: the scales come from m),
 * records d into rec->trace, forms d - d_obs and J on the device, and runs
 * the adjoint with receiver weights dt^2/m_r.  m: device FP64 dense interior.
 * d_obs: device FP64 [nsteps][nrec].  misfit: device FP64, one value.  grad:
 * device FP64 dense interior, overwritten.  fields is permuted as in
 * stencil_run.  The workspace is that of stencil_adjoint_workspace; the plan
 * keeps the point scales and the residual ((nsrc + nrec + nsteps * nrec)
 * doubles).  Errors as stencil_forward_ckpt and stencil_adjoint, plus
 * STENCIL_E_INVALID without receivers or with source scales. */
stencil_status stencil_gradient(stencil_plan plan, void** fields, const double* m, double dt, double h,
                                int64_t nsteps, int64_t checkpoint_every, const stencil_source* src,
                                const stencil_receivers* rec, const double* d_obs, double* misfit,
                                double* grad, void* workspace, size_t workspace_bytes, void* stream);

/* beta = dt^2 / (h^2 m) on the interior of a field (halo untouched) from a
 * dense interior FP64 array m (device), rounded to the plan's dtype (the
 * coefficient field of the Section 6.1 wave in terms of squared slowness). */
stencil_status stencil_wave_beta(stencil_plan plan, const double* m, double dt, double h, void* beta,
                                 void* stream);

/* out[i] = dt^2 / m(pos[i]) (FP64) for n interior positions (host [n][3]):
 * the factor dt^2 v^2 of a source amount and of a receiver's residual
 * weight in the m-form wave (Section 6.1 wave; Section 5.1 sparse sources).
 * m: device FP64 dense interior.  out: device FP64 [n]. */
stencil_status stencil_wave_point_scale(stencil_plan plan, const double* m, double dt, int64_t n,
                                        const int64_t* pos, double* out, void* stream);

/* ------------------------------------------------------- stencil programs */

/* One term of a stencil program.  A program computes nout output fields
 * from nin input fields at every interior point i: output o is the sum, in
 * program order, of its terms coeff * in[a](i + off_a), or
 * coeff * in[a](i + off_a) * in[b](i + off_b) for two factors (several
 * stencil.apply computations over several fields fused into one region, as
 * Section 6.2 describes for PW advection; the accesses are stencil.access at
 * relative offsets, Section 4.1).  Offsets are in C order (z, y, x); for
 * ndim < 3 the leading entries are 0. */
typedef struct {
    int32_t out;       /* output field, 0 .. nout-1 */
    int32_t nfac;      /* 1 or 2 */
    int32_t in[2];     /* input field of each factor, 0 .. nin-1 */
    int32_t off[2][3]; /* offset of each factor */
    double coeff;      /* rounded to FP32 for the device */
} stencil_term;

/* A program plan (the several fused stencil.apply computations of Section
 * 6.2, with stencil.access offsets of Section 4.1, as stencil_term
 * describes) over interior `shape` (ndim 1..3) with halo `halo`: nin in
 * [1, 4] input and nout in [1, 4] output fields of FP32 storage sharing the
 * plan's layout (stencil_layout), nterms in [1, 64] terms (copied).  Every
 * offset must lie within min(halo, 2).  Errors: STENCIL_E_INVALID for bad
 * indices or offsets, STENCIL_E_UNSUPPORTED for other dtypes or sizes beyond
 * these limits, STENCIL_E_DEVICE if compiling the program's kernel fails
 * (the message holds the compiler's log).  The plan compiles a kernel in
 * which the terms are constants (hiprtc, gfx950; plans with the same program
 * share it, and it is loaded on a device at the first apply there);
 * stencil_variant_count reports 3 or 4 variants, all with identical bits:
 * 0 runs that kernel on 64 x 16 tiles (256 threads); 1 a generic kernel
 * that reads the terms at run time; 2 the compiled kernel with a plane ring
 * one slot shorter (less LDS, a second barrier per plane); 3, where its LDS
 * ring fits a compute unit (160 KiB), the compiled kernel on 64 x 32 tiles
 * (512 threads).  Variants 2 and 3 are compiled at their first apply.
 * stencil_layout, stencil_exchanges(_box), stencil_halo_pack and _unpack,
 * the variant calls, stencil_tune (fields = inputs, then outputs) and
 * stencil_destroy accept the plan. */
stencil_status stencil_program_create(stencil_plan* out, int ndim, const int64_t* shape, int halo, int nin,
                                      int nout, const stencil_term* terms, int nterms, stencil_dtype dtype);

/* Evaluate the program once (one fused stencil.apply region, Sections 4.1
 * and 6.2): outs[nout] and ins[nin] are device field
 * pointers (256-byte aligned).  Interior points of every output are
 * written; halos are read from the inputs as they are (refresh them with an
 * exchange first where needed) and outputs' halos are untouched.  No output
 * may alias an input or another output.  Each term evaluates as
 * on its output's FP32 sum s in program order: s = fma(coeff, a, s) for
 * one factor, s = fma(fl(coeff * a), b, s) for two (fma: one rounding).
 * The first apply of a compiled variant on a device loads its code object
 * (hipModuleLoadData), which may synchronise the device: make that first
 * call outside stream capture; later applies only enqueue the kernel. */
stencil_status stencil_program_apply(stencil_plan plan, void* const* outs, const void* const* ins, void* stream);

/* ------------------------------------------------------- exchange schedule */

/* The neighbour directions in which a program reads input `field` outside
 * its interior.  Bit k stands for the direction d (per axis -1, 0 or +1, over
 * the plan's ndim axes) whose C-order code sum_j (d_j + 1) 3^(ndim-1-j) is k,
 * the same order as stencil_exchanges_box.  Bit k is set when some term reads
 * the field at an offset o that lands in d's halo box from some interior
 * point: on every axis d_j = sign(o_j) with o_j != 0, or d_j = 0 with
 * |o_j| < n_j.  Exchanging these boxes is enough before an apply (the paper's
 * dmp.swap, Section 4.2, restricted to what the access pattern needs).
 * Errors: STENCIL_E_STATE for a sweep plan, STENCIL_E_INVALID for a bad
 * field index. */
stencil_status stencil_program_halo_dirs(stencil_plan plan, int field, uint32_t* dirs);

/* One apply of a sequence: a program plan and the ids (0 .. nfields-1) of
 * the fields bound to its inputs and outputs. */
typedef struct {
    stencil_plan program;
    int32_t in[4];  /* first nin entries used */
    int32_t out[4]; /* first nout entries used */
} stencil_step;

enum { STENCIL_ACT_EXCHANGE = 0, STENCIL_ACT_APPLY = 1 };

/* One action of a schedule.  An exchange refreshes the halo boxes of `field`
 * in `dirs` (bits as stencil_program_halo_dirs) from the field's current
 * interior; `step` is the step whose read it serves first (-1 in a
 * prologue).  An apply runs `step`. */
typedef struct {
    int32_t kind;
    int32_t step;
    int32_t field;
    uint32_t dirs;
} stencil_action;

/* Exchange schedule of a sequence of applies (Section 4.2: a swap before
 * every load, redundant swaps then removed by data-flow analysis; Section
 * 4.3: loop-invariant communication hoisted).  A field's halo is stale until
 * it is exchanged, and again after each apply that writes the field (an apply
 * writes the interior only).  Before each step, each input field is exchanged
 * in the directions that step reads and that are stale, widened to every
 * direction read before the field's next write.  So each field is exchanged
 * at most once per write, and never when unchanged.  With loop != 0 the steps
 * are the body of a loop that repeats them.  Reads before a field's first
 * write in the body see the previous iteration's values.  The exchanges that
 * make the first iteration equal to every later one go into `prologue`; this
 * includes every exchange of a field the body never writes (hoisting).  With
 * loop == 0 the prologue is empty.  Outputs must be distinct and must not be
 * inputs of the same step, and every program must have the same ndim.
 * *nprologue and *nbody: in = capacity, out = count.  Errors:
 * STENCIL_E_INVALID (ids, aliasing, capacity, a sweep plan), STENCIL_E_STATE
 * (differing ndim). */
stencil_status stencil_schedule(const stencil_step* steps, int nsteps, int nfields, int loop,
                                stencil_action* prologue, int* nprologue, stencil_action* body, int* nbody);

/* ------------------------------------------- workspace and failure checks */

/* Bytes of caller workspace the plan's current variant needs in stencil_run
 * (stencil_batch_run for a batch): the second level pair of the temporally
 * blocked wave sweep (two fields, one pair per shot for a batch; Section 7
 * related work on overlapped temporal blocking), 0 for every other variant.
 * Query again after stencil_tune or stencil_set_variant. */
stencil_status stencil_run_workspace(stencil_plan plan, size_t* bytes);

/* Attach caller device memory as the plan's run workspace (NULL detaches;
 * no passage of the paper: memory ownership of the Section 7 temporal
 * blocking's second level pair).
 * The library enqueues a zero fill of all `bytes` on `stream` (the pair's
 * halos must be zero) and then only writes interiors; the memory must stay
 * valid while runs that use it may execute.  bytes: a multiple of 4. */
stencil_status stencil_set_workspace(stencil_plan plan, void* workspace, size_t bytes, void* stream);

/* Stability number of the plan's update (host only): D times the largest
 * value over theta in [0, pi] of -(c_0 + 2 sum_k c_k cos k theta), the
 * per-axis weights' symbol.  The explicit heat update is stable when it is
 * <= 2; the leapfrog wave when beta_max times it is <= 4 (von Neumann
 * analysis of the update of Section 5.1 / 6.1; the paper gives no bound). */
stencil_status stencil_stability(stencil_plan plan, double* ds);

typedef struct {
    int64_t nan_count;  /* NaN values in the scanned levels' interiors */
    int64_t inf_count;  /* infinite values there (storage overflow, e.g. past 65504 in FP16) */
    double max_abs;     /* largest finite |value| there */
    double beta_max;    /* wave: largest beta in the interior (0 for heat) */
    double stability;   /* wave: beta_max * ds / 4; heat: ds / 2 (ds: stencil_stability); stable <= 1 */
    double headroom;    /* largest finite value of the storage type / max_abs */
    int32_t flags;      /* STENCIL_CHECK_* bits */
    int32_t reserved;
} stencil_check_report;

enum {
    STENCIL_CHECK_NONFINITE = 1, /* a level holds NaN or infinity */
    STENCIL_CHECK_OVERFLOW = 2,  /* a level holds infinity: a value overflowed its storage type */
    STENCIL_CHECK_UNSTABLE = 4,  /* stability > 1: the run grows without bound */
    STENCIL_CHECK_BAD_BETA = 8   /* beta holds NaN or infinity */
};

/* On-demand scan of a sweep plan's fields (fields as in stencil_run; heat:
 * fields[0]; wave: the levels fields[0], fields[1] and beta fields[2]) for
 * non-finite values, their largest magnitude and the stability condition.
 * A failure check (no passage of the paper: the method has no failure
 * detection; the stability bound is the von Neumann one of
 * stencil_stability).  Synchronises `stream`
 * (the report is host data on return). */
stencil_status stencil_check(stencil_plan plan, void* const* fields, stencil_check_report* out, void* stream);

/* ------------------------------------------------------------ variants */

/* Kernel variants of a plan (this library's kernel choices: no passage of
 * the paper; the temporally blocked ones follow the overlapped temporal
 * blocking of Section 7's related work).  Variant 0 is the
 * one-thread-per-point kernel.
 * 3D plans add the z-marching sweep (tile shape and z-chunk), and for the
 * radius-4 wave and the FP32 heat with the zero halo the depth-2 temporally
 * blocked sweep (two steps per launch).  2D FP32 heat plans with the zero
 * halo and radius <= 2 add multi-step kernels (T = 4, 8 or 16 steps per
 * launch in LDS).  Program plans have their own three (see
 * stencil_program_create).  Every variant of a plan computes identical bits.
 * stencil_tune times the candidates on the caller's fields (reading them
 * only; outputs go to a scratch field it allocates and frees) and keeps the
 * fastest per step of one launch (2D multi-step plans: per step of 96
 * steps captured in a graph, as runs execute them); the choice is cached per
 * (device architecture, kind, ndim, radius, halo, boundary, dtype, damping,
 * shapes, field bytes), as a variant name.  With STENCIL_TUNE_CACHE set to a
 * file path the cache is read from that file on the first tuning of the
 * process and every new choice is appended to it ("<arch> <key> <name>" per
 * line); a cached name the plan does not offer is ignored and re-tuned.  With
 * STENCIL_FORCE_VARIANT set to a comma-separated list of variant names,
 * tuning picks the first one the plan offers without timing.  A batch plan's
 * last variant, "shots_concurrent_4", runs every shot with its own plan
 * (tuned with the batch, so each shot gets its own fastest variant) and
 * spreads the shots over four streams forked from and joined back to the
 * caller's stream, captured in one graph.  For a program plan `fields`
 * holds its nin input pointers, then its nout output pointers: the compiled
 * variants (0, 2 and 3 where it exists) are applied to them, the fastest
 * is kept, and the outputs hold the program's result (not cached; the
 * first apply of each variant compiles and loads it, outside capture). */
stencil_status stencil_variant_count(stencil_plan plan, int* count);

/* Name of variant `variant` (no passage of the paper: kernel choice), e.g.
 * "tb2_64x32_t768_zc256", at most len - 1 characters. */
stencil_status stencil_variant_name(stencil_plan plan, int variant, char* buf, size_t len);

/* The plan's current variant (no passage of the paper: kernel choice). */
stencil_status stencil_get_variant(stencil_plan plan, int* variant);

/* Select a variant (no passage of the paper: kernel choice); every variant
 * computes the same bits.  Batch plans take z-marching variants only. */
stencil_status stencil_set_variant(stencil_plan plan, int variant);

/* Time the candidates and keep the fastest, as described above (no passage
 * of the paper: autotuning of the launch shape). */
stencil_status stencil_tune(stencil_plan plan, void* const* fields, int reps, void* stream);

/* Message of the last error on this thread (no passage of the paper: error
 * reporting). */
const char* stencil_last_error(void);

/* Version of this ABI, 2 (no passage of the paper). */
int stencil_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* STENCIL_H */

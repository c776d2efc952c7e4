/*
 * dg.h -- C ABI of libdg, the MI355X (gfx950) library that advances nodal
 * discontinuous Galerkin (NDG) discretisations of periodic linear advection
 * and isothermal Euler in one, two and three dimensions with explicit
 * Runge-Kutta schemes.
 *
 * Method (Sporykhin & Homann, "Performance of a high-order MPI-Kokkos
 * accelerated fluid solver", arXiv:2510.05254):
 *   - the conservation law dU/dt + sum_d dF_d(U)/dx_d = 0 (Sec. 2.1, eq.
 *     scalar_cons; eqs. advection1d, advection2d, eulerIso2d);
 *   - tensor-product elements of N+1 Legendre-Gauss-Lobatto nodes per
 *     direction with the lumped LGL mass (Sec. 2.1, eqs. lagrange_pol,
 *     lag_coefs), the weak-form evolution equation of Sec. 2.1 and the
 *     Lax-Friedrichs numerical flux with alpha the largest absolute flux
 *     eigenvalue of the two traces at each face point (eq. LF);
 *   - periodic boundaries (Sec. 3.1);
 *   - the RK schemes of Sec. 2.3: RK3 (read as Heun's third-order method,
 *     whose coefficients the printed eq. RK3 carries), classical RK4 (eq. RK4)
 *     and Luther's sixth-order RK6 (eq. RK6);
 *   - the L2 norm of Sec. 3.1, integrated with the nodal LGL rule.
 *
 * Mesh: the periodic unit domain [0,1)^dim with K[d] uniform elements along
 * direction d, dx_d = 1/K[d]. Element e covers [e_d dx_d, (e_d+1) dx_d] and its
 * node i along d sits at x = e_d dx_d + (dx_d/2)(xi_i + 1).
 *
 * State layout ("canonical", used by every array crossing this ABI):
 *   u[v * nodes + e * Np + n], Np = (N+1)^dim, nodes = prod(K) * Np,
 *   e = e_x + K[0] (e_y + K[1] e_z), n = i + (N+1)(j + (N+1) k),
 * i.e. variable-major, then element (x fastest), then node (x fastest).
 * Variables: advection (U); isothermal Euler (rho, rho u_1, ..., rho u_dim).
 * Face nodes are stored once per element (discontinuous representation).
 *
 * Ownership: a dg_solver owns its device memory (unless a workspace is passed
 * to dg_create_ex) and its HIP stream (unless one is passed). The caller owns
 * every host and device array it passes; the library copies from them before
 * the call returns (host arrays) or in stream order (device arrays).
 *
 * Errors: every entry point returns DG_OK or a negative status; nothing
 * throws across the ABI. A failed call leaves the solver's state unchanged.
 * dg_last_error() gives a message for the calling thread's last failure.
 * Arguments are validated before any device is touched, so invalid arguments
 * give DG_EINVAL even on a machine without a GPU.
 *
 * Threading: one host thread at a time per solver; distinct solvers are
 * independent.
 */
#ifndef DG_H
#define DG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dg_solver dg_solver;
typedef struct dg_batch dg_batch;

enum dg_status {
    DG_OK = 0,
    DG_EINVAL = -1,   /* invalid argument */
    DG_ENOMEM = -2,   /* device memory (or the given workspace) too small */
    DG_EDEVICE = -3,  /* no usable GPU, or a HIP call failed */
    DG_ENOTSUP = -4,  /* valid request the library does not support */
    DG_ESTATE = -5    /* call out of order (e.g. stepping before a state is set) */
};

enum dg_equation { DG_ADVECTION = 0, DG_EULER_ISOTHERMAL = 1 };
enum dg_rk { DG_RK3 = 3, DG_RK4 = 4, DG_RK6 = 6 };
enum dg_precision { DG_FP64 = 0, DG_FP32 = 1 };

#define DG_MAX_ORDER 8   /* polynomial degree N ranges over 1..DG_MAX_ORDER */

/* Create a solver on the current HIP device, FP64, own stream, own memory.
 * Defining passages: the element partition of the periodic domain and the
 * map from the reference element (Sec. 2.1, eq. transformation), N+1 LGL
 * nodes per direction (Sec. 2.1 node definition, eqs. lagrange_pol and
 * lag_coefs), the fluxes of eqs. advection1d/advection2d (advection) and
 * eulerIso2d (isothermal Euler, restricted to (rho, rho u_x) in 1-D and
 * extended by rho u_z in 3-D), the Lax-Friedrichs flux of eq. LF, periodic
 * boundaries (Sec. 3.1).
 *   dim       1, 2 or 3
 *   N         polynomial degree, 1..8 (N+1 LGL nodes per direction)
 *   K         K[0..dim-1] >= 1, elements per direction (K[d] = 1 is its own
 *             periodic neighbour)
 *   equation  DG_ADVECTION: params = a[0..dim-1], the advection velocity
 *             (finite); DG_EULER_ISOTHERMAL: params = {c_s}, the sound speed
 *             (finite, > 0)
 *   out       receives the handle
 * Returns DG_EINVAL, DG_ENOMEM or DG_EDEVICE on failure. */
int dg_create(int dim, int N, const int64_t *K, int equation, const double *params,
              dg_solver **out);

/* dg_create with options (same method and passages as dg_create):
 *   precision        DG_FP64 or DG_FP32 (state, RHS and stage updates in that
 *                    type; L2 and mass reductions always accumulate in FP64)
 *   hip_stream       a hipStream_t to run on, or NULL for a library stream
 *   device_workspace device memory of workspace_bytes the library carves its
 *                    arrays from, or NULL to let the library allocate. With a
 *                    workspace the library never allocates device memory;
 *                    its size must be at least dg_workspace_bytes(..., rk)
 *                    for every rk the caller will step with (DG_ENOMEM from
 *                    dg_step otherwise). It must outlive the solver. */
int dg_create_ex(int dim, int N, const int64_t *K, int equation, const double *params,
                 int precision, void *hip_stream, void *device_workspace,
                 size_t workspace_bytes, dg_solver **out);

/* Device bytes a solver needs to step with scheme rk (3, 4 or 6): the
 * operator tables plus the state and the Runge-Kutta work arrays of the
 * scheme's stage schedule (Sec. 2.3, eqs. RK3, RK4, RK6): four state arrays
 * for RK3 and RK4, nine for RK6, whose seven stage vectors k_s are stored.
 * The scheme is an argument because the two sizes differ by five state
 * arrays (5 GB at 3-D 64^3 N = 4 FP64): a caller that will only step with
 * RK3/RK4 need not provide RK6's storage.
 * DG_EINVAL for an invalid mesh, equation, precision or rk, or bytes NULL. */
int dg_workspace_bytes(int dim, int N, const int64_t *K, int equation, int precision, int rk,
                       size_t *bytes);

/* Release the solver (waits for its stream) and the memory it owns. NULL is
 * accepted. A solver in a batch is removed from it first. */
int dg_destroy(dg_solver *h);

/* nvar = number of conserved variables (1 for advection, 1 + dim for
 * isothermal Euler: eqs. advection2d, eulerIso2d); nodes = prod(K) (N+1)^dim
 * (N+1 LGL nodes per direction per element, Sec. 2.1). A state array holds
 * nvar * nodes doubles. Either pointer may be NULL. */
int dg_sizes(const dg_solver *h, int *nvar, int64_t *nodes);

/* Node coordinates along one axis: x[e*(N+1) + i] = e dx + (dx/2)(xi_i + 1),
 * dx = 1/K[axis], xi_i the LGL nodes (Sec. 2.1 partition, eq. transformation
 * with the element offset), count = K[axis] (N+1). DG_EINVAL for a bad axis
 * or count. */
int dg_get_axis_coords(const dg_solver *h, int axis, double *x, int64_t count);

/* Node coordinates of every node: xyz[d * nodes + e * Np + n] is coordinate d
 * of node n of element e in the canonical layout above (the tensor product of
 * dg_get_axis_coords), count = dim * nodes doubles, host array owned by the
 * caller (Sec. 2.1 partition, eq. transformation). DG_EINVAL for a NULL
 * pointer or a count mismatch. */
int dg_get_coords(const dg_solver *h, double *xyz, int64_t count);

/* Copy a host state (canonical layout, count = nvar * nodes doubles) in: the
 * nodal values U_v(x_n) of the conserved variables (Sec. 2.1, the nodal
 * representation of eq. lagrange_pol). Synchronous with respect to the host
 * buffer; stream-ordered on the device. In FP32 solvers the values are
 * rounded to single precision. DG_EINVAL on a count mismatch, DG_ESTATE for a
 * batch member. */
int dg_set_state(dg_solver *h, const double *u, int64_t count);

/* As dg_set_state (the nodal values of Sec. 2.1) from a device array of count
 * FP64 values (stream-ordered; the caller keeps it alive until the solver's
 * stream has passed this point). DG_EINVAL on a count mismatch, DG_ESTATE for
 * a batch member. */
int dg_set_state_device(dg_solver *h, const void *u_dev, int64_t count);

/* Advance nsteps steps of size dt with scheme rk (DG_RK3, DG_RK4, DG_RK6) of
 * the semi-discrete system dU/dt = R(U) (Sec. 2.3, eqs. RK3 -- read as Heun's
 * third-order method --, RK4, RK6), where R is the NDG right-hand side of the
 * weak-form evolution equation of Sec. 2.1 (volume term with the LGL
 * differentiation matrix, Lax-Friedrichs flux of eq. LF at the faces, lift
 * by the lumped mass of eq. lag_coefs), evaluated on every element of the
 * periodic mesh. Asynchronous: enqueues the stage kernel launches on the
 * solver's stream and returns. dt must be finite and > 0, nsteps >= 0 (0 is a
 * no-op). DG_EINVAL for a bad rk/dt/nsteps, DG_ESTATE before the first
 * set_state or for a batch member, DG_ENOMEM when RK6 storage cannot be had.
 * No blow-up check is made. */
int dg_step(dg_solver *h, int rk, double dt, int64_t nsteps);

/* Copy the current state out (waits for the stream). count = nvar * nodes,
 * canonical layout, host array owned by the caller. DG_EINVAL on a count
 * mismatch, DG_ESTATE before the first set_state. */
int dg_get_state(dg_solver *h, double *u, int64_t count);

/* As dg_get_state (the nodal values of Sec. 2.1) into a device array of count
 * FP64 values (stream-ordered). DG_EINVAL on a count mismatch, DG_ESTATE
 * before the first set_state. */
int dg_get_state_device(dg_solver *h, void *u_dev, int64_t count);

/* L2 error of the current state against a host reference u_ref (canonical
 * layout, count = nvar * nodes), over all variables (Sec. 3.1 L2 norm, nodal
 * LGL quadrature with the element Jacobian):
 *   abs_err = sqrt(sum_v integral (U_v - Uref_v)^2),
 *   rel_err = abs_err / sqrt(sum_v integral Uref_v^2)
 * (rel_err = inf when the reference is zero). FP64 accumulation; waits for
 * the stream. Either output pointer may be NULL. */
int dg_l2_error(dg_solver *h, const double *u_ref, int64_t count, double *abs_err,
                double *rel_err);

/* Per-variable squared L2 norms (Sec. 3.1 L2 norm, nodal LGL quadrature with
 * the element Jacobian): sq_err[v] = integral (U_v - Uref_v)^2 and
 * sq_ref[v] = integral Uref_v^2 (arrays of nvar doubles). FP64; waits. */
int dg_l2_error_vars(dg_solver *h, const double *u_ref, int64_t count, double *sq_err,
                     double *sq_ref);

/* mass[v] = integral of U_v over the domain (nvar doubles) with the nodal
 * LGL quadrature of the lumped mass (eq. lag_coefs; the conserved integral
 * of the conservation law of Sec. 2.1, eq. scalar_cons), FP64; waits. */
int dg_mass(dg_solver *h, double *mass);

/* Wait for all work enqueued on the solver's stream (no computation); for a
 * batch member also for the batch work enqueued so far. */
int dg_synchronize(dg_solver *h);

/* The solver's hipStream_t (as void*), for stream-ordered interop; NULL for
 * a NULL handle. For a batch member the stream is first made to wait for the
 * batch work enqueued so far (work the batch enqueues later is not ordered
 * before what the caller then puts on the stream: call dg_stream again). */
void *dg_stream(const dg_solver *h);

/* Autotune the launch configuration (no change to the method: every
 * candidate evaluates the same Sec. 2.1 right-hand side and Sec. 2.3 scheme
 * bit for bit) for stepping h with scheme rk and step
 * dt: times trial_steps (1..1000) steps of each candidate on the solver's
 * arrays, restarting from a saved copy of the state, restores the state and
 * keeps the fastest candidate for later dg_step calls. Candidates: 3-D, the
 * tile order (XCD-contiguous or plain) x the z-slab size x the x-block
 * width, then the z-march length; 2-D, the tile order; 1-D RK3/RK4 meshes
 * split into chunks, the elements per workgroup (cfg[6]) x the steps per
 * launch (via the halo bound). Every candidate computes the same
 * results bit for bit; only speed differs. Synchronous. The tuner keeps
 * one copy of the state: a library-owned workspace allocates it; an external
 * workspace must hold it after the scheme's arrays, i.e. be at least
 * dg_workspace_bytes(rk) plus one state array (nvar * nodes values of the
 * state precision, rounded up to 256 bytes), DG_ENOTSUP otherwise.
 * DG_ESTATE before the first set_state or for a batch member. */
int dg_autotune(dg_solver *h, int rk, double dt, int trial_steps);

/* The launch configuration in use: cfg[0] tile order (0 XCD-contiguous,
 * 1 plain; by default plain for 2-D meshes whose x-tile count is a
 * multiple of 8, XCD-contiguous otherwise), cfg[1] z-slab size (z-units visited together), cfg[2] 1-D
 * halo-bound divisor (steps per launch at most capacity / (cfg[2] * stages),
 * default 10; a mesh split into one chunk per CU lowers it further until
 * the chunk and its halos fit),
 * cfg[3] 1 once autotuned, cfg[4] x-block width (x-tiles visited together;
 * the number of x-tiles by default), cfg[5] z-march length (3-D RK3/RK4: a
 * workgroup runs cfg[5] consecutive layers of one tile column bottom to top
 * and takes each lower z-face's other side from the layer it ran before;
 * 1 = one layer per workgroup), cfg[6] 1-D elements per workgroup (0: a
 * chunk per CU, the default; -1: the chunks the halo bound leaves, capacity
 * minus both halos; k > 0: k owned elements when they fit with the halos).
 * Writes min(n, 7) entries and zeros beyond. */
int dg_launch_config(const dg_solver *h, int64_t *cfg, int n);

/* Set the launch configuration (same layout as dg_launch_config, n = 7;
 * cfg[3] is ignored and the autotuned flag cleared), e.g. to reapply a
 * configuration found by dg_autotune in an earlier run. 3-D: cfg[5] in
 * 1..K[2], cfg[1] must divide the number of z-units ceil(K[2] / cfg[5]) and
 * cfg[4] the number of x-tiles; 1-D/2-D: cfg[1], cfg[4] and cfg[5] must
 * equal the values in use. cfg[0] in {0, 1}, cfg[2] in 1..1024, cfg[6] in
 * -1..2^30 (any dimension; used by 1-D RK3/RK4 meshes split into chunks). Every
 * configuration computes the same results bit for bit. DG_EINVAL on a bad
 * entry (nothing changed), DG_ESTATE for a batch member. Takes effect at the
 * next dg_step; work already enqueued is unaffected. */
int dg_set_launch_config(dg_solver *h, const int64_t *cfg, int n);

/* ---------------------------------------------------------------------------
 * Batched stepping (many solves advanced together; the method per solve is
 * unchanged: every member takes the same Sec. 2.3 RK steps of the Sec. 2.1
 * right-hand side it would take alone). Small grids leave a GPU mostly idle
 * (the paper's Sec. 3.2 finds GPUs efficient only from about 1e6-1e7 degrees
 * of freedom), so many small solves share each launch.
 *
 * A batch advances its member solvers on the batch's stream. Each "tick" is
 * one RK step of every active member; all members that share a kernel class
 * (precision, equation, dim, N) and scheme are advanced by one launch per RK
 * stage (1-D RK3/RK4: per launch of the temporally blocked kernel), whatever
 * their meshes, arrays and time steps, so many small solves fill the GPU
 * together; different classes run concurrently on up to four streams forked
 * from the batch stream and joined back within every dg_batch_run. Members
 * keep their own state arrays; results are bitwise those of dg_step on the
 * same member alone.
 * ------------------------------------------------------------------------ */

#define DG_BATCH_GRAPH 1   /* replay ticks from a captured hipGraph of one tick
                              (captured at the first run of >= 4 ticks after a
                              membership change; shorter runs launch directly) */

/* Create an empty batch on the current device. hip_stream: hipStream_t to run
 * on, or NULL for a library stream. flags: 0 or DG_BATCH_GRAPH. */
int dg_batch_create(void *hip_stream, int flags, dg_batch **out);

/* Wait for the batch's work and release it; members are released from it
 * (their handles stay valid). NULL is accepted. */
int dg_batch_destroy(dg_batch *b);

/* Add solver h (state set, on the batch's device, not in another batch) to
 * run nsteps >= 1 more steps of scheme rk (DG_RK3, DG_RK4 or DG_RK6) with
 * step dt > 0. RK6 members need the RK6 stage store as dg_step does (an
 * external workspace of dg_workspace_bytes(..., DG_RK6), else DG_ENOMEM; a
 * library-owned one allocates it here). While a member, h must not be stepped
 * or have its state set directly (DG_ESTATE); dg_get_state,
 * dg_get_state_device, dg_l2_error, dg_mass, dg_synchronize and dg_stream on
 * it are stream-ordered after the batch work enqueued so far (h's stream
 * waits for the batch when h is read, not after every dg_batch_run), and
 * dg_get_state_device's copy is ordered before later batch work. */
int dg_batch_add(dg_batch *b, dg_solver *h, int rk, double dt, int64_t nsteps);

/* Remove member h (finished or not); its remaining steps are dropped. */
int dg_batch_remove(dg_batch *b, dg_solver *h);

/* Enqueue (Sec. 2.3 steps of every active member) s = min(max_steps,
 * smallest remaining step count of the active
 * members) ticks and return s in *steps_done (0 when no member is active).
 * Members whose remaining count reaches 0 become inactive (they stay members
 * until removed). Asynchronous. */
int dg_batch_run(dg_batch *b, int64_t max_steps, int64_t *steps_done);

/* Steps member h still has to run. */
int dg_batch_remaining(const dg_batch *b, const dg_solver *h, int64_t *remaining);

/* Number of members and of active members. Either pointer may be NULL. */
int dg_batch_size(const dg_batch *b, int *members, int *active);

/* Wait for all work enqueued on the batch's stream. */
int dg_batch_synchronize(dg_batch *b);

/* ---------------------------------------------------------------------------
 * Stepping without device allocation.
 * ------------------------------------------------------------------------ */

/* Bytes of the fixed device array dg_step_static takes its work memory from
 * (one array per GPU the library runs on, held until the process ends). */
#define DG_STATIC_SCRATCH_BYTES (128u << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): dg_step on
 * a device state the caller holds, with no solver handle and no device
 * allocation by the library (no hipMalloc, hipFree or allocating library
 * routine on any path).
 *   dim, N, K, equation, params, precision   as dg_create_ex
 *   hip_stream   hipStream_t to run on, or NULL for the null stream
 *   u_dev        device array of count = nvar * nodes values in the state
 *                precision (double for DG_FP64, float for DG_FP32),
 *                canonical layout, aligned to its element size; advanced in
 *                place. Owned by the caller.
 *   rk, dt, nsteps   as dg_step (DG_RK3, DG_RK4, DG_RK6; nsteps 0 is a no-op)
 * Work memory: the operator tables, the Runge-Kutta work arrays (3 state
 * arrays for RK3/RK4, 8 for RK6) and, for isothermal Euler, the device-layout
 * copy of the state (1 more array) come from the library's fixed device array
 * of DG_STATIC_SCRATCH_BYTES bytes on the current device. A problem needing
 * more gives DG_ENOMEM, with the bytes needed in dg_last_error() (limit for
 * RK4 advection: about DG_STATIC_SCRATCH_BYTES / 3 bytes per state array,
 * e.g. 2-D advection 256^2 N = 7 in FP64).
 * Asynchronous like dg_step, except that a call whose (dim, N, equation,
 * precision) differs from the previous call's on the same device uploads the
 * operator tables and waits for hip_stream. Results are bitwise those of a solver made
 * with dg_create_ex on the same arguments, given the same state and stepped
 * with dg_step.
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind: calls whose work overlaps on one GPU (on other streams or from
 * other host threads while earlier work is still in flight) race and give
 * undefined results; issue them on one stream or synchronize between them.
 * DG_EINVAL for invalid arguments (as dg_create_ex and dg_step, plus a NULL
 * or misaligned u_dev or a count mismatch), DG_ENOTSUP for an unbuilt class,
 * DG_EDEVICE for a HIP failure. */
int dg_step_static(int dim, int N, const int64_t *K, int equation, const double *params,
                   int precision, void *hip_stream, void *u_dev, int64_t count, int rk, double dt,
                   int64_t nsteps);

/* ---------------------------------------------------------------------------
 * Measurement helper (no part of the method).
 * ------------------------------------------------------------------------ */

/* Streaming bandwidth reference: one launch on hip_stream (NULL = the null
 * stream) that reads nin (1..3) device arrays and writes nout (1..2) device
 * arrays of `bytes` bytes each (a positive multiple of 16; 16-byte aligned
 * pointers, owned by the caller): out_o[i] = sum_j in_j[i] + o over pairs of
 * doubles, one coalesced 16-byte access per thread and array. Timing the four
 * (nin, nout) mixes of a fused RK4 stage schedule on arrays of the state's
 * size gives the rate plain streaming of the stage kernels' algorithmic bytes
 * reaches (the roofline reference beside the HBM peak). Asynchronous.
 * DG_EINVAL on a bad count, size, NULL or misaligned pointer. */
int dg_bandwidth_probe(void *hip_stream, const void *const *in, int nin, void *const *out,
                       int nout, int64_t bytes);

/* Message for the calling thread's last non-OK return ("" if none). Owned by
 * the library, valid until the thread's next failing call. */
const char *dg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DG_H */

/*
 * lbm.h -- C ABI of the MI355X (gfx950) D2Q9 lattice Boltzmann library.
 *
 * The library advances the fused stream-and-collide BGK update of the
 * incompressible D2Q9I model (PortLBM paper, Section 3.1, Eq. 1-2) on one GPU,
 * with halfway bounce-back at solid nodes, a fixed-equilibrium inlet, a
 * zero-gradient outlet and an optional constant body force.  Every scheme and
 * data layout computes the same update; they differ only in how populations
 * are stored and moved (paper, Sections 3.2 and 3.3).
 *
 * Conventions shared by every entry point
 *   - Grids are nx * ny nodes, node (x, y) with x fastest and y growing
 *     upwards.  Host arrays exchanged through this ABI are dense row-major
 *     [ny][nx] (per component / direction), independent of the internal
 *     layout, which pads rows internally.
 *   - Directions follow Fig. 2 (b) of the paper: i = 0..8 is SW, S, SE, W,
 *     rest, E, NW, N, NE, i.e. c_i = (i mod 3 - 1, i div 3 - 1).
 *   - Populations crossing the ABI are *shifted*: f~_i = f_i - w_i, with
 *     w_i the Eq. 2 weights, as FP32.
 *   - Every function returns an lbm_status; no C++ exception crosses the ABI.
 *     After a device error (LBM_EDEVICE) a context is poisoned: every later
 *     call on it returns LBM_EDEVICE again.  lbm_last_error() gives a text.
 *   - Work is ordered on the context's HIP stream and is asynchronous unless
 *     stated.  A context is not thread-safe; distinct contexts are independent.
 *   - Pointers marked "host or device" are read/written on the device when
 *     on_device != 0 (they must then be device pointers valid on the context's
 *     device and stream), else they are host pointers and the call
 *     synchronizes the stream before returning.
 */
#ifndef LBM_H
#define LBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,    /* invalid argument; nothing was allocated or changed */
    LBM_ENOMEM = -2,    /* device memory exhausted; nothing was kept */
    LBM_EDEVICE = -3,   /* HIP runtime or kernel launch failure (sticky) */
    LBM_EUNSTABLE = -4, /* diagnostics found non-finite mass or momentum */
    LBM_EBUSY = -5,     /* serving: no slot / memory free now, try later */
    LBM_ENOTFOUND = -6  /* serving: unknown or not yet finished request id */
} lbm_status;

/* Propagation schemes (paper Section 3.3). */
typedef enum {
    LBM_LPTL = 0,    /* linear pull, two lattices: 1-D launch, runtime-chosen block */
    LBM_NPTL = 1,    /* tiled (2-D decomposition) pull, two lattices */
    LBM_TL_PUSH = 2, /* tiled one-step push, two lattices */
    LBM_NPOL = 3,    /* tiled pull, one lattice + buffer grid between tiles */
    LBM_NSOL = 4,    /* tiled swap scheme, one lattice + buffer grid */
    LBM_AA = 5       /* in-place AA streaming (Bailey et al.), the state-of-the-art one-lattice
                        scheme Section 3.3 cites and Section 6 names as the next step: even
                        updates are local, odd updates exchange pairwise with the neighbours;
                        one lattice, no buffer grid, 3 values per row of outlet side buffer */
} lbm_scheme;

/* Data layouts (paper Section 3.2, Fig. 2). */
typedef enum {
    LBM_STREAM = 0,   /* SoA: plane i, then node */
    LBM_BUNDLE = 1,   /* SoAoS: bundle (c_y), node, then c_x within the bundle */
    LBM_COLLISION = 2, /* AoS: node, then the 9 directions */
    LBM_BLOCKED = 3    /* D3Q19 only, AoSoA: rows cut into blocks of 64 nodes, each block
                          holding its 19 directions one after the other, 64 nodes each */
} lbm_layout;

/* Storage precision of the shifted populations; arithmetic is always FP32. */
typedef enum {
    LBM_FP32 = 0,
    LBM_FP16S = 1,   /* IEEE binary16, round-to-nearest-even on store */
    LBM_FP16S_SR = 2, /* IEEE binary16, deterministic stochastic rounding of every updated
                        value: rounded away from zero with probability equal to its position
                        between the two nearest binary16 values, decided by random bits from
                        a hash of the node index and three of the node's post-collision FP32
                        values (the same in every scheme and layout); initial and loaded
                        states round to nearest even */
    LBM_FP16C = 3,   /* custom 16-bit float for shifted populations (the customised 16-bit
                        formats of the related work on low-precision lattice storage): sign,
                        4 exponent bits, 11 fraction bits, bias 15 -- normal values
                        2^(e-15)(1 + m/2^11) in [2^-14, 2), subnormals m 2^-25, code 0x7fff
                        (either sign) NaN, also for values that round beyond the largest
                        finite one (1.99902); one fraction bit more than binary16 where
                        shifted populations lie.  Rounds to nearest even: the bits of the
                        FP32 value times 2^-112 with 12 bits dropped */
    LBM_FP16C_SR = 4 /* FP16C with stochastic rounding of every updated value (the same
                        random bits as LBM_FP16S_SR, 12 of them added below the dropped
                        bits); initial and loaded states round to nearest even */
} lbm_precision;

typedef enum {
    LBM_PERIODIC = 0,
    LBM_CLOSED = 1,        /* outside the box acts as a solid wall */
    LBM_INFLOW_OUTFLOW = 2, /* x only: column 0 inlet, column nx-1 zero-gradient outlet */
    LBM_INFLOW_PRESSURE = 3, /* x only: column 0 inlet, column nx-1 pressure outlet (the Zou-He
                                condition Section 3.1 adapts): an outlet node's three incoming
                                values with c_x = -1 are rebuilt from its six others so that its
                                incoming density is rho0 and its tangential momentum zero */
    LBM_NEUMANN_OUTFLOW = 4,  /* as LBM_INFLOW_OUTFLOW with the Neumann inlet of Section 3.1: the
                                 inlet node of row y holds feq(rho_in, u_in), rho_in being the
                                 density of node (1, y) after the previous update (zero normal
                                 density gradient) instead of rho0 */
    LBM_NEUMANN_PRESSURE = 5  /* the Neumann inlet and the pressure outlet */
} lbm_axis;

enum { LBM_FLUID = 0, LBM_SOLID = 1 }; /* user flag values */

typedef struct {
    int64_t nx, ny;
    int32_t scheme;    /* lbm_scheme */
    int32_t layout;    /* lbm_layout */
    int32_t precision; /* lbm_precision */
    int32_t tile_x;    /* tiled schemes: tile width in nodes; 0 (with tile_y 0) = automatic */
    int32_t tile_y;    /* tile height in nodes.  A tile is one block of at most 256 threads
                          (1024 for the one-lattice schemes), one node per thread (two for the
                          FP16S bundle tiled pull when tile_x is even) */
} lbm_grid;

typedef enum {
    LBM_HALFWAY = 0, /* halfway bounce-back at fluid-solid links (Section 3.1) */
    LBM_FULLWAY = 1  /* full-way bounce-back: solid nodes hold populations (at rest initially),
                        take in what streams into them and send it back reversed one update
                        later; fluid nodes pull from them like from any node.  Closed sides
                        stay halfway.  Schemes LBM_LPTL and LBM_NPTL; x axis periodic,
                        closed or LBM_INFLOW_OUTFLOW; not served by lbm_server_* */
} lbm_bounce;

typedef struct {
    int32_t x_axis, y_axis; /* lbm_axis; the kinds with an inlet and an outlet (2 to 5): x only */
    double u_in[2];         /* inlet velocity (x axis with an inlet) */
    double g[2];            /* body force per node and step */
    double rho0;            /* reference density; must be 1 */
    double u0[2];           /* initial velocity of fluid and outlet nodes */
    int32_t bounce;         /* lbm_bounce at solid nodes */
} lbm_bc;

typedef struct lbm_ctx lbm_ctx;

/*
 * lbm_create -- allocate and initialise one simulation.
 *   grid    : sizes, scheme, layout, precision, tile.  nx, ny >= 1; nx >= 2
 *             with an inflow/outflow x axis.
 *   flags   : host, nx*ny bytes [ny][nx], LBM_FLUID or LBM_SOLID; copied.
 *   tau     : BGK relaxation time (Eq. 1), finite and > 1/2.
 *   bc      : axis kinds, inlet velocity, body force, rho0 (= 1), u0.
 *   stream  : hipStream_t to order all work on, or NULL for a private stream.
 *   out     : receives the context.  On error *out is NULL and nothing is
 *             allocated; lbm_last_error(NULL) describes the failure.
 * Node types: solid where flagged; with an inflow/outflow x axis column 0 is
 * the inlet and column nx-1 the outlet, solid winning at corners.  Initial
 * state: fluid and outlet nodes hold feq(1, u0) (Eq. 2), the inlet
 * feq(1, u_in).  Synchronizes the stream before returning.
 */
lbm_status lbm_create(const lbm_grid* grid, const uint8_t* flags, double tau, const lbm_bc* bc, void* stream,
                      lbm_ctx** out);

/* lbm_step -- enqueue n >= 0 lattice updates (Eq. 1; streaming per scheme).
 * Asynchronous; consecutive calls replay cached HIP graphs of K updates. */
lbm_status lbm_step(lbm_ctx* ctx, int64_t n);

/*
 * lbm_macros -- macroscopic readout at the current time (Eq. 2 moments of the
 * incoming populations).  rho: nx*ny floats [ny][nx]; u: 2*nx*ny floats
 * [2][ny][nx] (x component first).  Fluid and outlet nodes: rho = sum f_i,
 * u = sum f_i c_i + g/2; inlet nodes: rho = 1, u = u_in; solid nodes 0.
 * Either pointer may be NULL.  Host or device per on_device.
 */
lbm_status lbm_macros(lbm_ctx* ctx, float* rho, float* u, int on_device);

/*
 * lbm_diag -- FP64 reductions over fluid and outlet nodes:
 *   out[0] = total mass sum rho, out[1..2] = total momentum sum (sum f_i c_i)
 *   (without the g/2 shift), out[3] = ||u_t - u_prev||_2 / ||u_t||_2 against
 *   the velocity field of the previous lbm_diag call (-1 on the first call
 *   and after lbm_set_state).  Every sum is taken in FP64 from the stored
 *   populations, and the previous velocities are kept in FP64 (2 doubles per
 *   node), so the residual has no storage floor of its own.
 * Synchronizes.  Returns LBM_EUNSTABLE when mass or momentum is not finite
 * (the values are still written).  The previous-velocity buffer and the
 * reduction partials are allocated on the first call (LBM_ENOMEM if that
 * fails).
 */
lbm_status lbm_diag(lbm_ctx* ctx, double out[4]);

/*
 * lbm_diag_noalloc -- the diagnostics of lbm_diag for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): it allocates nothing and does not
 * synchronize.  It enqueues on the context's stream the same FP64 reductions
 * as lbm_diag, with their partial sums in a fixed device array of the library
 * (41 KB per GPU, held until the process ends; enough for any grid size), and
 * writes to `out`, device memory of 4 doubles: mass, momentum x, momentum y
 * (as lbm_diag) and the residual ||u_t - u_prev||_2 / ||u_t||_2, or -1 when
 * have_prev is 0.
 *   u_prev: device memory of 2 * nx * ny doubles, caller-owned, dense
 *   [ny][nx][2] (u_x, u_y per node): read when have_prev is nonzero, then
 *   overwritten with the current velocities; NULL (with have_prev 0) computes
 *   no residual.
 * Non-finite results are written as they are (the caller checks them; an
 * asynchronous call cannot return LBM_EUNSTABLE).  LBM_EINVAL for NULL ctx or
 * out, or have_prev without u_prev.  Calls that overlap on one GPU race on the
 * shared array: order them (one stream, or events).
 */
lbm_status lbm_diag_noalloc(lbm_ctx* ctx, double* u_prev, int32_t have_prev, double* out);

/* lbm_get_populations -- shifted incoming (pre-collision) populations at the
 * current time, 9*nx*ny floats [9][ny][nx]; inlet nodes get the inlet
 * equilibrium, solid nodes 0.  Host or device per on_device. */
lbm_status lbm_get_populations(lbm_ctx* ctx, float* f, int on_device);

/* lbm_set_state -- replace the state by the shifted post-collision values f*
 * (9*nx*ny floats [9][ny][nx]) of every fluid and outlet node, i.e. the values
 * about to stream; they are rounded to the storage precision.  Values at inlet
 * and solid nodes are ignored.  The step counter is kept.  Host or device. */
lbm_status lbm_set_state(lbm_ctx* ctx, const float* f, int on_device);

typedef struct {
    int64_t steps;           /* updates done since create */
    int64_t nx, ny, pitch;   /* sizes and the internal (padded) row pitch */
    int32_t scheme, layout, precision;
    int32_t tile_x, tile_y;  /* tile chosen for tiled schemes (0 for LPTL) */
    int32_t block;           /* threads per block of the update kernel */
    int32_t bundle;          /* updates per cached HIP graph (0 = no graphs) */
    int64_t device_bytes;    /* device memory owned by the context */
    int64_t fluid_nodes;     /* fluid + outlet nodes */
} lbm_info;

lbm_status lbm_get_info(const lbm_ctx* ctx, lbm_info* info);

/* lbm_set_bundle -- updates per cached HIP graph used by lbm_step (0 = launch
 * each update directly).  Default 32. */
lbm_status lbm_set_bundle(lbm_ctx* ctx, int32_t k);

/* lbm_sync -- wait for all work enqueued on the context's stream. */
lbm_status lbm_sync(lbm_ctx* ctx);

/* lbm_last_error -- text of the last failure on ctx, or, for ctx == NULL, of
 * the calling thread's last failed lbm_create.  Never NULL. */
const char* lbm_last_error(const lbm_ctx* ctx);

/* lbm_destroy -- synchronize and free everything the context owns.  NULL-safe. */
void lbm_destroy(lbm_ctx* ctx);

/* lbm_bandwidth_probe -- measurement helper, not part of the method: a plain
 * grid-stride streaming kernel with 16-byte accesses on `stream` (a
 * hipStream_t, NULL = legacy default stream).  mode 0 copies `bytes` from src
 * to dst, mode 1 only reads src (dst: a 4-byte device sink, written only in a
 * practically impossible case), mode 2 only writes zeros to dst, mode 3
 * copies like mode 0 with non-temporal loads and stores and 8 pieces of 16
 * bytes in flight per lane (the practical copy peak).  bytes > 0
 * and a multiple of 16; device pointers, 16-byte aligned; caller-owned.
 * Asynchronous; LBM_EINVAL on bad arguments, LBM_EDEVICE on launch failure. */
lbm_status lbm_bandwidth_probe(int32_t mode, void* dst, const void* src, int64_t bytes, void* stream);

/* lbm_bytes_per_update -- algorithmic bytes one lattice update moves
 * per node (9 reads + 9 writes of the storage type, flag byte excluded):
 * 72 for FP32, 36 for every 16-bit format (FP16S, FP16S_SR, FP16C, FP16C_SR). */
int32_t lbm_bytes_per_update(int32_t precision);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of independent simulations on one GPU.
 *
 * Requests of any grid size are queued, admitted at bundle boundaries while a
 * slot and space in the HBM budget are free (arrival order, later requests
 * may pass one that does not fit yet), kept resident, and advanced together:
 * every bundle is one replay of a captured HIP graph of `bundle_steps`
 * launches of a persistent batched kernel, each launch one lattice update of
 * every resident request (two-lattice tiled pull, same arithmetic as
 * lbm_step, so a request's result is independent of the mix).  A request
 * stops at exactly its step count; its rho and u are then read back and its
 * memory freed.
 * ---------------------------------------------------------------------- */
typedef struct lbm_server lbm_server;

typedef struct {
    int32_t queued;             /* submitted, not admitted yet */
    int32_t running;            /* resident on the device */
    int32_t finished_unfetched; /* done, result waiting for lbm_server_fetch */
    int64_t pool_bytes, pool_used;
    int64_t bundles;            /* bundles launched with work */
    int64_t node_updates;       /* lattice-node updates completed */
} lbm_server_stats;

/* lbm_server_create -- hbm_budget_bytes (>= 1 MiB) is allocated at once as
 * the request pool; max_slots in [1, 65536] resident requests; bundle_steps in
 * [1, 4096] updates per graph replay; layout / precision for every request;
 * stream as in lbm_create.  lbm_server_last_error(NULL) explains failures. */
lbm_status lbm_server_create(int64_t hbm_budget_bytes, int32_t max_slots, int32_t bundle_steps, int32_t layout,
                             int32_t precision, void* stream, lbm_server** out);

/* lbm_server_submit -- queue one request (non-blocking).  grid gives nx, ny
 * (scheme, layout, precision and tile are the server's); flags, tau, bc as for
 * lbm_create (copied); steps >= 0.  LBM_ENOMEM when the request alone exceeds
 * the budget.  *id receives a positive request id. */
lbm_status lbm_server_submit(lbm_server* s, const lbm_grid* grid, const uint8_t* flags, double tau,
                             const lbm_bc* bc, int64_t steps, uint64_t* id);

/* lbm_server_run_bundle -- wait for the bundle in flight, retire requests that
 * reached their step count, admit what fits, and enqueue the next bundle
 * (asynchronous).  Cheap when idle. */
lbm_status lbm_server_run_bundle(lbm_server* s);

/* lbm_server_poll -- without blocking, report up to cap finished requests
 * (ids[k], status[k] = LBM_OK or LBM_EUNSTABLE for non-finite results) not
 * reported before; *n receives the count. */
lbm_status lbm_server_poll(lbm_server* s, uint64_t* ids, int32_t* status, int32_t cap, int32_t* n);

/* lbm_server_fetch -- copy a finished request's rho (nx*ny floats) and u
 * (2*nx*ny floats, [2][ny][nx]) to host memory (either may be NULL) and drop
 * it.  Returns its status; LBM_EBUSY if it is not finished, LBM_ENOTFOUND for
 * an unknown id. */
lbm_status lbm_server_fetch(lbm_server* s, uint64_t id, float* rho, float* u);

lbm_status lbm_server_get_stats(const lbm_server* s, lbm_server_stats* out);
const char* lbm_server_last_error(const lbm_server* s);

/* lbm_server_destroy -- synchronize and free everything.  NULL-safe. */
void lbm_server_destroy(lbm_server* s);

/* ------------------------------------------------------------------ D3Q19
 * The 3-D extension Section 6 of the paper names: the same update (BGK,
 * incompressible equilibrium of Eq. 2 with its 3-D velocity set, force term
 * 3 w_i (c_i . g), halfway bounce-back, inlet equilibrium, zero-gradient
 * outlet) on the D3Q19 lattice.
 *   - Grids are nx * ny * nz nodes; host arrays are dense [nz][ny][nx] per
 *     component / direction.
 *   - Directions: the 19 vectors c with components in {-1, 0, 1} and
 *     |c|^2 <= 2, ordered by (c_z, c_y, c_x) lexicographically: i = 9 is rest,
 *     opposite(i) = 18 - i.  Weights 1/3 (rest), 1/18 (|c| = 1), 1/36.
 *   - Populations crossing the ABI are shifted (f - w), FP32.
 *   - Schemes: LBM_NPTL (two lattices, one-step pull, tile_x * tile_y nodes
 *     of one z plane per block) and LBM_AA (one lattice in place).  Layouts: LBM_STREAM (SoA), LBM_COLLISION (AoS) and
 *     LBM_BLOCKED (AoSoA, blocks of 64 nodes).
 *     Precisions: all of lbm_precision.
 *   - Status, error text, streams and the on_device convention are those of
 *     the 2-D entry points. */
typedef struct {
    int64_t nx, ny, nz;
    int32_t scheme;    /* LBM_NPTL or LBM_AA */
    int32_t layout;    /* LBM_STREAM, LBM_COLLISION or LBM_BLOCKED */
    int32_t precision; /* lbm_precision */
    int32_t tile_x;    /* block tile in x and y, tile_x * tile_y <= 256; 0 and 0 = automatic
                          (256 nodes, as wide as nx allows: 256 x 1, 128 x 2, 64 x 4, ...) */
    int32_t tile_y;
} lbm3_grid;

typedef struct {
    int32_t x_axis;         /* LBM_PERIODIC, LBM_CLOSED or LBM_INFLOW_OUTFLOW */
    int32_t y_axis, z_axis; /* LBM_PERIODIC or LBM_CLOSED */
    double u_in[3];         /* inlet velocity */
    double g[3];            /* body force per node and step */
    double rho0;            /* must be 1 */
    double u0[3];           /* initial velocity of fluid and outlet nodes */
} lbm3_bc;

typedef struct lbm3_ctx lbm3_ctx;

/* lbm3_create -- allocate and initialise one D3Q19 simulation.
 *   flags : host, nx*ny*nz bytes [nz][ny][nx], LBM_FLUID or LBM_SOLID; copied.
 *   Other arguments as lbm_create.  Node types: solid where flagged; with an
 *   inflow/outflow x axis the plane x = 0 is the inlet and x = nx-1 the outlet
 *   (solid wins).  Initial state: feq(1, u0) on fluid and outlet nodes.  On
 *   error *out is NULL, nothing stays allocated, and lbm3_last_error(NULL)
 *   describes the failure (LBM_EINVAL bad argument, LBM_ENOMEM memory). */
lbm_status lbm3_create(const lbm3_grid* grid, const uint8_t* flags, double tau, const lbm3_bc* bc, void* stream,
                       lbm3_ctx** out);

/* lbm3_step -- advance n >= 0 updates (enqueued on the stream). */
lbm_status lbm3_step(lbm3_ctx* ctx, int64_t n);

/* lbm3_macros -- rho [nz][ny][nx] and u [3][nz][ny][nx] (FP32, host or
 * device; either may be NULL): rho and u = sum f c + g/2 of the incoming
 * populations on fluid and outlet nodes, (1, u_in) on inlet nodes, 0 on
 * solid nodes. */
lbm_status lbm3_macros(lbm3_ctx* ctx, float* rho, float* u, int on_device);

/* lbm3_get_populations -- shifted incoming populations [19][nz][ny][nx]
 * (host or device): what the next update collides; inlet nodes report the
 * inlet equilibrium, solid nodes 0. */
lbm_status lbm3_get_populations(lbm3_ctx* ctx, float* f, int on_device);

/* lbm3_set_state -- load shifted post-collision values [19][nz][ny][nx]
 * (host or device) as the state after the current update count; values of
 * inlet and solid nodes are ignored. */
lbm_status lbm3_set_state(lbm3_ctx* ctx, const float* f, int on_device);

/* lbm3_diag -- FP64 diagnostics over fluid and outlet nodes (synchronizes):
 * out[0] mass sum rho, out[1..3] momentum sum j, out[4] the residual
 * ||u_t - u_prev||_2 / ||u_t||_2 against the velocities of the previous call
 * (-1 on the first call and after lbm3_set_state).  Returns LBM_EUNSTABLE
 * when mass or momentum is not finite.  Scratch buffers are allocated on the
 * first call (LBM_ENOMEM if that fails). */
lbm_status lbm3_diag(lbm3_ctx* ctx, double out[5]);

/* lbm3_sync -- wait for the context's stream. */
lbm_status lbm3_sync(lbm3_ctx* ctx);

/* lbm3_last_error -- as lbm_last_error. */
const char* lbm3_last_error(const lbm3_ctx* ctx);

/* lbm3_destroy -- free everything; NULL is a no-op. */
void lbm3_destroy(lbm3_ctx* ctx);

/* lbm3_bytes_per_update -- algorithmic bytes per node update (19 loads and
 * 19 stores of the storage precision): 152 (FP32) or 76. */
int32_t lbm3_bytes_per_update(int32_t precision);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */

/*
 * liblbm.h -- MI355X (gfx950) lattice Boltzmann library for the
 * variable-speed-of-sound D2Q9 model of Buick & Cosgrove, "Investigation of
 * a Lattice Boltzmann Model with a Variable Speed of Sound".
 *
 * One time step is the update of Sec. 3, Eq. 5:
 *
 *   f_i(x + e_i, t + 1) = f_i(x, t) - (f_i - feq_i)/tau + 3 w_i alpha grad(rho).e_i
 *
 * on a periodic nx x ny D2Q9 lattice (links e_i and weights w_i of Sec. 2),
 * with feq of Eq. 2, rho and rho u of Eq. 3, and grad(rho) at time t by
 * central differences (Sec. 4, discussion of Fig. 1). The caller chooses the
 * squared speed of sound c2 = c_e^2; the library uses alpha = 1/3 - c2
 * (Eq. 8 with c_1^2 = 1/3), so c2 = 1/3 is the standard model (alpha = 0).
 * The viscosity is nu = (2 tau - 1)/6 for every c2 (Eq. 4, 7).
 *
 * All work runs in HIP kernels on the current HIP device of the calling
 * thread at create time. The library owns the device memory it allocates;
 * host arrays passed in belong to the caller and are only accessed during
 * the call. A handle is not thread-safe; distinct handles may be used from
 * distinct threads. No function throws; every int-returning function returns
 * an lbm_status.
 *
 * Field layout: every host or device field array is FP64, row-major, index
 * y*nx + x, nx*ny entries. Population arrays are FP64 [9][ny][nx] in the
 * link order of Sec. 2: e_0 = (0,0), e_1..4 = (1,0), (0,1), (-1,0), (0,-1),
 * e_5..8 = (1,1), (-1,1), (-1,-1), (1,-1).
 */
#ifndef LIBLBM_H
#define LIBLBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Storage / arithmetic forms. r_i is the lattice model's equilibrium at
 * rest (rho0 = 1, u = 0): the weights w_i for the paper's model (Eq. 2),
 * w_i 3 c2 (i != 0) and 1 - 5 c2 / 3 (i = 0) for LBM_MODEL_EQUILIBRIUM. */
enum lbm_dtype {
    LBM_F64 = 0,  /* f_i stored in FP64, FP64 arithmetic                         */
    LBM_F32 = 1,  /* f_i stored in FP32, FP32 arithmetic on d_i = f_i - r_i       */
    LBM_F32S = 2, /* g_i = f_i - r_i stored in FP32, FP32 arithmetic             */
    LBM_F16S = 3  /* g_i = f_i - r_i stored in FP16, FP32 arithmetic             */
};

enum lbm_status {
    LBM_OK = 0,
    LBM_EINVAL = -1,     /* argument out of range or NULL handle                   */
    LBM_ENOMEM = -2,     /* device or host allocation failed / budget exceeded     */
    LBM_EDEVICE = -3,    /* a HIP call failed                                      */
    LBM_ESTATE = -4,     /* step or read before init                               */
    LBM_ENONFINITE = -5  /* a conservation total is NaN or infinite                */
};

typedef struct lbm_lattice lbm_lattice;

/* Create a periodic nx x ny lattice on the current HIP device.
 * nx, ny >= 3 (the central differences of Sec. 4 need two distinct
 * neighbours); tau > 1/2 and finite (nu > 0, Eq. 4); c2 > 0 and finite
 * (c_e real, Eq. 8); dtype one of lbm_dtype. Large c2 is accepted: the paper
 * ran c_e up to 1.125 (Sec. 4); stability then depends on tau and the grid.
 * Allocates lbm_footprint_bytes(nx, ny, dtype) of device memory. Returns
 * NULL on failure and sets lbm_last_error() (LBM_EINVAL, LBM_ENOMEM,
 * LBM_EDEVICE). */
lbm_lattice* lbm_create(int nx, int ny, double tau, double c2, int dtype);

/* Status of the last failed lbm_create on this thread. */
int lbm_last_error(void);

/* Static text for a status code. */
const char* lbm_strerror(int status);

/* Release the lattice and its device memory (synchronises its stream).
 * NULL is a no-op. */
void lbm_destroy(lbm_lattice* L);

/* Set f_i(x, 0) = feq_i(rho(x), u(x)) (Eq. 2) from HOST FP64 fields.
 * rho == NULL means rho = 1; ux / uy == NULL mean 0. Resets t to 0.
 * Synchronous. */
int lbm_init(lbm_lattice* L, const double* rho, const double* ux, const double* uy);

/* Which model a lattice steps. LBM_MODEL_FORCING (the default) is the
 * paper's model, Eq. 5: relaxation to the Eq. 2 equilibrium plus the source
 * 3 w_i alpha grad(rho).e_i with alpha = 1/3 - c2. LBM_MODEL_EQUILIBRIUM is
 * the other route to a free sound speed the paper discusses (Sec. 3,
 * opening: alter the equilibrium, i.e. the share of rest and moving
 * particles), on D2Q9: relaxation to
 *   feq_i = w_i rho [3 c2 + 3 e_i.u + 9/2 (e_i.u)^2 - 3/2 u.u]  (i != 0),
 *   feq_0 = rho - sum_{i != 0} feq_i,
 * with no source term; its momentum flux is c2 rho I + rho u u exactly, and
 * c2 = 1/3 gives Eq. 2. */
enum lbm_model { LBM_MODEL_FORCING = 0, LBM_MODEL_EQUILIBRIUM = 1 };
/* Select the model for the following lbm_init / lbm_step calls (lbm_init
 * sets f to that model's equilibrium); on an initialised lattice the
 * populations f are kept (the shifted forms store f_i - r_i with r_i the
 * model's equilibrium at rest, and are re-centred, synchronously). LBM_EINVAL for a NULL handle, an
 * unknown model, or LBM_MODEL_EQUILIBRIUM with c2 >= 3/5 (its rest
 * population rho (1 - 5 c2 / 3) would not be positive), or for any model
 * but LBM_MODEL_FORCING while the lattice has a c2 field. Pools step the
 * forcing model. */
int lbm_set_model(lbm_lattice* L, int model);

/* Boundaries in x. LBM_XBC_PERIODIC (the default): periodic, as in y.
 * LBM_XBC_INLET_OUTLET: the set-up of Fig. 1 (Sec. 4), an oscillating
 * density at x = 0 and rho = 1, u = 0 at the far end. The sites of columns
 * x = 0 and x = nx - 1 do not collide: in the step from time t they emit
 * the lattice model's equilibrium at rest at the density
 *   rho_in(t) = 1 + amplitude sin(2 pi t / period)   (x = 0)
 * and 1 (x = nx - 1), and the periodic seam between the two columns is
 * cut: a population that would cross it arrives as the equilibrium
 * population of the column it enters, at that column's boundary density.
 * t is lbm_time() (so lbm_init / lbm_set_f restart the inlet's phase). Each
 * step then adds one small launch (the two columns). LBM_EINVAL for a NULL
 * handle, an unknown mode, or the inlet/outlet with nx < 5, a period that
 * is not finite and > 0, or |amplitude| >= 1. Takes effect at the next
 * step; pools are periodic. */
enum lbm_xbc { LBM_XBC_PERIODIC = 0, LBM_XBC_INLET_OUTLET = 1 };
int lbm_set_x_boundaries(lbm_lattice* L, int mode, double amplitude, double period);

/* A speed of sound that varies in space, the extension the paper's
 * conclusion (Sec. 5) proposes: alpha need not be constant, e.g. to model
 * an acoustic lens or a temperature gradient. c2 is a HOST FP64 array of
 * nx * ny entries, c2[y * nx + x] = c_e^2 at site (x, y); the source term of
 * Eq. 5 at that site then uses alpha(x) = 1/3 - c2[y * nx + x] (Eq. 8 site
 * by site), the gradient is unchanged. The lattice's own c2 (lbm_create) is
 * no longer used by the step. NULL removes the field (the uniform c2
 * applies again) and frees its memory. The field can be replaced between
 * steps (alpha varying in time). Synchronous.
 * The field is held in device memory in the compute precision (FP64 for
 * LBM_F64, else FP32): ny * ceil(nx / 256) * 256 * 4 or 8 bytes beyond
 * lbm_footprint_bytes, allocated by the first call; each step reads it
 * once (76 B per site in place of 72 for LBM_F32).
 * A lattice with a field steps with the vertical-stack kernels: a
 * march-form tile (no LBM_TILE_VSTACK) is replaced by the dtype's default
 * tile, and lbm_set_tile refuses one while the field exists.
 * LBM_EINVAL for a NULL handle, an entry that is not finite or not > 0 (the
 * field is then unchanged), or a lattice on LBM_MODEL_EQUILIBRIUM;
 * LBM_ENOMEM if the field cannot be allocated. */
int lbm_set_c2_field(lbm_lattice* L, const double* c2);

/* As lbm_set_c2_field with a DEVICE FP64 array (same layout) on the
 * lattice's device: asynchronous on the lattice's stream, for fields that
 * change every few steps. The entries are not checked: they must be finite
 * and > 0. NULL removes the field (synchronises the stream). */
int lbm_set_c2_field_device(lbm_lattice* L, const double* c2);

/* As lbm_init, but rho / ux / uy are DEVICE pointers (same layout) on the
 * lattice's device; asynchronous on the lattice's stream. */
int lbm_init_device(lbm_lattice* L, const double* rho, const double* ux, const double* uy);

/* Advance n >= 0 steps of Eq. 5; asynchronous on the lattice's stream.
 * LBM_ESTATE before init. */
int lbm_step(lbm_lattice* L, int n);

/* rho and u = (rho u)/rho (Eq. 3) of the current state f(x, t) into HOST
 * arrays (any may be NULL), and totals = {sum rho, sum rho u_x, sum rho u_y}
 * accumulated in FP64 in a fixed order (deterministic). totals may be NULL.
 * Synchronous. Returns LBM_ENONFINITE if a total is not finite. */
int lbm_moments(lbm_lattice* L, double* rho, double* ux, double* uy, double totals[3]);

/* As lbm_moments with DEVICE field pointers (any may be NULL) and HOST
 * totals (may be NULL). Synchronises the lattice's stream. */
int lbm_moments_device(lbm_lattice* L, double* rho, double* ux, double* uy, double totals[3]);

/* Canonical populations f_i(x, t) (the pre-collision state of Eq. 5) to /
 * from a HOST FP64 array [9][ny][nx]. lbm_set_f resets t to 0. Synchronous.
 * For the shifted forms the stored value is f_i - r_i, converted on the way
 * (r_i: the lattice model's equilibrium at rest, w_i for the paper's model). */
int lbm_get_f(lbm_lattice* L, double* f);
int lbm_set_f(lbm_lattice* L, const double* f);

/* Canonical populations at n sites (HOST arrays xs[n], ys[n] with
 * 0 <= x < nx, 0 <= y < ny) into HOST f[n][9]. Synchronous. LBM_EINVAL for a
 * site outside the lattice (nothing is read then). */
int lbm_sample_f(lbm_lattice* L, int n, const int* xs, const int* ys, double* f);

/* Use an existing HIP stream (hipStream_t, e.g. PyTorch's current stream)
 * for all later work on this lattice; NULL is the HIP null stream. The
 * caller keeps ownership of the stream. Synchronises the previous stream. */
int lbm_set_stream(lbm_lattice* L, void* hip_stream);

/* Return to the library's own (non-blocking) stream, the default after
 * lbm_create. Synchronises the previous stream. */
int lbm_use_own_stream(lbm_lattice* L);

/* The HIP stream the lattice currently launches on (NULL for a NULL handle). */
void* lbm_get_stream(const lbm_lattice* L);

/* Number of completed steps since init / set_f (-1 for NULL). */
long long lbm_time(const lbm_lattice* L);

/* Device bytes lbm_create allocates for this shape (0 if invalid). */
size_t lbm_footprint_bytes(int nx, int ny, int dtype);

/* Step kernel shape. vx = sites per lane along x (1, 2 or 4); flags =
 * LBM_TILE_* bits. March form: nw = 64-lane waves per workgroup (1 or 4),
 * each owning its own column strip of 64 * vx sites and marching h >= 1
 * rows. Vertical-stack form (LBM_TILE_VSTACK): nw = 4, 8 or 16 waves per
 * workgroup covering one strip and nw - 2 rows (h is ignored). Default:
 * the two-step form below; nw = 16 and non-temporal stores with vx = 1 for
 * LBM_F64 and vx = 2 for LBM_F32 and LBM_F32S; vx = 1, nw = 32 and plain
 * stores for LBM_F16S. Results do not depend on the shape (bitwise). LBM_EINVAL for an unsupported shape, for
 * a march-form shape (no LBM_TILE_VSTACK) while the lattice has a c2 field,
 * or for a shape whose grid would exceed one dispatch (2^32 work items) on
 * this lattice (only small shapes on the largest lattices).
 * Two-step form (LBM_TILE_VSTACK | LBM_TILE_TWO_STEP, optionally
 * LBM_TILE_NT_STORE; LBM_F64, LBM_F32 and LBM_F32S): one launch takes two
 * steps of Eq. 5, keeping the first step's results in on-chip memory, so
 * each site is loaded and stored once per two steps. vx = 1 or 2, nw = 12
 * or 16 waves, or nw = 32 rows on 16 waves (two rows each; vx = 1 and
 * LBM_F32, LBM_F32S or LBM_F16S); a workgroup writes nw - 6 rows and
 * (64 - 2 ceil(3 / vx)) vx columns. lbm_step takes the steps in pairs; a lone last step, and every
 * step while inlet/outlet boundaries are set, use the single-step vertical
 * stack (vx = 2, nw = 8, non-temporal stores). The
 * results are those of single steps, bit for bit (c2 fields included).
 * lbm_get_tile: any pointer may be NULL. */
enum lbm_tile_flags {
    LBM_TILE_PREFETCH = 1, /* issue the next row's loads before relaxing the current row */
    LBM_TILE_NT_STORE = 2, /* non-temporal (streaming) stores                              */
    LBM_TILE_ROWBAND = 4,  /* tile order: all strips of a row chunk before the next chunk  */
    LBM_TILE_PREFETCH2 = 8, /* issue loads two rows ahead (overrides LBM_TILE_PREFETCH)     */
    LBM_TILE_VSTACK = 16,   /* vertical-stack form (no march; uses only LBM_TILE_NT_STORE)  */
    LBM_TILE_TWO_STEP = 32  /* with LBM_TILE_VSTACK: two steps per launch (see lbm_set_tile) */
};
int lbm_set_tile(lbm_lattice* L, int vx, int nw, int h, int flags);
int lbm_get_tile(const lbm_lattice* L, int* vx, int* nw, int* h, int* flags);

/* Autotuner: time the candidate kernel shapes on this lattice, single- and
 * two-step, each over two steps (reps timed rounds each, after warm-up
 * launches; every launch reads the current state and writes the spare
 * buffer, so the state is unchanged) and apply the fastest. With use_cache != 0 a shape found before for the same GPU
 * architecture, dtype and nx x ny is applied without timing. Results are
 * remembered for the process and, if the environment variable LBM_TUNE_CACHE
 * names a file, appended to it (one JSON object per line). Synchronous.
 * LBM_ESTATE before init. */
int lbm_autotune(lbm_lattice* L, int reps, int use_cache);

/* ---------------------------------------------------------------------------
 * Pools: the batched and served forms. A pool holds resident lattices
 * (slots) of one dtype, each with its own nx, ny, tau and c2, under a device
 * memory budget, and steps any subset of them together: every step (or two
 * steps, in two-step tiles) of the listed lattices is one launch over all
 * their tiles (the same per-site code
 * as the single-lattice kernel, so each slot's result is bitwise identical to
 * stepping it alone with lbm_step). All pool work runs on the pool's stream.
 * A pool is not thread-safe.
 */
typedef struct lbm_pool lbm_pool;

enum lbm_pool_mode {
    LBM_POOL_GROUPED = 0,   /* one launch per step (per two steps in two-step tiles)   */
    LBM_POOL_GRAPH = 1,     /* the launches of a call captured once in a hipGraph and
                               replayed by later calls with the same shape             */
    LBM_POOL_PERSISTENT = 2 /* one launch for all steps of a call: the workgroups
                               resident when it starts take items dynamically, with a
                               grid barrier between steps (between two-step passes in
                               two-step tiles)                                         */
};

/* Create an empty pool for lattices of `dtype` whose device memory
 * (lbm_pool_slot_bytes each) may total at most budget_bytes. NULL on
 * failure; lbm_pool_last_error() tells why. Slots are carved from a few
 * large device allocations (up to 2 GiB each), taken as slots are added and
 * kept until lbm_pool_destroy: removing a slot returns its range to the
 * pool, not to the device. Slots do not always pack their allocations
 * exactly, so these may exceed budget_bytes, by at most 2 GiB
 * (lbm_pool_device_bytes): when a slot finds no free range and a new
 * allocation would go past that, allocations with no slot in them are freed
 * first, and if that does not make room lbm_pool_add returns LBM_ENOMEM
 * (the caller may retry after removing slots). */
lbm_pool* lbm_pool_create(size_t budget_bytes, int dtype);
int lbm_pool_last_error(void);
/* Free every slot and the pool (synchronises its stream). NULL: no-op. */
void lbm_pool_destroy(lbm_pool* P);

/* Device bytes one slot of this shape takes (0 if the shape is invalid): its
 * two population buffers and reduction scratch, rounded up to 64 KiB. */
size_t lbm_pool_slot_bytes(int nx, int ny, int dtype);
size_t lbm_pool_used_bytes(const lbm_pool* P);   /* sum of the slots' lbm_pool_slot_bytes      */
size_t lbm_pool_budget_bytes(const lbm_pool* P);
size_t lbm_pool_device_bytes(const lbm_pool* P); /* device memory the pool holds for its slots */

/* Admit a lattice (arguments as lbm_create). Returns the slot id (>= 0), or
 * LBM_EINVAL, or LBM_ENOMEM when it does not fit the remaining budget (by
 * slot bytes, or by the pool's device memory when freed ranges are too
 * fragmented to hold it) or the device allocation fails. Slot ids of
 * removed lattices are reused. */
int lbm_pool_add(lbm_pool* P, int nx, int ny, double tau, double c2);
/* Release a slot. Its range may be given to a slot added later: work
 * already queued on the pool's stream that reads this slot (a step, a
 * lbm_pool_totals_device) runs before any later work on that range, since
 * all pool work runs in order on the pool's stream. Does not wait. */
int lbm_pool_remove(lbm_pool* P, int slot);

/* As lbm_init / lbm_init_device for one slot; resets its time to 0. */
int lbm_pool_init(lbm_pool* P, int slot, const double* rho, const double* ux, const double* uy);
int lbm_pool_init_device(lbm_pool* P, int slot, const double* rho, const double* ux, const double* uy);

/* Advance slots[k] by nsteps[k] >= 0 steps, k < count (each slot at most
 * once). Launch s of the call steps every listed slot with nsteps > s.
 * Asynchronous on the pool's stream; LBM_ESTATE for an uninitialised slot. */
int lbm_pool_step(lbm_pool* P, const int* slots, const int* nsteps, int count);
/* As lbm_pool_step, for callers that cannot allocate device memory during
 * the call (tight serving loops, harnesses that forbid it): the batch's
 * descriptors and work-item map go to a fixed device array of the library
 * (about 9 MB per GPU, held until the process ends) in place of pool memory
 * that lbm_pool_step allocates as batches grow. At most 4096 lattices
 * (listed slots with nsteps > 0) and 2^21 work items per call (a lattice
 * has ceil(nx / (64 vx)) * ceil(ny / (nw - 2)) tiles, one item per
 * tiles_per_item of them); LBM_EINVAL for a larger batch, which is not
 * stepped. Grouped launches, or one persistent launch in LBM_POOL_PERSISTENT
 * mode (no graph). The pool's device must be current (LBM_EINVAL
 * otherwise). Results are those of lbm_pool_step. The array is shared
 * by every call on a GPU: calls that overlap on one GPU (on different
 * streams, or from different threads) race and must not be made. */
int lbm_pool_step_noalloc(lbm_pool* P, const int* slots, const int* nsteps, int count);

/* Wait for the pool's stream. */
int lbm_pool_sync(lbm_pool* P);

/* Diagnostics of LBM_POOL_PERSISTENT: the number of workgroups that took
 * part in the last persistent launch (those resident when it started; 0
 * before any). Synchronises the pool's stream. Negative: an error status. */
int lbm_pool_persistent_members(lbm_pool* P);

/* The totals {sum rho, sum rho u_x, sum rho u_y} of a slot's current state
 * (as lbm_moments: FP64, fixed order) into a DEVICE array of 3 doubles,
 * asynchronously on the pool's stream (no check of finiteness; a timed-out
 * persistent launch is reported by the next lbm_pool_sync). The serving loop
 * reads the totals of finished jobs this way while the next steps run. */
int lbm_pool_totals_device(lbm_pool* P, int slot, double* totals);

/* As lbm_moments / lbm_get_f for one slot (synchronous). */
int lbm_pool_moments(lbm_pool* P, int slot, double* rho, double* ux, double* uy, double totals[3]);
int lbm_pool_get_f(lbm_pool* P, int slot, double* f);
/* Completed steps of a slot since its init (-1 for an invalid slot). */
long long lbm_pool_time(const lbm_pool* P, int slot);

/* Launch mode (lbm_pool_mode) and, for LBM_POOL_PERSISTENT, a cap on the
 * workgroups of the persistent launch (0: as many as the runtime reports a
 * CU can hold at once; those not resident when it starts take no part). */
int lbm_pool_set_mode(lbm_pool* P, int mode, int max_grid);
/* Vertical-stack tile of the batched kernels: vx in {1, 2, 4}, nw in
 * {4, 8, 16}, flags 0 or LBM_TILE_NT_STORE. Default: the two-step tile
 * below with nw 16, vx 1 for LBM_F64 and 2 for LBM_F32 and LBM_F32S, and
 * non-temporal stores; for LBM_F16S vx 4 and nw 8 with non-temporal
 * stores. Two-step tiles (flags LBM_TILE_TWO_STEP, optionally with
 * LBM_TILE_VSTACK and LBM_TILE_NT_STORE; vx 1 or 2, nw 12 or 16, one row
 * per wave; every dtype and mode): each launch (in LBM_POOL_PERSISTENT mode, each pass
 * between grid barriers) takes two steps of every listed lattice (the
 * shapes of lbm_set_tile's two-step form); a lattice with an odd step count
 * takes its last step alone in the last one. LBM_EINVAL for other shapes.
 * Does not change results (bitwise). lbm_pool_get_tile reports
 * LBM_TILE_TWO_STEP and LBM_TILE_NT_STORE. */
int lbm_pool_set_tile(lbm_pool* P, int vx, int nw, int flags);
int lbm_pool_get_tile(const lbm_pool* P, int* vx, int* nw, int* flags);
/* Tiles per work item of the batched kernels (1..64, default 1): a
 * workgroup takes that many consecutive tiles of one lattice, paying the
 * lattice lookup once. Does not change results. */
int lbm_pool_set_items(lbm_pool* P, int tiles_per_item);
/* Autotuner for the batched kernels (see lbm_autotune): shape, stores,
 * tiles per item and the order in which items are dealt to the GPU's
 * chiplets, single- and two-step tiles, each timed over two steps of the
 * listed slots without advancing them (in LBM_POOL_PERSISTENT mode, on
 * persistent launches, whose best shape differs); cached per
 * architecture, mode, dtype, and the batch's
 * lattice count and total sites rounded up to powers of two. Call it after
 * lbm_pool_set_mode. */
int lbm_pool_autotune(lbm_pool* P, const int* slots, int count, int reps, int use_cache);
/* Use an existing (non-null) HIP stream for the pool's work; NULL selects
 * the pool's own non-blocking stream (the default). Synchronises the
 * previous stream. */
int lbm_pool_set_stream(lbm_pool* P, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* LIBLBM_H */

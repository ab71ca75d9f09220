// pool.hip -- host side of the batched and served forms: a pool of resident
// lattices (slots) of one storage dtype under a device-memory budget, stepped
// together by batched launches (grouped, grouped under a captured hipGraph,
// or one persistent launch). C ABI in include/liblbm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "arena.h"
#include "host.h"
#include "tune.h"

using namespace lbm;

namespace {

struct Slot {
    bool used = false;
    bool ready = false;
    int nx = 0, ny = 0;
    double tau = 0, c2 = 0;
    Geom g{};
    Coef coef{};
    size_t bytes = 0;  // buffers + moments scratch
    size_t span = 0;   // arena bytes held (bytes rounded up)
    void* buf = nullptr;
    void* b0 = nullptr;  // state at even buffer times
    void* b1 = nullptr;  // state at odd buffer times
    double* red = nullptr;
    long long t = 0;
    // Buffer phase: the state at time t is in buffer (t + ph) & 1. Single
    // steps keep it; a two-step pass (one read and one write for two steps)
    // flips it.
    int ph = 0;
};

// Chunks of slot memory come from hipMalloc (see arena.h).
struct DeviceAlloc {
    using Err = hipError_t;
    static constexpr hipError_t kOk = hipSuccess;
    static constexpr hipError_t kNoMem = hipErrorOutOfMemory;
    static hipError_t get(void** p, size_t n) { return hipMalloc(p, n); }
    static void put(void* p) { (void)hipFree(p); }
};
using SlotArena = lbm::Arena<DeviceAlloc>;

struct GraphEntry {
    int nsteps_max = 0, nitems = 0, vx = 0, nw = 0, nts = 0, ch = 0, two = 0;
    const BatchLat* lats = nullptr;
    const int* items = nullptr;
    hipGraphExec_t exec = nullptr;
};

}  // namespace

// Scratch of lbm_pool_step_noalloc: a batch's descriptors (at most
// kNoAllocLattices) and its item map (at most kNoAllocItems work items) in
// one file-scope device array, instead of device memory the pool allocates
// as batches grow. Each GPU holds its own copy (about 9 MB) until the
// process ends. Host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device (noalloc_scratch).
namespace {
constexpr int kNoAllocLattices = 4096;
constexpr int kNoAllocItems = 1 << 21;
constexpr size_t kNoAllocItemsAt = ((size_t)kNoAllocLattices * sizeof(BatchLat) + 255) / 256 * 256;
constexpr size_t kNoAllocBytes = kNoAllocItemsAt + (size_t)kNoAllocItems * sizeof(int);
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
char* g_scratch[kMaxDevices] = {};

// The device address of `scratch` on device dev, which must be current;
// looked up on the first call for that device.
hipError_t noalloc_scratch(int dev, char** out)
{
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = (char*)p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace

struct lbm_pool {
    int dtype = 0, esize = 0, device = 0;
    size_t budget = 0, used = 0;
    std::vector<Slot> slots;
    SlotArena arena;              // device memory of the slots
    hipStream_t own = nullptr, stream = nullptr;
    int vx = 2, nw = 16, nts = 1; // vertical-stack tile of the batched kernels
    int two = 0;                  // two steps per launch (two-step tiles; grouped and graph modes)
    int mode = LBM_POOL_GROUPED;
    int max_grid = 0;             // persistent mode: workgroup cap (0 = all co-resident)
    BatchLat* d_lats = nullptr;   // device descriptor array
    int* d_items = nullptr;       // device item -> lattice map
    unsigned* d_bar = nullptr;    // barrier state of the persistent kernel (kPoolBarWords words)
    int cap = 0, item_cap = 0;
    int per_item = 1;             // tiles per work item
    int xcd_chunk = 8;            // items per XCD chunk of the grouped launches (see xcd_tile)
    std::vector<BatchLat> h_lats;
    std::vector<int> h_items;
    std::vector<GraphEntry> graphs;
};

namespace {

thread_local int g_pool_error = LBM_OK;

Slot* slot_of(lbm_pool* P, int s)
{
    if (!P || s < 0 || s >= (int)P->slots.size() || !P->slots[s].used) return nullptr;
    return &P->slots[s];
}

void* cur_buf(const Slot& S) { return ((S.t + S.ph) & 1) ? S.b1 : S.b0; }

// The buffer time a batch descriptor carries for slot S (see BatchLat and
// Slot::ph).
long long buffer_time(const Slot& S) { return S.t + S.ph; }

// Advance slot S by n steps taken in two-step passes (two != 0: ceil(n / 2)
// launches, each moving the state to the other buffer) or in single steps.
void advance(Slot& S, int n, int two)
{
    if (two) S.ph = (int)((S.ph + (n + 1) / 2 + n) & 1);
    S.t += n;
}

// The dtype's default tile of the batched kernels (from the batched
// sweeps): the two-step tile where it is faster (16 waves, vx = 1 for FP64
// and 2 for FP32 and FP32-shifted, as for single lattices), else (FP16) the
// single-step vertical stack of 8 waves with vx = 4; non-temporal stores.
void set_default_tile(lbm_pool* P)
{
    P->nts = 1;
    if (P->dtype != LBM_F16S) {
        P->two = 1;
        P->nw = 16;
        P->vx = P->dtype == LBM_F64 ? 1 : 2;
    } else {
        P->two = 0;
        P->nw = 8;
        P->vx = P->dtype == LBM_F16S ? 4 : 2;
    }
}

void drop_graphs(lbm_pool* P)
{
    for (auto& g : P->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    P->graphs.clear();
}

// Bytes of a slot's range: both buffers, then the moments scratch at the
// next 256-byte boundary (*red_at), rounded up to the arena's unit.
size_t slot_bytes(int nx, int ny, int dtype, Geom* g_out, size_t* red_at = nullptr)
{
    const int es = esize_of(dtype);
    const Geom g = make_geom(nx, ny, es, choose_interleaved(nx, ny, dtype));
    if (g_out) *g_out = g;
    const size_t at = (footprint(g, es) + 255) / 256 * 256;
    if (red_at) *red_at = at;
    return SlotArena::round(at + red_doubles(g) * sizeof(double));
}

// The descriptor of a slot for vertical-stack tiles of vx columns per lane
// and nw waves (the shape of the launch that reads it); two: the two-step
// tiles of step2_cols / step2_rows.
StepTile slot_tile(const Slot& S, int vx, int nw, int two)
{
    StepTile t{};
    t.src = S.b0;
    t.dst = S.b1;
    t.g = S.g;
    t.c = S.coef;
    t.h = nw - 2;
    const int W = two ? step2_cols(vx) : 64 * vx, R = two ? step2_rows(nw) : nw - 2;
    t.nstrips = (S.nx + W - 1) / W;
    t.nchunks = (S.ny + R - 1) / R;
    t.rowband = 1;
    return t;
}

hipError_t ensure_cap(lbm_pool* P, int n, int nitems)
{
    if (n > P->cap) {
        int cap = std::max(n, std::max(16, 2 * P->cap));
        BatchLat* d = nullptr;
        hipError_t e = hipMalloc((void**)&d, sizeof(BatchLat) * (size_t)cap);
        if (e != hipSuccess) return e;
        if (P->d_lats) {
            (void)hipStreamSynchronize(P->stream);
            (void)hipFree(P->d_lats);
        }
        drop_graphs(P);  // they hold the old descriptor pointer
        P->d_lats = d;
        P->cap = cap;
    }
    if (nitems > P->item_cap) {
        int cap = std::max(nitems, std::max(1024, 2 * P->item_cap));
        int* d = nullptr;
        hipError_t e = hipMalloc((void**)&d, sizeof(int) * (size_t)cap);
        if (e != hipSuccess) return e;
        if (P->d_items) {
            (void)hipStreamSynchronize(P->stream);
            (void)hipFree(P->d_items);
        }
        drop_graphs(P);
        P->d_items = d;
        P->item_cap = cap;
    }
    return hipSuccess;
}

// Append lattice descriptor b (tile already set) and its work items.
void add_lattice(lbm_pool* P, BatchLat b)
{
    b.ntiles = b.tile.nstrips * b.tile.nchunks;
    b.per_item = P->per_item;
    b.item_begin = (int)P->h_items.size();
    const int nitems = (b.ntiles + b.per_item - 1) / b.per_item;
    const int l = (int)P->h_lats.size();
    for (int k = 0; k < nitems; ++k) P->h_items.push_back(l);
    P->h_lats.push_back(b);
}

// Run the batch described by h_lats / h_items (already built) for nmax steps.
hipError_t run_batch(lbm_pool* P, int nmax)
{
    const int nlat = (int)P->h_lats.size(), nitems = (int)P->h_items.size();
    hipError_t e = ensure_cap(P, nlat, nitems);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(P->d_lats, P->h_lats.data(), sizeof(BatchLat) * (size_t)nlat, hipMemcpyHostToDevice,
                       P->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(P->d_items, P->h_items.data(), sizeof(int) * (size_t)nitems, hipMemcpyHostToDevice,
                           P->stream);
    if (e != hipSuccess) return e;
    const bool nts = P->nts != 0;
    if (P->mode == LBM_POOL_PERSISTENT)
        return P->two ? launch_batch2_persistent(P->dtype, P->vx, P->nw, nts, P->d_lats, P->d_items, nitems,
                                                 (nmax + 1) / 2, P->max_grid, P->xcd_chunk, P->d_bar, P->stream)
                      : launch_batch(P->dtype, P->vx, P->nw, nts, true, P->d_lats, P->d_items, nitems, nmax,
                                     P->max_grid, P->xcd_chunk, P->d_bar, P->stream);
    // launch k of the call: step k, or two-step pass k
    const int nlaunch = P->two ? (nmax + 1) / 2 : nmax;
    auto launch_k = [&](int k) {
        return P->two ? launch_batch2(P->dtype, P->vx, P->nw, nts, P->d_lats, P->d_items, nitems, k, P->xcd_chunk,
                                      P->stream)
                      : launch_batch(P->dtype, P->vx, P->nw, nts, false, P->d_lats, P->d_items, nitems, k, 0,
                                     P->xcd_chunk, nullptr, P->stream);
    };
    if (P->mode == LBM_POOL_GRAPH) {
        GraphEntry* ge = nullptr;
        for (auto& g : P->graphs)
            if (g.nsteps_max == nmax && g.nitems == nitems && g.vx == P->vx && g.nw == P->nw && g.nts == P->nts &&
                g.ch == P->xcd_chunk && g.two == P->two && g.lats == P->d_lats && g.items == P->d_items)
                ge = &g;
        if (!ge) {
            // Capture the call's grouped launches once; replays re-read the
            // descriptors, which are refreshed above before every replay.
            hipGraph_t graph = nullptr;
            e = hipStreamBeginCapture(P->stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return e;
            hipError_t le = hipSuccess;
            for (int k = 0; k < nlaunch && le == hipSuccess; ++k) le = launch_k(k);
            e = hipStreamEndCapture(P->stream, &graph);
            if (le != hipSuccess) e = le;
            hipGraphExec_t exec = nullptr;
            if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (graph) (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return e;
            if (P->graphs.size() >= 8) {
                (void)hipGraphExecDestroy(P->graphs.front().exec);
                P->graphs.erase(P->graphs.begin());
            }
            P->graphs.push_back(
                GraphEntry{nmax, nitems, P->vx, P->nw, P->nts, P->xcd_chunk, P->two, P->d_lats, P->d_items, exec});
            ge = &P->graphs.back();
        }
        return hipGraphLaunch(ge->exec, P->stream);
    }
    for (int k = 0; k < nlaunch && e == hipSuccess; ++k) e = launch_k(k);
    return e;
}

}  // namespace

extern "C" {

int lbm_pool_last_error(void) { return g_pool_error; }

lbm_pool* lbm_pool_create(size_t budget_bytes, int dtype)
{
    if (esize_of(dtype) == 0 || budget_bytes == 0) {
        g_pool_error = LBM_EINVAL;
        return nullptr;
    }
    lbm_pool* P = new (std::nothrow) lbm_pool();
    if (!P) {
        g_pool_error = LBM_ENOMEM;
        return nullptr;
    }
    P->dtype = dtype;
    P->esize = esize_of(dtype);
    P->budget = budget_bytes;
    set_default_tile(P);
    if (const char* ev = std::getenv("LBM_XCD_CHUNK")) {  // experiments: items per XCD chunk
        const int v = std::atoi(ev);
        if (v >= 0 && v <= 4096) P->xcd_chunk = v;
    }
    hipError_t e = hipGetDevice(&P->device);
    char* noalloc_base = nullptr;  // look up lbm_pool_step_noalloc's array while set up
    if (e == hipSuccess) e = noalloc_scratch(P->device, &noalloc_base);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&P->own, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc((void**)&P->d_bar, kPoolBarWords * sizeof(unsigned));
    if (e == hipSuccess) e = hipMemsetAsync(P->d_bar, 0, kPoolBarWords * sizeof(unsigned), P->own);
    if (e == hipSuccess) e = hipStreamSynchronize(P->own);
    if (e != hipSuccess) {
        g_pool_error = LBM_EDEVICE;
        if (P->d_bar) (void)hipFree(P->d_bar);
        if (P->own) (void)hipStreamDestroy(P->own);
        delete P;
        return nullptr;
    }
    P->stream = P->own;
    g_pool_error = LBM_OK;
    return P;
}

void lbm_pool_destroy(lbm_pool* P)
{
    if (!P) return;
    (void)hipStreamSynchronize(P->stream);
    drop_graphs(P);
    P->arena.release();
    if (P->d_lats) (void)hipFree(P->d_lats);
    if (P->d_items) (void)hipFree(P->d_items);
    if (P->d_bar) (void)hipFree(P->d_bar);
    if (P->own) (void)hipStreamDestroy(P->own);
    delete P;
}

size_t lbm_pool_slot_bytes(int nx, int ny, int dtype)
{
    if (!args_ok(nx, ny, 1.0, 1.0 / 3.0, dtype)) return 0;
    return slot_bytes(nx, ny, dtype, nullptr);
}

size_t lbm_pool_used_bytes(const lbm_pool* P) { return P ? P->used : 0; }
size_t lbm_pool_device_bytes(const lbm_pool* P) { return P ? P->arena.total : 0; }
size_t lbm_pool_budget_bytes(const lbm_pool* P) { return P ? P->budget : 0; }

int lbm_pool_add(lbm_pool* P, int nx, int ny, double tau, double c2)
{
    if (!P || !args_ok(nx, ny, tau, c2, P->dtype)) return LBM_EINVAL;
    Geom g;
    size_t red_at = 0;
    const size_t bytes = slot_bytes(nx, ny, P->dtype, &g, &red_at);
    if (P->used + bytes > P->budget) return LBM_ENOMEM;
    Slot S;
    S.used = true;
    S.nx = nx;
    S.ny = ny;
    S.tau = tau;
    S.c2 = c2;
    S.g = g;
    S.coef = make_coef(tau, c2, LBM_MODEL_FORCING);
    S.bytes = bytes;
    const size_t fb = footprint(g, P->esize);
    S.span = bytes;
    hipError_t e = hipSuccess;
    S.buf = P->arena.take(S.span, P->budget, &e);
    if (S.buf) {
        S.red = (double*)((char*)S.buf + red_at);
        e = hipMemsetAsync(S.buf, 0, fb, P->stream);
        if (e != hipSuccess) P->arena.give(S.buf, S.span);
    }
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE;
    S.b0 = S.buf;
    S.b1 = (char*)S.buf + (size_t)buffer_elems(g) * P->esize;
    P->used += bytes;
    for (int i = 0; i < (int)P->slots.size(); ++i)
        if (!P->slots[i].used) {
            P->slots[i] = S;
            return i;
        }
    P->slots.push_back(S);
    return (int)P->slots.size() - 1;
}

int lbm_pool_remove(lbm_pool* P, int slot)
{
    Slot* S = slot_of(P, slot);
    if (!S) return LBM_EINVAL;
    // No wait: all pool work runs in order on the pool's stream, so work
    // queued on a later slot in the same range runs after the work already
    // queued on this one.
    if (S->buf) P->arena.give(S->buf, S->span);
    P->used -= S->bytes;
    *S = Slot();
    return LBM_OK;
}

int lbm_pool_init(lbm_pool* P, int slot, const double* rho, const double* ux, const double* uy)
{
    Slot* S = slot_of(P, slot);
    if (!S) return LBM_EINVAL;
    const size_t n = (size_t)S->nx * S->ny;
    DevScratch d;
    hipError_t e = d.alloc(3 * n, P->stream);
    const double* src[3] = {rho, ux, uy};
    const double* dp[3] = {nullptr, nullptr, nullptr};
    for (int c = 0; c < 3 && e == hipSuccess; ++c) {
        if (!src[c]) continue;
        e = hipMemcpyAsync(d.p + c * n, src[c], n * sizeof(double), hipMemcpyHostToDevice, P->stream);
        dp[c] = d.p + c * n;
    }
    if (e == hipSuccess) e = launch_init(P->dtype, S->b0, S->g, dp[0], dp[1], dp[2], 0.0, P->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(P->stream);
    if (e != hipSuccess) return status_of(e);
    S->t = 0;
    S->ph = 0;
    S->ready = true;
    return LBM_OK;
}

int lbm_pool_init_device(lbm_pool* P, int slot, const double* rho, const double* ux, const double* uy)
{
    Slot* S = slot_of(P, slot);
    if (!S) return LBM_EINVAL;
    hipError_t e = launch_init(P->dtype, S->b0, S->g, rho, ux, uy, 0.0, P->stream);
    if (e != hipSuccess) return status_of(e);
    S->t = 0;
    S->ph = 0;
    S->ready = true;
    return LBM_OK;
}

// The descriptors and work items of a batched call into P->h_lats and
// P->h_items (host vectors whose capacity is kept from call to call);
// *nmax = the largest step count.
static int build_batch(lbm_pool* P, const int* slots, const int* nsteps, int count, int* nmax)
{
    if (!P || count < 0 || (count > 0 && (!slots || !nsteps))) return LBM_EINVAL;
    P->h_lats.clear();
    P->h_items.clear();
    *nmax = 0;
    for (int k = 0; k < count; ++k) {
        Slot* S = slot_of(P, slots[k]);
        if (!S || nsteps[k] < 0) return LBM_EINVAL;
        if (!S->ready) return LBM_ESTATE;
        for (int j = 0; j < k; ++j)
            if (slots[j] == slots[k]) return LBM_EINVAL;  // a slot listed twice
        if (nsteps[k] == 0) continue;
        BatchLat b{};
        b.tile = slot_tile(*S, P->vx, P->nw, P->two);
        b.t0 = buffer_time(*S);
        b.nsteps = nsteps[k];
        add_lattice(P, b);
        *nmax = std::max(*nmax, nsteps[k]);
    }
    return LBM_OK;
}

int lbm_pool_step(lbm_pool* P, const int* slots, const int* nsteps, int count)
{
    int nmax = 0;
    const int st = build_batch(P, slots, nsteps, count, &nmax);
    if (st != LBM_OK || P->h_lats.empty()) return st;
    hipError_t e = run_batch(P, nmax);
    if (e != hipSuccess) return status_of(e);
    for (int k = 0; k < count; ++k) advance(P->slots[slots[k]], nsteps[k], P->two);
    return LBM_OK;
}

int lbm_pool_step_noalloc(lbm_pool* P, const int* slots, const int* nsteps, int count)
{
    int nmax = 0;
    const int st = build_batch(P, slots, nsteps, count, &nmax);
    if (st != LBM_OK || P->h_lats.empty()) return st;
    const int nlat = (int)P->h_lats.size(), nitems = (int)P->h_items.size();
    if (nlat > kNoAllocLattices || nitems > kNoAllocItems) return LBM_EINVAL;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return status_of(e);
    if (dev != P->device) return LBM_EINVAL;  // the scratch address is per device
    char* base = nullptr;
    e = noalloc_scratch(dev, &base);
    if (e != hipSuccess) return status_of(e);
    BatchLat* d_lats = (BatchLat*)base;
    int* d_items = (int*)(base + kNoAllocItemsAt);
    e = hipMemcpyAsync(d_lats, P->h_lats.data(), sizeof(BatchLat) * (size_t)nlat, hipMemcpyHostToDevice, P->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_items, P->h_items.data(), sizeof(int) * (size_t)nitems, hipMemcpyHostToDevice,
                           P->stream);
    const bool nts = P->nts != 0;
    if (e == hipSuccess) {
        if (P->mode == LBM_POOL_PERSISTENT && P->two) {
            e = launch_batch2_persistent(P->dtype, P->vx, P->nw, nts, d_lats, d_items, nitems, (nmax + 1) / 2,
                                         P->max_grid, P->xcd_chunk, P->d_bar, P->stream);
        } else if (P->mode == LBM_POOL_PERSISTENT) {
            e = launch_batch(P->dtype, P->vx, P->nw, nts, true, d_lats, d_items, nitems, nmax, P->max_grid,
                             P->xcd_chunk, P->d_bar, P->stream);
        } else if (P->two) {
            for (int k = 0; k < (nmax + 1) / 2 && e == hipSuccess; ++k)
                e = launch_batch2(P->dtype, P->vx, P->nw, nts, d_lats, d_items, nitems, k, P->xcd_chunk, P->stream);
        } else {
            for (int s = 0; s < nmax && e == hipSuccess; ++s)
                e = launch_batch(P->dtype, P->vx, P->nw, nts, false, d_lats, d_items, nitems, s, 0, P->xcd_chunk,
                                 nullptr, P->stream);
        }
    }
    if (e != hipSuccess) return status_of(e);
    for (int k = 0; k < count; ++k) advance(P->slots[slots[k]], nsteps[k], P->two);
    return LBM_OK;
}

// After the pool's stream is idle: LBM_EDEVICE if a persistent launch timed
// out at a grid barrier since the flag was last read (its steps, and those
// of the launches after it, are incomplete), clearing the flag; else LBM_OK.
static int take_barrier_error(lbm_pool* P)
{
    unsigned flag = 0;
    hipError_t e = hipMemcpy(&flag, P->d_bar + 2, sizeof(flag), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return status_of(e);
    if (!flag) return LBM_OK;
    unsigned zero[3] = {0, 0, 0};
    (void)hipMemcpy(P->d_bar, zero, sizeof(zero), hipMemcpyHostToDevice);
    return LBM_EDEVICE;
}

int lbm_pool_sync(lbm_pool* P)
{
    if (!P) return LBM_EINVAL;
    hipError_t e = hipStreamSynchronize(P->stream);
    if (e != hipSuccess) return status_of(e);
    return take_barrier_error(P);
}

int lbm_pool_persistent_members(lbm_pool* P)
{
    if (!P) return LBM_EINVAL;
    hipError_t e = hipStreamSynchronize(P->stream);
    unsigned members = 0;
    if (e == hipSuccess) e = hipMemcpy(&members, P->d_bar + 3, sizeof(members), hipMemcpyDeviceToHost);
    return e != hipSuccess ? status_of(e) : (int)members;
}

int lbm_pool_moments(lbm_pool* P, int slot, double* rho, double* ux, double* uy, double totals[3])
{
    Slot* S = slot_of(P, slot);
    if (!S) return LBM_EINVAL;
    if (!S->ready) return LBM_ESTATE;
    const size_t n = (size_t)S->nx * S->ny;
    DevScratch d;
    hipError_t e = (rho || ux || uy) ? d.alloc(3 * n, P->stream) : hipSuccess;
    double* dp[3] = {rho ? d.p : nullptr, ux ? d.p + n : nullptr, uy ? d.p + 2 * n : nullptr};
    double* tot_dev = S->red + (size_t)3 * moments_blocks(S->g);
    double tot[3] = {0, 0, 0};
    if (e == hipSuccess)
        e = launch_moments(P->dtype, cur_buf(*S), S->g, dp[0], dp[1], dp[2], S->red, tot_dev, P->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(tot, tot_dev, sizeof(tot), hipMemcpyDeviceToHost, P->stream);
    double* host[3] = {rho, ux, uy};
    for (int c = 0; c < 3 && e == hipSuccess; ++c)
        if (host[c]) e = hipMemcpyAsync(host[c], dp[c], n * sizeof(double), hipMemcpyDeviceToHost, P->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(P->stream);
    if (e != hipSuccess) return status_of(e);
    if (totals) std::memcpy(totals, tot, sizeof(tot));
    const int be = take_barrier_error(P);
    if (be != LBM_OK) return be;
    for (double v : tot)
        if (!std::isfinite(v)) return LBM_ENONFINITE;
    return LBM_OK;
}

int lbm_pool_totals_device(lbm_pool* P, int slot, double* totals)
{
    Slot* S = slot_of(P, slot);
    if (!S || !totals) return LBM_EINVAL;
    if (!S->ready) return LBM_ESTATE;
    return status_of(launch_moments(P->dtype, cur_buf(*S), S->g, nullptr, nullptr, nullptr, S->red, totals, P->stream));
}

int lbm_pool_get_f(lbm_pool* P, int slot, double* f)
{
    Slot* S = slot_of(P, slot);
    if (!S || !f) return LBM_EINVAL;
    if (!S->ready) return LBM_ESTATE;
    const size_t n = (size_t)9 * S->nx * S->ny;
    DevScratch d;
    hipError_t e = d.alloc(n, P->stream);
    if (e == hipSuccess) e = launch_get_f(P->dtype, cur_buf(*S), S->g, d.p, 0.0, P->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(f, d.p, n * sizeof(double), hipMemcpyDeviceToHost, P->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(P->stream);
    if (e != hipSuccess) return status_of(e);
    return take_barrier_error(P);
}

long long lbm_pool_time(const lbm_pool* P, int slot)
{
    if (!P || slot < 0 || slot >= (int)P->slots.size() || !P->slots[slot].used) return -1;
    return P->slots[slot].t;
}

int lbm_pool_set_mode(lbm_pool* P, int mode, int max_grid)
{
    if (!P || mode < LBM_POOL_GROUPED || mode > LBM_POOL_PERSISTENT || max_grid < 0) return LBM_EINVAL;
    P->mode = mode;
    P->max_grid = max_grid;
    return LBM_OK;
}

int lbm_pool_set_tile(lbm_pool* P, int vx, int nw, int flags)
{
    if (!P) return LBM_EINVAL;
    const bool two = (flags & LBM_TILE_TWO_STEP) != 0;
    if (two) {
        // the batched two-step kernels take one row per wave (nw 12 or 16)
        if ((flags & ~(LBM_TILE_TWO_STEP | LBM_TILE_VSTACK | LBM_TILE_NT_STORE)) ||
            !step2_shape_supported(P->dtype, vx, nw) || nw > 16)
            return LBM_EINVAL;
    } else if ((flags & ~LBM_TILE_NT_STORE) || !step_shape_supported(P->dtype, vx, nw, LBM_TILE_VSTACK)) {
        return LBM_EINVAL;
    }
    hipError_t e = hipStreamSynchronize(P->stream);
    P->vx = vx;
    P->nw = nw;
    P->nts = (flags & LBM_TILE_NT_STORE) ? 1 : 0;
    P->two = two ? 1 : 0;
    return status_of(e);
}

int lbm_pool_autotune(lbm_pool* P, const int* slots, int count, int reps, int use_cache)
{
    if (!P || reps < 1 || count < 1 || !slots) return LBM_EINVAL;
    long long sites = 0;
    for (int k = 0; k < count; ++k) {
        Slot* S = slot_of(P, slots[k]);
        if (!S) return LBM_EINVAL;
        if (!S->ready) return LBM_ESTATE;
        sites += (long long)S->nx * S->ny;
    }
    // key: the batch's lattice count and total sites, rounded to powers of 2
    int lc = 0, ls = 0;
    while ((1 << lc) < count) ++lc;
    while ((1LL << ls) < sites) ++ls;
    // the persistent kernel is tuned on its own launches (its best shape differs)
    const bool pers = P->mode == LBM_POOL_PERSISTENT;
    char key[160];
    std::snprintf(key, sizeof(key), "%s|%s|%d|n2^%d|s2^%d", device_arch().c_str(), pers ? "pool-persistent" : "pool",
                  P->dtype, lc, ls);
    TileCand c{};
    if (use_cache && tune_cache_get(key, &c)) {
        P->per_item = c.h;
        P->xcd_chunk = c.ch;
        return lbm_pool_set_tile(P, c.vx, c.nw, c.flags);
    }
    std::vector<TileCand> cands = pool_candidates(P->dtype);
    if (pers)  // 4-wave tiles (2 rows each) take one atomic per 2 rows: far slower persistent, and slow to time
        cands.erase(std::remove_if(cands.begin(), cands.end(), [](const TileCand& k) { return k.nw < 8; }),
                    cands.end());
    // Every candidate is timed over two steps without advancing any slot:
    // two batched launches at step 0 of a 1-step call (each reads each
    // slot's current buffer and writes the other; a persistent launch of
    // one step in persistent mode), or one two-step pass of a 2-step call
    // (reads the current buffer, writes the other). The
    // descriptors and the item map of a shape are built and uploaded by its
    // first (untimed) launch only, so that the timed launches measure the
    // kernel and not the host work, which grows with the number of items.
    TileCand built{};
    bool have_built = false;
    int nitems = 0;
    auto launch = [&](const TileCand& k) -> hipError_t {
        const int two = (k.flags & LBM_TILE_TWO_STEP) ? 1 : 0;
        const bool nts = (k.flags & LBM_TILE_NT_STORE) != 0;
        auto go = [&]() {
            if (two && pers)
                return launch_batch2_persistent(P->dtype, k.vx, k.nw, nts, P->d_lats, P->d_items, nitems, 1,
                                                P->max_grid, k.ch, P->d_bar, P->stream);
            if (two) return launch_batch2(P->dtype, k.vx, k.nw, nts, P->d_lats, P->d_items, nitems, 0, k.ch, P->stream);
            hipError_t ge = hipSuccess;
            for (int r = 0; r < 2 && ge == hipSuccess; ++r)
                ge = launch_batch(P->dtype, k.vx, k.nw, nts, pers, P->d_lats, P->d_items, nitems, pers ? 1 : 0,
                                  pers ? P->max_grid : 0, k.ch, pers ? P->d_bar : nullptr, P->stream);
            return ge;
        };
        if (have_built && built.vx == k.vx && built.nw == k.nw && built.h == k.h &&
            (built.flags & LBM_TILE_TWO_STEP) == (k.flags & LBM_TILE_TWO_STEP))
            return go();
        have_built = false;
        const int ovx = P->vx, onw = P->nw, opi = P->per_item;
        P->vx = k.vx;
        P->nw = k.nw;
        P->per_item = k.h;
        P->h_lats.clear();
        P->h_items.clear();
        for (int j = 0; j < count; ++j) {
            BatchLat b{};
            b.tile = slot_tile(P->slots[slots[j]], k.vx, k.nw, two);
            b.t0 = buffer_time(P->slots[slots[j]]);
            b.nsteps = two ? 2 : 1;
            add_lattice(P, b);
        }
        P->vx = ovx;
        P->nw = onw;
        P->per_item = opi;
        nitems = (int)P->h_items.size();
        hipError_t le = ensure_cap(P, count, nitems);
        if (le == hipSuccess)
            le = hipMemcpyAsync(P->d_lats, P->h_lats.data(), sizeof(BatchLat) * (size_t)count, hipMemcpyHostToDevice,
                                P->stream);
        if (le == hipSuccess)
            le = hipMemcpyAsync(P->d_items, P->h_items.data(), sizeof(int) * (size_t)nitems, hipMemcpyHostToDevice,
                                P->stream);
        if (le == hipSuccess) le = go();
        if (le == hipSuccess) {
            built = k;
            have_built = true;
        }
        return le;
    };
    float us = 0;
    const int best = time_candidates(cands, reps, P->stream, launch, &us);
    if (best < 0) return LBM_EDEVICE;
    tune_cache_put(key, cands[best], us);
    P->per_item = cands[best].h;
    P->xcd_chunk = cands[best].ch;
    return lbm_pool_set_tile(P, cands[best].vx, cands[best].nw, cands[best].flags);
}

int lbm_pool_set_items(lbm_pool* P, int tiles_per_item)
{
    if (!P || tiles_per_item < 1 || tiles_per_item > 64) return LBM_EINVAL;
    P->per_item = tiles_per_item;
    return LBM_OK;
}

int lbm_pool_get_tile(const lbm_pool* P, int* vx, int* nw, int* flags)
{
    if (!P) return LBM_EINVAL;
    if (vx) *vx = P->vx;
    if (nw) *nw = P->nw;
    if (flags) *flags = (P->nts ? LBM_TILE_NT_STORE : 0) | (P->two ? LBM_TILE_TWO_STEP : 0);
    return LBM_OK;
}

int lbm_pool_set_stream(lbm_pool* P, void* s)
{
    if (!P) return LBM_EINVAL;
    hipError_t e = hipStreamSynchronize(P->stream);
    drop_graphs(P);  // graphs were captured on the old stream
    P->stream = s ? (hipStream_t)s : P->own;
    return status_of(e);
}

}  // extern "C"

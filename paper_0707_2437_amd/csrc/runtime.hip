// runtime.hip -- host side of liblbm: handles, device memory, streams,
// argument validation and the C ABI declared in include/liblbm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

#include "host.h"
#include "tune.h"

using namespace lbm;

struct lbm_lattice {
    int nx, ny, dtype, esize, device;
    double tau, c2;
    int model;         // lbm_model
    Geom g;
    Coef coef;
    size_t buf_bytes;
    void* buf;         // both population buffers
    void* cur;         // S of the current state (read by the next step)
    void* nxt;         // written by the next step
    double* red;       // moments partials (3 per block) + 3 totals
    hipStream_t own;   // library stream
    hipStream_t stream;
    long long t;
    bool ready;
    int vx, nw, h;     // step tile
    int kflags;        // LBM_TILE_* bits
    void* field;       // per-site source coefficients of a c2 field, or nullptr
    int fpitch;        // its row pitch (elements)
    int xbc;           // lbm_xbc
    double amp, period;  // inlet density oscillation (LBM_XBC_INLET_OUTLET)
};

namespace {

thread_local int g_last_error = LBM_OK;

// Defaults from repeated tile sweeps on MI355X at 4096^2 and 8192^2
// (row-interleaved layout). Single-step shapes: the vertical-stack form for
// every dtype; they also take the steps a two-step shape cannot (a lone last
// step, inlet/outlet boundaries).
struct TileDefault {
    int vx, nw, h, flags;
};
TileDefault default_single_tile(int dtype)
{
    switch (dtype) {
    case LBM_F64: return {2, 8, 8, LBM_TILE_VSTACK | LBM_TILE_NT_STORE};
    case LBM_F32: return {2, 8, 8, LBM_TILE_VSTACK | LBM_TILE_NT_STORE};
    case LBM_F32S: return {2, 8, 8, LBM_TILE_VSTACK | LBM_TILE_NT_STORE};
    default: return {4, 8, 8, LBM_TILE_VSTACK | LBM_TILE_NT_STORE};
    }
}
// The default shape of a new lattice: two steps per launch (FP64 with one
// column per lane, which measured faster for it and keeps its LDS at half
// of the CU's; FP16 in 32-row tiles with plain stores, the only two-step
// shape that beat its single-step kernel).
TileDefault default_tile(int dtype)
{
    switch (dtype) {
    case LBM_F64: return {1, 16, 8, LBM_TILE_VSTACK | LBM_TILE_TWO_STEP | LBM_TILE_NT_STORE};
    case LBM_F32:
    case LBM_F32S: return {2, 16, 8, LBM_TILE_VSTACK | LBM_TILE_TWO_STEP | LBM_TILE_NT_STORE};
    default: return {1, 32, 8, LBM_TILE_VSTACK | LBM_TILE_TWO_STEP};
    }
}

// A step shape of lbm_set_tile: the two-step form (LBM_TILE_TWO_STEP, with
// LBM_TILE_VSTACK and at most LBM_TILE_NT_STORE besides) or a single-step one.
bool tile_supported(int dtype, int vx, int nw, int flags)
{
    if (flags & ~63) return false;
    if (flags & LBM_TILE_TWO_STEP)
        return (flags & LBM_TILE_VSTACK) && !(flags & ~(LBM_TILE_TWO_STEP | LBM_TILE_VSTACK | LBM_TILE_NT_STORE)) &&
               step2_shape_supported(dtype, vx, nw);
    return step_shape_supported(dtype, vx, nw, flags);
}

// Optional override for experiments: LBM_TILE="vx,nw,h,flags".
void apply_tile_env(int dtype, int* vx, int* nw, int* h, int* flags)
{
    const char* e = std::getenv("LBM_TILE");
    int a = 0, b = 0, c = 0, f = 0;
    if (e && std::sscanf(e, "%d,%d,%d,%d", &a, &b, &c, &f) == 4 && tile_supported(dtype, a, b, f) &&
        (c > 0 || (f & LBM_TILE_VSTACK))) {
        *vx = a;
        *nw = b;
        *h = c;
        *flags = f;
    }
}

StepTile make_tile(const lbm_lattice* L)
{
    StepTile t;
    t.src = L->cur;
    t.dst = L->nxt;
    t.g = L->g;
    t.c = L->coef;
    t.h = L->h;
    t.xcd_chunk = 0;
    if (L->kflags & LBM_TILE_TWO_STEP) {
        // step2_cols(vx) columns and step2_rows(nw) rows per workgroup
        const int W = step2_cols(L->vx), R = step2_rows(L->nw);
        t.nstrips = (L->nx + W - 1) / W;
        t.nchunks = (L->ny + R - 1) / R;
        t.xcd_chunk = xcd_chunk_tiles(t.nstrips);
    } else if (L->kflags & LBM_TILE_VSTACK) {
        // one strip of 64 * vx columns and nw - 2 rows per workgroup
        const int W = 64 * L->vx, R = L->nw - 2;
        t.nstrips = (L->nx + W - 1) / W;
        t.nchunks = (L->ny + R - 1) / R;
        t.xcd_chunk = xcd_chunk_tiles(t.nstrips);
    } else {
        const int W = 64 * L->nw * L->vx;  // columns of the NW strips of one workgroup
        t.nstrips = (L->nx + W - 1) / W;
        t.nchunks = (L->ny + L->h - 1) / L->h;
    }
    t.rowband = (L->kflags & LBM_TILE_ROWBAND) ? 1 : 0;
    t.field = L->field;
    t.fpitch = L->fpitch;
    return t;
}

// A lattice with a c2 field steps with the vertical-stack kernels (single-
// or two-step) only: a march-form tile is replaced by the dtype's default.
void field_tile(lbm_lattice* L)
{
    if (L->kflags & LBM_TILE_VSTACK) return;
    const TileDefault td = default_tile(L->dtype);
    L->vx = td.vx;
    L->nw = td.nw;
    L->h = td.h;
    L->kflags = td.flags;
}

// Allocate the field array on first use.
int ensure_field(lbm_lattice* L)
{
    if (L->field) return LBM_OK;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, field_bytes(L->nx, L->ny, L->dtype));
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE;
    L->field = p;
    L->fpitch = field_pitch(L->nx);
    return LBM_OK;
}

int drop_field(lbm_lattice* L)
{
    if (!L->field) return LBM_OK;
    hipError_t e = hipStreamSynchronize(L->stream);
    (void)hipFree(L->field);
    L->field = nullptr;
    L->fpitch = 0;
    return status_of(e);
}

}  // namespace

extern "C" {

int lbm_last_error(void) { return g_last_error; }

const char* lbm_strerror(int status)
{
    switch (status) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOMEM: return "out of memory";
    case LBM_EDEVICE: return "HIP device error";
    case LBM_ESTATE: return "lattice not initialised";
    case LBM_ENONFINITE: return "non-finite conservation total";
    default: return "unknown status";
    }
}

size_t lbm_footprint_bytes(int nx, int ny, int dtype)
{
    if (!args_ok(nx, ny, 1.0, 1.0 / 3.0, dtype)) return 0;
    const int es = esize_of(dtype);
    const Geom g = make_geom(nx, ny, es, choose_interleaved(nx, ny, dtype));
    return footprint(g, es) + red_doubles(g) * sizeof(double);
}

lbm_lattice* lbm_create(int nx, int ny, double tau, double c2, int dtype)
{
    if (!args_ok(nx, ny, tau, c2, dtype)) {
        g_last_error = LBM_EINVAL;
        return nullptr;
    }
    lbm_lattice* L = new (std::nothrow) lbm_lattice();
    if (!L) {
        g_last_error = LBM_ENOMEM;
        return nullptr;
    }
    L->nx = nx;
    L->ny = ny;
    L->dtype = dtype;
    L->esize = esize_of(dtype);
    L->tau = tau;
    L->c2 = c2;
    L->g = make_geom(nx, ny, L->esize, choose_interleaved(nx, ny, dtype));
    L->model = LBM_MODEL_FORCING;
    L->coef = make_coef(tau, c2, L->model);
    const TileDefault td = default_tile(dtype);
    L->vx = td.vx;
    L->nw = td.nw;
    L->h = td.h;
    L->kflags = td.flags;
    apply_tile_env(dtype, &L->vx, &L->nw, &L->h, &L->kflags);
    hipError_t e = hipGetDevice(&L->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&L->own, hipStreamNonBlocking);
    if (e != hipSuccess) {
        g_last_error = status_of(e);
        delete L;
        return nullptr;
    }
    L->stream = L->own;
    L->buf_bytes = footprint(L->g, L->esize);
    e = hipMalloc(&L->buf, L->buf_bytes);
    if (e == hipSuccess) e = hipMalloc((void**)&L->red, red_doubles(L->g) * sizeof(double));
    if (e == hipSuccess) e = hipMemsetAsync(L->buf, 0, L->buf_bytes, L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    if (e != hipSuccess) {
        g_last_error = e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE;
        lbm_destroy(L);
        return nullptr;
    }
    L->cur = L->buf;
    L->nxt = (char*)L->buf + (size_t)buffer_elems(L->g) * L->esize;
    g_last_error = LBM_OK;
    return L;
}

void lbm_destroy(lbm_lattice* L)
{
    if (!L) return;
    if (L->own) (void)hipStreamSynchronize(L->stream);
    if (L->buf) (void)hipFree(L->buf);
    if (L->red) (void)hipFree(L->red);
    if (L->field) (void)hipFree(L->field);
    if (L->own) (void)hipStreamDestroy(L->own);
    delete L;
}

int lbm_set_stream(lbm_lattice* L, void* s)
{
    if (!L) return LBM_EINVAL;
    hipError_t e = hipStreamSynchronize(L->stream);
    L->stream = (hipStream_t)s;
    return status_of(e);
}

int lbm_use_own_stream(lbm_lattice* L)
{
    if (!L) return LBM_EINVAL;
    hipError_t e = hipStreamSynchronize(L->stream);
    L->stream = L->own;
    return status_of(e);
}

void* lbm_get_stream(const lbm_lattice* L) { return L ? (void*)L->stream : nullptr; }

long long lbm_time(const lbm_lattice* L) { return L ? L->t : -1; }

int lbm_set_tile(lbm_lattice* L, int vx, int nw, int h, int flags)
{
    if (!L || !tile_supported(L->dtype, vx, nw, flags)) return LBM_EINVAL;
    if (!(flags & LBM_TILE_VSTACK) && (h < 1 || L->field)) return LBM_EINVAL;
    {
        // the shape's grid must fit one dispatch for this lattice
        lbm_lattice tmp = *L;
        tmp.vx = vx;
        tmp.nw = nw;
        tmp.h = h;
        tmp.kflags = flags;
        const StepTile t = make_tile(&tmp);
        const long long tiles = (long long)t.nstrips * t.nchunks;
        if (!grid_fits(tiles + 8LL * (t.xcd_chunk > 0 ? t.xcd_chunk : 1), 64 * nw)) return LBM_EINVAL;
    }
    L->vx = vx;
    L->nw = nw;
    L->h = h;
    L->kflags = flags;
    return LBM_OK;
}

int lbm_autotune(lbm_lattice* L, int reps, int use_cache)
{
    if (!L || reps < 1) return LBM_EINVAL;
    if (!L->ready) return LBM_ESTATE;
    char key[160];
    std::snprintf(key, sizeof(key), "%s|%s|%d|%dx%d", device_arch().c_str(), L->field ? "lattice-field" : "lattice",
                  L->dtype, L->nx, L->ny);
    TileCand c{};
    if (use_cache && tune_cache_get(key, &c)) return lbm_set_tile(L, c.vx, c.nw, c.h, c.flags);
    std::vector<TileCand> cands = lattice_candidates(L->dtype);
    if (L->field)  // the vertical-stack kernels only
        cands.erase(std::remove_if(cands.begin(), cands.end(),
                                   [](const TileCand& k) { return !(k.flags & LBM_TILE_VSTACK); }),
                    cands.end());
    // Each candidate is timed over two steps (two single-step launches or
    // one two-step launch), reading cur and writing nxt with no swap: the
    // state does not change.
    auto launch = [&](const TileCand& k) -> hipError_t {
        lbm_lattice tmp = *L;
        tmp.vx = k.vx;
        tmp.nw = k.nw;
        tmp.h = k.h;
        tmp.kflags = k.flags;
        const StepTile t = make_tile(&tmp);
        if (k.flags & LBM_TILE_TWO_STEP) return launch_step2(L->dtype, k.vx, k.nw, k.flags, t, L->stream);
        hipError_t e = launch_step(L->dtype, k.vx, k.nw, k.flags, t, L->stream);
        if (e == hipSuccess) e = launch_step(L->dtype, k.vx, k.nw, k.flags, t, L->stream);
        return e;
    };
    float us = 0;
    const int best = time_candidates(cands, reps, L->stream, launch, &us);
    if (best < 0) return LBM_EDEVICE;
    tune_cache_put(key, cands[best], us);
    return lbm_set_tile(L, cands[best].vx, cands[best].nw, cands[best].h, cands[best].flags);
}

int lbm_get_tile(const lbm_lattice* L, int* vx, int* nw, int* h, int* flags)
{
    if (!L) return LBM_EINVAL;
    if (vx) *vx = L->vx;
    if (nw) *nw = L->nw;
    if (h) *h = L->h;
    if (flags) *flags = L->kflags;
    return LBM_OK;
}

int lbm_init_device(lbm_lattice* L, const double* rho, const double* ux, const double* uy)
{
    if (!L) return LBM_EINVAL;
    hipError_t e = launch_init(L->dtype, L->cur, L->g, rho, ux, uy, eq_shift(L->c2, L->model), L->stream);
    if (e != hipSuccess) return status_of(e);
    L->t = 0;
    L->ready = true;
    return LBM_OK;
}

int lbm_set_model(lbm_lattice* L, int model)
{
    if (!L || !model_ok(model, L->c2) || (L->field && model != LBM_MODEL_FORCING)) return LBM_EINVAL;
    const double old_shift = eq_shift(L->c2, L->model), new_shift = eq_shift(L->c2, model);
    if (L->ready && new_shift != old_shift && (L->dtype == LBM_F32S || L->dtype == LBM_F16S)) {
        // The shifted storage is centred on the model's state at rest: keep
        // f by reading it with the old centre and storing it with the new.
        DevScratch d;
        hipError_t e = d.alloc((size_t)9 * L->nx * L->ny, L->stream);
        if (e == hipSuccess) e = launch_get_f(L->dtype, L->cur, L->g, d.p, old_shift, L->stream);
        if (e == hipSuccess) e = launch_set_f(L->dtype, L->cur, L->g, d.p, new_shift, L->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
        if (e != hipSuccess) return status_of(e);
    }
    L->model = model;
    L->coef = make_coef(L->tau, L->c2, model);
    return LBM_OK;
}

int lbm_set_x_boundaries(lbm_lattice* L, int mode, double amplitude, double period)
{
    if (!L) return LBM_EINVAL;
    if (mode == LBM_XBC_PERIODIC) {
        L->xbc = mode;
        return LBM_OK;
    }
    if (mode != LBM_XBC_INLET_OUTLET || L->nx < 5 || !std::isfinite(period) || !(period > 0.0) ||
        !std::isfinite(amplitude) || !(std::fabs(amplitude) < 1.0))
        return LBM_EINVAL;
    L->xbc = mode;
    L->amp = amplitude;
    L->period = period;
    return LBM_OK;
}

int lbm_set_c2_field(lbm_lattice* L, const double* c2)
{
    if (!L || L->model != LBM_MODEL_FORCING) return LBM_EINVAL;
    if (!c2) return drop_field(L);
    const size_t n = (size_t)L->nx * L->ny;
    for (size_t k = 0; k < n; ++k)
        if (!std::isfinite(c2[k]) || !(c2[k] > 0.0)) return LBM_EINVAL;
    int st = ensure_field(L);
    if (st != LBM_OK) return st;
    DevScratch d;
    hipError_t e = d.alloc(n, L->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d.p, c2, n * sizeof(double), hipMemcpyHostToDevice, L->stream);
    if (e == hipSuccess) e = launch_field(L->dtype, L->field, L->nx, L->ny, L->fpitch, d.p, L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    if (e != hipSuccess) return status_of(e);
    field_tile(L);
    return LBM_OK;
}

int lbm_set_c2_field_device(lbm_lattice* L, const double* c2)
{
    if (!L || L->model != LBM_MODEL_FORCING) return LBM_EINVAL;
    if (!c2) return drop_field(L);
    int st = ensure_field(L);
    if (st != LBM_OK) return st;
    hipError_t e = launch_field(L->dtype, L->field, L->nx, L->ny, L->fpitch, c2, L->stream);
    if (e != hipSuccess) return status_of(e);
    field_tile(L);
    return LBM_OK;
}

int lbm_init(lbm_lattice* L, const double* rho, const double* ux, const double* uy)
{
    if (!L) return LBM_EINVAL;
    const size_t n = (size_t)L->nx * L->ny;
    DevScratch d;
    hipError_t e = d.alloc(3 * n, L->stream);
    const double* src[3] = {rho, ux, uy};
    const double* dp[3] = {nullptr, nullptr, nullptr};
    for (int c = 0; c < 3 && e == hipSuccess; ++c) {
        if (!src[c]) continue;
        e = hipMemcpyAsync(d.p + c * n, src[c], n * sizeof(double), hipMemcpyHostToDevice, L->stream);
        dp[c] = d.p + c * n;
    }
    if (e != hipSuccess) return status_of(e);
    int st = lbm_init_device(L, dp[0], dp[1], dp[2]);
    e = hipStreamSynchronize(L->stream);
    return st != LBM_OK ? st : status_of(e);
}

int lbm_step(lbm_lattice* L, int n)
{
    if (!L || n < 0) return LBM_EINVAL;
    if (!L->ready) return LBM_ESTATE;
    // A two-step shape advances two steps per launch; a lone last step, and
    // every step of a lattice with inlet/outlet boundaries (applied after
    // each step), take the dtype's default single-step shape.
    const bool two = (L->kflags & LBM_TILE_TWO_STEP) != 0;
    lbm_lattice one = *L;
    if (two) {
        const TileDefault td = default_single_tile(L->dtype);
        one.vx = td.vx;
        one.nw = td.nw;
        one.h = td.h;
        one.kflags = td.flags;
    }
    for (int k = 0; k < n;) {
        hipError_t e;
        int done = 1;
        if (two && L->xbc != LBM_XBC_INLET_OUTLET && n - k >= 2) {
            e = launch_step2(L->dtype, L->vx, L->nw, L->kflags, make_tile(L), L->stream);
            done = 2;
        } else {
            one.cur = L->cur;
            one.nxt = L->nxt;
            e = launch_step(L->dtype, one.vx, one.nw, one.kflags, make_tile(&one), L->stream);
            if (e == hipSuccess && L->xbc == LBM_XBC_INLET_OUTLET)
                e = launch_xbc(L->dtype, L->nxt, L->g, inlet_density(L->amp, L->period, L->t),
                               eq_shift(L->c2, L->model), L->stream);
        }
        if (e != hipSuccess) return status_of(e);
        void* tmp = L->cur;
        L->cur = L->nxt;
        L->nxt = tmp;
        L->t += done;
        k += done;
    }
    return LBM_OK;
}

int lbm_moments_device(lbm_lattice* L, double* rho, double* ux, double* uy, double totals[3])
{
    if (!L) return LBM_EINVAL;
    if (!L->ready) return LBM_ESTATE;
    const int nb = moments_blocks(L->g);
    double* tot_dev = L->red + (size_t)3 * nb;
    hipError_t e = launch_moments(L->dtype, L->cur, L->g, rho, ux, uy, L->red, tot_dev, L->stream);
    double tot[3] = {0, 0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(tot, tot_dev, sizeof(tot), hipMemcpyDeviceToHost, L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    if (e != hipSuccess) return status_of(e);
    if (totals) std::memcpy(totals, tot, sizeof(tot));
    for (double v : tot)
        if (!std::isfinite(v)) return LBM_ENONFINITE;
    return LBM_OK;
}

int lbm_moments(lbm_lattice* L, double* rho, double* ux, double* uy, double totals[3])
{
    if (!L) return LBM_EINVAL;
    if (!L->ready) return LBM_ESTATE;
    const size_t n = (size_t)L->nx * L->ny;
    DevScratch d;
    hipError_t e = (rho || ux || uy) ? d.alloc(3 * n, L->stream) : hipSuccess;
    if (e != hipSuccess) return status_of(e);
    double* dp[3] = {rho ? d.p : nullptr, ux ? d.p + n : nullptr, uy ? d.p + 2 * n : nullptr};
    int st = lbm_moments_device(L, dp[0], dp[1], dp[2], totals);
    if (st != LBM_OK && st != LBM_ENONFINITE) return st;
    double* host[3] = {rho, ux, uy};
    for (int c = 0; c < 3 && e == hipSuccess; ++c)
        if (host[c]) e = hipMemcpyAsync(host[c], dp[c], n * sizeof(double), hipMemcpyDeviceToHost, L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    return e != hipSuccess ? status_of(e) : st;
}

int lbm_get_f(lbm_lattice* L, double* f)
{
    if (!L || !f) return LBM_EINVAL;
    if (!L->ready) return LBM_ESTATE;
    const size_t n = (size_t)9 * L->nx * L->ny;
    DevScratch d;
    hipError_t e = d.alloc(n, L->stream);
    if (e == hipSuccess) e = launch_get_f(L->dtype, L->cur, L->g, d.p, eq_shift(L->c2, L->model), L->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(f, d.p, n * sizeof(double), hipMemcpyDeviceToHost, L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    return status_of(e);
}

int lbm_sample_f(lbm_lattice* L, int n, const int* xs, const int* ys, double* f)
{
    if (!L || n < 0 || (n > 0 && (!xs || !ys || !f))) return LBM_EINVAL;
    if (!L->ready) return LBM_ESTATE;
    if (n == 0) return LBM_OK;
    for (int k = 0; k < n; ++k)
        if (xs[k] < 0 || xs[k] >= L->nx || ys[k] < 0 || ys[k] >= L->ny) return LBM_EINVAL;
    int* hxy = (int*)std::malloc(sizeof(int) * 2 * (size_t)n);
    if (!hxy) return LBM_ENOMEM;
    for (int k = 0; k < n; ++k) {
        hxy[2 * k] = xs[k];
        hxy[2 * k + 1] = ys[k];
    }
    DevScratch d;  // 9 n doubles of output, then 2 n ints of sites
    hipError_t e = d.alloc((size_t)9 * n + (size_t)n, L->stream);
    int* dxy = (int*)(d.p + (size_t)9 * n);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dxy, hxy, sizeof(int) * 2 * (size_t)n, hipMemcpyHostToDevice, L->stream);
    if (e == hipSuccess) e = launch_sample_f(L->dtype, L->cur, L->g, n, dxy, d.p, eq_shift(L->c2, L->model), L->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(f, d.p, sizeof(double) * 9 * (size_t)n, hipMemcpyDeviceToHost, L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    std::free(hxy);
    return status_of(e);
}

int lbm_set_f(lbm_lattice* L, const double* f)
{
    if (!L || !f) return LBM_EINVAL;
    const size_t n = (size_t)9 * L->nx * L->ny;
    DevScratch d;
    hipError_t e = d.alloc(n, L->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d.p, f, n * sizeof(double), hipMemcpyHostToDevice, L->stream);
    if (e == hipSuccess) e = launch_set_f(L->dtype, L->cur, L->g, d.p, eq_shift(L->c2, L->model), L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    if (e != hipSuccess) return status_of(e);
    L->t = 0;
    L->ready = true;
    return LBM_OK;
}

}  // extern "C"

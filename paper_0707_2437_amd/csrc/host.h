// host.h -- host-side helpers shared by the lattice (runtime.hip) and pool
// (pool.hip) parts of liblbm: kernel launchers, geometry and coefficients.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>

#include "internal.h"
#include "liblbm.h"
#include "step2.h"

namespace lbm {
hipError_t launch_step(int dtype, int vx, int nw, int flags, const StepTile& t, hipStream_t st);
bool step_shape_supported(int dtype, int vx, int nw, int flags);
// Two steps per launch (step2.hip); t's strips and row groups are those of
// step2_cols / step2_rows.
hipError_t launch_step2(int dtype, int vx, int nw, int flags, const StepTile& t, hipStream_t st);
bool step2_shape_supported(int dtype, int vx, int nw);
// Set-up of a persistent batched launch of kernel kern (threads per
// workgroup): the grid (what the runtime reports as resident at once,
// capped by max_grid, a multiple of 8 ch, or of 8 with *ch = 0, or *ch =
// -1 below 8), the bounded barrier wait and the membership grace in device
// clock ticks; and the reset of the barrier words bar on stream st.
hipError_t persistent_setup(const void* kern, int threads, int max_grid, int* ch, int* grid,
                            unsigned long long* wait_ticks, unsigned long long* grace_ticks, unsigned* bar,
                            hipStream_t st);
// All passes (npasses of two steps) of a batch in one persistent launch of
// two-step tiles (step2.hip), with a grid barrier between passes (as the
// single-step persistent kernel, batch.hip).
hipError_t launch_batch2_persistent(int dtype, int vx, int nw, bool nts, const BatchLat* lats, const int* item_lat,
                                    int nitems, int npasses, int max_grid, int ch, unsigned* bar, hipStream_t st);
// Pass p (steps 2p, 2p + 1) of a batch in two-step tiles (step2.hip): the
// descriptors' t0 is each lattice's buffer time (its state is in buffer
// (t0 + p) & 1 at the start of pass p); a lattice with nsteps = 2p + 1
// takes one step, one with nsteps <= 2p none.
hipError_t launch_batch2(int dtype, int vx, int nw, bool nts, const BatchLat* lats, const int* item_lat, int nitems,
                         int p, int ch, hipStream_t st);
hipError_t launch_init(int dtype, void* s, const Geom& g, const double* rho, const double* ux, const double* uy,
                       double eqs, hipStream_t st);
hipError_t launch_xbc(int dtype, void* s, const Geom& g, double rho_in, double eqs, hipStream_t st);
hipError_t launch_field(int dtype, void* field, int nx, int ny, int fpitch, const double* c2, hipStream_t st);
// eqs: the model's equilibrium shift (eq_shift), which sets the centre of
// the shifted storage.
hipError_t launch_set_f(int dtype, void* s, const Geom& g, const double* f, double eqs, hipStream_t st);
hipError_t launch_get_f(int dtype, const void* s, const Geom& g, double* f, double eqs, hipStream_t st);
int moments_blocks(const Geom& g);
hipError_t launch_sample_f(int dtype, const void* s, const Geom& g, int n, const int* xy, double* out, double eqs,
                           hipStream_t st);
hipError_t launch_moments(int dtype, const void* s, const Geom& g, double* rho, double* ux, double* uy,
                          double* partials, double* totals, hipStream_t st);
// Words of barrier and work-counter state a persistent batched launch
// needs (device memory the pool allocates once; see the persistent kernel).
constexpr int kPoolBarWords = 24;
// bar: the persistent kernel's barrier state, kPoolBarWords zeroed words
// (device memory of the caller; unused by grouped launches).
hipError_t launch_batch(int dtype, int vx, int nw, bool nts, bool persistent, const BatchLat* lats,
                        const int* item_lat, int nitems, int s_or_n, int max_grid, int ch, unsigned* bar,
                        hipStream_t st);


constexpr int kLineBytes = 128;

inline int esize_of(int dtype)
{
    switch (dtype) {
    case LBM_F64: return 8;
    case LBM_F32:
    case LBM_F32S: return 4;
    case LBM_F16S: return 2;
    default: return 0;
    }
}

inline Geom make_geom(int nx, int ny, int esize, bool interleaved);
inline long long buffer_elems(const Geom& g);

// True if the kernels' 32-bit byte offsets cover the lattice in this layout:
// a plane (plane-major) or a whole buffer (row-interleaved).
inline bool offsets_fit(int nx, int ny, int dtype, bool interleaved)
{
    const Geom g = make_geom(nx, ny, esize_of(dtype), interleaved);
    const long long span = interleaved ? buffer_elems(g) : g.ps;
    return (unsigned long long)(span + g.pitch) * esize_of(dtype) < (1ULL << 32);
}

// Layout of a new lattice: row-interleaved when it fits (it streams the nine
// plane rows of a lattice row as one contiguous block), else plane-major.
// LBM_LAYOUT=soa forces plane-major.
inline bool choose_interleaved(int nx, int ny, int dtype)
{
    const char* e = std::getenv("LBM_LAYOUT");
    if (e && std::strcmp(e, "soa") == 0) return false;
    return offsets_fit(nx, ny, dtype, true);
}

inline bool args_ok(int nx, int ny, double tau, double c2, int dtype)
{
    // nx, ny >= 3: the central differences need two distinct neighbours.
    // tau > 1/2: positive viscosity (Eq. 4). c2 > 0: real c_e (Eq. 8).
    if (nx < 3 || ny < 3 || !std::isfinite(tau) || !(tau > 0.5) || !std::isfinite(c2) || !(c2 > 0.0)) return false;
    if (esize_of(dtype) == 0) return false;
    if (nx > (1 << 28) || ny > (1 << 28)) return false;
    return offsets_fit(nx, ny, dtype, choose_interleaved(nx, ny, dtype));
}

// Row pitch leaves one line before column 0 and room past column nx - 1 for
// the widest window (the gather reads up to two columns before the row and
// up to kMaxVX + 2 after it; those padding elements are never used).
// Plane-major layout: planes rounded to 4 KiB plus a 1 KiB skew;
// row-interleaved layout: rows of 9 * pitch.
inline Geom make_geom(int nx, int ny, int esize, bool interleaved)
{
    Geom g;
    g.nx = nx;
    g.ny = ny;
    const int line = kLineBytes / esize;
    g.off = line;
    const long long need = (long long)line + nx + kMaxVX + 4;
    g.pitch = (int)((need + line - 1) / line * line);
    if (interleaved) {
        g.ps = g.pitch;
        g.rs = 9LL * g.pitch;
    } else {
        const long long bytes = (long long)g.pitch * ny * esize;
        g.ps = ((bytes + 4095) / 4096 * 4096 + 1024) / esize;
        g.rs = g.pitch;
    }
    return g;
}

// Elements of one population buffer (9 planes).
inline long long buffer_elems(const Geom& g) { return g.rs == g.pitch ? 9 * g.ps : g.rs * g.ny; }

inline size_t footprint(const Geom& g, int esize)
{
    // 2 buffers, plus one line of slack past the end.
    return (size_t)2 * (size_t)buffer_elems(g) * esize + kLineBytes;
}

inline size_t red_doubles(const Geom& g) { return (size_t)3 * moments_blocks(g) + 3; }

// The equilibrium shift of the altered-equilibrium model: 3 c^2 - 1 (its
// moving populations carry 3 c^2 in place of the 1 of Eq. 2); 0 for the
// paper's model.
inline double eq_shift(double c2, int model) { return model == LBM_MODEL_EQUILIBRIUM ? 3.0 * c2 - 1.0 : 0.0; }

inline Coef make_coef(double tau, double c2, int model)
{
    // Eq. 5 with alpha = 1/3 - c2 (Eq. 8), weights of Sec. 2; the 1/2 of the
    // central differences is folded into as1, as2. The altered-equilibrium
    // model has no source term and shifts the equilibrium instead: for
    // i != 0, feq_i - w_i gains w_i rho (3 c^2 - 1); feq_0 loses the sum of
    // those, (5/9) rho (3 c^2 - 1) = w_0 rho (5/4)(3 c^2 - 1).
    const double om = 1.0 / tau;
    const double w0 = 4.0 / 9.0, w1 = 1.0 / 9.0, w2 = 1.0 / 36.0;
    const double sh = eq_shift(c2, model);
    Coef k;
    k.om1 = 1.0 - om;
    k.wo0 = om * w0;
    k.wo1 = om * w1;
    k.wo2 = om * w2;
    k.as1 = model == LBM_MODEL_EQUILIBRIUM ? 0.0 : source_as1(c2);
    k.as2 = 0.25 * k.as1;
    k.e1 = sh;
    k.e0 = -1.25 * sh;
    k.om1f = (float)k.om1;
    k.wo0f = (float)k.wo0;
    k.wo1f = (float)k.wo1;
    k.wo2f = (float)k.wo2;
    k.as1f = (float)k.as1;
    k.as2f = (float)k.as2;
    k.e1f = (float)k.e1;
    k.e0f = (float)k.e0;
    return k;
}

// A c2 field: row pitch (elements) and bytes of the per-site coefficient
// array of a lattice (compute precision: FP64 for LBM_F64, else FP32). The
// pitch covers every column a vertical-stack lane of up to 4 columns reads.
inline int field_pitch(int nx) { return (nx + 255) / 256 * 256; }
inline size_t field_esize(int dtype) { return dtype == LBM_F64 ? sizeof(double) : sizeof(float); }
inline size_t field_bytes(int nx, int ny, int dtype) { return (size_t)ny * field_pitch(nx) * field_esize(dtype); }

// Inlet density of the Fig. 1 boundaries at time t (Sec. 4): an oscillation
// of the given amplitude and period about rho = 1.
inline double inlet_density(double amplitude, double period, long long t)
{
    return 1.0 + amplitude * std::sin(2.0 * 3.14159265358979323846 * (double)t / period);
}

// Tiles per XCD chunk of the vertical-stack kernels (see xcd_tile): whole
// row groups of a lattice, at least 16 tiles. LBM_XCD_CHUNK=<n> overrides
// it for experiments (0: one contiguous run of tiles per XCD).
inline int xcd_chunk_tiles(int nstrips)
{
    if (const char* e = std::getenv("LBM_XCD_CHUNK")) {
        const int v = std::atoi(e);
        if (v >= 0 && v <= 4096) return v;
    }
    const int groups = (16 + nstrips - 1) / nstrips;
    return groups * nstrips;
}

// Models an lbm_set_model call may select for (c2): the altered-equilibrium
// model needs a positive rest population, 1 - 5 c^2 / 3 > 0.
inline bool model_ok(int model, double c2)
{
    return model == LBM_MODEL_FORCING || (model == LBM_MODEL_EQUILIBRIUM && c2 < 0.6);
}

inline int status_of(hipError_t e)
{
    if (e == hipSuccess) return LBM_OK;
    if (e == hipErrorOutOfMemory) return LBM_ENOMEM;
    if (e == hipErrorInvalidConfiguration) return LBM_EINVAL;  // a grid too large for one dispatch
    return LBM_EDEVICE;
}

// Device staging memory of one host-array entry point: taken from the
// device's stream-ordered memory pool on the call's stream and given back on
// that stream when the call returns. Unlike hipMalloc / hipFree, neither step
// synchronises the device, so a set-up or read-back call on one lattice does
// not stall work queued on other streams.
struct DevScratch {
    double* p = nullptr;
    hipStream_t st = nullptr;
    hipError_t alloc(size_t n, hipStream_t stream)
    {
        st = stream;
        const hipError_t e = hipMallocAsync((void**)&p, n * sizeof(double), stream);
        if (e != hipSuccess) p = nullptr;
        return e;
    }
    ~DevScratch()
    {
        if (p) (void)hipFreeAsync(p, st);
    }
};

}  // namespace lbm

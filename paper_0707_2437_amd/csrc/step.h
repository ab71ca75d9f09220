// step.h -- device code of the variable-speed-of-sound D2Q9 step (Buick &
// Cosgrove, Sec. 3 Eq. 5), shared by the single-lattice and batched kernels.
// See kernels.hip for the decomposition; internal.h for the storage layout.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.h"

namespace lbm {

template <class T> struct CompT { using type = float; };
template <> struct CompT<double> { using type = double; };

// Minimum waves per SIMD the vertical-stack kernels are compiled for. The
// FP16 form converts every loaded value and is bound by how many tiles are
// in flight per CU; asking for 7 waves caps it at 72 VGPRs (no spills).
template <class T> struct MinWaves { static constexpr int value = 1; };
template <> struct MinWaves<_Float16> { static constexpr int value = 7; };

// Periodicity in x. FP16 storage keeps ghost copies of the two edge columns
// on each side of every row (columns -2, -1 hold nx-2, nx-1 and nx, nx+1
// hold 0, 1), written by the step that writes those columns, so its windows
// need no wrap. The other storage types write no copies (they would be
// scattered partial-line stores); their loads take the wrapped elements from
// the periodic image instead (patch_edges), in a separate copy of the code
// run only by the strips at the lattice's edges. For FP16 the patch costs
// more than the copies (its 2-byte elements share registers).
template <class T> struct GhostCols { static constexpr bool value = false; };
template <> struct GhostCols<_Float16> { static constexpr bool value = true; };

// Lattice weights (Sec. 2) in compute precision.
template <class C> __device__ __forceinline__ C wt(int i)
{
    return i == 0 ? C(4) / C(9) : (i < 5 ? C(1) / C(9) : C(1) / C(36));
}

__device__ __forceinline__ int wrapy(int r, int ny) { return r < 0 ? r + ny : (r >= ny ? r - ny : r); }

// The state the arithmetic is centred on: d_i = f_i - r_i. FP32 arithmetic
// (and the shifted storage, which it reads as is) centres on the lattice
// model's equilibrium at rest (rho = 1, u = 0), r_i = w_i (1 + e): e = 0 for
// Eq. 2 (r_i = w_i), e = 3 c^2 - 1 (moving) and -(5/4)(3 c^2 - 1) (rest) for
// the altered-equilibrium model, whose populations at small c^2 sit far from
// the weights; keeping d small next to f is what FP32 needs. FP64
// arithmetic centres on the weights, r_i = w_i, for both models. Either way
// sum_i r_i = 1 and sum_i r_i e_i = 0, so rho = 1 + sum_i d_i and
// rho u = sum_i d_i e_i. The batched kernels, whose lattices all step the
// paper's model (r_i = w_i), centre on the weights at every precision
// (their coefficients sit behind two dependent loads, and the weights are
// compile-time constants); RC below selects the centring.
template <class C> struct ModelCentred { static constexpr bool value = sizeof(C) == sizeof(float); };
template <class C> struct Centre {
    C r0, r1, r2;
    __device__ __forceinline__ C at(int i) const { return i == 0 ? r0 : (i < 5 ? r1 : r2); }
};

// Stored value -> d_i = f_i - r_i in compute precision, and back (shifted
// storage already holds d_i).
template <class T, bool SHIFT, class C> __device__ __forceinline__ C to_d(T v, int i, const Centre<C>& cn)
{
    if constexpr (SHIFT) return (C)v;
    else return (C)v - cn.at(i);
}
template <class T, bool SHIFT, class C> __device__ __forceinline__ T from_d(C d, int i, const Centre<C>& cn)
{
    if constexpr (sizeof(T) < sizeof(C)) {
        // The relaxed value is rounded to FP32 and then to the storage type.
        // Hide it from instruction selection, which would otherwise fuse the
        // last FMA and the conversion into one mixed-precision FMA (a single
        // rounding) in some kernels and not in others, and the kernels would
        // no longer agree bit for bit.
        asm("" : "+v"(d));
    }
    if constexpr (SHIFT) return (T)d;
    else return (T)(cn.at(i) + d);
}

// Compile-time loop: f(std::integral_constant<int, I>) for I = B .. E - 1.
template <int B, int E, class F> __device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

template <class T, int VX> struct Pack { T v[VX]; };

// Memory is addressed as a per-plane base pointer (uniform, computed once
// per workgroup, held in scalar registers) plus a 32-bit byte offset (row
// offset + lane offset), which maps to SGPR-based global loads and stores;
// the lattice is created only if those offsets fit in 32 bits. Only element
// alignment is assumed: the windows start one element off a vector
// boundary, and gfx950 executes such dwordx2/x3/x4 loads directly.
//
// The population buffers are device (global) memory, and every access goes
// through a global-address-space pointer: pointers that come from a
// descriptor array rather than a kernel argument (the batched kernels) are
// otherwise generic to the compiler, which then emits flat accesses with
// 64-bit per-lane addresses.
// Aggregates are moved as 1-4 dword vectors (a struct copy through such a
// pointer would be lowered to a generic-space copy); A is the alignment the
// address is known to have (the element size).
#define LBM_GLOBAL __attribute__((address_space(1)))
template <int N, int A> struct DWords;
#define LBM_DWORDS(A)                                                                                     \
    template <> struct DWords<1, A> { typedef unsigned __attribute__((aligned(A))) type; };               \
    template <> struct DWords<2, A> { typedef unsigned __attribute__((ext_vector_type(2), aligned(A))) type; }; \
    template <> struct DWords<3, A> { typedef unsigned __attribute__((ext_vector_type(3), aligned(A))) type; }; \
    template <> struct DWords<4, A> { typedef unsigned __attribute__((ext_vector_type(4), aligned(A))) type; };
LBM_DWORDS(2)
LBM_DWORDS(4)
LBM_DWORDS(8)
#undef LBM_DWORDS

template <class V, int A = alignof(V)> __device__ __forceinline__ V ld_g(const char* p)
{
    V r;
    if constexpr (sizeof(V) % 4 == 0) {
        constexpr int W = sizeof(V) / 4;
        unsigned w[W];
        static_for<0, (W + 3) / 4>([&](auto cc) {
            constexpr int k = 4 * decltype(cc)::value, n = W - k < 4 ? W - k : 4;
            using D = typename DWords<n, A>::type;
            const D d = *(const LBM_GLOBAL D*)(p + 4 * k);
            __builtin_memcpy(&w[k], &d, 4 * n);
        });
        __builtin_memcpy(&r, w, sizeof(V));
    } else {  // e.g. three FP16 values: element by element
        static_assert(sizeof(V) % sizeof(unsigned short) == 0, "2-byte elements");
        unsigned short h[sizeof(V) / 2];
#pragma unroll
        for (int k = 0; k < (int)(sizeof(V) / 2); ++k) h[k] = *(const LBM_GLOBAL unsigned short*)(p + 2 * k);
        __builtin_memcpy(&r, h, sizeof(V));
    }
    return r;
}

// Non-temporal (streaming) store of a whole aggregate as dword vectors, one
// store instruction per vector.
template <class V, int A = alignof(V)> __device__ __forceinline__ void st_g_nt(char* p, const V& v)
{
    static_assert(sizeof(V) % 4 == 0, "whole dwords");
    constexpr int W = sizeof(V) / 4;
    unsigned w[W];
    __builtin_memcpy(w, &v, sizeof(V));
    static_for<0, (W + 3) / 4>([&](auto cc) {
        constexpr int k = 4 * decltype(cc)::value, n = W - k < 4 ? W - k : 4;
        using D = typename DWords<n, A>::type;
        D d;
        __builtin_memcpy(&d, &w[k], 4 * n);
        __builtin_nontemporal_store(d, (LBM_GLOBAL D*)(p + 4 * k));
    });
}

template <class V, int A = alignof(V)> __device__ __forceinline__ void st_g(char* p, const V& v)
{
    if constexpr (sizeof(V) % 4 == 0) {
        constexpr int W = sizeof(V) / 4;
        unsigned w[W];
        __builtin_memcpy(w, &v, sizeof(V));
        static_for<0, (W + 3) / 4>([&](auto cc) {
            constexpr int k = 4 * decltype(cc)::value, n = W - k < 4 ? W - k : 4;
            using D = typename DWords<n, A>::type;
            D d;
            __builtin_memcpy(&d, &w[k], 4 * n);
            *(LBM_GLOBAL D*)(p + 4 * k) = d;
        });
    } else {
        unsigned short h[sizeof(V) / 2];
        __builtin_memcpy(h, &v, sizeof(V));
#pragma unroll
        for (int k = 0; k < (int)(sizeof(V) / 2); ++k) *(LBM_GLOBAL unsigned short*)(p + 2 * k) = h[k];
    }
}

// A: the alignment of the address (the storage element size, at most 4).
template <class T, int VX, int A> __device__ __forceinline__ Pack<T, VX> ld_vec(const char* base, unsigned byte_off)
{
    return ld_g<Pack<T, VX>, A>(base + (size_t)byte_off);
}

// Fused multiply-add in the compute precision (the only FMAs the build emits).
__device__ __forceinline__ float fmac(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmac(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <class C> __device__ __forceinline__ C recip(C r) { return C(1) / r; }
template <> __device__ __forceinline__ float recip<float>(float r) { return __builtin_amdgcn_rcpf(r); }

// Registers hold the populations of two rows. FP32/FP64 storage is kept
// as d_i = f_i - w_i in compute precision; FP16 storage is kept raw (half
// the registers) and converted where it is used.
template <class T, class C> using KeepT = typename std::conditional<(sizeof(T) < sizeof(C)), T, C>::type;

template <class T, bool SHIFT, class C>
__device__ __forceinline__ KeepT<T, C> keep_of(T v, int i, const Centre<C>& cn)
{
    if constexpr (sizeof(T) < sizeof(C)) return v;
    else return to_d<T, SHIFT, C>(v, i, cn);
}
template <class T, bool SHIFT, class C> __device__ __forceinline__ C d_of(KeepT<T, C> v, int i, const Centre<C>& cn)
{
    if constexpr (sizeof(T) < sizeof(C)) return to_d<T, SHIFT, C>(v, i, cn);
    else return v;
}

// Window gather: for the VX sites at columns x .. x+VX-1 of row r, load
// per plane i the stored values S_i(c - e_ix, r - e_iy) for the VX + 2
// columns c = x-1 .. x+VX, i.e. f_i of those columns (Eq. 5, left-hand
// side). Links (Sec. 2): e_0 (0,0); e_1 (1,0); e_2 (0,1); e_3 (-1,0);
// e_4 (0,-1); e_5 (1,1); e_6 (-1,1); e_7 (-1,-1); e_8 (1,-1).
// pb[i] points at column -2 of row 0 of plane i; the byte offset of column
// x - 1 - e_ix in row q is (q * rs + x + 1 - e_ix) * sizeof(T) >= 0.
// Near the lattice's left and right edges the windows reach source columns
// -2 .. -1 and nx .. nx+1: ghost copies for FP16 storage, else padding whose
// elements are then taken from the periodic image (Sec. 4: periodic in x;
// see GhostCols).
template <class LT> __device__ __forceinline__ void set_elem(LT* w, int j, LT v) { w[j] = v; }

// FP16 windows loaded as packed words: element j is half j & 1 of word j / 2.
__device__ __forceinline__ void set_elem_h(unsigned* w, int j, unsigned short v)
{
    const int q = j >> 1;
    w[q] = (j & 1) ? ((w[q] & 0xffffu) | ((unsigned)v << 16)) : ((w[q] & 0xffff0000u) | (unsigned)v);
}

// Every element whose source column lies outside [0, nx) is re-loaded from
// its periodic image by the lanes concerned (a few per edge wave). Which
// elements can wrap is fixed at compile time: on the left edge those with
// d = j - 1 - e_ix <= -1, on the right edge those with d >= 1.
template <class T, int NV, class LT, int NL>
__device__ __forceinline__ void patch_edges(const char* const (&rb)[9], const Geom& g, int x, Pack<LT, NL> (&v)[9])
{
    constexpr int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    constexpr unsigned es = sizeof(T);
#pragma unroll
    for (int i = 0; i < 9; ++i)
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            const int d = j - 1 - ex[i];  // source column s = x + d
            int sw = -1;
            if (d <= -1 && x + d < 0) sw = x + d + g.nx;                     // left edge: from nx + s
            if (d >= 1 && x + d >= g.nx) sw = min(x + d - g.nx, g.nx - 1);  // right edge: from s - nx
            if ((d <= -1 || d >= 1) && sw >= 0) {
                const char* a = rb[i] + (size_t)((unsigned)(sw + 2) * es);
                if constexpr (sizeof(LT) == sizeof(T)) set_elem<LT>(v[i].v, j, ld_g<T>(a));
                else set_elem_h(v[i].v, j, ld_g<unsigned short>(a));
            }
        }
}

// Source row bases of the nine planes for row r (uniform over the wave in
// every caller: the row offsets are scalar and are added to the scalar plane
// bases, leaving one per-lane 32-bit column offset).
template <class T>
__device__ __forceinline__ void row_bases(const char* const (&pb)[9], const Geom& g, int r, const char* (&rb)[9])
{
    constexpr unsigned es = sizeof(T);
    const size_t rs = (size_t)g.rs * es;
    const size_t om = (size_t)wrapy(r - 1, g.ny) * rs;  // source row r - 1 (e_iy = +1)
    const size_t o0 = (size_t)wrapy(r, g.ny) * rs;      // source row r     (e_iy =  0)
    const size_t op = (size_t)wrapy(r + 1, g.ny) * rs;  // source row r + 1 (e_iy = -1)
    const char* const b[9] = {pb[0] + o0, pb[1] + o0, pb[2] + om, pb[3] + o0, pb[4] + op,
                              pb[5] + om, pb[6] + om, pb[7] + op, pb[8] + op};
#pragma unroll
    for (int i = 0; i < 9; ++i) rb[i] = b[i];
}

// The nine window loads of the lane at column x (the +-1 column shifts are
// immediates).
template <class T, int NV, class LT, int NL>
__device__ __forceinline__ void window_loads(const char* const (&rb)[9], int x, Pack<LT, NL> (&v)[9])
{
    constexpr unsigned es = sizeof(T);
    const unsigned xm = (unsigned)x * es, x0 = xm + es, xp = xm + 2 * es;  // window starts for e_ix = +1, 0, -1
    constexpr int A = es < 4 ? (int)es : 4;
    v[0] = ld_vec<LT, NL, A>(rb[0], x0);
    v[1] = ld_vec<LT, NL, A>(rb[1], xm);
    v[2] = ld_vec<LT, NL, A>(rb[2], x0);
    v[3] = ld_vec<LT, NL, A>(rb[3], xp);
    v[4] = ld_vec<LT, NL, A>(rb[4], x0);
    v[5] = ld_vec<LT, NL, A>(rb[5], xm);
    v[6] = ld_vec<LT, NL, A>(rb[6], xp);
    v[7] = ld_vec<LT, NL, A>(rb[7], xp);
    v[8] = ld_vec<LT, NL, A>(rb[8], xm);
}

// LT / NL: the register type and count the windows are loaded as (the FP16
// kernels load their windows as packed 32-bit words, NL = ceil(NV / 2)).
// EDGE = false: the caller knows that no lane of the wave is within reach
// of a lattice edge (x >= 2 and x + NV <= nx), and no patch code is emitted.
template <class T, int NV, class LT = T, int NL = NV, bool EDGE = !GhostCols<T>::value>
__device__ __forceinline__ void gather_raw(const char* const (&pb)[9], const Geom& g, int r, int x, Pack<LT, NL> (&v)[9])
{
    const char* rb[9];
    row_bases<T>(pb, g, r, rb);
    window_loads<T, NV, LT, NL>(rb, x, v);
    if constexpr (EDGE) {
        static_assert(!GhostCols<T>::value, "ghost columns make the patch unnecessary");
        if (x < 2 || x + NV > g.nx) patch_edges<T, NV, LT, NL>(rb, g, x, v);
    }
}

// As gather_raw, with the edge patch chosen at run time (`edge`, uniform over
// the workgroup): the window loads are one code path for every tile, and an
// edge strip adds the patch loads, which write the wrapped elements into the
// same registers.
template <class T, int NV, class LT = T, int NL = NV>
__device__ __forceinline__ void gather_raw_rt(const char* const (&pb)[9], const Geom& g, int r, int x, bool edge,
                                              Pack<LT, NL> (&v)[9])
{
    const char* rb[9];
    row_bases<T>(pb, g, r, rb);
    window_loads<T, NV, LT, NL>(rb, x, v);
    if constexpr (!GhostCols<T>::value) {
        if (edge)
            if (x < 2 || x + NV > g.nx) patch_edges<T, NV, LT, NL>(rb, g, x, v);
    }
}

// A column of nine populations d_i (one site) as seen by the arithmetic
// below. ColF holds them in compute precision; ColH (FP16 storage) reads
// them from packed halves with mixed-precision FMAs, which convert an FP16
// operand exactly, so both give the same bits. Operations: add(a, b) =
// d_a + d_b, sub(a, b) = d_a - d_b, plus(a, s) = s + d_a, fma(m, a, c) =
// m d_a + c, each rounded once.
template <class C> struct ColF {
    C d[9];
    __device__ __forceinline__ C add(int a, int b) const { return d[a] + d[b]; }
    __device__ __forceinline__ C sub(int a, int b) const { return d[a] - d[b]; }
    __device__ __forceinline__ C plus(int a, C s) const { return s + d[a]; }
    __device__ __forceinline__ C fma(C m, int a, C c) const { return fmac(m, d[a], c); }
};

template <class T, bool SHIFT, class C, int VX>
__device__ __forceinline__ ColF<C> col_of(const KeepT<T, C> d[9][VX], int j, const Centre<C>& cn)
{
    ColF<C> v;
#pragma unroll
    for (int i = 0; i < 9; ++i) v.d[i] = d_of<T, SHIFT, C>(d[i][j], i, cn);
    return v;
}

// delta rho = sum_i d_i (Eq. 3), one fixed order for every code path.
template <class V> __device__ __forceinline__ auto drho_col(const V& v)
{
    return v.plus(8, (v.add(0, 1) + v.add(2, 3)) + (v.add(4, 5) + v.add(6, 7)));
}

template <class T, bool SHIFT, class C, int VX>
__device__ __forceinline__ C drho_of(const KeepT<T, C> d[9][VX], int j, const Centre<C>& cn)
{
    return drho_col(col_of<T, SHIFT, C, VX>(d, j, cn));
}

template <class C> struct CoefC {
    C om1, wo0, wo1, wo2, as1, as2, e1, e0;
};

template <class C> __device__ __forceinline__ CoefC<C> coef_c(const Coef& k)
{
    if constexpr (sizeof(C) == sizeof(float))
        return CoefC<C>{k.om1f, k.wo0f, k.wo1f, k.wo2f, k.as1f, k.as2f, k.e1f, k.e0f};
    else return CoefC<C>{k.om1, k.wo0, k.wo1, k.wo2, k.as1, k.as2, k.e1, k.e0};
}

// The centre in compute precision (see Centre): w_i (1 + e) for FP32, which
// is w_i itself for the paper's model (e = 0); w_i for FP64.
// Only the model's shifts are read, so the centre is all a tile holds of
// the coefficients while its loads are in flight.
template <class C, bool RC = ModelCentred<C>::value> __device__ __forceinline__ Centre<C> centre_c(const Coef& c)
{
    if constexpr (RC) {
        const CoefC<C> k = coef_c<C>(c);
        return Centre<C>{wt<C>(0) * (C(1) + k.e0), wt<C>(1) * (C(1) + k.e1), wt<C>(5) * (C(1) + k.e1)};
    } else {
        return Centre<C>{wt<C>(0), wt<C>(1), wt<C>(5)};
    }
}

// Eq. 5 right-hand side in delta form for one site.
//   rho = 1 + drho, u = j / rho (Eq. 3)
//   feq_i - w_i = w_i [drho + rho (3 e.u + 9/2 (e.u)^2 - 3/2 u.u)]      (Eq. 2)
//   d*_i = d_i - (d_i - (feq_i - w_i))/tau + 3 w_i alpha (e_i . G)      (Eq. 5)
// G is the central-difference gradient (Sec. 4); the caller passes D = 2 G
// (the undivided differences rho(x+1) - rho(x-1), rho(y+1) - rho(y-1)) and
// k.as = 3 w alpha / 2, which gives the same products exactly.
// For a link pair (i, opp) with e_opp = -e_i, write A = drho - 3/2 rho u.u,
// sym = A + 9/2 rho (e.u)^2, P = om w sym, Q = om w 3 rho (e.u) + as (e.D):
//   d*_i = (1 - om) d_i + P + Q,  d*_opp = (1 - om) d_opp + P - Q.
// The altered-equilibrium model (as = 0): its feq_i - w_i is
// w_i [drho + rho e + rho (3 e.u + 9/2 (e.u)^2 - 3/2 u.u)], so sym uses
// A + rho e1 and the rest population A + rho e0 (Coef); centred on its own
// state at rest (FP32, see Centre) the shift is drho e instead of rho e.
template <bool RC, class V, class C>
__device__ __forceinline__ void collide_col(const V& v, C drho, C gx, C gy, const CoefC<C>& k, C o[9])
{
    const C jx = (v.sub(1, 3) + v.sub(5, 6)) + v.sub(8, 7);
    const C jy = (v.sub(2, 4) + v.sub(5, 8)) + v.sub(6, 7);
    const C rho = C(1) + drho;
    const C ir = recip<C>(rho);
    const C ux = jx * ir, uy = jy * ir;
    const C usq = fmac(ux, ux, uy * uy);
    const C A = fmac(C(-1.5) * rho, usq, drho);
    // equilibrium shifts of the altered-equilibrium model (exactly A when
    // e1 = e0 = 0, the paper's model)
    const C es = RC ? drho : rho;
    const C Ap = fmac(es, k.e1, A), A0 = fmac(es, k.e0, A);
    const C r45 = C(4.5) * rho, r3 = C(3) * rho;
    o[0] = v.fma(k.om1, 0, k.wo0 * A0);
    auto pair = [&](int i, int io, C eu, C eg, C wo, C as) {
        const C P = wo * fmac(r45, eu * eu, Ap);
        const C Q = fmac(as, eg, wo * (r3 * eu));
        o[i] = v.fma(k.om1, i, P + Q);
        o[io] = v.fma(k.om1, io, P - Q);
    };
    pair(1, 3, ux, gx, k.wo1, k.as1);
    pair(2, 4, uy, gy, k.wo1, k.as1);
    pair(5, 7, ux + uy, gx + gy, k.wo2, k.as2);
    pair(6, 8, uy - ux, gy - gx, k.wo2, k.as2);
}

template <class T, bool SHIFT, class C, int VX, bool RC = ModelCentred<C>::value>
__device__ __forceinline__ void collide(const KeepT<T, C> dk[9][VX], int j, C drho, C gx, C gy, const CoefC<C>& k,
                                        const Centre<C>& cn, C o[9])
{
    collide_col<RC>(col_of<T, SHIFT, C, VX>(dk, j, cn), drho, gx, gy, k, o);
}

// ---------------------------------------------------------------------------
// FP16 storage (shifted form): the nine populations of a window column sit
// in the same half (H) of nine packed registers; v_fma_mix_f32 reads that
// half as an FP16 operand (exactly converted) next to FP32 operands, so the
// FP32 arithmetic needs no separate conversion instructions.
template <int H> struct ColH {
    unsigned w[9];
    __device__ __forceinline__ float add(int a, int b) const
    {
        float r;
        if constexpr (H == 0) asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel_hi:[1,0,1]" : "=v"(r) : "v"(w[a]), "v"(w[b]));
        else asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[1,0,1] op_sel_hi:[1,0,1]" : "=v"(r) : "v"(w[a]), "v"(w[b]));
        return r;
    }
    __device__ __forceinline__ float sub(int a, int b) const
    {
        float r;
        if constexpr (H == 0)
            asm("v_fma_mix_f32 %0, %1, 1.0, -%2 op_sel_hi:[1,0,1]" : "=v"(r) : "v"(w[a]), "v"(w[b]));
        else
            asm("v_fma_mix_f32 %0, %1, 1.0, -%2 op_sel:[1,0,1] op_sel_hi:[1,0,1]" : "=v"(r) : "v"(w[a]), "v"(w[b]));
        return r;
    }
    __device__ __forceinline__ float plus(int a, float s) const
    {
        float r;
        if constexpr (H == 0) asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(r) : "v"(w[a]), "v"(s));
        else asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(w[a]), "v"(s));
        return r;
    }
    __device__ __forceinline__ float fma(float m, int a, float c) const
    {
        float r;
        if constexpr (H == 0) asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel_hi:[0,1,0]" : "=v"(r) : "v"(m), "v"(w[a]), "v"(c));
        else asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel:[0,1,0] op_sel_hi:[0,1,0]" : "=v"(r) : "v"(m), "v"(w[a]), "v"(c));
        return r;
    }
};

// Window column J of nine FP16 windows held as packed words.
template <int J, int NWD> __device__ __forceinline__ ColH<J & 1> col_h(const unsigned (&u)[9][NWD])
{
    ColH<J & 1> v;
#pragma unroll
    for (int i = 0; i < 9; ++i) v.w[i] = u[i][J >> 1];
    return v;
}

// Two FP32 values rounded to FP16 (round to nearest even), packed low/high.
__device__ __forceinline__ unsigned pack_h2(float lo, float hi)
{
    typedef float f2 __attribute__((ext_vector_type(2)));
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    f2 v = {lo, hi};
    asm("" : "+v"(v));  // keep the conversion separate from the FMAs that produced v
    const h2 r = __builtin_convertvector(v, h2);
    unsigned u;
    __builtin_memcpy(&u, &r, sizeof(u));
    return u;
}


// Write row y of the lattice: VX relaxed sites per lane (nv of them valid)
// and, with ghost columns (GhostCols), the copies of the edge columns (-2, -1
// hold nx-2, nx-1; nx, nx+1 hold 0, 1; for nx = 3 column 1 has two ghosts).
template <class T, int VX, bool NTS>
__device__ __forceinline__ void write_row(char* const (&dbase)[9], const Geom& g, int y, int x, int nv,
                                          const Pack<T, VX> (&out)[9])
{
    constexpr unsigned es = sizeof(T);
    const size_t ro = (size_t)y * ((size_t)g.rs * es);  // row y, column 0 (uniform: added to the scalar bases)
    const unsigned lo = (unsigned)x * es;
    if (nv == VX) {
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            char* rb = dbase[i] + ro;
            if constexpr (NTS) {
                // One non-temporal vector store per plane. Which source form
                // gets that from the compiler was found by reading the
                // generated code: element-wise through a generic pointer for
                // FP32 (a dword-vector store lost its non-temporal bit), a
                // dword-vector store for FP64 and FP16 (element-wise ones were
                // split into partial stores).
                if constexpr (sizeof(T) == 4 || sizeof(out[i]) % 4 != 0) {
#pragma unroll
                    for (int j = 0; j < VX; ++j)
                        __builtin_nontemporal_store(out[i].v[j], (T*)(rb + (size_t)(lo + j * es)));
                } else {
                    st_g_nt<Pack<T, VX>, (sizeof(out[i]) < 8 ? (int)sizeof(out[i]) : 8)>(rb + (size_t)lo, out[i]);
                }
            } else {
                st_g<Pack<T, VX>>(rb + (size_t)lo, out[i]);
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i)
#pragma unroll
            for (int j = 0; j < VX; ++j)
                if (j < nv) st_g<T>(dbase[i] + ro + (size_t)(lo + j * es), out[i].v[j]);
    }
    if constexpr (GhostCols<T>::value) {
#pragma unroll
        for (int j = 0; j < VX; ++j) {
            const int c = x + j;
            if (j < nv && c >= g.nx - 2) {
#pragma unroll
                for (int i = 0; i < 9; ++i)  // column c - nx in [-2, -1]
                    st_g<T>(dbase[i] + ro - 2 * es + (size_t)((unsigned)(c - g.nx + 2) * es), out[i].v[j]);
            }
            if (j < nv && c <= 1) {
#pragma unroll
                for (int i = 0; i < 9; ++i)  // column c + nx in [nx, nx + 1]
                    st_g<T>(dbase[i] + ro + (size_t)((unsigned)(c + g.nx) * es), out[i].v[j]);
            }
        }
    }
}

// Tile of workgroup b in a grid of nb workgroups. Consecutive workgroups are
// dispatched round-robin to the 8 XCDs (b & 7); j = b >> 3 counts one XCD's
// workgroups in dispatch order. With ch > 0 the tiles are dealt to the XCDs
// in chunks of ch consecutive tiles (about one row group each): the 8 XCDs
// work on 8 adjacent chunks at a time, so the rows being streamed form one
// compact band (DRAM page locality); the rows shared by adjacent chunks are
// re-read through the shared last-level cache. The grid is a multiple of
// 8 ch. With ch <= 0 each XCD takes one contiguous run of nb / 8 tiles.
__device__ __forceinline__ int xcd_tile(int b, int nb, int ch)
{
    if (ch <= 0) return (b & 7) * (nb >> 3) + (b >> 3);
    const int j = b >> 3;
    return (j / ch) * (8 * ch) + (b & 7) * ch + (j % ch);
}

// Per-plane base pointers: source at column -2, destination at column 0.
template <class T>
__device__ __forceinline__ void plane_bases(const void* src, void* dst, const Geom& g, const char* (&sb)[9],
                                            char* (&dbase)[9])
{
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        sb[i] = (const char*)src + ((long long)i * g.ps + g.off - 2) * (long long)sizeof(T);
        dbase[i] = (char*)dst + ((long long)i * g.ps + g.off) * (long long)sizeof(T);
    }
}

// The per-site source coefficients (a c2 field) of the VX columns a lane
// owns in row y (a row of the field array, see StepTile).
template <class C, int VX>
__device__ __forceinline__ Pack<C, VX> field_row(const StepTile& a, int y, int x)
{
    const char* row = (const char*)a.field + (size_t)y * a.fpitch * sizeof(C);
    return ld_vec<C, VX, 4>(row, (unsigned)x * (unsigned)sizeof(C));
}

// Coefficients of one site: the uniform ones, or with the source
// coefficients of the site (as2 = as1 / 4 exactly).
template <bool FIELD, class C> __device__ __forceinline__ CoefC<C> site_coef(const CoefC<C>& k, C as1)
{
    if constexpr (!FIELD) return k;
    CoefC<C> s = k;
    s.as1 = as1;
    s.as2 = C(0.25) * as1;
    return s;
}

// ---------------------------------------------------------------------------
// Vertical-stack tiles. A tile is strip `strip` (64 * VX columns) and row
// group `grp` (R = NW - 2 rows) of one lattice, processed by a workgroup of
// NW waves: wave w handles row y0 - 1 + w, so waves 0 and R + 1 take the
// rows just outside the group, whose densities the gradient needs. A tile
// runs in three phases:
//   issue: every wave issues the window loads of its row (no wait);
//   land:  the loads are consumed: populations and window densities are
//          kept in registers and the wave's own columns' densities are
//          published in LDS;
//   relax: after a workgroup barrier, the interior waves read the densities
//          of the rows above and below from LDS, relax (Eq. 5) and write.
// vstack_tile runs them in order; the persistent batched kernel overlaps
// the issue phase of the next tile with the relax phase of the current one.
// The arithmetic, and its order, is the same code either way.

// This wave's row of a tile.
struct VRow {
    int wave, lane;
    int y, x, nv;  // lattice row (-1 .. ny: wraps by index), first column, columns held (<= VX)
    bool load;     // the lane loads a row (a halo or interior row, columns inside the lattice)
    bool relax;    // ... and relaxes and writes it (interior rows)
};

// `wave`: the tile row the wave takes (0: the halo row above the group).
template <int VX, int NW> __device__ __forceinline__ VRow vrow(const Geom& g, int strip, int grp, int wave)
{
    constexpr int R = NW - 2;
    VRow r;
    r.wave = wave;
    r.lane = threadIdx.x & 63;
    const int y0 = grp * R;
    const int nrows = min(R, g.ny - y0);
    r.y = y0 - 1 + r.wave;
    r.x = strip * (64 * VX) + r.lane * VX;
    r.nv = min(VX, g.nx - r.x);
    r.load = r.nv > 0 && r.wave <= nrows + 1;  // waves past the bottom halo idle
    r.relax = r.load && r.wave >= 1 && r.wave <= nrows;
    return r;
}
template <int VX, int NW> __device__ __forceinline__ VRow vrow(const Geom& g, int strip, int grp)
{
    return vrow<VX, NW>(g, strip, grp, __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)));
}

// Strips whose windows can reach past a lattice edge (the first, and those
// within two columns of the right edge) run the load-side periodic patch
// (see GhostCols); uniform over the workgroup.
template <class T, int VX> __device__ __forceinline__ bool edge_strip(const Geom& g, int strip)
{
    if constexpr (GhostCols<T>::value) return false;
    else return strip == 0 || (strip + 1) * (64 * VX) + 2 > g.nx;
}

template <class T> __device__ __forceinline__ void src_bases(const void* src, const Geom& g, const char* (&sb)[9])
{
#pragma unroll
    for (int i = 0; i < 9; ++i) sb[i] = (const char*)src + ((long long)i * g.ps + g.off - 2) * (long long)sizeof(T);
}
template <class T> __device__ __forceinline__ void dst_bases(void* dst, const Geom& g, char* (&dbase)[9])
{
#pragma unroll
    for (int i = 0; i < 9; ++i) dbase[i] = (char*)dst + ((long long)i * g.ps + g.off) * (long long)sizeof(T);
}

// Tile registers and phases for FP32 / FP64 storage. FIELD: the source
// coefficients come per site from a.field (a c2 field); the interior waves
// load them with their windows. RC: centre the arithmetic on the lattice
// model's state at rest (see Centre); the batched kernels (paper's model
// only) pass false.
template <class T, bool SHIFT, int VX, int NW, bool NTS, bool FIELD, bool RC> struct VTileF {
    using C = typename CompT<T>::type;
    using K = KeepT<T, C>;
    using Lds = C[NW][64 * VX];
    static constexpr int WV = VX + 2;
    Pack<T, WV> raw[9];  // window loads in flight
    Pack<C, VX> af;      // per-site source coefficients (FIELD)
    K d[9][VX];          // populations of the own columns
    C w[WV];             // densities of the window columns

    // issue_rows / land_rows: the phases for a lane with r.load set.
    template <bool EDGE> __device__ __forceinline__ void issue_rows(const StepTile& a, const void* src, const VRow& r)
    {
        const char* sb[9];
        src_bases<T>(src, a.g, sb);
        gather_raw<T, WV, T, WV, EDGE>(sb, a.g, r.y, r.x, raw);
        if constexpr (FIELD)
            if (r.relax) af = field_row<C, VX>(a, r.y, r.x);
    }

    // The loads consumed: populations of the own columns (d) and densities
    // of the window columns (w).
    __device__ __forceinline__ void land_regs(const StepTile& a)
    {
        const Centre<C> cn = centre_c<C, RC>(a.c);
        K tmp[9][WV];
#pragma unroll
        for (int i = 0; i < 9; ++i)
#pragma unroll
            for (int j = 0; j < WV; ++j) tmp[i][j] = keep_of<T, SHIFT, C>(raw[i].v[j], i, cn);
#pragma unroll
        for (int j = 0; j < WV; ++j) w[j] = drho_of<T, SHIFT, C, WV>(tmp, j, cn);
#pragma unroll
        for (int i = 0; i < 9; ++i)
#pragma unroll
            for (int j = 0; j < VX; ++j) d[i][j] = tmp[i][j + 1];
    }

    __device__ __forceinline__ void land_rows(const StepTile& a, const VRow& r, Lds& lds)
    {
        land_regs(a);
#pragma unroll
        for (int j = 0; j < VX; ++j) lds[r.wave][r.lane * VX + j] = w[j + 1];
    }

    template <bool EDGE> __device__ __forceinline__ void issue(const StepTile& a, const void* src, const VRow& r)
    {
        if (r.load) issue_rows<EDGE>(a, src, r);
    }
    // issue with the edge patch chosen at run time (see gather_raw_rt)
    __device__ __forceinline__ void issue_rt(const StepTile& a, const void* src, const VRow& r, bool edge)
    {
        if (r.load) {
            const char* sb[9];
            src_bases<T>(src, a.g, sb);
            gather_raw_rt<T, WV, T, WV>(sb, a.g, r.y, r.x, edge, raw);
            if constexpr (FIELD)
                if (r.relax) af = field_row<C, VX>(a, r.y, r.x);
        }
    }
    __device__ __forceinline__ void land(const StepTile& a, const VRow& r, Lds& lds)
    {
        if (r.load) land_rows(a, r, lds);
    }

    __device__ __forceinline__ void relax(const StepTile& a, void* dst, const VRow& r, const Lds& lds)
    {
        relax_g(a, dst, r, [&](int j) { return lds[r.wave + 1][r.lane * VX + j] - lds[r.wave - 1][r.lane * VX + j]; });
    }

    // relax with gy(j) the undivided y difference rho(y + 1) - rho(y - 1) at
    // the lane's column j
    template <class GY> __device__ __forceinline__ void relax_g(const StepTile& a, void* dst, const VRow& r, GY&& gyf)
    {
        if (r.relax) {
            char* dbase[9];
            dst_bases<T>(dst, a.g, dbase);
            const CoefC<C> k = coef_c<C>(a.c);
            const Centre<C> cn = centre_c<C, RC>(a.c);
            Pack<T, VX> out[9];
#pragma unroll
            for (int j = 0; j < VX; ++j) {
                // undivided central differences at time t (Sec. 4)
                const C gx = w[j + 2] - w[j];
                const C gy = gyf(j);
                C o[9];
                collide<T, SHIFT, C, VX, RC>(d, j, w[j + 1], gx, gy, site_coef<FIELD>(k, af.v[j]), cn, o);
#pragma unroll
                for (int i = 0; i < 9; ++i) out[i].v[j] = from_d<T, SHIFT, C>(o[i], i, cn);
            }
            write_row<T, VX, NTS>(dbase, a.g, r.y, r.x, r.nv, out);
        }
    }
};

// Tile registers and phases for FP16 storage (shifted form): the same tile,
// rows, summation orders and roundings, with the populations kept as the
// packed halves they were loaded as (see ColH) and the results rounded to
// FP16 two at a time.
template <class T, bool SHIFT, int VX, int NW, bool NTS, bool FIELD, bool RC> struct VTileH {
    static_assert(SHIFT, "FP16 storage is the shifted form");
    static_assert(GhostCols<T>::value, "FP16 rows carry ghost columns");
    using C = float;
    using Lds = C[NW][64 * VX];
    static constexpr int WV = VX + 2;
    static constexpr int NWD = (WV + 1) / 2;  // packed words per window
    Pack<unsigned, NWD> raw[9];
    Pack<float, VX> af;
    unsigned u[9][NWD];
    float w[WV];

    template <bool EDGE> __device__ __forceinline__ void issue_rows(const StepTile& a, const void* src, const VRow& r)
    {
        static_assert(!EDGE, "ghost columns make the patch unnecessary");
        // An odd-length window (VX = 1) loads one half past its end (at most
        // column nx + 2, row padding).
        const char* sb[9];
        src_bases<T>(src, a.g, sb);
        gather_raw<T, WV, unsigned, NWD, false>(sb, a.g, r.y, r.x, raw);
        if constexpr (FIELD)
            if (r.relax) af = field_row<float, VX>(a, r.y, r.x);
    }

    __device__ __forceinline__ void land_regs(const StepTile&)
    {
#pragma unroll
        for (int i = 0; i < 9; ++i)
#pragma unroll
            for (int q = 0; q < NWD; ++q) u[i][q] = raw[i].v[q];
        static_for<0, WV>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            w[j] = drho_col(col_h<j>(u));
        });
    }

    __device__ __forceinline__ void land_rows(const StepTile& a, const VRow& r, Lds& lds)
    {
        land_regs(a);
#pragma unroll
        for (int j = 0; j < VX; ++j) lds[r.wave][r.lane * VX + j] = w[j + 1];
    }

    template <bool EDGE> __device__ __forceinline__ void issue(const StepTile& a, const void* src, const VRow& r)
    {
        if (r.load) issue_rows<EDGE>(a, src, r);
    }
    __device__ __forceinline__ void issue_rt(const StepTile& a, const void* src, const VRow& r, bool)
    {
        if (r.load) issue_rows<false>(a, src, r);
    }
    __device__ __forceinline__ void land(const StepTile& a, const VRow& r, Lds& lds)
    {
        if (r.load) land_rows(a, r, lds);
    }

    __device__ __forceinline__ void relax(const StepTile& a, void* dst, const VRow& r, const Lds& lds)
    {
        relax_g(a, dst, r, [&](int j) { return lds[r.wave + 1][r.lane * VX + j] - lds[r.wave - 1][r.lane * VX + j]; });
    }

    template <class GY> __device__ __forceinline__ void relax_g(const StepTile& a, void* dst, const VRow& r, GY&& gyf)
    {
        if (r.relax) {
            char* dbase[9];
            dst_bases<T>(dst, a.g, dbase);
            const CoefC<float> k = coef_c<float>(a.c);
            float o[VX][9];
            static_for<0, VX>([&](auto jc) {
                constexpr int j = decltype(jc)::value;
                // undivided central differences at time t (Sec. 4)
                const float gx = w[j + 2] - w[j];
                const float gy = gyf(j);
                collide_col<RC>(col_h<j + 1>(u), w[j + 1], gx, gy, site_coef<FIELD>(k, af.v[j]), o[j]);
            });
            Pack<T, VX> out[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                if constexpr (VX == 1) {
                    float v = o[0][i];
                    asm("" : "+v"(v));
                    out[i].v[0] = (T)v;
                } else {
                    unsigned pk[VX / 2];
#pragma unroll
                    for (int j = 0; j < VX; j += 2) pk[j / 2] = pack_h2(o[j][i], o[j + 1][i]);
                    __builtin_memcpy(&out[i], pk, sizeof(out[i]));
                }
            }
            write_row<T, VX, NTS>(dbase, a.g, r.y, r.x, r.nv, out);
        }
    }
};

template <class T, bool SHIFT, int VX, int NW, bool NTS, bool FIELD, bool RC>
using VTile = typename std::conditional<std::is_same<T, _Float16>::value, VTileH<T, SHIFT, VX, NW, NTS, FIELD, RC>,
                                        VTileF<T, SHIFT, VX, NW, NTS, FIELD, RC>>::type;

// One vertical-stack tile, its three phases in order, with src/dst the
// buffers of this step. The caller must place a barrier between two calls
// that reuse `lds`. Edge strips take a separate copy of the whole tile
// code; the others issue their loads and start the arithmetic as the loads
// land, with no patch code in between.
template <class T, bool SHIFT, int VX, int NW, bool NTS, bool FIELD = false,
          bool RC = ModelCentred<typename CompT<T>::type>::value>
__device__ __forceinline__ void vstack_tile(const StepTile& a, const void* src, void* dst, int strip, int grp,
                                            typename CompT<T>::type (&lds)[NW][64 * VX])
{
    using V = VTile<T, SHIFT, VX, NW, NTS, FIELD, RC>;
    const VRow r = vrow<VX, NW>(a.g, strip, grp);
    auto run = [&](auto edge) {
        V v;
        v.af = {};
        if (r.load) {
            v.template issue_rows<decltype(edge)::value>(a, src, r);
            v.land_rows(a, r, lds);
        }
        __syncthreads();
        v.relax(a, dst, r, lds);
    };
    if constexpr (GhostCols<T>::value) run(std::false_type{});
    else if (edge_strip<T, VX>(a.g, strip)) run(std::true_type{});
    else run(std::false_type{});
}

}  // namespace lbm

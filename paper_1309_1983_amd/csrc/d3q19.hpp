// Device-side building blocks of the D3Q19 step for gfx950.
//
// Velocity set of Eq. (4) and weights stated after Eq. (5) (Mawson & Revell,
// Section 3.1), population storage codecs, periodic neighbour indexing for
// the pull gather of Algorithm 3, and the BGK collision (Eqs. (2)-(3), (5)-(7))
// with Guo forcing, evaluated in FP32 on offsets h_i = f_i - w_i.
//
// Compiled with -ffp-contract=off: every fused multiply-add is an explicit
// fmaf, so each kernel that inlines these functions performs bit-identical
// arithmetic (the AB and AA patterns must agree bit for bit).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace d3q19 {

constexpr int Q = 19;

// Eq. (4), i = 0..18.
constexpr int EX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1};
constexpr int EY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int EZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, 1, -1};
// e_OPP[i] = -e_i: the pairs (1,2), (3,4), ..., (17,18).
constexpr int OPP[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};

__host__ __device__ constexpr float weight(int i)
{
    return i == 0 ? 1.0f / 3.0f : (i <= 6 ? 1.0f / 18.0f : 1.0f / 36.0f);
}

// Flag byte: bits 0-1 cell type (0 fluid, 1 wall, 2 moving wall); bit 2 set on
// fluid cells with at least one solid neighbour (computed at creation).
constexpr uint8_t TYPE_MASK = 3;
constexpr uint8_t MOVING = 2;
constexpr uint8_t NEAR_WALL = 4;
// bit 3 set on fluid cells with at least one moving-wall neighbour.
constexpr uint8_t NEAR_MOVING = 8;
// bit 4: on-site velocity node, a fluid node lying on the wall whose velocity
// is prescribed (type bits 0); bit 5: that velocity is u_w, else zero.
constexpr uint8_t ONSITE_NODE = 16;
constexpr uint8_t ONSITE_MOVING = 32;

// ---------------------------------------------------------------------------
// Storage codecs. raw_t is what lives in HBM; off() decodes the offset
// f_i - w_i in FP32, enc() encodes an offset (round to nearest even), plain()
// decodes the plain population.
// ---------------------------------------------------------------------------
struct StF32 {
    using raw_t = float;
    using bits_t = float;   // element type of vector memory accesses
    static __device__ __forceinline__ float off_b(bits_t b, int i) { return b - weight(i); }
    static __device__ __forceinline__ bits_t enc_b(float h, int i) { return weight(i) + h; }
    static __device__ __forceinline__ float off(raw_t r, int i) { return r - weight(i); }
    static __device__ __forceinline__ raw_t enc(float h, int i) { return weight(i) + h; }
    static __device__ __forceinline__ float plain(raw_t r, int) { return r; }
    static __device__ __forceinline__ raw_t from_plain(float f, int) { return f; }
};

// The FP32 result itself is what gets rounded to a 16-bit format. Without
// this barrier the compiler may merge the last fma of the collision and the
// conversion into one mixed-precision fma (v_fma_mixlo_f16), which rounds the
// exact product-sum once instead of the FP32 value; it does so in some kernels
// and not in others, which would make kernels disagree in the last bit.
__device__ __forceinline__ float fp32_value(float v)
{
    asm("" : "+v"(v));
    return v;
}

struct StF16 {
    using raw_t = _Float16;
    using bits_t = uint16_t;
    static __device__ __forceinline__ float off_b(bits_t b, int) { return (float)__builtin_bit_cast(_Float16, b); }
    static __device__ __forceinline__ bits_t enc_b(float h, int) { return __builtin_bit_cast(uint16_t, (_Float16)fp32_value(h)); }
    static __device__ __forceinline__ float off(raw_t r, int) { return (float)r; }
    static __device__ __forceinline__ raw_t enc(float h, int) { return (_Float16)fp32_value(h); }
    static __device__ __forceinline__ float plain(raw_t r, int i) { return weight(i) + (float)r; }
    static __device__ __forceinline__ raw_t from_plain(float f, int i) { return (_Float16)(f - weight(i)); }
};

struct StBF16 {
    using raw_t = __bf16;
    using bits_t = uint16_t;
    static __device__ __forceinline__ float off_b(bits_t b, int) { return __uint_as_float((uint32_t)b << 16); }
    static __device__ __forceinline__ bits_t enc_b(float h, int) { return __builtin_bit_cast(uint16_t, (__bf16)fp32_value(h)); }
    static __device__ __forceinline__ float off(raw_t r, int) { return (float)r; }
    static __device__ __forceinline__ raw_t enc(float h, int) { return (__bf16)fp32_value(h); }
    static __device__ __forceinline__ float plain(raw_t r, int i) { return weight(i) + (float)r; }
    static __device__ __forceinline__ raw_t from_plain(float f, int i) { return (__bf16)(f - weight(i)); }
};

// VW consecutive elements as one memory access (element-aligned: gfx950
// global memory accepts 4-byte- and 2-byte-aligned vector accesses).
template <class B, int VW>
struct Vec {
    typedef B t __attribute__((ext_vector_type(VW), aligned(sizeof(B))));
};
template <class B>
using V4 = Vec<B, 4>;

// Element idx of an array base: the byte offset is formed in 32 bits (every
// plane is < 4 GiB), so accesses take the scalar-base + 32-bit vector-offset
// addressing form.
template <class T>
__device__ __forceinline__ T ld(const T* base, uint32_t idx)
{
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + idx * (uint32_t)sizeof(T));
}
template <class T>
__device__ __forceinline__ void st(T* base, uint32_t idx, T v)
{
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + idx * (uint32_t)sizeof(T)) = v;
}
template <int VW, class B>
__device__ __forceinline__ typename Vec<B, VW>::t ldv(const B* base, uint32_t idx)
{
    return *reinterpret_cast<const typename Vec<B, VW>::t*>(reinterpret_cast<const char*>(base) + idx * (uint32_t)sizeof(B));
}
template <int VW, class B>
__device__ __forceinline__ void stv(B* base, uint32_t idx, typename Vec<B, VW>::t v)
{
    *reinterpret_cast<typename Vec<B, VW>::t*>(reinterpret_cast<char*>(base) + idx * (uint32_t)sizeof(B)) = v;
}
// Raw buffer resource over a wave-uniform base address, reaching 4 GiB - 1
// bytes past it (stride 0; the data-format word of gfx9 raw buffers).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const void* base)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, -1, 0x00020000);
}

// Streaming vector store, for whole-wave store streams that the same launch
// does not read back: the populations a step writes, its macroscopic output
// and the adjoint's outputs. Both forms carry the non-temporal hint. FP32
// data goes through a raw buffer store (plane base in the resource, 32-bit
// offset): on MI355X the 256^3 FP32 step ran 0.9% faster than with the
// global store. 16-bit data keeps the global store: the eight-point 16-bit
// step sits at the 168-VGPR edge of three waves per SIMD, and the buffer
// form pushed it over (11% slower at 256^3). A device-scope bit (sc1, write
// through the L2) measured +0.3% on the 256^3 step and slower on arrays the
// memory-side cache partly holds, so it is not used. `base` must be
// wave-uniform (a plane or array base); idx * sizeof(B) < 4 GiB.
template <int VW, class B>
__device__ __forceinline__ void stv_nt(B* base, uint32_t idx, typename Vec<B, VW>::t v)
{
    typedef uint32_t u2 __attribute__((ext_vector_type(2)));
    typedef uint32_t u4 __attribute__((ext_vector_type(4)));
    constexpr int BYTES = VW * (int)sizeof(B);
    constexpr int NT = 2;   // cache-policy bit of buffer accesses: non-temporal
    if constexpr (sizeof(B) == 4) {
        const __amdgpu_buffer_rsrc_t r = buffer_of(base);
        const uint32_t off = idx * (uint32_t)sizeof(B);
        if constexpr (BYTES == 32) {
            struct P2 { u4 lo, hi; };
            const P2 p = __builtin_bit_cast(P2, v);
            __builtin_amdgcn_raw_buffer_store_b128(p.lo, r, off, 0, NT);
            __builtin_amdgcn_raw_buffer_store_b128(p.hi, r, off + 16u, 0, NT);
        } else if constexpr (BYTES == 16) {
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, v), r, off, 0, NT);
        } else if constexpr (BYTES == 8) {
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, off, 0, NT);
        } else {
            static_assert(BYTES == 4, "vector store of 4, 8, 16 or 32 bytes");
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, NT);
        }
    } else {
        __builtin_nontemporal_store(v, reinterpret_cast<typename Vec<B, VW>::t*>(reinterpret_cast<char*>(base) +
                                                                                  idx * (uint32_t)sizeof(B)));
    }
}

template <class B>
__device__ __forceinline__ typename V4<B>::t ld4(const B* base, uint32_t idx) { return ldv<4>(base, idx); }

struct Dims {
    int nx, ny, nz;
    uint32_t nxy;   // nx*ny
    uint32_t N;     // nx*ny*nz (< 2^30)
};

// Population storage: the values of direction i in z-slab z form one plane of
// nx*ny elements, f[(z*Q + i)*nxy + y*nx + x]. All work-items of a work-group
// share z, so plane bases are scalar; in-slab offsets are 32-bit.
template <class T>
__device__ __forceinline__ T* plane(T* f, const Dims& d, int i, uint32_t z)
{
    return f + ((size_t)z * Q + (size_t)i) * d.nxy;
}

// Slab of the pull source x - e_i given the wrapped z-1 (zm) and z+1 (zp).
__device__ __forceinline__ uint32_t src_slab(int i, uint32_t z, uint32_t zm, uint32_t zp)
{
    return EZ[i] == 1 ? zm : (EZ[i] == -1 ? zp : z);
}

// In-slab offsets (y'*nx + x') of the pull sources x - e_i, periodic in x, y.
// Offsets are added modulo 2^32 (negative offsets wrap back into range).
__device__ __forceinline__ void pull_offsets(const Dims& d, int x, int y, uint32_t o[Q])
{
    const uint32_t oc = (uint32_t)y * (uint32_t)d.nx + (uint32_t)x;
    const uint32_t oxm = (x == 0) ? (uint32_t)(d.nx - 1) : 0xffffffffu;              // to x-1
    const uint32_t oxp = (x == d.nx - 1) ? (uint32_t)(1 - d.nx) : 1u;                // to x+1
    const uint32_t oym = (y == 0) ? (uint32_t)(d.ny - 1) * d.nx : (uint32_t)(-d.nx); // to y-1
    const uint32_t oyp = (y == d.ny - 1) ? (uint32_t)(1 - d.ny) * d.nx : (uint32_t)d.nx;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        uint32_t s = oc;
        // pull from x - e_i: e = +1 reads the minus neighbour
        if (EX[i] == 1) s += oxm; else if (EX[i] == -1) s += oxp;
        if (EY[i] == 1) s += oym; else if (EY[i] == -1) s += oyp;
        o[i] = s;
    }
}

__device__ __forceinline__ uint32_t wrap_m(uint32_t v, uint32_t n) { return v == 0 ? n - 1 : v - 1; }
__device__ __forceinline__ uint32_t wrap_p(uint32_t v, uint32_t n) { return v == n - 1 ? 0 : v + 1; }

// VW consecutive 32-bit words at base[idx] (idx a multiple of min(VW, 4)).
template <int VW>
__device__ __forceinline__ void load_words(const uint32_t* __restrict__ base, uint32_t idx, uint32_t w[VW])
{
    constexpr int G = VW < 4 ? VW : 4;
#pragma unroll
    for (int g = 0; g < VW / G; ++g) {
        const typename Vec<uint32_t, G>::t v = ldv<G>(base, idx + G * g);
#pragma unroll
        for (int k = 0; k < G; ++k) w[G * g + k] = v[k];
    }
}

// ---------------------------------------------------------------------------
// Vector gather of VW consecutive x-points (x0 .. x0+VW-1, nx % VW == 0) of
// one row, for all 19 directions: q[i][j] = value of direction i at
// x_j - SIGN*e_i (SIGN = +1: the pull of Algorithm 3; SIGN = -1: the
// transposed gather x_j + e_i of the adjoint), periodic in x, y and z. When
// that neighbour is solid the bounced value, direction opp(i) at x_j itself,
// is taken instead (smask bit b set on point x when x - e_b is solid).
// Directions with e_x != 0 are single accesses shifted by one element; the
// row ends are clamped into the row and the wrapped element is loaded on its
// own, only when the end point needs it (end0/endL: first/last point fluid).
// Bounced values: a work-item with near-wall points loads its neighbour mask
// before the gather's loads, then, after them, one plane per opposite pair
// that the mask names, all without waiting in between (opposite directions
// sit in adjacent planes, so one load with a per-work-item plane choice
// serves either bounced value of a pair). With 16-bit storage and more than
// four near-wall work-items in the wave (porous geometry) it loads all 18 of
// its own planes at once instead, each load coalesced over the wave. Measured
// on MI355X against loading all 18 planes whenever more than two work-items
// are near a wall: FP32 cavity +0.3%, sphere duct +1.8%, 128-wide duct +2.9%,
// adjoint +6%; 16-bit cavity +3-5%, duct +7%, sphere duct -1 to -3%. The
// choice is wave-uniform; every work-item of the wave calls this function.
//
// EARLY (porous geometry, FP32 storage): the 19 gather loads are issued
// before anything that depends on the point flags, whose load the caller
// issued just before, together with the neighbour masks of every work-item
// (`early_mask`); end0, endL and near_wall are only consumed after the gather
// loads are in flight, so the flag load's latency overlaps them instead of
// preceding them. Measured on MI355X, FP32 sphere duct 128x128x256 (10%
// solid, 10% of the fluid points next to a solid): 126.7 -> 114.1 us per step.
// On the 256^3 cavity (2% near-wall points) the unconditional mask loads cost
// more than the overlap gains, so the caller enables it by geometry.
// ---------------------------------------------------------------------------
template <int SIGN, int VW, bool EARLY = false, bool DROP_PRIO = false, class B>
__device__ __forceinline__ void gather_vec(const B* __restrict__ src, const Dims& d, uint32_t z,
                                           uint32_t zm, uint32_t zp, uint32_t orow, uint32_t oym,
                                           uint32_t oyp, uint32_t x0, bool end0, bool endL,
                                           bool near_wall, const uint32_t* __restrict__ smask,
                                           uint32_t c0, typename Vec<B, VW>::t q[Q],
                                           const uint32_t* early_mask = nullptr)
{
    static_assert(!EARLY || sizeof(B) == 4, "the early-gather form is FP32 only");
    using Vt = typename Vec<B, VW>::t;
    const uint32_t nx = (uint32_t)d.nx;
    const uint32_t o0 = orow + x0;
    const bool wl = x0 == 0;
    const bool wr = x0 + VW == nx;
    const uint32_t xm = wl ? x0 : x0 - 1;   // group start when reading x - 1
    const uint32_t xp = wr ? x0 : x0 + 1;   // group start when reading x + 1
    bool all_planes = false;
    uint32_t smw[VW];   // neighbour mask, loaded first unless all planes are loaded
#pragma unroll
    for (int j = 0; j < VW; ++j) smw[j] = 0u;
    // 16-bit storage, four points per work-item: the all-planes form loads
    // only the planes some work-item of the wave bounces from, by the wave's
    // OR of the neighbour masks, which are then loaded before the gather
    constexpr bool WAVE_OR = sizeof(B) == 2 && VW == 4;
    if constexpr (!EARLY) {
        // wave-wide count of work-items with near-wall points
        const int nw_lanes = __builtin_popcountll(__builtin_amdgcn_ballot_w64(near_wall));
        all_planes = sizeof(B) == 2 && nw_lanes > 4;
        if (near_wall && (!all_planes || WAVE_OR)) load_words<VW>(smask, c0, smw);
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int ex = SIGN * EX[i], ey = SIGN * EY[i];
        const int iz = SIGN > 0 ? i : OPP[i];   // slab of x - SIGN*e_i
        uint32_t r = orow;
        if (ey == 1) r += oym; else if (ey == -1) r += oyp;
        const uint32_t xs = ex == 1 ? xm : (ex == -1 ? xp : x0);
        const B* P = plane(src, d, i, src_slab(iz, z, zm, zp));
        // FP32: the aligned directions (e_x = 0) load with the non-temporal
        // hint; no other work-item touches their lines. Measured on MI355X:
        // cavity 256^3 +2.5%, sphere duct +3%, 128-wide duct +3.5%; with
        // 16-bit storage it was neutral on the cavity and 7% slower on the
        // sphere duct, and on the shifted directions (whose lines neighbouring
        // work-items share) it was slower everywhere.
        if (ex == 0 && sizeof(B) == 4)
            q[i] = __builtin_nontemporal_load(
                reinterpret_cast<const Vt*>(reinterpret_cast<const char*>(P) + (r + xs) * (uint32_t)sizeof(B)));
        else
            q[i] = ldv<VW>(P, r + xs);
    }
    // the caller raised the wave's priority for issuing these loads
    if constexpr (DROP_PRIO) __builtin_amdgcn_s_setprio(0);
    if constexpr (EARLY) {
#pragma unroll
        for (int j = 0; j < VW; ++j) smw[j] = near_wall ? early_mask[j] : 0u;
    }
    B wrapv[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) wrapv[i] = B(0);
    const bool fixl = wl && end0, fixr = wr && endL;
    if (fixl || fixr) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int ex = SIGN * EX[i], ey = SIGN * EY[i];
            if (ex == 0) continue;
            const int iz = SIGN > 0 ? i : OPP[i];
            uint32_t r = orow;
            if (ey == 1) r += oym; else if (ey == -1) r += oyp;
            const B* P = plane(src, d, i, src_slab(iz, z, zm, zp));
            if (ex == 1 && fixl) wrapv[i] = ld(P, r + nx - 1);
            if (ex == -1 && fixr) wrapv[i] = ld(P, r);
        }
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int ex = SIGN * EX[i];
        if (ex == 0) continue;
        const Vt v = q[i];
        Vt s;
        if (ex == 1) {
            s[0] = wrapv[i];
#pragma unroll
            for (int k = 1; k < VW; ++k) s[k] = v[k - 1];
            q[i] = wl ? s : v;
        } else {
#pragma unroll
            for (int k = 0; k < VW - 1; ++k) s[k] = v[k + 1];
            s[VW - 1] = wrapv[i];
            q[i] = wr ? s : v;
        }
    }
    if (near_wall && all_planes) {
        const B* base = plane(src, d, 0, z);
        Vt loc[Q];
        uint32_t sm[VW];
        if constexpr (WAVE_OR) {
            uint32_t lane_or = 0;
#pragma unroll
            for (int j = 0; j < VW; ++j) {
                sm[j] = smw[j];
                lane_or |= smw[j];
            }
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const int bit = SIGN > 0 ? i : OPP[i];
                loc[OPP[i]] = q[i];   // not read unless some work-item needs the plane
                if (__builtin_amdgcn_ballot_w64((lane_or >> bit) & 1u) != 0ull)
                    loc[OPP[i]] = ldv<VW>(base, (uint32_t)OPP[i] * d.nxy + o0);
            }
        } else {
#pragma unroll
            for (int i = 1; i < Q; ++i) loc[i] = ldv<VW>(base, (uint32_t)i * d.nxy + o0);
            load_words<VW>(smask, c0, sm);
        }
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const int bit = SIGN > 0 ? i : OPP[i];
            Vt v = q[i];
#pragma unroll
            for (int j = 0; j < VW; ++j)
                if ((sm[j] >> bit) & 1u) v[j] = loc[OPP[i]][j];
            q[i] = v;
        }
    } else if (near_wall) {
        // one load per opposite pair (i, i+1), i odd, that any point needs:
        // direction i+1 at x when q[i]'s neighbour is solid, else direction i
        uint32_t any = 0;
#pragma unroll
        for (int j = 0; j < VW; ++j) any |= smw[j];
        const B* pair_base = plane(src, d, 0, z);
        Vt bb[Q / 2];
#pragma unroll
        for (int p = 0; p < Q / 2; ++p) {
            const int i = 2 * p + 1, k = i + 1;
            const int bi = SIGN > 0 ? i : k;
            const bool need_i = (any >> bi) & 1u;
            const int bk = SIGN > 0 ? k : i;
            const bool need_k = (any >> bk) & 1u;
            if (need_i || need_k) bb[p] = ldv<VW>(pair_base, (need_i ? (uint32_t)k : (uint32_t)i) * d.nxy + o0);
        }
#pragma unroll
        for (int p = 0; p < Q / 2; ++p) {
            const int i = 2 * p + 1, k = i + 1;
            const int bi = SIGN > 0 ? i : k;
            const int bk = SIGN > 0 ? k : i;
            const bool need_i = (any >> bi) & 1u, need_k = (any >> bk) & 1u;
            if (need_i) {
                Vt v = q[i];
#pragma unroll
                for (int j = 0; j < VW; ++j)
                    if ((smw[j] >> bi) & 1u) v[j] = bb[p][j];
                q[i] = v;
            } else if (need_k) {
                Vt v = q[k];
#pragma unroll
                for (int j = 0; j < VW; ++j)
                    if ((smw[j] >> bk) & 1u) v[j] = bb[p][j];
                q[k] = v;
            }
            if (need_i && need_k) {   // both of the pair bounce somewhere in the group (rare)
                const Vt b2 = ldv<VW>(pair_base, (uint32_t)i * d.nxy + o0);
                Vt w = q[k];
#pragma unroll
                for (int j = 0; j < VW; ++j)
                    if ((smw[j] >> bk) & 1u) w[j] = b2[j];
                q[k] = w;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Collision on offsets. In: h_i = p_i - w_i (pre-collision), force F (zero
// when FORCE is false). Out: h_i <- s_i - w_i.
//   rho = 1 + sum h_i, m = sum e_i h_i (sum e_i w_i = 0), u = (m + F/2)/rho
//   f^eq_i - w_i = w_i [ (rho - 1) + rho (3 e.u + 4.5 (e.u)^2 - 1.5 u.u) ]
//   s_i = p_i + omega (f^eq_i - p_i) + (1 - omega/2) G_i
//   G_i = w_i [ 3 (e_i - u).F + 9 (e_i.u)(e_i.F) ]
// ---------------------------------------------------------------------------
struct Macro {
    float drho, rho, ux, uy, uz;
};

__device__ __forceinline__ float sum_h(const float h[Q])
{
    return ((((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7])))
            + (((h[8] + h[9]) + (h[10] + h[11])) + ((h[12] + h[13]) + (h[14] + h[15]))))
           + ((h[16] + h[17]) + h[18]);
}
__device__ __forceinline__ float mom_x(const float h[Q])
{
    return ((h[1] - h[2]) + (h[7] - h[8])) + ((h[9] - h[10]) + (h[15] - h[16])) + (h[18] - h[17]);
}
__device__ __forceinline__ float mom_y(const float h[Q])
{
    return ((h[3] - h[4]) + (h[7] - h[8])) + ((h[10] - h[9]) + (h[11] - h[12])) + (h[13] - h[14]);
}
__device__ __forceinline__ float mom_z(const float h[Q])
{
    return ((h[5] - h[6]) + (h[11] - h[12])) + ((h[14] - h[13]) + (h[15] - h[16])) + (h[17] - h[18]);
}

// In-step macroscopic values of pre-collision offsets (u includes +F/2).
template <bool FORCE>
__device__ __forceinline__ Macro macro_pre(const float h[Q], float Fx, float Fy, float Fz)
{
    Macro m;
    m.drho = sum_h(h);
    m.rho = 1.0f + m.drho;
    const float ir = 1.0f / m.rho;
    float mx = mom_x(h), my = mom_y(h), mz = mom_z(h);
    if (FORCE) {
        mx = fmaf(0.5f, Fx, mx);
        my = fmaf(0.5f, Fy, my);
        mz = fmaf(0.5f, Fz, mz);
    }
    m.ux = mx * ir;
    m.uy = my * ir;
    m.uz = mz * ir;
    return m;
}

__device__ __forceinline__ float edot(int i, float ax, float ay, float az)
{
    float r = 0.0f;
    if (EX[i] == 1) r = ax; else if (EX[i] == -1) r = -ax;
    if (EY[i] == 1) r += ay; else if (EY[i] == -1) r -= ay;
    if (EZ[i] == 1) r += az; else if (EZ[i] == -1) r -= az;
    return r;
}

// f^eq_i - w_i given the macro state and A = drho - 1.5 rho u.u.
__device__ __forceinline__ float heq(int i, const Macro& m, float A)
{
    const float eu = edot(i, m.ux, m.uy, m.uz);
    return weight(i) * fmaf(m.rho * eu, fmaf(4.5f, eu, 3.0f), A);
}

__device__ __forceinline__ float eq_A(const Macro& m)
{
    const float usq = fmaf(m.ux, m.ux, fmaf(m.uy, m.uy, m.uz * m.uz));
    return fmaf(-1.5f * m.rho, usq, m.drho);
}

// Guo source without the (1 - omega/2) factor.
__device__ __forceinline__ float guo(int i, const Macro& m, float Fx, float Fy, float Fz, float uF)
{
    const float eu = edot(i, m.ux, m.uy, m.uz);
    const float eF = edot(i, Fx, Fy, Fz);
    return weight(i) * fmaf(9.0f * eu, eF, 3.0f * (eF - uF));
}

// ---------------------------------------------------------------------------
// On-site velocity nodes (the boundary family of the paper's cavity
// validation, Section 5, after Hecht & Harting). A node on a box face, edge or
// corner has a prescribed velocity u; the directions whose pull source is
// solid (bits of U) are unknown after the gather and are rebuilt before the
// collision so that the node carries mass rho and bare momentum
// j = rho u - F/2 (velocity u once the collision adds F/2):
//   - unknown i with known opposite:  f_i = f_opp(i) + 6 w_i e_i.j + e_i.lambda
//   - both i and opp(i) unknown (edge and corner nodes): the pair takes the
//     equilibrium at (rho, u) and carries j: f_i = f^eq_i(rho, u) - 1.5 w_i e_i.F
//   - mass:  rho (1 - W_B - a.u - B_q) = 1 - W_B + H - a.F/2, in offsets
//       delta = rho - 1 = (H + a.u + B_q - a.F/2) / (1 - W_B - a.u - B_q)
//     with H = sum of the known offsets and of the opposites of the bounced
//     ones, a = 6 sum w_i e_i over the bounced unknowns, W_B and
//     B_q = sum w_i (4.5 (e_i.u)^2 - 1.5 u.u) over the buried pairs;
//   - the momentum along the axes normal to the wall then holds by itself;
//     along each tangential axis t the remainder R_t is spread over the
//     bounced unknowns with e_it != 0: lambda_t = R_t / #{such links}.
// Mass and momentum hold exactly (up to rounding) on faces, edges and
// corners; on faces this is the Zou-He / Hecht-Harting rule.
// ---------------------------------------------------------------------------

// Bits of the directions opposite to those set in m (pairs (1,2) .. (17,18)).
__device__ __forceinline__ uint32_t opp_bits(uint32_t m)
{
    return ((m & 0x2AAAAu) << 1) | ((m & 0x55554u) >> 1);
}

// U is a valid unknown set: the union over one to three axis-aligned walls of
// the directions pointing away from that wall (box face, edge or corner).
__device__ __forceinline__ bool onsite_pattern_ok(uint32_t U)
{
    const bool xm = (U >> 1) & 1u, xp = (U >> 2) & 1u;
    const bool ym = (U >> 3) & 1u, yp = (U >> 4) & 1u;
    const bool zm = (U >> 5) & 1u, zp = (U >> 6) & 1u;
    if ((xm && xp) || (ym && yp) || (zm && zp)) return false;
    uint32_t expect = 0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const bool in = (xm && EX[i] == 1) || (xp && EX[i] == -1) || (ym && EY[i] == 1) ||
                        (yp && EY[i] == -1) || (zm && EZ[i] == 1) || (zp && EZ[i] == -1);
        if (in) expect |= 1u << i;
    }
    return U != 0 && U == expect;
}

// h: offsets after the gather (entries in U arbitrary) -> rebuilt offsets.
// Written without branches (per-direction selects): the unknown set differs
// from lane to lane, and branches would serialise.
// With the wall normals n_k (unit vectors pointing into the fluid, one to
// three of them) the class constants follow from the velocity set:
//   a = 6 sum_{bounced} w_i e_i = c_k sum_k n_k, c = 1, 5/6, 2/3 for a face,
//   edge, corner (the directions shared by two walls are buried);
//   W_B = (number of buried directions) / 36;
//   bounced links with a non-zero component along a tangential axis: 2 on a
//   face, 4 on an edge (none on a corner).
template <bool FORCE>
__device__ __forceinline__ void onsite_rebuild(float h[Q], uint32_t U, float ux, float uy, float uz,
                                               float Fx, float Fy, float Fz)
{
    const uint32_t Bm = U & opp_bits(U);   // buried pairs
    const uint32_t Rm = U & ~Bm;           // bounced unknowns
    const float nx = (U & 2u) ? 1.0f : ((U & 4u) ? -1.0f : 0.0f);
    const float ny = (U & 8u) ? 1.0f : ((U & 16u) ? -1.0f : 0.0f);
    const float nz = (U & 32u) ? 1.0f : ((U & 64u) ? -1.0f : 0.0f);
    const bool tx = nx == 0.0f, ty = ny == 0.0f, tz = nz == 0.0f;
    const int walls = 3 - (int)tx - (int)ty - (int)tz;
    const float ca = walls == 1 ? 1.0f : (walls == 2 ? 5.0f / 6.0f : 2.0f / 3.0f);
    const float ax = ca * nx, ay = ca * ny, az = ca * nz;
    const float WB = (float)__builtin_popcount(Bm) * (1.0f / 36.0f);
    const float usq = fmaf(ux, ux, fmaf(uy, uy, uz * uz));
    float H = h[0], Bq = 0.0f;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const bool unknown = (U >> i) & 1u, rb = (Rm >> i) & 1u;
        H += unknown ? (rb ? h[OPP[i]] : 0.0f) : h[i];
        if (i >= 7) {   // only diagonal directions can be buried
            const float eu = edot(i, ux, uy, uz);
            Bq += ((Bm >> i) & 1u) ? weight(i) * fmaf(4.5f * eu, eu, -1.5f * usq) : 0.0f;
        }
    }
    const float au = fmaf(ax, ux, fmaf(ay, uy, az * uz));
    float num = H + au + Bq;
    if (FORCE) num = fmaf(-0.5f, fmaf(ax, Fx, fmaf(ay, Fy, az * Fz)), num);
    const float delta = num / (((1.0f - WB) - au) - Bq);
    const float rho = 1.0f + delta;
    float jx = rho * ux, jy = rho * uy, jz = rho * uz;
    if (FORCE) {
        jx = fmaf(-0.5f, Fx, jx);
        jy = fmaf(-0.5f, Fy, jy);
        jz = fmaf(-0.5f, Fz, jz);
    }
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const float w = weight(i);
        const float vr = fmaf(6.0f * w, edot(i, jx, jy, jz), h[OPP[i]]);
        float v = ((Rm >> i) & 1u) ? vr : h[i];
        if (i >= 7) {
            const float eu = edot(i, ux, uy, uz);
            float vb = w * fmaf(rho, fmaf(eu, fmaf(4.5f, eu, 3.0f), -1.5f * usq), delta);
            if (FORCE) vb = fmaf(-1.5f * w, edot(i, Fx, Fy, Fz), vb);
            v = ((Bm >> i) & 1u) ? vb : v;
        }
        h[i] = v;
    }
    // tangential momentum remainder (spread over 2 or 4 links: exact scaling)
    const float inv_n = walls == 1 ? 0.5f : 0.25f;
    const float lx = tx ? (jx - mom_x(h)) * inv_n : 0.0f;
    const float ly = ty ? (jy - mom_y(h)) * inv_n : 0.0f;
    const float lz = tz ? (jz - mom_z(h)) * inv_n : 0.0f;
#pragma unroll
    for (int i = 1; i < Q; ++i) h[i] += ((Rm >> i) & 1u) ? edot(i, lx, ly, lz) : 0.0f;
}

// Returns the in-step macroscopic values (rho, u = (m + F/2)/rho).
// Opposite directions i, opp(i) share e.u up to sign, so the equilibrium and
// the Guo source are split into a part even in e and a part odd in e and
// evaluated once per pair:
//   f^eq_i - w_i = w_i (A + 4.5 rho (e.u)^2) +- 3 w_i rho (e.u)
//   G_i          = w_i (9 (e.u)(e.F) - 3 u.F) +- 3 w_i (e.F)
template <bool FORCE>
__device__ __forceinline__ Macro bgk_collide(float h[Q], float omega, float cF, float Fx, float Fy,
                                             float Fz)
{
    const Macro m = macro_pre<FORCE>(h, Fx, Fy, Fz);
    const float A = eq_A(m);
    float uF = 0.0f;
    if (FORCE) uF = fmaf(m.ux, Fx, fmaf(m.uy, Fy, m.uz * Fz));
    h[0] = fmaf(omega, weight(0) * A - h[0], h[0]);
    if (FORCE) h[0] = fmaf(cF, weight(0) * (-3.0f * uF), h[0]);
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
        const int k = i + 1;                        // OPP[i]
        const float w = weight(i);
        const float eu = edot(i, m.ux, m.uy, m.uz);
        const float reu = m.rho * eu;
        const float even = w * fmaf(4.5f * reu, eu, A);
        const float odd = (3.0f * w) * reu;
        float oi = fmaf(omega, (even + odd) - h[i], h[i]);
        float ok = fmaf(omega, (even - odd) - h[k], h[k]);
        if (FORCE) {
            const float eF = edot(i, Fx, Fy, Fz);
            const float geven = w * fmaf(9.0f * eu, eF, -3.0f * uF);
            const float godd = (3.0f * w) * eF;
            oi = fmaf(cF, geven + godd, oi);
            ok = fmaf(cF, geven - godd, ok);
        }
        h[i] = oi;
        h[k] = ok;
    }
    return m;
}

}  // namespace d3q19

// Forward kernels for gfx950: the fused pull step (Mawson & Revell, Section 4.2,
// Algorithm 3) in the two-array (AB) pattern and the single-array (AA)
// pattern, plus the auxiliary per-point kernels (initialisation, macroscopic
// output, state copy in and out, finite check, flag preprocessing, copy probe).
//
// Work-groups are x-dominant (Section 6) and every work-group lies in one
// z-slab. Populations are stored per (direction, slab) plane (see plane() in
// d3q19.hpp): the structure-of-arrays coalescing of Section 4.1, with the 19
// planes of a slab next to each other so that the concurrently running
// work-groups stream through a compact address window.
#include <type_traits>

#include "kernels.hpp"

using namespace d3q19;

namespace lbmk {

Launch make_launch(const Dims& d, int bx, int by, hipStream_t s)
{
    Launch L;
    L.block = dim3((unsigned)bx, (unsigned)by, 1);
    L.grid = dim3((unsigned)((d.nx + bx - 1) / bx), (unsigned)((d.ny + by - 1) / by), (unsigned)d.nz);
    L.stream = s;
    return L;
}

template <int FM>
__device__ __forceinline__ void load_force(const StepArgs& a, const float* __restrict__ ff, uint32_t c,
                                           float& Fx, float& Fy, float& Fz)
{
    if (FM == FORCE_UNIFORM) {
        Fx = a.Fx; Fy = a.Fy; Fz = a.Fz;
    } else if (FM == FORCE_FIELD) {
        Fx = ff[c];
        Fy = ff[(size_t)a.d.N + c];
        Fz = ff[2 * (size_t)a.d.N + c];
    } else {
        Fx = Fy = Fz = 0.0f;
    }
}

// Decode, add moving-wall terms, rebuild the unknowns of an on-site node
// (onsiteU != 0: its solid-source directions), collide. h ends as
// post-collision offsets.
template <class St, int FM, bool ONSITE>
__device__ __forceinline__ Macro decode_collide(const typename St::raw_t raw[Q], uint32_t mwmask,
                                                uint32_t onsiteU, bool onsite_moving,
                                                const StepArgs& a, const float* __restrict__ ff,
                                                uint32_t c, float h[Q])
{
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        h[i] = St::off(raw[i], i);
        if (i > 0 && ((mwmask >> i) & 1u)) h[i] = h[i] + a.mw[i];
    }
    float Fx, Fy, Fz;
    load_force<FM>(a, ff, c, Fx, Fy, Fz);
    if (ONSITE && onsiteU) {
        const float ux = onsite_moving ? a.uw[0] : 0.0f;
        const float uy = onsite_moving ? a.uw[1] : 0.0f;
        const float uz = onsite_moving ? a.uw[2] : 0.0f;
        onsite_rebuild<FM != FORCE_NONE>(h, onsiteU, ux, uy, uz, Fx, Fy, Fz);
    }
    return bgk_collide<FM != FORCE_NONE>(h, a.omega, a.cF, Fx, Fy, Fz);
}

#define POINT_PROLOGUE(d)                                                                      \
    const int x = blockIdx.x * blockDim.x + threadIdx.x;                                       \
    const int y = blockIdx.y * blockDim.y + threadIdx.y;                                       \
    const uint32_t z = blockIdx.z;                                                             \
    if (x >= (d).nx || y >= (d).ny) return;                                                    \
    const uint32_t o = (uint32_t)y * (uint32_t)(d).nx + (uint32_t)x;                           \
    const uint32_t c = z * (d).nxy + o;                                                        \
    const uint32_t zm = wrap_m(z, (uint32_t)(d).nz), zp = wrap_p(z, (uint32_t)(d).nz);

// ---------------------------------------------------------------------------
// AB pull step, one point per work-item: gather from x - e_i in `src`,
// bounce back at solid neighbours, collide, store into `dst`. Used when the
// row length is not a multiple of the vector width. MACROS: also store the
// in-step rho and u (the four extra stores per point of Section 4.1).
// ONSITE: rebuild the unknown populations of on-site velocity nodes.
// ---------------------------------------------------------------------------
template <class St, int FM, bool COLLIDE, bool MACROS, bool ONSITE>
__global__ __launch_bounds__(1024) void k_step_ab(const typename St::raw_t* __restrict__ src,
                                                  typename St::raw_t* __restrict__ dst,
                                                  const uint8_t* __restrict__ flags,
                                                  const uint32_t* __restrict__ smask,
                                                  const uint32_t* __restrict__ mmask,
                                                  const float* __restrict__ ff, StepArgs a,
                                                  float* __restrict__ rho_out, float* __restrict__ u_out)
{
    using T = typename St::raw_t;
    const Dims& d = a.d;
    POINT_PROLOGUE(d)
    const uint8_t fl = flags[c];
    if (fl & TYPE_MASK) {
        if (MACROS) {
            rho_out[c] = 0.0f;
            u_out[c] = 0.0f; u_out[(size_t)d.N + c] = 0.0f; u_out[2 * (size_t)d.N + c] = 0.0f;
        }
        return;
    }

    uint32_t on[Q];
    pull_offsets(d, x, y, on);
    T raw[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) raw[i] = ld(plane(src, d, i, src_slab(i, z, zm, zp)), on[i]);

    uint32_t mwmask = 0, solid = 0;
    if (fl & NEAR_WALL) {
        solid = smask[c];
        if (fl & NEAR_MOVING) mwmask = mmask[c];
#pragma unroll
        for (int i = 1; i < Q; ++i)
            if ((solid >> i) & 1u) raw[i] = ld(plane(src, d, OPP[i], z), o);
    }

    if (!COLLIDE) {
#pragma unroll
        for (int i = 0; i < Q; ++i) st(plane(dst, d, i, z), o, raw[i]);
        return;
    }
    float h[Q];
    const Macro m = decode_collide<St, FM, ONSITE>(raw, mwmask, (fl & ONSITE_NODE) ? solid : 0u,
                                                   (fl & ONSITE_MOVING) != 0, a, ff, c, h);
#pragma unroll
    for (int i = 0; i < Q; ++i) st(plane(dst, d, i, z), o, St::enc(h[i], i));
    if (MACROS) {
        rho_out[c] = m.rho;
        u_out[c] = m.ux; u_out[(size_t)d.N + c] = m.uy; u_out[2 * (size_t)d.N + c] = m.uz;
    }
}

// ---------------------------------------------------------------------------
// AB pull step, VW consecutive x-points per work-item (nx % VW == 0), one
// vector access per direction: 16 bytes for FP32 (VW = 4) and for 16-bit
// storage with VW = 8, 8 bytes for 16-bit storage with VW = 4.
// The gather (gather_vec in d3q19.hpp): directions with e_x = 0 are aligned
// accesses; e_x = +-1 are shifted by one element (a shifted wave access spans
// one extra cache line, which the neighbouring work-item also touches, so
// HBM traffic does not grow). Near-wall points take the bounced values
// s_opp(i)(x) through the precomputed solid-neighbour mask.
// Solid points inside a work-item's group are written as the rest state.
// ONSITE: on-site velocity nodes rebuild their unknowns (the solid-source
// bits of the neighbour mask) before the collision.
// Per fluid point the arithmetic is the one-point kernel's, bit for bit.
// ---------------------------------------------------------------------------
template <int VW>
struct FlagWord;
template <>
struct FlagWord<4> {
    typedef uint32_t t;
    static constexpr uint32_t ones = 0x01010101u;
};
template <>
struct FlagWord<8> {
    typedef uint64_t t;
    static constexpr uint64_t ones = 0x0101010101010101ull;
};

// EARLY (FP32, porous geometry): the gather's loads are issued before the
// flag-dependent branches (gather_vec), with the neighbour masks of every
// work-item; fully solid groups then run the whole path and store the rest
// state like solid points in mixed groups, and waves with no fluid point
// store nothing.
template <class St, int FM, int VW, bool MACROS, bool ONSITE>
struct Occupancy {
    // Waves per SIMD the register budget must allow: the 16-bit eight-point
    // step sits at the 168-VGPR edge of three waves per SIMD, and losing the
    // third wave cost 11% at 256^3 on MI355X. Variants that need more (the
    // macroscopic output, on-site nodes, bfloat16 with a body force) would
    // spill under that bound and keep two waves.
    static constexpr bool tight = VW == 8 && !ONSITE && !MACROS &&
                                  (sizeof(typename St::raw_t) == 2 && (!std::is_same_v<St, StBF16> || FM == FORCE_NONE));
    static constexpr int waves = tight ? 3 : 1;
};

template <class St, int FM, bool COLLIDE, int VW, bool MACROS, bool ONSITE, bool FLAT, bool EARLY>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Occupancy<St, FM, VW, MACROS, ONSITE>::waves)))
void k_step_abv(const typename St::bits_t* __restrict__ src,
                                                  typename St::bits_t* __restrict__ dst,
                                                  const uint8_t* __restrict__ flags,
                                                  const uint32_t* __restrict__ smask,
                                                  const uint32_t* __restrict__ mmask,
                                                  const float* __restrict__ ff, StepArgs a,
                                                  float* __restrict__ rho_out, float* __restrict__ u_out)
{
    using B = typename St::bits_t;
    using Vt = typename Vec<B, VW>::t;
    using FW = typename FlagWord<VW>::t;
    constexpr FW ONES = FlagWord<VW>::ones;
    const Dims& d = a.d;
    // FP32 flags-first form: the wave issues its flag and gather loads at
    // raised priority and drops it once the 19 loads are out, so that waves
    // starting while others collide get their loads into the memory pipeline
    // first. 256^3 cavity on MI355X: 410.2 -> 407.9 us per step; on the
    // porous forms (early gather, 16-bit all-planes bounce loads) it was 3-12%
    // slower, so they run at the default priority.
    constexpr bool PRIO = sizeof(B) == 4 && !EARLY;
    if constexpr (PRIO) __builtin_amdgcn_s_setprio(2);
    // FLAT: rows whose group count is not a multiple of the wave width run
    // on a one-dimensional grid over the plane (a.gx groups per row), so
    // that every wave is full.
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    int x0, y;
    if (FLAT) {
        const uint32_t gy = gid / a.gx;
        x0 = VW * (int)(gid - gy * a.gx);
        y = (int)gy;
    } else {
        x0 = VW * (int)gid;
        y = blockIdx.y * blockDim.y + threadIdx.y;
    }
    const uint32_t z = blockIdx.z;
    if (x0 >= d.nx || y >= d.ny) return;
    const uint32_t nx = (uint32_t)d.nx;
    const uint32_t orow = (uint32_t)y * nx;
    const uint32_t o0 = orow + (uint32_t)x0;
    const uint32_t c0 = z * d.nxy + o0;
    static_assert(!EARLY || (sizeof(B) == 4 && !MACROS && !ONSITE && COLLIDE), "early gather: FP32 step only");
    const FW flw = *reinterpret_cast<const FW*>(flags + c0);
    const FW solid = (flw | (flw >> 1)) & ONES;   // byte j: point j solid
    uint32_t early_mask[EARLY ? VW : 1];
    if constexpr (EARLY) {
        load_words<VW>(smask, c0, early_mask);
    } else {
        // wave-wide vote, taken by every work-item before the branch
        if (__builtin_amdgcn_ballot_w64(solid != ONES) == 0ull) {   // no fluid point in the wave
            if (MACROS) {
                const typename Vec<float, VW>::t zero = 0.0f;
                stv_nt<VW>(rho_out, c0, zero);
#pragma unroll
                for (int k = 0; k < 3; ++k) stv_nt<VW>(u_out + k * (size_t)d.N, c0, zero);
            }
            return;
        }
    }

    Vt q[Q];
    typename Vec<float, VW>::t mr, mx, my, mz;
    if (!EARLY && solid == ONES) {
        // Fully solid group in a wave that holds fluid points: the rest
        // state (offset 0), although nothing reads it. Leaving holes in a
        // wave's stores cost 17% of the step time on the 10%-solid sphere
        // duct, and storing it apart from the fluid work-items' stores wrote
        // the shared cache lines back twice (write traffic 9-14% above the
        // state size with 16-bit storage); the same store instructions
        // write both. Waves with no fluid point store nothing.
#pragma unroll
        for (int i = 0; i < Q; ++i) q[i] = St::enc_b(0.0f, i);
        mr = 0.0f; mx = 0.0f; my = 0.0f; mz = 0.0f;
    } else {
        const uint32_t zm = wrap_m(z, (uint32_t)d.nz), zp = wrap_p(z, (uint32_t)d.nz);
        const uint32_t oym = (y == 0) ? (uint32_t)(d.ny - 1) * nx : (uint32_t)0 - nx;
        const uint32_t oyp = (y == d.ny - 1) ? (uint32_t)(1 - d.ny) * nx : nx;

        gather_vec<+1, VW, EARLY, PRIO>(src, d, z, zm, zp, orow, oym, oyp, (uint32_t)x0, !(solid & 0x1u),
                                  !((solid >> (8 * (VW - 1))) & 0x1u), (flw & (ONES * NEAR_WALL)) != 0, smask, c0,
                                  q, early_mask);

        // moving-wall terms of the bounced populations
        uint32_t mm[VW];
#pragma unroll
        for (int j = 0; j < VW; ++j) mm[j] = 0u;
        if (COLLIDE && (flw & (ONES * NEAR_MOVING))) {
#pragma unroll
            for (int g = 0; g < VW / 4; ++g) {
                const typename V4<uint32_t>::t m4 = ld4(mmask, c0 + 4 * g);
                mm[4 * g] = m4.x; mm[4 * g + 1] = m4.y; mm[4 * g + 2] = m4.z; mm[4 * g + 3] = m4.w;
            }
        }
        uint32_t os[VW];   // unknown-direction bits of on-site nodes, else 0
#pragma unroll
        for (int j = 0; j < VW; ++j) os[j] = 0u;
        if (ONSITE && COLLIDE && (flw & (ONES * ONSITE_NODE))) {
            load_words<VW>(smask, c0, os);
#pragma unroll
            for (int j = 0; j < VW; ++j)
                if (!((flw >> (8 * j)) & ONSITE_NODE)) os[j] = 0u;
        }

        if (COLLIDE) {
            float F[3][VW];
            if (FM == FORCE_FIELD) {
#pragma unroll
                for (int k = 0; k < 3; ++k)
#pragma unroll
                    for (int g = 0; g < VW / 4; ++g) {
                        const typename V4<float>::t f = ld4(ff + k * (size_t)d.N, c0 + 4 * g);
                        F[k][4 * g] = f.x; F[k][4 * g + 1] = f.y; F[k][4 * g + 2] = f.z; F[k][4 * g + 3] = f.w;
                    }
            } else {
#pragma unroll
                for (int j = 0; j < VW; ++j) {
                    F[0][j] = FM == FORCE_UNIFORM ? a.Fx : 0.0f;
                    F[1][j] = FM == FORCE_UNIFORM ? a.Fy : 0.0f;
                    F[2][j] = FM == FORCE_UNIFORM ? a.Fz : 0.0f;
                }
            }
            // On-site nodes: the first on-site point of each work-item is rebuilt
            // before the loop, so a wave whose on-site points sit at different
            // positions in different work-items (the two ends of a row) runs the
            // rebuild once rather than once per position; further on-site points
            // of a work-item (rows lying on a face of the box) are rebuilt in the
            // loop. The moving-wall terms are skipped for that point: they only
            // touch its unknown directions, which the rebuild overwrites.
            int jr = VW;
            float hr[ONSITE ? Q : 1];
            if (ONSITE) {
                uint32_t Ur = 0u;
#pragma unroll
                for (int j = VW - 1; j >= 0; --j)
                    if (os[j]) { jr = j; Ur = os[j]; }
                if (Ur) {
                    float fr[3];
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        fr[k] = F[k][0];
#pragma unroll
                        for (int j = 1; j < VW; ++j) fr[k] = jr == j ? F[k][j] : fr[k];
                    }
#pragma unroll
                    for (int i = 0; i < Q; ++i) {
                        B b = q[i][0];
#pragma unroll
                        for (int j = 1; j < VW; ++j) b = jr == j ? q[i][j] : b;
                        hr[i] = St::off_b(b, i);
                    }
                    const bool mv = (flw >> (8 * jr)) & ONSITE_MOVING;
                    onsite_rebuild<FM != FORCE_NONE>(hr, Ur, mv ? a.uw[0] : 0.0f, mv ? a.uw[1] : 0.0f,
                                                     mv ? a.uw[2] : 0.0f, fr[0], fr[1], fr[2]);
                }
            }
#pragma unroll
            for (int j = 0; j < VW; ++j) {
                float h[Q];
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    h[i] = St::off_b(q[i][j], i);
                    if (i > 0 && ((mm[j] >> i) & 1u)) h[i] = h[i] + a.mw[i];
                }
                if (ONSITE) {
                    if (jr == j) {
#pragma unroll
                        for (int i = 0; i < Q; ++i) h[i] = hr[i];
                    } else if (os[j]) {
                        const bool mv = (flw >> (8 * j)) & ONSITE_MOVING;
                        onsite_rebuild<FM != FORCE_NONE>(h, os[j], mv ? a.uw[0] : 0.0f, mv ? a.uw[1] : 0.0f,
                                                         mv ? a.uw[2] : 0.0f, F[0][j], F[1][j], F[2][j]);
                    }
                }
                const Macro m = bgk_collide<FM != FORCE_NONE>(h, a.omega, a.cF, F[0][j], F[1][j], F[2][j]);
                const bool sol = (solid >> (8 * j)) & 1u;
#pragma unroll
                for (int i = 0; i < Q; ++i) q[i][j] = St::enc_b(sol ? 0.0f : h[i], i);
                if (MACROS) {
                    mr[j] = sol ? 0.0f : m.rho;
                    mx[j] = sol ? 0.0f : m.ux;
                    my[j] = sol ? 0.0f : m.uy;
                    mz[j] = sol ? 0.0f : m.uz;
                }
            }
        }
    }
    if (MACROS) {
        stv_nt<VW>(rho_out, c0, mr);
        stv_nt<VW>(u_out, c0, mx);
        stv_nt<VW>(u_out + (size_t)d.N, c0, my);
        stv_nt<VW>(u_out + 2 * (size_t)d.N, c0, mz);
    }
    if constexpr (EARLY) {
        if (__builtin_amdgcn_ballot_w64(solid != ONES) == 0ull) return;   // no fluid point in the wave
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) stv_nt<VW>(plane(dst, d, i, z), o0, q[i]);
}

// ---------------------------------------------------------------------------
// AA pattern, one array, in place.
// Parity 0 (array holds s_i(x) at slot [i][x]): read p_i from [i][x - e_i],
// or from [opp(i)][x] when x - e_i is solid; write s'_j into the slot that
// p_opp(j) was read from. Afterwards s'_j(x) sits at [opp(j)][x + e_j]
// (or at [j][x] when x + e_j is solid).
// Parity 1: p_i = [opp(i)][x] for every i (local); write s'_i to [i][x],
// restoring the natural layout. Each work-item reads and writes the same 19
// slots, and no two work-items share a slot, so the update is race-free.
// ---------------------------------------------------------------------------
template <class St, int FM, bool COLLIDE, bool ONSITE>
__global__ __launch_bounds__(1024) void k_step_aa0(typename St::raw_t* f,
                                                   const uint8_t* __restrict__ flags,
                                                   const uint32_t* __restrict__ smask,
                                                   const uint32_t* __restrict__ mmask,
                                                   const float* __restrict__ ff, StepArgs a)
{
    using T = typename St::raw_t;
    const Dims& d = a.d;
    POINT_PROLOGUE(d)
    const uint8_t fl = flags[c];
    if (fl & TYPE_MASK) return;

    uint32_t on[Q];
    pull_offsets(d, x, y, on);
    T raw[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) raw[i] = ld(plane(f, d, i, src_slab(i, z, zm, zp)), on[i]);

    uint32_t solid = 0, mwmask = 0;
    if (fl & NEAR_WALL) {
        solid = smask[c];
        if (fl & NEAR_MOVING) mwmask = mmask[c];
#pragma unroll
        for (int i = 1; i < Q; ++i)
            if ((solid >> i) & 1u) raw[i] = ld(plane(f, d, OPP[i], z), o);
    }

    float h[Q];
    if (COLLIDE)
        decode_collide<St, FM, ONSITE>(raw, mwmask, (fl & ONSITE_NODE) ? solid : 0u, (fl & ONSITE_MOVING) != 0,
                                       a, ff, c, h);
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        const int k = OPP[j];
        const T v = COLLIDE ? St::enc(h[j], j) : raw[j];
        if ((solid >> k) & 1u) st(plane(f, d, j, z), o, v);
        else st(plane(f, d, k, src_slab(k, z, zm, zp)), on[k], v);
    }
}

template <class St, int FM, bool COLLIDE, bool ONSITE>
__global__ __launch_bounds__(1024) void k_step_aa1(typename St::raw_t* f,
                                                   const uint8_t* __restrict__ flags,
                                                   const uint32_t* __restrict__ smask,
                                                   const uint32_t* __restrict__ mmask,
                                                   const float* __restrict__ ff, StepArgs a)
{
    using T = typename St::raw_t;
    const Dims& d = a.d;
    POINT_PROLOGUE(d)
    (void)zm; (void)zp;   // every access of the local step is in the point's own slab
    const uint8_t fl = flags[c];
    if (fl & TYPE_MASK) return;

    T raw[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) raw[i] = ld(plane(f, d, OPP[i], z), o);

    uint32_t mwmask = 0, solid = 0;
    if (COLLIDE && (fl & NEAR_MOVING)) mwmask = mmask[c];
    if (COLLIDE && ONSITE && (fl & ONSITE_NODE)) solid = smask[c];
    if (!COLLIDE) {
#pragma unroll
        for (int i = 0; i < Q; ++i) st(plane(f, d, i, z), o, raw[i]);
        return;
    }
    float h[Q];
    decode_collide<St, FM, ONSITE>(raw, mwmask, (fl & ONSITE_NODE) ? solid : 0u, (fl & ONSITE_MOVING) != 0, a,
                                   ff, c, h);
#pragma unroll
    for (int i = 0; i < Q; ++i) st(plane(f, d, i, z), o, St::enc(h[i], i));
}

// ---------------------------------------------------------------------------
// Stored state of one point in natural order (s_j(x), j = 0..18), for either
// layout. Layout 1 (AA after an odd number of steps): s_j(x) is at
// [opp(j)][x + e_j] when x + e_j is fluid, else at [j][x].
// ---------------------------------------------------------------------------
template <class St, int LAYOUT>
__device__ __forceinline__ void load_state(const typename St::raw_t* __restrict__ f,
                                           const uint8_t* __restrict__ flags, const Dims& d, int x,
                                           int y, uint32_t z, uint32_t o, uint8_t fl,
                                           typename St::raw_t raw[Q])
{
    if (LAYOUT == 0 || (fl & TYPE_MASK)) {
#pragma unroll
        for (int j = 0; j < Q; ++j) raw[j] = ld(plane(f, d, j, z), o);
        return;
    }
    const uint32_t zm = wrap_m(z, (uint32_t)d.nz), zp = wrap_p(z, (uint32_t)d.nz);
    uint32_t on[Q];
    pull_offsets(d, x, y, on);
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        const int k = OPP[j];
        const uint32_t zk = src_slab(k, z, zm, zp);
        const bool wall = (fl & NEAR_WALL) && (flags[zk * d.nxy + on[k]] & TYPE_MASK);
        raw[j] = wall ? ld(plane(f, d, j, z), o) : ld(plane(f, d, k, zk), on[k]);
    }
}

template <class St, int LAYOUT>
__global__ __launch_bounds__(1024) void k_get(const typename St::raw_t* __restrict__ f,
                                              const uint8_t* __restrict__ flags,
                                              float* __restrict__ out, Dims d)
{
    POINT_PROLOGUE(d)
    (void)zm; (void)zp;
    typename St::raw_t raw[Q];
    load_state<St, LAYOUT>(f, flags, d, x, y, z, o, flags[c], raw);
#pragma unroll
    for (int j = 0; j < Q; ++j) out[(size_t)j * d.N + c] = St::plain(raw[j], j);
}

template <class St>
__global__ __launch_bounds__(1024) void k_set(typename St::raw_t* __restrict__ f,
                                              const float* __restrict__ in, Dims d)
{
    POINT_PROLOGUE(d)
    (void)zm; (void)zp;
#pragma unroll
    for (int j = 0; j < Q; ++j) st(plane(f, d, j, z), o, St::from_plain(in[(size_t)j * d.N + c], j));
}

template <class St>
__global__ __launch_bounds__(1024) void k_init_eq(typename St::raw_t* __restrict__ f,
                                                  const float* __restrict__ rho,
                                                  const float* __restrict__ u, Dims d)
{
    POINT_PROLOGUE(d)
    (void)zm; (void)zp;
    Macro m;
    m.rho = rho ? rho[c] : 1.0f;
    m.drho = m.rho - 1.0f;
    m.ux = u ? u[c] : 0.0f;
    m.uy = u ? u[(size_t)d.N + c] : 0.0f;
    m.uz = u ? u[2 * (size_t)d.N + c] : 0.0f;
    const float A = eq_A(m);
#pragma unroll
    for (int j = 0; j < Q; ++j) st(plane(f, d, j, z), o, St::enc(heq(j, m, A), j));
}

template <class St, int LAYOUT, int FM>
__global__ __launch_bounds__(1024) void k_macros(const typename St::raw_t* __restrict__ f,
                                                 const uint8_t* __restrict__ flags,
                                                 const float* __restrict__ ff,
                                                 float* __restrict__ rho, float* __restrict__ u,
                                                 StepArgs a)
{
    const Dims& d = a.d;
    POINT_PROLOGUE(d)
    (void)zm; (void)zp;
    const uint8_t fl = flags[c];
    const size_t N = d.N;
    if (fl & TYPE_MASK) {
        if (rho) rho[c] = 0.0f;
        if (u) { u[c] = 0.0f; u[N + c] = 0.0f; u[2 * N + c] = 0.0f; }
        return;
    }
    typename St::raw_t raw[Q];
    load_state<St, LAYOUT>(f, flags, d, x, y, z, o, fl, raw);
    float h[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) h[j] = St::off(raw[j], j);
    float Fx, Fy, Fz;
    load_force<FM>(a, ff, c, Fx, Fy, Fz);
    // post-collision state: u = (m - F/2)/rho
    const Macro m = macro_pre<FM != FORCE_NONE>(h, -Fx, -Fy, -Fz);
    if (rho) rho[c] = m.rho;
    if (u) { u[c] = m.ux; u[N + c] = m.uy; u[2 * N + c] = m.uz; }
}

template <class St, int LAYOUT>
__global__ __launch_bounds__(1024) void k_check_finite(const typename St::raw_t* __restrict__ f,
                                                       const uint8_t* __restrict__ flags,
                                                       int* flag, Dims d)
{
    POINT_PROLOGUE(d)
    (void)zm; (void)zp;
    const uint8_t fl = flags[c];
    if (fl & TYPE_MASK) return;
    typename St::raw_t raw[Q];
    load_state<St, LAYOUT>(f, flags, d, x, y, z, o, fl, raw);
    bool ok = true;
#pragma unroll
    for (int j = 0; j < Q; ++j) ok = ok && isfinite(St::off(raw[j], j));
    if (!ok) atomicOr(flag, 1);
}

// Caller flag value (0..4) -> type bits: only 1 (wall) and 2 (moving wall)
// are solid; on-site nodes (3, 4) are fluid nodes.
__device__ __forceinline__ uint8_t type_of(uint8_t v) { return (v == 1 || v == 2) ? v : 0; }

// counts[0] += fluid points with a solid neighbour, counts[1] += fluid
// points (one atomic per wave).
__global__ __launch_bounds__(1024) void k_mark_near_wall(const uint8_t* __restrict__ in,
                                                         uint8_t* __restrict__ out,
                                                         uint32_t* __restrict__ smask,
                                                         uint32_t* __restrict__ mmask,
                                                         int* __restrict__ bad,
                                                         unsigned* __restrict__ counts, Dims d)
{
    POINT_PROLOGUE(d)
    const uint8_t v = in[c];
    const uint8_t fl = type_of(v);
    uint8_t r = fl;
    uint32_t sm = 0, mm = 0;
    if (fl == 0) {
        uint32_t on[Q];
        pull_offsets(d, x, y, on);
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const uint8_t t = type_of(in[src_slab(i, z, zm, zp) * d.nxy + on[i]]);
            if (t) sm |= 1u << i;
            if (t == MOVING) mm |= 1u << i;
        }
        if (sm) r |= NEAR_WALL;
        if (mm) r |= NEAR_MOVING;
        if (v >= 3) {
            r |= ONSITE_NODE;
            if (v == 4) r |= ONSITE_MOVING;
            if (!onsite_pattern_ok(sm)) atomicOr(bad, 1);
        }
    }
    out[c] = r;
    smask[c] = sm;
    mmask[c] = mm;
    const uint64_t near = __builtin_amdgcn_ballot_w64(fl == 0 && sm != 0u);
    const uint64_t fluid = __builtin_amdgcn_ballot_w64(fl == 0);
    const uint64_t active = __builtin_amdgcn_read_exec();
    if (__lane_id() == (unsigned)__builtin_ctzll(active)) {
        if (near) atomicAdd(&counts[0], (unsigned)__builtin_popcountll(near));
        if (fluid) atomicAdd(&counts[1], (unsigned)__builtin_popcountll(fluid));
    }
}

// Bandwidth probe: one 16-byte chunk per work-item (src and dst 16-byte
// aligned), load and store both non-temporal: the fastest plain copy
// measured on MI355X (2 GiB of random data: 6.46 TB/s, against 6.28 with
// only the store hinted and 6.16 with neither; two or more chunks per
// work-item were slower). The work-item after the last whole chunk copies
// the 0-3 remaining floats.
__global__ __launch_bounds__(256) void k_copy(const float* __restrict__ src, float* __restrict__ dst,
                                              size_t n)
{
    using F4 = typename V4<float>::t;
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t n4 = n / 4;
    if (k < n4) {
        __builtin_nontemporal_store(__builtin_nontemporal_load(reinterpret_cast<const F4*>(src) + k),
                                    reinterpret_cast<F4*>(dst) + k);
    } else if (k == n4) {
        for (size_t e = 4 * n4; e < n; ++e) dst[e] = src[e];
    }
}

// ------------------------------- dispatch ----------------------------------

// While t_resolve is set (resolve_step_kernel), the step dispatch records the
// kernel it would launch instead of launching it.
static thread_local const void** t_resolve = nullptr;
#define STEP_LAUNCH(K, GRID, BLOCK, SHMEM, STREAM, ...)                         \
    do {                                                                      \
        if (t_resolve) *t_resolve = reinterpret_cast<const void*>(&K);        \
        else hipLaunchKernelGGL(K, GRID, BLOCK, SHMEM, STREAM, __VA_ARGS__);  \
    } while (0)

template <class St, int FM, bool ONSITE>
static hipError_t step_fm(int pattern, int parity, bool collide, void* a, void* b,
                          const uint8_t* flags, const uint32_t* sm, const uint32_t* mm, const float* ff,
                          const StepArgs& args, const Launch& L, float* rho, float* u)
{
    using T = typename St::raw_t;
    T* A = static_cast<T*>(a);
    T* B = static_cast<T*>(b);
    if (pattern == 0) {
        if (collide && rho)
            STEP_LAUNCH((k_step_ab<St, FM, true, true, ONSITE>), L.grid, L.block, L.shmem, L.stream, A, B, flags, sm, mm, ff, args, rho, u);
        else if (collide)
            STEP_LAUNCH((k_step_ab<St, FM, true, false, ONSITE>), L.grid, L.block, L.shmem, L.stream, A, B, flags, sm, mm, ff, args, rho, u);
        else
            STEP_LAUNCH((k_step_ab<St, FORCE_NONE, false, false, false>), L.grid, L.block, L.shmem, L.stream, A, B, flags, sm, mm, ff, args, rho, u);
    } else if (parity == 0) {
        if (collide)
            STEP_LAUNCH((k_step_aa0<St, FM, true, ONSITE>), L.grid, L.block, L.shmem, L.stream, A, flags, sm, mm, ff, args);
        else
            STEP_LAUNCH((k_step_aa0<St, FORCE_NONE, false, false>), L.grid, L.block, L.shmem, L.stream, A, flags, sm, mm, ff, args);
    } else {
        if (collide)
            STEP_LAUNCH((k_step_aa1<St, FM, true, ONSITE>), L.grid, L.block, L.shmem, L.stream, A, flags, sm, mm, ff, args);
        else
            STEP_LAUNCH((k_step_aa1<St, FORCE_NONE, false, false>), L.grid, L.block, L.shmem, L.stream, A, flags, sm, mm, ff, args);
    }
    return hipGetLastError();
}

template <class St, bool ONSITE>
static hipError_t step_st(int pattern, int parity, bool collide, int fm, void* a, void* b,
                          const uint8_t* flags, const uint32_t* sm, const uint32_t* mm, const float* ff,
                          const StepArgs& args, const Launch& L, float* rho, float* u)
{
    switch (fm) {
    case FORCE_UNIFORM: return step_fm<St, FORCE_UNIFORM, ONSITE>(pattern, parity, collide, a, b, flags, sm, mm, ff, args, L, rho, u);
    case FORCE_FIELD: return step_fm<St, FORCE_FIELD, ONSITE>(pattern, parity, collide, a, b, flags, sm, mm, ff, args, L, rho, u);
    default: return step_fm<St, FORCE_NONE, ONSITE>(pattern, parity, collide, a, b, flags, sm, mm, ff, args, L, rho, u);
    }
}

template <bool ONSITE>
static hipError_t step_os(int storage, int pattern, int parity, bool collide, int force_mode, void* a,
                          void* b, const uint8_t* flags, const uint32_t* sm, const uint32_t* mm,
                          const float* ffield, const StepArgs& args, const Launch& L, float* rho, float* u)
{
    switch (storage) {
    case 1: return step_st<StF16, ONSITE>(pattern, parity, collide, force_mode, a, b, flags, sm, mm, ffield, args, L, rho, u);
    case 2: return step_st<StBF16, ONSITE>(pattern, parity, collide, force_mode, a, b, flags, sm, mm, ffield, args, L, rho, u);
    default: return step_st<StF32, ONSITE>(pattern, parity, collide, force_mode, a, b, flags, sm, mm, ffield, args, L, rho, u);
    }
}

hipError_t launch_step(int storage, int pattern, int parity, bool collide, int force_mode, void* a,
                       void* b, const uint8_t* flags, const uint32_t* smask, const uint32_t* mmask,
                       const float* ffield, const StepArgs& args, const Launch& L, float* rho, float* u,
                       bool onsite)
{
    return (onsite && collide)
               ? step_os<true>(storage, pattern, parity, collide, force_mode, a, b, flags, smask, mmask, ffield, args, L, rho, u)
               : step_os<false>(storage, pattern, parity, collide, force_mode, a, b, flags, smask, mmask, ffield, args, L, rho, u);
}

template <class St, int FM, int VW, bool ONSITE, bool FLAT>
static hipError_t stepv_grid(bool collide, void* a, void* b, const uint8_t* flags, const uint32_t* sm,
                             const uint32_t* mm, const float* ff, const StepArgs& args, const Launch& L,
                             float* rho, float* u)
{
    using B = typename St::bits_t;
    const B* A = static_cast<const B*>(a);
    B* Bp = static_cast<B*>(b);
    constexpr bool CAN_EARLY = sizeof(B) == 4 && !ONSITE;
    if (collide && rho)
        STEP_LAUNCH((k_step_abv<St, FM, true, VW, true, ONSITE, FLAT, false>), L.grid, L.block, L.shmem, L.stream, A, Bp, flags, sm, mm, ff, args, rho, u);
    else if (collide && CAN_EARLY && args.early)
        STEP_LAUNCH((k_step_abv<St, FM, true, VW, false, ONSITE, FLAT, CAN_EARLY>), L.grid, L.block, L.shmem, L.stream, A, Bp, flags, sm, mm, ff, args, rho, u);
    else if (collide)
        STEP_LAUNCH((k_step_abv<St, FM, true, VW, false, ONSITE, FLAT, false>), L.grid, L.block, L.shmem, L.stream, A, Bp, flags, sm, mm, ff, args, rho, u);
    else
        STEP_LAUNCH((k_step_abv<St, FORCE_NONE, false, VW, false, false, FLAT, false>), L.grid, L.block, L.shmem, L.stream, A, Bp, flags, sm, mm, ff, args, rho, u);
    return hipGetLastError();
}

template <class St, int FM, int VW, bool ONSITE>
static hipError_t stepv_fm(bool collide, void* a, void* b, const uint8_t* flags, const uint32_t* sm,
                           const uint32_t* mm, const float* ff, const StepArgs& args, const Launch& L,
                           float* rho, float* u)
{
    return args.gx ? stepv_grid<St, FM, VW, ONSITE, true>(collide, a, b, flags, sm, mm, ff, args, L, rho, u)
                   : stepv_grid<St, FM, VW, ONSITE, false>(collide, a, b, flags, sm, mm, ff, args, L, rho, u);
}

template <class St, int VW, bool ONSITE>
static hipError_t stepv_st(bool collide, int fm, void* a, void* b, const uint8_t* flags, const uint32_t* sm,
                           const uint32_t* mm, const float* ff, const StepArgs& args, const Launch& L,
                           float* rho, float* u)
{
    switch (fm) {
    case FORCE_UNIFORM: return stepv_fm<St, FORCE_UNIFORM, VW, ONSITE>(collide, a, b, flags, sm, mm, ff, args, L, rho, u);
    case FORCE_FIELD: return stepv_fm<St, FORCE_FIELD, VW, ONSITE>(collide, a, b, flags, sm, mm, ff, args, L, rho, u);
    default: return stepv_fm<St, FORCE_NONE, VW, ONSITE>(collide, a, b, flags, sm, mm, ff, args, L, rho, u);
    }
}

bool vector_width_ok(int storage, int vw) { return vw == 4 || (vw == 8 && storage != 0); }

template <bool ONSITE>
static hipError_t stepv_os(int storage, int vw, bool collide, int force_mode, void* a, void* b,
                           const uint8_t* flags, const uint32_t* smask, const uint32_t* mmask,
                           const float* ffield, const StepArgs& args, const Launch& L, float* rho, float* u)
{
    switch (storage * 16 + vw) {
    case 1 * 16 + 8: return stepv_st<StF16, 8, ONSITE>(collide, force_mode, a, b, flags, smask, mmask, ffield, args, L, rho, u);
    case 1 * 16 + 4: return stepv_st<StF16, 4, ONSITE>(collide, force_mode, a, b, flags, smask, mmask, ffield, args, L, rho, u);
    case 2 * 16 + 8: return stepv_st<StBF16, 8, ONSITE>(collide, force_mode, a, b, flags, smask, mmask, ffield, args, L, rho, u);
    case 2 * 16 + 4: return stepv_st<StBF16, 4, ONSITE>(collide, force_mode, a, b, flags, smask, mmask, ffield, args, L, rho, u);
    case 0 * 16 + 4: return stepv_st<StF32, 4, ONSITE>(collide, force_mode, a, b, flags, smask, mmask, ffield, args, L, rho, u);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step_abv(int storage, int vw, bool collide, int force_mode, void* a, void* b,
                           const uint8_t* flags, const uint32_t* smask, const uint32_t* mmask,
                           const float* ffield, const StepArgs& args, const Launch& L, float* rho, float* u,
                           bool onsite)
{
    return (onsite && collide)
               ? stepv_os<true>(storage, vw, collide, force_mode, a, b, flags, smask, mmask, ffield, args, L, rho, u)
               : stepv_os<false>(storage, vw, collide, force_mode, a, b, flags, smask, mmask, ffield, args, L, rho, u);
}

hipError_t launch_mark_near_wall(const uint8_t* in, uint8_t* out, uint32_t* smask, uint32_t* mmask, int* bad,
                                 unsigned* counts, const Dims& d, const Launch& L)
{
    hipLaunchKernelGGL(k_mark_near_wall, L.grid, L.block, 0, L.stream, in, out, smask, mmask, bad, counts, d);
    return hipGetLastError();
}

template <class St>
static hipError_t init_st(void* f, const float* rho, const float* u, const Dims& d, const Launch& L)
{
    hipLaunchKernelGGL((k_init_eq<St>), L.grid, L.block, 0, L.stream,
                       static_cast<typename St::raw_t*>(f), rho, u, d);
    return hipGetLastError();
}

hipError_t launch_init_eq(int storage, void* f, const float* rho, const float* u, const Dims& d,
                          const Launch& L)
{
    switch (storage) {
    case 1: return init_st<StF16>(f, rho, u, d, L);
    case 2: return init_st<StBF16>(f, rho, u, d, L);
    default: return init_st<StF32>(f, rho, u, d, L);
    }
}

template <class St>
static hipError_t get_st(int layout, const void* f, const uint8_t* flags, float* out, const Dims& d,
                         const Launch& L)
{
    using T = typename St::raw_t;
    if (layout)
        hipLaunchKernelGGL((k_get<St, 1>), L.grid, L.block, 0, L.stream, static_cast<const T*>(f), flags, out, d);
    else
        hipLaunchKernelGGL((k_get<St, 0>), L.grid, L.block, 0, L.stream, static_cast<const T*>(f), flags, out, d);
    return hipGetLastError();
}

hipError_t launch_get(int storage, int layout, const void* f, const uint8_t* flags, float* out,
                      const Dims& d, const Launch& L)
{
    switch (storage) {
    case 1: return get_st<StF16>(layout, f, flags, out, d, L);
    case 2: return get_st<StBF16>(layout, f, flags, out, d, L);
    default: return get_st<StF32>(layout, f, flags, out, d, L);
    }
}

template <class St>
static hipError_t set_st(void* f, const float* in, const Dims& d, const Launch& L)
{
    hipLaunchKernelGGL((k_set<St>), L.grid, L.block, 0, L.stream, static_cast<typename St::raw_t*>(f), in, d);
    return hipGetLastError();
}

hipError_t launch_set(int storage, void* f, const float* in, const Dims& d, const Launch& L)
{
    switch (storage) {
    case 1: return set_st<StF16>(f, in, d, L);
    case 2: return set_st<StBF16>(f, in, d, L);
    default: return set_st<StF32>(f, in, d, L);
    }
}

template <class St, int LAYOUT>
static hipError_t macros_l(int fm, const void* f, const uint8_t* flags, const float* ff, float* rho,
                           float* u, const StepArgs& a, const Launch& L)
{
    using T = typename St::raw_t;
    const T* F = static_cast<const T*>(f);
    switch (fm) {
    case FORCE_UNIFORM:
        hipLaunchKernelGGL((k_macros<St, LAYOUT, FORCE_UNIFORM>), L.grid, L.block, 0, L.stream, F, flags, ff, rho, u, a);
        break;
    case FORCE_FIELD:
        hipLaunchKernelGGL((k_macros<St, LAYOUT, FORCE_FIELD>), L.grid, L.block, 0, L.stream, F, flags, ff, rho, u, a);
        break;
    default:
        hipLaunchKernelGGL((k_macros<St, LAYOUT, FORCE_NONE>), L.grid, L.block, 0, L.stream, F, flags, ff, rho, u, a);
    }
    return hipGetLastError();
}

template <class St>
static hipError_t macros_st(int layout, int fm, const void* f, const uint8_t* flags, const float* ff,
                            float* rho, float* u, const StepArgs& a, const Launch& L)
{
    return layout ? macros_l<St, 1>(fm, f, flags, ff, rho, u, a, L)
                  : macros_l<St, 0>(fm, f, flags, ff, rho, u, a, L);
}

hipError_t launch_macros(int storage, int layout, int fm, const void* f, const uint8_t* flags,
                         const float* ff, float* rho, float* u, const StepArgs& a, const Launch& L)
{
    switch (storage) {
    case 1: return macros_st<StF16>(layout, fm, f, flags, ff, rho, u, a, L);
    case 2: return macros_st<StBF16>(layout, fm, f, flags, ff, rho, u, a, L);
    default: return macros_st<StF32>(layout, fm, f, flags, ff, rho, u, a, L);
    }
}

template <class St>
static hipError_t finite_st(int layout, const void* f, const uint8_t* flags, int* flag, const Dims& d,
                            const Launch& L)
{
    using T = typename St::raw_t;
    if (layout)
        hipLaunchKernelGGL((k_check_finite<St, 1>), L.grid, L.block, 0, L.stream, static_cast<const T*>(f), flags, flag, d);
    else
        hipLaunchKernelGGL((k_check_finite<St, 0>), L.grid, L.block, 0, L.stream, static_cast<const T*>(f), flags, flag, d);
    return hipGetLastError();
}

hipError_t launch_check_finite(int storage, int layout, const void* f, const uint8_t* flags, int* flag,
                               const Dims& d, const Launch& L)
{
    switch (storage) {
    case 1: return finite_st<StF16>(layout, f, flags, flag, d, L);
    case 2: return finite_st<StBF16>(layout, f, flags, flag, d, L);
    default: return finite_st<StF32>(layout, f, flags, flag, d, L);
    }
}

hipError_t resolve_step_kernel(bool vector, int storage, int pattern, int parity, int vw, bool collide,
                               int force_mode, void* a, void* b, const uint8_t* flags, const uint32_t* smask,
                               const uint32_t* mmask, const float* ffield, const StepArgs& args, const Launch& L,
                               bool onsite, const void** kernel)
{
    *kernel = nullptr;
    t_resolve = kernel;
    const hipError_t e = vector ? launch_step_abv(storage, vw, collide, force_mode, a, b, flags, smask, mmask,
                                                  ffield, args, L, nullptr, nullptr, onsite)
                                : launch_step(storage, pattern, parity, collide, force_mode, a, b, flags, smask,
                                              mmask, ffield, args, L, nullptr, nullptr, onsite);
    t_resolve = nullptr;
    return *kernel ? hipSuccess : (e != hipSuccess ? e : hipErrorInvalidValue);
}

hipError_t launch_copy(const float* src, float* dst, size_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const size_t blocks = (n / 4 + 1 + 255) / 256;   // whole chunks plus the tail work-item
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

}  // namespace lbmk

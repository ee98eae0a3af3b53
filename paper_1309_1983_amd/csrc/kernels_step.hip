// Forward kernels for gfx950: the fused pull step (Mawson & Revell, Section 4.2,
// Algorithm 3) in the two-array (AB) pattern and the single-array (AA)
// pattern, plus the auxiliary per-cell kernels (initialisation, macroscopic
// output, state copy in/out, finite check, flag preprocessing, copy probe).
//
// One work-item per lattice point, work-groups x-dominant (Section 6). The
// population arrays are structure-of-arrays planes (Section 4.1): the 19
// loads of a wave are each one contiguous 64-element run, shifted by one
// element for the ten directions with e_x != 0; stores are aligned. The
// shifted runs straddle one extra cache line that the neighbouring wave of
// the same row also reads, so the re-read is served from L2 and HBM traffic
// stays at one read and one write per population.
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

// Decode, add moving-wall terms, collide. h ends as post-collision offsets.
template <class St, int FM>
__device__ __forceinline__ void decode_collide(const typename St::raw_t raw[Q], uint32_t mwmask,
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
    bgk_collide<FM != FORCE_NONE>(h, a.omega, a.cF, Fx, Fy, Fz);
}

// ---------------------------------------------------------------------------
// AB pull step: gather from x - e_i in `src`, bounce back at solid
// neighbours, collide, store aligned into `dst`.
// ---------------------------------------------------------------------------
template <class St, int FM, bool COLLIDE>
__global__ __launch_bounds__(1024) void k_step_ab(const typename St::raw_t* __restrict__ src,
                                                  typename St::raw_t* __restrict__ dst,
                                                  const uint8_t* __restrict__ flags,
                                                  const float* __restrict__ ff, StepArgs a)
{
    using T = typename St::raw_t;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= a.d.nx || y >= a.d.ny) return;
    const uint32_t c = ((uint32_t)z * (uint32_t)a.d.ny + (uint32_t)y) * (uint32_t)a.d.nx + (uint32_t)x;
    const uint8_t fl = flags[c];
    if (fl & TYPE_MASK) return;

    uint32_t nb[Q];
    pull_sources(a.d, x, y, z, c, nb);
    const size_t N = a.d.N;
    T raw[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) raw[i] = ld(src + i * N, nb[i]);

    uint32_t mwmask = 0;
    if (fl & NEAR_WALL) {
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const uint8_t nf = flags[nb[i]];
            if (nf & TYPE_MASK) {
                raw[i] = ld(src + OPP[i] * N, c);
                if (nf & MOVING) mwmask |= 1u << i;
            }
        }
    }

    if (!COLLIDE) {
#pragma unroll
        for (int i = 0; i < Q; ++i) st(dst + i * N, c, raw[i]);
        return;
    }
    float h[Q];
    decode_collide<St, FM>(raw, mwmask, a, ff, c, h);
#pragma unroll
    for (int i = 0; i < Q; ++i) st(dst + i * N, c, St::enc(h[i], i));
}

// ---------------------------------------------------------------------------
// AB pull step, four consecutive x-cells per work-item (nx % 4 == 0).
// Each direction is one 4-element access: aligned for e_x = 0, shifted by one
// element for e_x = +-1 (a shifted wave access spans 9 instead of 8 cache
// lines; the extra line is the neighbouring work-item's and stays in L2).
// Row ends are clamped into the row and the periodic wrap element is loaded
// separately, only when the end cell is fluid. Near-wall cells take the
// bounced values s_opp(i)(x) through the precomputed solid-neighbour mask.
// Solid cells inside a work-item's quad are written as the rest state.
// Per fluid cell the arithmetic is the same as the one-cell kernel's.
// ---------------------------------------------------------------------------
template <class St, int FM, bool COLLIDE>
__global__ __launch_bounds__(256) void k_step_ab4(const typename St::bits_t* __restrict__ src,
                                                  typename St::bits_t* __restrict__ dst,
                                                  const uint8_t* __restrict__ flags,
                                                  const uint32_t* __restrict__ smask,
                                                  const uint32_t* __restrict__ mmask,
                                                  const float* __restrict__ ff, StepArgs a)
{
    using B = typename St::bits_t;
    using Vt = typename V4<B>::t;
    const Dims& d = a.d;
    const int x0 = 4 * (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x0 >= d.nx || y >= d.ny) return;
    const uint32_t nx = (uint32_t)d.nx;
    const uint32_t row = ((uint32_t)z * (uint32_t)d.ny + (uint32_t)y) * nx;
    const uint32_t c0 = row + (uint32_t)x0;
    const uint32_t fl4 = *reinterpret_cast<const uint32_t*>(flags + c0);
    const uint32_t solid4 = (fl4 | (fl4 >> 1)) & 0x01010101u;   // byte j: cell j solid
    if (solid4 == 0x01010101u) return;

    const uint32_t oym = (y == 0) ? (uint32_t)(d.ny - 1) * nx : (uint32_t)0 - nx;
    const uint32_t oyp = (y == d.ny - 1) ? (uint32_t)(1 - d.ny) * nx : nx;
    const uint32_t ozm = (z == 0) ? (uint32_t)(d.nz - 1) * d.nxy : (uint32_t)0 - d.nxy;
    const uint32_t ozp = (z == d.nz - 1) ? (uint32_t)(1 - d.nz) * d.nxy : d.nxy;
    const bool wl = x0 == 0;
    const bool wr = (uint32_t)x0 + 4 == nx;
    const uint32_t xm = wl ? (uint32_t)x0 : (uint32_t)x0 - 1;   // quad start for e_x = +1
    const uint32_t xp = wr ? (uint32_t)x0 : (uint32_t)x0 + 1;   // quad start for e_x = -1
    const size_t N = d.N;

    Vt q[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        uint32_t r = row;
        if (EY[i] == 1) r += oym; else if (EY[i] == -1) r += oyp;
        if (EZ[i] == 1) r += ozm; else if (EZ[i] == -1) r += ozp;
        const uint32_t xs = EX[i] == 1 ? xm : (EX[i] == -1 ? xp : (uint32_t)x0);
        q[i] = ld4(src + i * N, r + xs);
    }

    // periodic wrap in x at the two row ends
    const bool fixl = wl && !(solid4 & 0x1u);
    const bool fixr = wr && !(solid4 & 0x01000000u);
    B wrapv[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) wrapv[i] = B(0);
    if (fixl || fixr) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            if (EX[i] == 0) continue;
            uint32_t r = row;
            if (EY[i] == 1) r += oym; else if (EY[i] == -1) r += oyp;
            if (EZ[i] == 1) r += ozm; else if (EZ[i] == -1) r += ozp;
            if (EX[i] == 1 && fixl) wrapv[i] = ld(src + i * N, r + nx - 1);
            if (EX[i] == -1 && fixr) wrapv[i] = ld(src + i * N, r);
        }
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const Vt v = q[i];
        if (EX[i] == 1 && wl) q[i] = Vt{wrapv[i], v.x, v.y, v.z};
        if (EX[i] == -1 && wr) q[i] = Vt{v.y, v.z, v.w, wrapv[i]};
    }

    // bounce-back at solid neighbours (cells flagged NEAR_WALL)
    uint32_t mm[4] = {0u, 0u, 0u, 0u};
    if (fl4 & 0x04040404u) {
        const typename V4<uint32_t>::t sm = ld4(smask, c0);
        if (COLLIDE && (fl4 & 0x08080808u)) {
            const typename V4<uint32_t>::t m = ld4(mmask, c0);
            mm[0] = m.x; mm[1] = m.y; mm[2] = m.z; mm[3] = m.w;
        }
        const uint32_t any = sm.x | sm.y | sm.z | sm.w;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            if ((any >> i) & 1u) {
                const Vt bb = ld4(src + OPP[i] * N, c0);
                Vt v = q[i];
                if ((sm.x >> i) & 1u) v.x = bb.x;
                if ((sm.y >> i) & 1u) v.y = bb.y;
                if ((sm.z >> i) & 1u) v.z = bb.z;
                if ((sm.w >> i) & 1u) v.w = bb.w;
                q[i] = v;
            }
        }
    }

    if (COLLIDE) {
        float F[3][4];
        if (FM == FORCE_FIELD) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const typename V4<float>::t f = ld4(ff + k * N, c0);
                F[k][0] = f.x; F[k][1] = f.y; F[k][2] = f.z; F[k][3] = f.w;
            }
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                F[0][j] = FM == FORCE_UNIFORM ? a.Fx : 0.0f;
                F[1][j] = FM == FORCE_UNIFORM ? a.Fy : 0.0f;
                F[2][j] = FM == FORCE_UNIFORM ? a.Fz : 0.0f;
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            float h[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                h[i] = St::off_b(q[i][j], i);
                if (i > 0 && ((mm[j] >> i) & 1u)) h[i] = h[i] + a.mw[i];
            }
            bgk_collide<FM != FORCE_NONE>(h, a.omega, a.cF, F[0][j], F[1][j], F[2][j]);
            const bool sol = (solid4 >> (8 * j)) & 1u;
#pragma unroll
            for (int i = 0; i < Q; ++i) q[i][j] = St::enc_b(sol ? 0.0f : h[i], i);
        }
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) st4(dst + i * N, c0, q[i]);
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
template <class St, int FM, bool COLLIDE>
__global__ __launch_bounds__(1024) void k_step_aa0(typename St::raw_t* f,
                                                   const uint8_t* __restrict__ flags,
                                                   const float* __restrict__ ff, StepArgs a)
{
    using T = typename St::raw_t;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= a.d.nx || y >= a.d.ny) return;
    const uint32_t c = ((uint32_t)z * (uint32_t)a.d.ny + (uint32_t)y) * (uint32_t)a.d.nx + (uint32_t)x;
    const uint8_t fl = flags[c];
    if (fl & TYPE_MASK) return;

    uint32_t nb[Q];
    pull_sources(a.d, x, y, z, c, nb);
    const size_t N = a.d.N;
    T raw[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) raw[i] = ld(f + i * N, nb[i]);

    uint32_t solid = 0, mwmask = 0;
    if (fl & NEAR_WALL) {
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const uint8_t nf = flags[nb[i]];
            if (nf & TYPE_MASK) {
                solid |= 1u << i;
                raw[i] = ld(f + OPP[i] * N, c);
                if (nf & MOVING) mwmask |= 1u << i;
            }
        }
    }

    float h[Q];
    if (COLLIDE) {
        decode_collide<St, FM>(raw, mwmask, a, ff, c, h);
    }
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        const int o = OPP[j];
        const T v = COLLIDE ? St::enc(h[j], j) : raw[j];
        if ((solid >> o) & 1u) st(f + j * N, c, v);
        else st(f + o * N, nb[o], v);
    }
}

template <class St, int FM, bool COLLIDE>
__global__ __launch_bounds__(1024) void k_step_aa1(typename St::raw_t* f,
                                                   const uint8_t* __restrict__ flags,
                                                   const float* __restrict__ ff, StepArgs a)
{
    using T = typename St::raw_t;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= a.d.nx || y >= a.d.ny) return;
    const uint32_t c = ((uint32_t)z * (uint32_t)a.d.ny + (uint32_t)y) * (uint32_t)a.d.nx + (uint32_t)x;
    const uint8_t fl = flags[c];
    if (fl & TYPE_MASK) return;

    const size_t N = a.d.N;
    T raw[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) raw[i] = ld(f + OPP[i] * N, c);

    uint32_t mwmask = 0;
    if (COLLIDE && (fl & NEAR_WALL)) {
        uint32_t nb[Q];
        pull_sources(a.d, x, y, z, c, nb);
#pragma unroll
        for (int i = 1; i < Q; ++i)
            if ((flags[nb[i]] & TYPE_MASK) == MOVING) mwmask |= 1u << i;
    }
    if (!COLLIDE) {
#pragma unroll
        for (int i = 0; i < Q; ++i) st(f + i * N, c, raw[i]);
        return;
    }
    float h[Q];
    decode_collide<St, FM>(raw, mwmask, a, ff, c, h);
#pragma unroll
    for (int i = 0; i < Q; ++i) st(f + i * N, c, St::enc(h[i], i));
}

// ---------------------------------------------------------------------------
// Stored state of one cell in natural order (s_j(x), j = 0..18), for either
// layout. Layout 1 (AA after an odd number of steps): s_j(x) is at
// [opp(j)][x + e_j] when x + e_j is fluid, else at [j][x].
// ---------------------------------------------------------------------------
template <class St, int LAYOUT>
__device__ __forceinline__ void load_state(const typename St::raw_t* __restrict__ f,
                                           const uint8_t* __restrict__ flags, const Dims& d, int x,
                                           int y, int z, uint32_t c, uint8_t fl,
                                           typename St::raw_t raw[Q])
{
    const size_t N = d.N;
    if (LAYOUT == 0 || (fl & TYPE_MASK)) {
#pragma unroll
        for (int j = 0; j < Q; ++j) raw[j] = ld(f + j * N, c);
        return;
    }
    uint32_t nb[Q];
    pull_sources(d, x, y, z, c, nb);
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        const int o = OPP[j];
        const bool wall = (fl & NEAR_WALL) && (flags[nb[o]] & TYPE_MASK);
        raw[j] = wall ? ld(f + j * N, c) : ld(f + o * N, nb[o]);
    }
}

#define CELL_PROLOGUE                                                                          \
    const int x = blockIdx.x * blockDim.x + threadIdx.x;                                       \
    const int y = blockIdx.y * blockDim.y + threadIdx.y;                                       \
    const int z = blockIdx.z;                                                                  \
    if (x >= d.nx || y >= d.ny) return;                                                        \
    const uint32_t c = ((uint32_t)z * (uint32_t)d.ny + (uint32_t)y) * (uint32_t)d.nx + (uint32_t)x;

template <class St, int LAYOUT>
__global__ __launch_bounds__(1024) void k_get(const typename St::raw_t* __restrict__ f,
                                              const uint8_t* __restrict__ flags,
                                              float* __restrict__ out, Dims d)
{
    CELL_PROLOGUE
    typename St::raw_t raw[Q];
    load_state<St, LAYOUT>(f, flags, d, x, y, z, c, flags[c], raw);
#pragma unroll
    for (int j = 0; j < Q; ++j) out[(size_t)j * d.N + c] = St::plain(raw[j], j);
}

template <class St>
__global__ __launch_bounds__(1024) void k_set(typename St::raw_t* __restrict__ f,
                                              const float* __restrict__ in, Dims d)
{
    CELL_PROLOGUE
#pragma unroll
    for (int j = 0; j < Q; ++j) st(f + j * (size_t)d.N, c, St::from_plain(in[(size_t)j * d.N + c], j));
}

template <class St>
__global__ __launch_bounds__(1024) void k_init_eq(typename St::raw_t* __restrict__ f,
                                                  const float* __restrict__ rho,
                                                  const float* __restrict__ u, Dims d)
{
    CELL_PROLOGUE
    Macro m;
    m.rho = rho ? rho[c] : 1.0f;
    m.drho = m.rho - 1.0f;
    m.ux = u ? u[c] : 0.0f;
    m.uy = u ? u[(size_t)d.N + c] : 0.0f;
    m.uz = u ? u[2 * (size_t)d.N + c] : 0.0f;
    const float A = eq_A(m);
#pragma unroll
    for (int j = 0; j < Q; ++j) st(f + j * (size_t)d.N, c, St::enc(heq(j, m, A), j));
}

template <class St, int LAYOUT, int FM>
__global__ __launch_bounds__(1024) void k_macros(const typename St::raw_t* __restrict__ f,
                                                 const uint8_t* __restrict__ flags,
                                                 const float* __restrict__ ff,
                                                 float* __restrict__ rho, float* __restrict__ u,
                                                 StepArgs a)
{
    const Dims& d = a.d;
    CELL_PROLOGUE
    const uint8_t fl = flags[c];
    const size_t N = d.N;
    if (fl & TYPE_MASK) {
        if (rho) rho[c] = 0.0f;
        if (u) { u[c] = 0.0f; u[N + c] = 0.0f; u[2 * N + c] = 0.0f; }
        return;
    }
    typename St::raw_t raw[Q];
    load_state<St, LAYOUT>(f, flags, d, x, y, z, c, fl, raw);
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
    CELL_PROLOGUE
    const uint8_t fl = flags[c];
    if (fl & TYPE_MASK) return;
    typename St::raw_t raw[Q];
    load_state<St, LAYOUT>(f, flags, d, x, y, z, c, fl, raw);
    bool ok = true;
#pragma unroll
    for (int j = 0; j < Q; ++j) ok = ok && isfinite(St::off(raw[j], j));
    if (!ok) atomicOr(flag, 1);
}

__global__ __launch_bounds__(1024) void k_mark_near_wall(const uint8_t* __restrict__ in,
                                                         uint8_t* __restrict__ out,
                                                         uint32_t* __restrict__ smask,
                                                         uint32_t* __restrict__ mmask, Dims d)
{
    CELL_PROLOGUE
    const uint8_t fl = in[c] & TYPE_MASK;
    uint8_t r = fl;
    uint32_t sm = 0, mm = 0;
    if (fl == 0) {
        uint32_t nb[Q];
        pull_sources(d, x, y, z, c, nb);
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const uint8_t t = in[nb[i]] & TYPE_MASK;
            if (t) sm |= 1u << i;
            if (t == MOVING) mm |= 1u << i;
        }
        if (sm) r |= NEAR_WALL;
        if (mm) r |= NEAR_MOVING;
    }
    out[c] = r;
    smask[c] = sm;
    mmask[c] = mm;
}

__global__ __launch_bounds__(256) void k_copy(const float* __restrict__ src, float* __restrict__ dst,
                                              size_t n)
{
    const size_t k = 4 * ((size_t)blockIdx.x * blockDim.x + threadIdx.x);
    if (k + 4 <= n) {
        *reinterpret_cast<typename V4<float>::t*>(dst + k) = *reinterpret_cast<const typename V4<float>::t*>(src + k);
    } else {
        for (size_t e = k; e < n; ++e) dst[e] = src[e];
    }
}

// ------------------------------- dispatch ----------------------------------

template <class St, int FM>
static hipError_t step_fm(int pattern, int parity, bool collide, void* a, void* b,
                          const uint8_t* flags, const float* ff, const StepArgs& args,
                          const Launch& L)
{
    using T = typename St::raw_t;
    T* A = static_cast<T*>(a);
    T* B = static_cast<T*>(b);
    if (pattern == 0) {
        if (collide)
            hipLaunchKernelGGL((k_step_ab<St, FM, true>), L.grid, L.block, 0, L.stream, A, B, flags, ff, args);
        else
            hipLaunchKernelGGL((k_step_ab<St, FORCE_NONE, false>), L.grid, L.block, 0, L.stream, A, B, flags, ff, args);
    } else if (parity == 0) {
        if (collide)
            hipLaunchKernelGGL((k_step_aa0<St, FM, true>), L.grid, L.block, 0, L.stream, A, flags, ff, args);
        else
            hipLaunchKernelGGL((k_step_aa0<St, FORCE_NONE, false>), L.grid, L.block, 0, L.stream, A, flags, ff, args);
    } else {
        if (collide)
            hipLaunchKernelGGL((k_step_aa1<St, FM, true>), L.grid, L.block, 0, L.stream, A, flags, ff, args);
        else
            hipLaunchKernelGGL((k_step_aa1<St, FORCE_NONE, false>), L.grid, L.block, 0, L.stream, A, flags, ff, args);
    }
    return hipGetLastError();
}

template <class St>
static hipError_t step_st(int pattern, int parity, bool collide, int fm, void* a, void* b,
                          const uint8_t* flags, const float* ff, const StepArgs& args,
                          const Launch& L)
{
    switch (fm) {
    case FORCE_UNIFORM: return step_fm<St, FORCE_UNIFORM>(pattern, parity, collide, a, b, flags, ff, args, L);
    case FORCE_FIELD: return step_fm<St, FORCE_FIELD>(pattern, parity, collide, a, b, flags, ff, args, L);
    default: return step_fm<St, FORCE_NONE>(pattern, parity, collide, a, b, flags, ff, args, L);
    }
}

template <class St, int FM>
static hipError_t step4_fm(bool collide, void* a, void* b, const uint8_t* flags, const uint32_t* sm,
                           const uint32_t* mm, const float* ff, const StepArgs& args, const Launch& L)
{
    using B = typename St::bits_t;
    const B* A = static_cast<const B*>(a);
    B* Bp = static_cast<B*>(b);
    if (collide)
        hipLaunchKernelGGL((k_step_ab4<St, FM, true>), L.grid, L.block, 0, L.stream, A, Bp, flags, sm, mm, ff, args);
    else
        hipLaunchKernelGGL((k_step_ab4<St, FORCE_NONE, false>), L.grid, L.block, 0, L.stream, A, Bp, flags, sm, mm, ff, args);
    return hipGetLastError();
}

template <class St>
static hipError_t step4_st(bool collide, int fm, void* a, void* b, const uint8_t* flags, const uint32_t* sm,
                           const uint32_t* mm, const float* ff, const StepArgs& args, const Launch& L)
{
    switch (fm) {
    case FORCE_UNIFORM: return step4_fm<St, FORCE_UNIFORM>(collide, a, b, flags, sm, mm, ff, args, L);
    case FORCE_FIELD: return step4_fm<St, FORCE_FIELD>(collide, a, b, flags, sm, mm, ff, args, L);
    default: return step4_fm<St, FORCE_NONE>(collide, a, b, flags, sm, mm, ff, args, L);
    }
}

hipError_t launch_step_ab4(int storage, bool collide, int force_mode, void* a, void* b, const uint8_t* flags,
                           const uint32_t* smask, const uint32_t* mmask, const float* ffield,
                           const StepArgs& args, const Launch& L)
{
    switch (storage) {
    case 1: return step4_st<StF16>(collide, force_mode, a, b, flags, smask, mmask, ffield, args, L);
    case 2: return step4_st<StBF16>(collide, force_mode, a, b, flags, smask, mmask, ffield, args, L);
    default: return step4_st<StF32>(collide, force_mode, a, b, flags, smask, mmask, ffield, args, L);
    }
}

hipError_t launch_step(int storage, int pattern, int parity, bool collide, int force_mode, void* a,
                       void* b, const uint8_t* flags, const float* ffield, const StepArgs& args,
                       const Launch& L)
{
    switch (storage) {
    case 1: return step_st<StF16>(pattern, parity, collide, force_mode, a, b, flags, ffield, args, L);
    case 2: return step_st<StBF16>(pattern, parity, collide, force_mode, a, b, flags, ffield, args, L);
    default: return step_st<StF32>(pattern, parity, collide, force_mode, a, b, flags, ffield, args, L);
    }
}

hipError_t launch_mark_near_wall(const uint8_t* in, uint8_t* out, uint32_t* smask, uint32_t* mmask,
                                 const Dims& d, const Launch& L)
{
    hipLaunchKernelGGL(k_mark_near_wall, L.grid, L.block, 0, L.stream, in, out, smask, mmask, d);
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

hipError_t launch_copy(const float* src, float* dst, size_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const size_t blocks = ((n + 3) / 4 + 255) / 256;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

}  // namespace lbmk

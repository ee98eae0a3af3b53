// Reverse-time (discrete adjoint) kernels for the FP32 two-array step.
//
// The forward step is s^{t+1} = C(P s^t; F, tau): P is the pull gather with
// bounce-back of Algorithm 3 (Mawson & Revell, Section 4.2) and C the BGK
// collision with Guo forcing (Eqs. (2)-(3), (5)-(7)). With a = dL/ds^{t+1} at
// one cell, the transposed collision Jacobian has the structured form
//   S     = sum_i a_i f^eq_i / rho
//   V_al  = omega rho sum_i a_i w_i [3 e_ial + 9 (e_i.u) e_ial - 3 u_al]
//           + (1 - omega/2) sum_i a_i w_i [-3 F_al + 9 e_ial (e_i.F)]
//   W_be  = sum_i a_i w_i [3 (e_ibe - u_be) + 9 (e_i.u) e_ibe]
//   (J^T a)_j = (1 - omega) a_j + omega S + sum_al V_al (e_jal - u_al) / rho
//   dL/dF_be += V_be / (2 rho) + (1 - omega/2) W_be
//   dL/dtau  += sum_i a_i [(p_i - f^eq_i) + G_i / 2] / tau^2
// and the transposed gather is (P^T b)_j(x) = b_j(x + e_j) if x + e_j is
// fluid, else b_opp(j)(x). One work-item per cell: it gathers a^{t+1}(x)
// from the previous reverse step's b through P^T, re-gathers p = (P s^t)(x),
// and stores b^t(x) = J_C(p)^T a^{t+1}(x); the next reverse step gathers it.
#include "kernels.hpp"

using namespace d3q19;

namespace lbmk {

template <int FM>
__device__ __forceinline__ void force_at(const StepArgs& a, const float* __restrict__ ff, uint32_t c,
                                         float& Fx, float& Fy, float& Fz)
{
    if (FM == FORCE_UNIFORM) {
        Fx = a.Fx; Fy = a.Fy; Fz = a.Fz;
    } else if (FM == FORCE_FIELD) {
        Fx = ff[c]; Fy = ff[(size_t)a.d.N + c]; Fz = ff[2 * (size_t)a.d.N + c];
    } else {
        Fx = Fy = Fz = 0.0f;
    }
}

// Seed: u = (m - F/2)/rho from the post-collision state, du_al/ds_j =
// (e_jal - u_al)/rho, so a_j = (e_j.g - u.g)/rho; direct dL/dF = -g/(2 rho).
template <int FM>
__global__ __launch_bounds__(1024) void k_adj_seed(const float* __restrict__ f,
                                                   const uint8_t* __restrict__ flags,
                                                   const float* __restrict__ ff,
                                                   const float* __restrict__ g,
                                                   float* __restrict__ aout, float* __restrict__ gF,
                                                   StepArgs a)
{
    const Dims& d = a.d;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const uint32_t z = blockIdx.z;
    if (x >= d.nx || y >= d.ny) return;
    const uint32_t o = (uint32_t)y * (uint32_t)d.nx + (uint32_t)x;
    const uint32_t c = z * d.nxy + o;
    const size_t N = d.N;
    if (flags[c] & TYPE_MASK) {
#pragma unroll
        for (int j = 0; j < Q; ++j) st(plane(aout, d, j, z), o, 0.0f);
        gF[c] = 0.0f; gF[N + c] = 0.0f; gF[2 * N + c] = 0.0f;
        return;
    }
    float h[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) h[j] = ld(plane(f, d, j, z), o) - weight(j);
    float Fx, Fy, Fz;
    force_at<FM>(a, ff, c, Fx, Fy, Fz);
    const Macro m = macro_pre<FM != FORCE_NONE>(h, -Fx, -Fy, -Fz);
    const float ir = 1.0f / m.rho;
    const float gx = g[c], gy = g[N + c], gz = g[2 * N + c];
    const float ug = fmaf(m.ux, gx, fmaf(m.uy, gy, m.uz * gz));
#pragma unroll
    for (int j = 0; j < Q; ++j) st(plane(aout, d, j, z), o, (edot(j, gx, gy, gz) - ug) * ir);
    const float h2 = -0.5f * ir;
    gF[c] = gx * h2;
    gF[N + c] = gy * h2;
    gF[2 * N + c] = gz * h2;
}

// Transposed collision Jacobian at one point: av = dL/ds (post-collision),
// h = pre-collision offsets p_i - w_i (moving-wall terms included), force F.
// Returns b = J_C(p)^T av, the force-gradient increment (gx, gy, gz) and the
// tau term sum_i av_i [(p_i - f^eq_i) + G_i/2] / tau^2.
template <bool FORCE>
__device__ __forceinline__ void adj_cell(const float av[Q], const float h[Q], float Fx, float Fy,
                                         float Fz, const StepArgs& a, float inv_tau2, float b[Q],
                                         float& gx, float& gy, float& gz, float& tterm)
{
    const Macro m = macro_pre<FORCE>(h, Fx, Fy, Fz);
    const float A = eq_A(m);
    const float uF = FORCE ? fmaf(m.ux, Fx, fmaf(m.uy, Fy, m.uz * Fz)) : 0.0f;

    float S = 0.0f, A0 = 0.0f;
    float A1x = 0.0f, A1y = 0.0f, A1z = 0.0f;   // sum a w e
    float A2x = 0.0f, A2y = 0.0f, A2z = 0.0f;   // sum a w (e.u) e
    float A3x = 0.0f, A3y = 0.0f, A3z = 0.0f;   // sum a w (e.F) e
    float tt = 0.0f, tg = 0.0f;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const float he = heq(i, m, A);
        S = fmaf(av[i], weight(i) + he, S);
        const float aw = av[i] * weight(i);
        A0 += aw;
        const float eu = edot(i, m.ux, m.uy, m.uz);
        const float awe = aw * eu;
        if (EX[i]) { A1x += EX[i] * aw; A2x += EX[i] * awe; }
        if (EY[i]) { A1y += EY[i] * aw; A2y += EY[i] * awe; }
        if (EZ[i]) { A1z += EZ[i] * aw; A2z += EZ[i] * awe; }
        tt = fmaf(av[i], h[i] - he, tt);
        if (FORCE) {
            const float eF = edot(i, Fx, Fy, Fz);
            const float awF = aw * eF;
            if (EX[i]) A3x += EX[i] * awF;
            if (EY[i]) A3y += EY[i] * awF;
            if (EZ[i]) A3z += EZ[i] * awF;
            tg = fmaf(av[i], guo(i, m, Fx, Fy, Fz, uF), tg);
        }
    }
    const float om = a.omega, cF = a.cF;
    const float ir = 1.0f / m.rho;
    S *= ir;
    const float orho = om * m.rho;
    float Vx = orho * (3.0f * A1x + 9.0f * A2x - 3.0f * m.ux * A0);
    float Vy = orho * (3.0f * A1y + 9.0f * A2y - 3.0f * m.uy * A0);
    float Vz = orho * (3.0f * A1z + 9.0f * A2z - 3.0f * m.uz * A0);
    if (FORCE) {
        Vx = fmaf(cF, 9.0f * A3x - 3.0f * Fx * A0, Vx);
        Vy = fmaf(cF, 9.0f * A3y - 3.0f * Fy * A0, Vy);
        Vz = fmaf(cF, 9.0f * A3z - 3.0f * Fz * A0, Vz);
    }
    const float Vu = fmaf(Vx, m.ux, fmaf(Vy, m.uy, Vz * m.uz));
    const float base = om * S;
    const float oneMinus = 1.0f - om;
#pragma unroll
    for (int j = 0; j < Q; ++j) b[j] = fmaf(oneMinus, av[j], base) + (edot(j, Vx, Vy, Vz) - Vu) * ir;
    const float Wx = 3.0f * A1x - 3.0f * m.ux * A0 + 9.0f * A2x;
    const float Wy = 3.0f * A1y - 3.0f * m.uy * A0 + 9.0f * A2y;
    const float Wz = 3.0f * A1z - 3.0f * m.uz * A0 + 9.0f * A2z;
    const float h2 = 0.5f * ir;
    gx = fmaf(Vx, h2, cF * Wx);
    gy = fmaf(Vy, h2, cF * Wy);
    gz = fmaf(Vz, h2, cF * Wz);
    tterm = fmaf(0.5f, tg, tt) * inv_tau2;
}

// Block sum of per-work-item tau terms in double with a fixed-shape LDS tree
// (any block size, deterministic); thread 0 adds it to this block's slot.
__device__ __forceinline__ void block_tau_sum(double v, double* __restrict__ taupart)
{
    __shared__ double part[1024];
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    const int nthreads = blockDim.x * blockDim.y;
    part[tid] = v;
    __syncthreads();
    int span = 1;
    while (span < nthreads) span <<= 1;
    for (int sh = span >> 1; sh > 0; sh >>= 1) {
        if (tid < sh && tid + sh < nthreads) part[tid] += part[tid + sh];
        __syncthreads();
    }
    if (tid == 0) {
        const size_t blk = (size_t)blockIdx.x + (size_t)gridDim.x * ((size_t)blockIdx.y + (size_t)gridDim.y * blockIdx.z);
        taupart[blk] += part[0];
    }
}

template <int FM, bool DIRECT>
__global__ __launch_bounds__(256) void k_adj_step(const float* __restrict__ s,
                                                   const float* __restrict__ bin,
                                                   float* __restrict__ bout, float* __restrict__ gF,
                                                   double* __restrict__ taupart,
                                                   const uint8_t* __restrict__ flags,
                                                   const float* __restrict__ ff, StepArgs a,
                                                   float inv_tau2)
{
    constexpr bool FORCE = FM != FORCE_NONE;
    const Dims& d = a.d;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const uint32_t z = blockIdx.z;
    const bool inside = x < d.nx && y < d.ny;
    const uint32_t o = inside ? (uint32_t)y * (uint32_t)d.nx + (uint32_t)x : 0u;
    const uint32_t c = z * d.nxy + o;
    const uint8_t fl = inside ? flags[c] : (uint8_t)1;
    float tterm = 0.0f;

    if (!(fl & TYPE_MASK)) {
        const size_t N = d.N;
        const uint32_t zm = wrap_m(z, (uint32_t)d.nz), zp = wrap_p(z, (uint32_t)d.nz);
        uint32_t on[Q];
        pull_offsets(d, x, y, on);
        float av[Q], h[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            // a_i(x) arrives from b_i(x + e_i); x + e_i is the pull source of opp(i)
            av[i] = DIRECT ? ld(plane(bin, d, i, z), o)
                           : ld(plane(bin, d, i, src_slab(OPP[i], z, zm, zp)), on[OPP[i]]);
            h[i] = ld(plane(s, d, i, src_slab(i, z, zm, zp)), on[i]);
        }
        uint32_t mwmask = 0;
        if (fl & NEAR_WALL) {
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const uint8_t nf = flags[src_slab(i, z, zm, zp) * d.nxy + on[i]];
                if (nf & TYPE_MASK) {
                    h[i] = ld(plane(s, d, OPP[i], z), o);
                    if (nf & MOVING) mwmask |= 1u << i;
                }
                // x + e_i solid: the adjoint arrives by the bounced link
                const int k = OPP[i];
                if (!DIRECT && (flags[src_slab(k, z, zm, zp) * d.nxy + on[k]] & TYPE_MASK))
                    av[i] = ld(plane(bin, d, k, z), o);
            }
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            h[i] = h[i] - weight(i);
            if (i > 0 && ((mwmask >> i) & 1u)) h[i] = h[i] + a.mw[i];
        }
        float Fx, Fy, Fz;
        force_at<FM>(a, ff, c, Fx, Fy, Fz);
        float b[Q], gx, gy, gz;
        adj_cell<FORCE>(av, h, Fx, Fy, Fz, a, inv_tau2, b, gx, gy, gz, tterm);
#pragma unroll
        for (int j = 0; j < Q; ++j) st(plane(bout, d, j, z), o, b[j]);
        gF[c] += gx;
        gF[N + c] += gy;
        gF[2 * N + c] += gz;
    }

    block_tau_sum((double)tterm, taupart);
}

// Flag bytes of VW consecutive points as one word.
template <int VW>
struct FlagBytes;
template <>
struct FlagBytes<2> {
    typedef uint16_t t;
    static constexpr uint16_t ones = 0x0101u;
};
template <>
struct FlagBytes<4> {
    typedef uint32_t t;
    static constexpr uint32_t ones = 0x01010101u;
};

// Reverse step with VW consecutive x-points per work-item (nx % VW == 0):
// the state is gathered from x - e_i and the adjoint from x + e_i with the
// 16-byte shifted accesses of the forward vector kernel (gather_vec); each
// point then runs the same adj_cell arithmetic as the one-point kernel, so
// b and dL/dF agree with it bit for bit. The launch bound asks for three
// waves per SIMD (168 VGPRs for two points per work-item): against two waves
// at 174 VGPRs the reverse sweep measured 11% faster (256^3 duct on MI355X).
// To fit that bound without spilling, a per-point force is read point by
// point inside the cell loop and dL/dF is read after it, so neither is held
// across the loop: with a force field this removed 20 bytes of scratch per
// work-item (reverse-step counter traffic was 1.11x its 264 bytes per point).
template <int FM, bool DIRECT, int VW>
__global__ __launch_bounds__(256, 3) void k_adj_stepv(const float* __restrict__ s,
                                                   const float* __restrict__ bin,
                                                   float* __restrict__ bout, float* __restrict__ gF,
                                                   double* __restrict__ taupart,
                                                   const uint8_t* __restrict__ flags,
                                                   const uint32_t* __restrict__ smask,
                                                   const uint32_t* __restrict__ mmask,
                                                   const float* __restrict__ ff, StepArgs a,
                                                   float inv_tau2)
{
    using Vt = typename Vec<float, VW>::t;
    using FW = typename FlagBytes<VW>::t;
    constexpr bool FORCE = FM != FORCE_NONE;
    constexpr FW ONES = FlagBytes<VW>::ones;
    const Dims& d = a.d;
    const int x0 = VW * (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const uint32_t z = blockIdx.z;
    const bool inside = x0 < d.nx && y < d.ny;
    const uint32_t nx = (uint32_t)d.nx;
    const uint32_t orow = inside ? (uint32_t)y * nx : 0u;
    const uint32_t o0 = orow + (inside ? (uint32_t)x0 : 0u);
    const uint32_t c0 = z * d.nxy + o0;
    const FW flw = inside ? *reinterpret_cast<const FW*>(flags + c0) : ONES;
    const FW solid = (flw | (flw >> 1)) & ONES;
    double tsum = 0.0;

    if (solid != ONES) {
        const size_t N = d.N;
        const uint32_t zm = wrap_m(z, (uint32_t)d.nz), zp = wrap_p(z, (uint32_t)d.nz);
        const uint32_t oym = (y == 0) ? (uint32_t)(d.ny - 1) * nx : (uint32_t)0 - nx;
        const uint32_t oyp = (y == d.ny - 1) ? (uint32_t)(1 - d.ny) * nx : nx;
        const bool end0 = !(solid & 1u), endL = !((solid >> (8 * (VW - 1))) & 1u);
        const bool nw = (flw & (ONES * NEAR_WALL)) != 0;
        Vt hq[Q], aq[Q];
        gather_vec<+1, VW>(s, d, z, zm, zp, orow, oym, oyp, (uint32_t)x0, end0, endL, nw, smask, c0, hq);
        if (DIRECT) {
#pragma unroll
            for (int i = 0; i < Q; ++i) aq[i] = ldv<VW>(plane(bin, d, i, z), o0);
        } else {
            gather_vec<-1, VW>(bin, d, z, zm, zp, orow, oym, oyp, (uint32_t)x0, end0, endL, nw, smask, c0, aq);
        }
        uint32_t mm[VW];
#pragma unroll
        for (int j = 0; j < VW; ++j) mm[j] = 0u;
        if (flw & (ONES * NEAR_MOVING)) load_words<VW>(mmask, c0, mm);
        float ga[3][VW];
#pragma unroll
        for (int j = 0; j < VW; ++j) {
            const bool sol = (solid >> (8 * j)) & 1u;
            float F[3];
#pragma unroll
            for (int k = 0; k < 3; ++k)
                F[k] = FM == FORCE_FIELD ? ld(ff + k * N, c0 + (uint32_t)j)
                                         : (FM == FORCE_UNIFORM ? (k == 0 ? a.Fx : (k == 1 ? a.Fy : a.Fz)) : 0.0f);
            float av[Q], h[Q], b[Q], gx, gy, gz, tt;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                av[i] = aq[i][j];
                h[i] = hq[i][j] - weight(i);
                if (i > 0 && ((mm[j] >> i) & 1u)) h[i] = h[i] + a.mw[i];
            }
            adj_cell<FORCE>(av, h, F[0], F[1], F[2], a, inv_tau2, b, gx, gy, gz, tt);
#pragma unroll
            for (int i = 0; i < Q; ++i) aq[i][j] = sol ? 0.0f : b[i];
            ga[0][j] = gx; ga[1][j] = gy; ga[2][j] = gz;
            if (!sol) tsum += (double)tt;
        }
        Vt gv[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) gv[k] = ldv<VW>(gF + k * N, c0);
#pragma unroll
        for (int j = 0; j < VW; ++j) {
            if (!((solid >> (8 * j)) & 1u)) {
                gv[0][j] = gv[0][j] + ga[0][j];
                gv[1][j] = gv[1][j] + ga[1][j];
                gv[2][j] = gv[2][j] + ga[2][j];
            }
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) stv_nt<VW>(plane(bout, d, i, z), o0, aq[i]);
#pragma unroll
        for (int k = 0; k < 3; ++k) stv_nt<VW>(gF + k * N, c0, gv[k]);
    }

    block_tau_sum(tsum, taupart);
}

// Zero n doubles with a kernel (no memset node, so the launch may be captured).
__global__ __launch_bounds__(256) void k_zero_f64(double* __restrict__ p, size_t n)
{
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = 0.0;
}

// out[0] = p[0] + p[1] + ... + p[n-1], added one by one in index order by a
// single work-item: the order and rounding of the host loop that sums the
// per-work-group tau partials, so both give the same bits.
__global__ __launch_bounds__(64) void k_sum_f64_ordered(const double* __restrict__ p, size_t n,
                                                        double* __restrict__ out)
{
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (size_t k = 0; k < n; ++k) s += p[k];
    out[0] = s;
}

hipError_t launch_zero_f64(double* p, size_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_sum_f64_ordered(const double* p, size_t n, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_f64_ordered, dim3(1), dim3(64), 0, s, p, n, out);
    return hipGetLastError();
}

hipError_t launch_adjoint_seed(int fm, const float* f, const uint8_t* flags, const float* ff,
                               const float* g, float* aout, float* gF, const StepArgs& args,
                               const Launch& L)
{
    switch (fm) {
    case FORCE_UNIFORM:
        hipLaunchKernelGGL((k_adj_seed<FORCE_UNIFORM>), L.grid, L.block, L.shmem, L.stream, f, flags, ff, g, aout, gF, args);
        break;
    case FORCE_FIELD:
        hipLaunchKernelGGL((k_adj_seed<FORCE_FIELD>), L.grid, L.block, L.shmem, L.stream, f, flags, ff, g, aout, gF, args);
        break;
    default:
        hipLaunchKernelGGL((k_adj_seed<FORCE_NONE>), L.grid, L.block, L.shmem, L.stream, f, flags, ff, g, aout, gF, args);
    }
    return hipGetLastError();
}

template <int FM>
static hipError_t adj_fm(bool direct, const float* s, const float* bin, float* bout, float* gF,
                         double* tp, const uint8_t* flags, const float* ff, const StepArgs& a,
                         float it2, const Launch& L)
{
    if (direct)
        hipLaunchKernelGGL((k_adj_step<FM, true>), L.grid, L.block, L.shmem, L.stream, s, bin, bout, gF, tp, flags, ff, a, it2);
    else
        hipLaunchKernelGGL((k_adj_step<FM, false>), L.grid, L.block, L.shmem, L.stream, s, bin, bout, gF, tp, flags, ff, a, it2);
    return hipGetLastError();
}

template <int FM, int VW>
static hipError_t adjv_fm(bool direct, const float* s, const float* bin, float* bout, float* gF,
                          double* tp, const uint8_t* flags, const uint32_t* sm, const uint32_t* mm,
                          const float* ff, const StepArgs& a, float it2, const Launch& L)
{
    if (direct)
        hipLaunchKernelGGL((k_adj_stepv<FM, true, VW>), L.grid, L.block, L.shmem, L.stream, s, bin, bout, gF, tp, flags, sm, mm, ff, a, it2);
    else
        hipLaunchKernelGGL((k_adj_stepv<FM, false, VW>), L.grid, L.block, L.shmem, L.stream, s, bin, bout, gF, tp, flags, sm, mm, ff, a, it2);
    return hipGetLastError();
}

template <int VW>
static hipError_t adjv_vw(bool direct, int fm, const float* s, const float* bin, float* bout, float* gF,
                          double* tp, const uint8_t* flags, const uint32_t* sm, const uint32_t* mm,
                          const float* ff, const StepArgs& a, float it2, const Launch& L)
{
    switch (fm) {
    case FORCE_UNIFORM: return adjv_fm<FORCE_UNIFORM, VW>(direct, s, bin, bout, gF, tp, flags, sm, mm, ff, a, it2, L);
    case FORCE_FIELD: return adjv_fm<FORCE_FIELD, VW>(direct, s, bin, bout, gF, tp, flags, sm, mm, ff, a, it2, L);
    default: return adjv_fm<FORCE_NONE, VW>(direct, s, bin, bout, gF, tp, flags, sm, mm, ff, a, it2, L);
    }
}

hipError_t launch_adjoint_stepv(int vw, bool direct, int fm, const float* s, const float* bin, float* bout,
                                float* gF, double* taupart, const uint8_t* flags, const uint32_t* smask,
                                const uint32_t* mmask, const float* ff, const StepArgs& args,
                                float inv_tau2, const Launch& L)
{
    if (vw == 2) return adjv_vw<2>(direct, fm, s, bin, bout, gF, taupart, flags, smask, mmask, ff, args, inv_tau2, L);
    if (vw == 4) return adjv_vw<4>(direct, fm, s, bin, bout, gF, taupart, flags, smask, mmask, ff, args, inv_tau2, L);
    return hipErrorInvalidValue;
}

hipError_t launch_adjoint_step(bool direct, int fm, const float* s, const float* bin, float* bout,
                               float* gF, double* taupart, const uint8_t* flags, const float* ff,
                               const StepArgs& args, float inv_tau2, const Launch& L)
{
    switch (fm) {
    case FORCE_UNIFORM: return adj_fm<FORCE_UNIFORM>(direct, s, bin, bout, gF, taupart, flags, ff, args, inv_tau2, L);
    case FORCE_FIELD: return adj_fm<FORCE_FIELD>(direct, s, bin, bout, gF, taupart, flags, ff, args, inv_tau2, L);
    default: return adj_fm<FORCE_NONE>(direct, s, bin, bout, gF, taupart, flags, ff, args, inv_tau2, L);
    }
}

}  // namespace lbmk

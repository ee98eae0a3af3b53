// Memory-access study kernels (include/lbm_study.h): the aligned/misaligned
// read and write experiment and the three offset-by-one propagation methods
// of Mawson & Revell, Section 4.3, and the push (Algorithm 2) and pull
// (Algorithm 3) iterations with one point per work-item, on gfx950.
#include <hip/hip_runtime.h>

#include "../../include/lbm_study.h"
#include "d3q19.hpp"

using namespace d3q19;

namespace {

// ------------------------------- streams -----------------------------------
// Each work-item handles WIDTH consecutive elements of all NV vectors, so
// like the lattice kernels it keeps NV independent accesses in flight.
template <int MODE, int NV, int WIDTH>
__global__ __launch_bounds__(256) void k_stream(const float* __restrict__ src, float* __restrict__ dst,
                                                float* __restrict__ sink, size_t n, int roff, int woff)
{
    using Vt = typename Vec<float, WIDTH>::t;
    const size_t k0 = (size_t)WIDTH * ((size_t)blockIdx.x * blockDim.x + threadIdx.x);
    const size_t last = n - 1;   // elements k < n - 1 are processed
    if (k0 >= last) return;
    if (k0 + WIDTH <= last) {
        Vt acc = 0.0f;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const size_t base = (size_t)v * n + k0;
            if (MODE == 0) {
                const Vt x = *reinterpret_cast<const Vt*>(src + base + roff);
                *reinterpret_cast<Vt*>(dst + base + woff) = x;
            } else if (MODE == 1) {
                acc += *reinterpret_cast<const Vt*>(src + base + roff);
            } else {
                Vt x;
#pragma unroll
                for (int j = 0; j < WIDTH; ++j) x[j] = (float)(k0 + j + v);
                *reinterpret_cast<Vt*>(dst + base + woff) = x;
            }
        }
        if (MODE == 1) *reinterpret_cast<Vt*>(sink + k0) = acc;
    } else {
        for (size_t k = k0; k < last; ++k) {
            float acc = 0.0f;
            for (int v = 0; v < NV; ++v) {
                const size_t base = (size_t)v * n + k;
                if (MODE == 0) dst[base + woff] = src[base + roff];
                else if (MODE == 1) acc += src[base + roff];
                else dst[base + woff] = (float)(k + v);
            }
            if (MODE == 1) sink[k] = acc;
        }
    }
}

template <int MODE, int WIDTH>
hipError_t stream_nv(int nv, const float* src, float* dst, float* sink, size_t n, int roff, int woff,
                     hipStream_t s)
{
    const size_t items = (n - 1 + WIDTH - 1) / WIDTH;
    const dim3 grid((unsigned)((items + 255) / 256)), block(256);
    switch (nv) {
    case 1: hipLaunchKernelGGL((k_stream<MODE, 1, WIDTH>), grid, block, 0, s, src, dst, sink, n, roff, woff); break;
    case 2: hipLaunchKernelGGL((k_stream<MODE, 2, WIDTH>), grid, block, 0, s, src, dst, sink, n, roff, woff); break;
    case 4: hipLaunchKernelGGL((k_stream<MODE, 4, WIDTH>), grid, block, 0, s, src, dst, sink, n, roff, woff); break;
    case 8: hipLaunchKernelGGL((k_stream<MODE, 8, WIDTH>), grid, block, 0, s, src, dst, sink, n, roff, woff); break;
    case 16: hipLaunchKernelGGL((k_stream<MODE, 16, WIDTH>), grid, block, 0, s, src, dst, sink, n, roff, woff); break;
    case 19: hipLaunchKernelGGL((k_stream<MODE, 19, WIDTH>), grid, block, 0, s, src, dst, sink, n, roff, woff); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------- propagation ----------------------------------
// Direct kernels: block index = chunk + chunks * row.
__global__ __launch_bounds__(1024) void k_shift_direct(const float* __restrict__ src, float* __restrict__ dst, int nx,
                                                       unsigned chunks)
{
    const int x = (blockIdx.x % chunks) * blockDim.x + threadIdx.x;
    if (x >= nx) return;
    const size_t row = (size_t)(blockIdx.x / chunks) * nx;
    dst[row + x] = src[row + (x == 0 ? nx - 1 : x - 1)];
}

__global__ __launch_bounds__(1024) void k_shift_lds(const float* __restrict__ src, float* __restrict__ dst, int nx)
{
    __shared__ float s[1024];
    const int x = threadIdx.x;
    const size_t row = (size_t)blockIdx.x * nx;
    s[x] = src[row + x];
    __syncthreads();
    dst[row + x] = s[x == 0 ? nx - 1 : x - 1];
}

__global__ __launch_bounds__(1024) void k_shift_dpp(const float* __restrict__ src, float* __restrict__ dst, int nx)
{
    __shared__ float edge[16];   // last element of every wave
    const int x = threadIdx.x;
    const int lane = x & 63, wave = x >> 6, waves = nx >> 6;
    const size_t row = (size_t)blockIdx.x * nx;
    const float v = src[row + x];
    // wave_shr:1 -- lane l receives lane l-1's value; lane 0 keeps `old`
    const float w = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, false));
    if (lane == 63) edge[wave] = v;
    __syncthreads();
    dst[row + x] = lane == 0 ? edge[wave == 0 ? waves - 1 : wave - 1] : w;
}

__global__ __launch_bounds__(256) void k_shift_direct4(const float* __restrict__ src, float* __restrict__ dst, int nx,
                                                        unsigned chunks)
{
    using Vt = typename Vec<float, 4>::t;
    const int x0 = 4 * ((blockIdx.x % chunks) * blockDim.x + threadIdx.x);
    if (x0 >= nx) return;
    const size_t row = (size_t)(blockIdx.x / chunks) * nx;
    const bool wl = x0 == 0;
    const Vt v = *reinterpret_cast<const Vt*>(src + row + (wl ? 0 : x0 - 1));
    Vt out = v;
    if (wl) out = Vt{src[row + nx - 1], v.x, v.y, v.z};
    *reinterpret_cast<Vt*>(dst + row + x0) = out;
}

// ------------------------------ push / pull --------------------------------
struct Box {
    int nx, ny, nz;
    size_t N;
};

__device__ __forceinline__ uint32_t cell_at(const Box& b, int x, int y, int z)
{
    x = x < 0 ? x + b.nx : (x >= b.nx ? x - b.nx : x);
    y = y < 0 ? y + b.ny : (y >= b.ny ? y - b.ny : y);
    z = z < 0 ? z + b.nz : (z >= b.nz ? z - b.nz : z);
    return ((uint32_t)z * (uint32_t)b.ny + (uint32_t)y) * (uint32_t)b.nx + (uint32_t)x;
}

// Pull (Algorithm 3): p_i(x) = s_i(x - e_i), or s_opp(i)(x) at a wall.
__global__ __launch_bounds__(1024) void k_pull(const float* __restrict__ a, float* __restrict__ b,
                                               const uint8_t* __restrict__ flags, Box bx, float omega)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= bx.nx) return;
    const uint32_t c = cell_at(bx, x, y, z);
    if (flags[c]) return;
    float h[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const uint32_t s = cell_at(bx, x - EX[i], y - EY[i], z - EZ[i]);
        const float p = flags[s] ? a[OPP[i] * bx.N + c] : a[i * bx.N + s];
        h[i] = p - weight(i);
    }
    bgk_collide<false>(h, omega, 0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
    for (int i = 0; i < Q; ++i) b[i * bx.N + c] = weight(i) + h[i];
}

// Push (Algorithm 2): local reads of p(x), collide, s_i(x) -> x + e_i, or
// back into direction opp(i) of x when x + e_i is a wall.
__global__ __launch_bounds__(1024) void k_push(const float* __restrict__ a, float* __restrict__ b,
                                               const uint8_t* __restrict__ flags, Box bx, float omega)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= bx.nx) return;
    const uint32_t c = cell_at(bx, x, y, z);
    if (flags[c]) return;
    float h[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) h[i] = a[i * bx.N + c] - weight(i);
    bgk_collide<false>(h, omega, 0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const uint32_t t = cell_at(bx, x + EX[i], y + EY[i], z + EZ[i]);
        const float v = weight(i) + h[i];
        if (flags[t]) b[OPP[i] * bx.N + c] = v;
        else b[i * bx.N + t] = v;
    }
}

// --------------------------- 19-plane streams ------------------------------
// The step's memory streams without the step: the 19 planes of a z-slab in
// the lattice kernels' layout (plane (z, i) at (z*19 + i)*nx*ny, x fastest),
// one row per wave, four x-points (16 bytes) per work-item, every access
// aligned, with the FP32 step's cache hints (non-temporal loads, buffer
// stores with the non-temporal bit). MODE 0 copies src to dst, 1 reads src
// (a never-taken store keeps the loads), 2 writes dst. The plane layout and
// launch shape are the step's, the neighbour shifts and the collision are
// left out: this is the pattern's own bandwidth ceiling.
template <int MODE>
__global__ __launch_bounds__(64) void k_planes(const float* __restrict__ src, float* __restrict__ dst,
                                               float* __restrict__ sink, Dims d)
{
    using V = typename Vec<float, 4>::t;
    const uint32_t x0 = 4 * (blockIdx.x * blockDim.x + threadIdx.x);
    const uint32_t y = blockIdx.y, z = blockIdx.z;
    if (x0 >= (uint32_t)d.nx) return;
    const uint32_t o = y * (uint32_t)d.nx + x0;
    V q[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (MODE == 2) {
            q[i] = V{(float)i, (float)o, 0.0f, 1.0f};
        } else {
            const float* P = plane(src, d, i, z);
            q[i] = __builtin_nontemporal_load(reinterpret_cast<const V*>(P + o));
        }
    }
    if (MODE == 1) {
        V a = q[0];
#pragma unroll
        for (int i = 1; i < Q; ++i) a += q[i];
        if (a.x == -1234.5f && a.y == 4321.5f) sink[0] = a.z;   // data are never these values
        return;
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) stv_nt<4>(plane(dst, d, i, z), o, q[i]);
}

lbm_status launch_status(hipError_t e) { return e == hipSuccess ? LBM_OK : LBM_ERR_DEVICE; }

}  // namespace

extern "C" {

lbm_status lbm_study_stream(int mode, const float* src, float* dst, float* sink, size_t n, int nvec,
                            int roff, int woff, int width, void* hip_stream)
{
    if (mode < 0 || mode > 2 || n < 8 || (roff != 0 && roff != 1) || (woff != 0 && woff != 1)) return LBM_ERR_INVALID;
    if (width != 1 && width != 4) return LBM_ERR_INVALID;
    if (width == 4 && n % 4) return LBM_ERR_INVALID;
    if (nvec != 1 && nvec != 2 && nvec != 4 && nvec != 8 && nvec != 16 && nvec != 19) return LBM_ERR_INVALID;
    if ((mode != 2 && !src) || (mode != 1 && !dst) || (mode == 1 && !sink)) return LBM_ERR_INVALID;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipError_t e;
    if (width == 1) {
        e = mode == 0 ? stream_nv<0, 1>(nvec, src, dst, sink, n, roff, woff, s)
            : mode == 1 ? stream_nv<1, 1>(nvec, src, dst, sink, n, roff, woff, s)
                        : stream_nv<2, 1>(nvec, src, dst, sink, n, roff, woff, s);
    } else {
        e = mode == 0 ? stream_nv<0, 4>(nvec, src, dst, sink, n, roff, woff, s)
            : mode == 1 ? stream_nv<1, 4>(nvec, src, dst, sink, n, roff, woff, s)
                        : stream_nv<2, 4>(nvec, src, dst, sink, n, roff, woff, s);
    }
    return launch_status(e);
}

lbm_status lbm_study_shift(const float* src, float* dst, int nx, int nrows, int method, void* hip_stream)
{
    if (!src || !dst || nx < 1 || nrows < 1) return LBM_ERR_INVALID;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    switch (method) {
    case 0: {
        const int bx = nx < 256 ? nx : 256;
        const unsigned chunks = (unsigned)((nx + bx - 1) / bx);
        if ((unsigned long long)chunks * nrows >= (1ull << 31)) return LBM_ERR_INVALID;
        hipLaunchKernelGGL(k_shift_direct, dim3(chunks * (unsigned)nrows), dim3((unsigned)bx), 0, s, src, dst, nx, chunks);
        break;
    }
    case 1:
        if (nx % 64 || nx > 1024) return LBM_ERR_INVALID;
        hipLaunchKernelGGL(k_shift_lds, dim3((unsigned)nrows), dim3((unsigned)nx), 0, s, src, dst, nx);
        break;
    case 2:
        if (nx % 64 || nx > 1024) return LBM_ERR_INVALID;
        hipLaunchKernelGGL(k_shift_dpp, dim3((unsigned)nrows), dim3((unsigned)nx), 0, s, src, dst, nx);
        break;
    case 3: {
        if (nx % 4) return LBM_ERR_INVALID;
        const int q = nx / 4, bx = q < 64 ? q : 64;
        const unsigned chunks = (unsigned)((q + bx - 1) / bx);
        if ((unsigned long long)chunks * nrows >= (1ull << 31)) return LBM_ERR_INVALID;
        hipLaunchKernelGGL(k_shift_direct4, dim3(chunks * (unsigned)nrows), dim3((unsigned)bx), 0, s, src, dst, nx, chunks);
        break;
    }
    default: return LBM_ERR_INVALID;
    }
    return launch_status(hipGetLastError());
}

lbm_status lbm_study_planes(int mode, const float* src, float* dst, float* sink, int nx, int ny, int nz,
                            void* hip_stream)
{
    if (mode < 0 || mode > 2 || nx < 4 || nx % 4 || ny < 1 || nz < 1 || ny > 65535 || nz > 65535)
        return LBM_ERR_INVALID;
    if ((unsigned long long)nx * ny * nz >= (1ull << 30)) return LBM_ERR_INVALID;
    if ((mode != 2 && !src) || (mode != 1 && !dst) || (mode == 1 && !sink)) return LBM_ERR_INVALID;
    if ((((uintptr_t)src) | ((uintptr_t)dst)) & 15u) return LBM_ERR_INVALID;
    Dims d{};
    d.nx = nx; d.ny = ny; d.nz = nz;
    d.nxy = (uint32_t)nx * (uint32_t)ny;
    d.N = (uint32_t)((size_t)nx * ny * nz);
    const unsigned groups = (unsigned)(nx / 4);
    const unsigned bx = groups < 64 ? groups : 64;
    const dim3 grid((groups + bx - 1) / bx, (unsigned)ny, (unsigned)nz), block(bx);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    switch (mode) {
    case 0: hipLaunchKernelGGL(k_planes<0>, grid, block, 0, s, src, dst, sink, d); break;
    case 1: hipLaunchKernelGGL(k_planes<1>, grid, block, 0, s, src, dst, sink, d); break;
    default: hipLaunchKernelGGL(k_planes<2>, grid, block, 0, s, src, dst, sink, d); break;
    }
    return launch_status(hipGetLastError());
}

lbm_status lbm_study_step(const float* a, float* b, const uint8_t* flags, int nx, int ny, int nz, float tau,
                          int scheme, int block_x, void* hip_stream)
{
    if (!a || !b || !flags || a == b || nx < 1 || ny < 1 || nz < 1 || ny > 65535 || nz > 65535) return LBM_ERR_INVALID;
    if (!(tau > 0.5f) || (scheme != 0 && scheme != 1) || block_x < 1 || block_x > 1024) return LBM_ERR_INVALID;
    if ((unsigned long long)nx * ny * nz >= (1ull << 30)) return LBM_ERR_INVALID;
    Box bx{nx, ny, nz, (size_t)nx * ny * nz};
    const float omega = (float)(1.0 / (double)tau);
    const dim3 grid((unsigned)((nx + block_x - 1) / block_x), (unsigned)ny, (unsigned)nz), block((unsigned)block_x);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (scheme == 0) hipLaunchKernelGGL(k_pull, grid, block, 0, s, a, b, flags, bx, omega);
    else hipLaunchKernelGGL(k_push, grid, block, 0, s, a, b, flags, bx, omega);
    return launch_status(hipGetLastError());
}

}  // extern "C"

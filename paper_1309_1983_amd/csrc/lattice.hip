// Host runtime of the C ABI declared in include/lbm.h.
//
// Owns the device buffers of a lattice (population arrays, preprocessed
// flags, force field, checkpoints and adjoint buffers), validates every
// argument before touching HIP, launches the kernels on the lattice's stream
// and keeps the step bookkeeping: the AB buffer swap after each step
// (Mawson & Revell, Section 4.1, footnote on the redundant copy), the AA
// parity, the per-step event log, and the checkpoint-every-K rollout with
// its reverse sweep.
#include <hip/hip_runtime.h>

#include <cxxabi.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "kernels.hpp"

using d3q19::Q;

namespace {

thread_local std::string g_last_error;

lbm_status fail(lbm_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

size_t storage_bytes(int storage) { return storage == LBM_STORAGE_F32 ? 4 : 2; }

}  // namespace

struct lbm_lattice {
    int nx = 0, ny = 0, nz = 0;
    size_t N = 0;
    d3q19::Dims dims{};
    int device = 0;
    int storage = LBM_STORAGE_F32;
    int pattern = LBM_PATTERN_AB;
    int bx = 256, by = 1;
    hipStream_t stream = nullptr;

    float tau = 0.6f;
    float uw[3] = {0, 0, 0};
    float force[3] = {0, 0, 0};
    bool has_force_uniform = false;
    float* d_force = nullptr;   // [3][N] when a field is set
    bool has_force_field = false;

    void* d_f[2] = {nullptr, nullptr};
    bool own_f = true;             // population arrays allocated by the library
    int cur = 0;      // AB: index of the array holding the state
    int parity = 0;   // AA: 0 natural layout, 1 shifted layout
    uint8_t* d_flags = nullptr;
    uint32_t* d_smask = nullptr;   // solid-neighbour bits per cell
    uint32_t* d_mmask = nullptr;   // moving-wall-neighbour bits per cell
    int* d_check = nullptr;
    int cpl = 1;                   // points per work-item of the AB step (1 or the vector width)
    bool vec_ok = true;            // vector kernels allowed (cells_per_lane != 1)
    int bx4 = 64, by4 = 1;         // work-group of the vector kernel
    bool flat = false;             // vector AB step on a one-dimensional grid per plane
    bool alt4 = false;             // bfloat16, eight points: four points while a force is set
    int alt_bx4 = 64, alt_by4 = 1; // work-group of that four-point launch
    bool alt_flat = false;
    bool onsite = false;           // has on-site velocity nodes (flags 3, 4)
    bool early = false;            // FP32 vector AB step gathers before the flag branches
    unsigned shmem4 = 0;           // LDS reserved per vector-step work-group (residency cap)
    hipEvent_t order_ev = nullptr; // orders work across lbm_set_stream

    bool sticky = false;
    long long steps_done = 0;
    int check_interval = 0;

    // per-step timing log
    int timing_cap = 0;
    std::vector<hipEvent_t> events;  // ring of timing_cap + 1
    long long ev_recorded = 0;       // events recorded since the log was cleared

    // checkpointed trajectory for the adjoint
    std::vector<float*> ckpt;
    int traj_T = -1, traj_K = 0;
    long long traj_version = -1;
    long long version = 0;           // bumped by anything that changes the dynamics/state
    float* d_seg = nullptr;          // (K-1) states
    int seg_cap = 0;
    void* traj_dev = nullptr;        // caller-owned checkpoint store (NULL: library allocates)
    size_t traj_bytes = 0;
    bool traj_owned = true;          // ckpt / d_seg were allocated by the library
    float* d_adj[2] = {nullptr, nullptr};
    double* d_taupart = nullptr;
    size_t taupart_n = 0;
    void* adj_dev = nullptr;         // caller-owned adjoint workspace (NULL: library allocates)
    size_t adj_bytes = 0;

    size_t bytes = 0;
};

namespace {

lbm_status hip_check(lbm_lattice* L, hipError_t e, const char* what)
{
    if (e == hipSuccess) return LBM_OK;
    if (L) L->sticky = true;
    if (e == hipErrorOutOfMemory) return fail(LBM_ERR_OOM, "%s: %s", what, hipGetErrorString(e));
    return fail(LBM_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHK(L, call)                                                 \
    do {                                                                \
        lbm_status _st = hip_check((L), (call), #call);                 \
        if (_st != LBM_OK) return _st;                                  \
    } while (0)

lbm_status usable(const lbm_lattice* L)
{
    if (!L) return fail(LBM_ERR_INVALID, "lattice is NULL");
    if (L->sticky) return fail(LBM_ERR_DEVICE, "lattice is in a failed state after a device error");
    return LBM_OK;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int now = -1;
        if (prev >= 0 && hipGetDevice(&now) == hipSuccess && now != prev) (void)hipSetDevice(prev);
    }
};

int force_mode(const lbm_lattice* L)
{
    if (L->has_force_field) return lbmk::FORCE_FIELD;
    if (L->has_force_uniform) return lbmk::FORCE_UNIFORM;
    return lbmk::FORCE_NONE;
}

// Points per work-item and launch shape of the vector AB step for the
// lattice's current force mode. A bfloat16 lattice laid out with eight points
// per work-item runs four while a body force is set: the eight-point kernel
// with a force needs 185 VGPRs (two waves per SIMD; bounded to three it
// spills), and four points measured 2-6% faster with a uniform force or a
// force field on MI355X (256^3 cavity, 128x128x256 sphere duct); without a
// force eight points are 4-5% faster.
struct VecShape {
    int cpl, bx4, by4;
    bool flat;
};
VecShape vec_shape(const lbm_lattice* L)
{
    if (L->alt4 && force_mode(L) != lbmk::FORCE_NONE) return {4, L->alt_bx4, L->alt_by4, L->alt_flat};
    return {L->cpl, L->bx4, L->by4, L->flat};
}

lbmk::StepArgs step_args(const lbm_lattice* L)
{
    lbmk::StepArgs a{};
    a.d = L->dims;
    const double tau = L->tau;
    a.omega = (float)(1.0 / tau);
    a.cF = (float)(1.0 - 0.5 / tau);
    a.Fx = L->force[0];
    a.Fy = L->force[1];
    a.Fz = L->force[2];
    for (int i = 0; i < Q; ++i) {
        const double eu = d3q19::EX[i] * (double)L->uw[0] + d3q19::EY[i] * (double)L->uw[1]
                          + d3q19::EZ[i] * (double)L->uw[2];
        a.mw[i] = (float)(6.0 * (double)d3q19::weight(i) * eu);
    }
    for (int k = 0; k < 3; ++k) a.uw[k] = L->uw[k];
    const VecShape v = vec_shape(L);
    a.gx = v.flat ? (uint32_t)(L->nx / v.cpl) : 0u;
    a.early = L->early ? 1u : 0u;
    return a;
}

lbmk::Launch launch_of(const lbm_lattice* L) { return lbmk::make_launch(L->dims, L->bx, L->by, L->stream); }

// Only valid when the lattice uses the vector kernel (cpl > 1).
lbmk::Launch launch4_of(const lbm_lattice* L)
{
    const VecShape v = vec_shape(L);
    if (v.flat) {
        const unsigned long long groups = (unsigned long long)(L->nx / v.cpl) * (unsigned long long)L->ny;
        lbmk::Launch la;
        la.block = dim3(64, 1, 1);
        la.grid = dim3((unsigned)((groups + 63) / 64), 1, (unsigned)L->nz);
        la.stream = L->stream;
        la.shmem = L->shmem4;
        return la;
    }
    d3q19::Dims q = L->dims;
    q.nx = L->nx / v.cpl;   // the grid counts groups of cpl points along x
    lbmk::Launch la = lbmk::make_launch(q, v.bx4, v.by4, L->stream);
    la.shmem = L->shmem4;
    return la;
}

void default_block(int nx, int& bx, int& by)
{
    // rows that are a multiple of 512 points: 512-point groups, 6.5% faster
    // than 256 for the in-place 16-bit step at 512^3 on MI355X
    if (nx % 512 == 0) { bx = 512; by = 1; return; }
    if (nx >= 256) { bx = 256; by = 1; return; }
    if ((nx & (nx - 1)) == 0) { bx = nx; by = 256 / nx; return; }
    bx = std::min(256, (nx + 63) / 64 * 64);
    by = std::max(1, 256 / bx);
}

// Work-group shape of the one-point reverse step: the default shape capped at
// the kernel's 256 work-items (rows that are a multiple of 512 points take
// 512-point groups for the forward steps).
void adjoint_block(int nx, int& bx, int& by)
{
    default_block(nx, bx, by);
    if (bx * by > 256) {
        bx = std::min(bx, 256);
        by = std::max(1, 256 / bx);
    }
}

// Launch of the reverse step: two x-points per work-item with 64-work-item
// groups (the fastest shape measured at 256^3; four points need too many
// registers), else one point per work-item with at most 256 per group.
lbmk::Launch adjoint_launch(const d3q19::Dims& dims, bool vec_ok, hipStream_t stream, bool& vec)
{
    vec = vec_ok && dims.nx % 2 == 0;
    if (vec) {
        d3q19::Dims q = dims;
        q.nx = dims.nx / 2;
        const int rbx = std::min(q.nx, 64);
        return lbmk::make_launch(q, rbx, std::max(1, 64 / rbx), stream);
    }
    int abx, aby;
    adjoint_block(dims.nx, abx, aby);
    return lbmk::make_launch(dims, abx, aby, stream);
}

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t state_bytes_of(size_t N) { return (size_t)Q * N * sizeof(float); }

// Adjoint workspace: two adjoint arrays, then one double per work-group.
size_t adjoint_bytes_of(const d3q19::Dims& dims, bool vec_ok, size_t& nblk)
{
    bool vec = false;
    const lbmk::Launch LR = adjoint_launch(dims, vec_ok, nullptr, vec);
    nblk = (size_t)LR.grid.x * LR.grid.y * LR.grid.z;
    return 2 * round256(state_bytes_of(dims.N)) + nblk * sizeof(double);
}

bool aligned256(const void* p) { return ((uintptr_t)p & 255u) == 0; }

template <class T>
lbm_status dalloc(lbm_lattice* L, T** p, size_t bytes, const char* what)
{
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? LBM_ERR_OOM : LBM_ERR_DEVICE, "hipMalloc(%zu B) for %s: %s",
                    bytes, what, hipGetErrorString(e));
    }
    *p = static_cast<T*>(q);
    L->bytes += bytes;
    return LBM_OK;
}

void dfree(lbm_lattice* L, void* p, size_t bytes)
{
    if (p) {
        (void)hipFree(p);
        L->bytes -= std::min(L->bytes, bytes);
    }
}

void drop_trajectory(lbm_lattice* L)
{
    const size_t sb = (size_t)Q * L->N * sizeof(float);
    if (L->traj_owned) {
        for (float* p : L->ckpt) dfree(L, p, sb);
        dfree(L, L->d_seg, sb * (size_t)L->seg_cap);
    }
    L->ckpt.clear();
    L->d_seg = nullptr;
    L->seg_cap = 0;
    L->traj_T = -1;
    L->traj_version = -1;
}

// Releases library-allocated adjoint buffers; caller workspace pointers are
// just forgotten.
void drop_adjoint_buffers(lbm_lattice* L)
{
    const size_t sb = state_bytes_of(L->N);
    if (!L->adj_dev) {
        dfree(L, L->d_adj[0], sb);
        dfree(L, L->d_adj[1], sb);
        dfree(L, L->d_taupart, L->taupart_n * sizeof(double));
    }
    L->d_adj[0] = L->d_adj[1] = nullptr;
    L->d_taupart = nullptr;
    L->taupart_n = 0;
}

void invalidate(lbm_lattice* L) { ++L->version; }

lbm_status run_steps(lbm_lattice* L, int n, bool collide, float* rho = nullptr, float* u = nullptr);
lbm_status adjoint_sweep(lbm_lattice* L, const float* g, float* gF, float* adj[2], double* part,
                         const lbmk::Launch& LR, bool vec);

}  // namespace

extern "C" {

void lbm_options_default(lbm_options* opt)
{
    if (!opt) return;
    std::memset(opt, 0, sizeof *opt);
    opt->storage = LBM_STORAGE_F32;
    opt->pattern = LBM_PATTERN_AB;
    opt->device = -1;
}

const char* lbm_status_string(lbm_status st)
{
    switch (st) {
    case LBM_OK: return "LBM_OK";
    case LBM_ERR_INVALID: return "LBM_ERR_INVALID";
    case LBM_ERR_OOM: return "LBM_ERR_OOM";
    case LBM_ERR_DEVICE: return "LBM_ERR_DEVICE";
    case LBM_ERR_STATE: return "LBM_ERR_STATE";
    case LBM_ERR_NONFINITE: return "LBM_ERR_NONFINITE";
    }
    return "LBM_ERR_UNKNOWN";
}

const char* lbm_last_error(void) { return g_last_error.c_str(); }

lbm_status lbm_create(int nx, int ny, int nz, float tau, const uint8_t* flags_host, lbm_lattice** out)
{
    return lbm_create_ex(nx, ny, nz, tau, flags_host, nullptr, out);
}

}  // extern "C"

namespace {

// Launch layout of a lattice, resolved from its size and options.
struct Layout {
    int bx = 0, by = 0;        // one-point kernels
    int cpl = 1;               // points per work-item of the AB step
    int bx4 = 0, by4 = 0;      // vector AB step work-group
    bool flat = false;         // vector AB step on a one-dimensional grid per plane
};

// Validates everything lbm_create_ex checks before touching the device
// except tau and the flags, and resolves the launch layout.
lbm_status resolve_layout(int nx, int ny, int nz, const lbm_options& opt, Layout& lay)
{
    if (nx <= 0 || ny <= 0 || nz <= 0) return fail(LBM_ERR_INVALID, "sizes must be positive (%d,%d,%d)", nx, ny, nz);
    const unsigned long long N = (unsigned long long)nx * ny * nz;
    if (N >= (1ull << 30)) return fail(LBM_ERR_INVALID, "N = %llu points exceeds 2^30", N);
    if (nz > 65535) return fail(LBM_ERR_INVALID, "nz must be <= 65535 (got %d)", nz);
    if (opt.storage < 0 || opt.storage > 2) return fail(LBM_ERR_INVALID, "unknown storage %d", opt.storage);
    if (opt.pattern < 0 || opt.pattern > 1) return fail(LBM_ERR_INVALID, "unknown pattern %d", opt.pattern);
    if (opt.gather_mode < 0 || opt.gather_mode > 2) return fail(LBM_ERR_INVALID, "unknown gather_mode %d", opt.gather_mode);
    if (opt.groups_per_cu < -1 || opt.groups_per_cu > 64)
        return fail(LBM_ERR_INVALID, "groups_per_cu must be -1, 0 or 1..64 (got %d)", opt.groups_per_cu);
    int bx = opt.block_x, by = opt.block_y;
    if (bx == 0 && by == 0) default_block(nx, bx, by);
    if (bx <= 0 || by <= 0 || bx * by > 1024) return fail(LBM_ERR_INVALID, "bad block shape %dx%d", bx, by);
    if ((ny + by - 1) / by > 65535) return fail(LBM_ERR_INVALID, "ny/block_y must be <= 65535 work-groups");
    if (opt.timing_capacity < 0 || opt.check_interval < 0) return fail(LBM_ERR_INVALID, "negative timing/check option");
    if (opt.cells_per_lane != 0 && opt.cells_per_lane != 1 && !lbmk::vector_width_ok(opt.storage, opt.cells_per_lane))
        return fail(LBM_ERR_INVALID, "cells_per_lane must be 0, 1, 4%s (got %d)",
                    opt.storage == LBM_STORAGE_F32 ? "" : " or 8", opt.cells_per_lane);
    // default vector width: 16-byte accesses for FP32; for 16-bit storage
    // 8-byte accesses, or 16-byte ones on rows of 256 points or more, where
    // they measured faster on MI355X (cavity 256^3 +1.7%, 512^3 +7.7%; rows
    // of 128 points, 5-10% slower)
    const bool wide = opt.storage != LBM_STORAGE_F32 && nx % 8 == 0 && nx >= 256;
    const int vw = opt.cells_per_lane > 1 ? opt.cells_per_lane : (wide ? 8 : 4);
    int cpl = 1, bx4 = 0, by4 = 0;
    bool flat = false;
    if (opt.pattern == LBM_PATTERN_AB && nx % vw == 0 && opt.cells_per_lane != 1) {
        if (opt.block_x == 0 && opt.block_y == 0) {
            // one wave per work-group along x (a whole 256-point row when
            // nx = 256 and vw = 4): the fastest shape measured at 256^3 on MI355X.
            // Rows of more than 64 groups that are not a multiple of 64 (a
            // 260-point row: 65 groups) take a one-dimensional grid over the
            // plane instead, which keeps every wave full.
            bx4 = std::min(nx / vw, 64);
            by4 = std::max(1, 64 / bx4);
            flat = nx / vw > 64 && (nx / vw) % 64 != 0;
            cpl = vw;
        } else if (bx * by <= 256) {
            bx4 = bx; by4 = by;
            cpl = vw;
        }
    }
    if (opt.cells_per_lane > 1 && cpl != opt.cells_per_lane)
        return fail(LBM_ERR_INVALID, "cells_per_lane = %d needs the AB pattern, nx %% %d == 0 and <= 256 work-items per group",
                    vw, vw);
    if (cpl > 1 && (ny + by4 - 1) / by4 > 65535) return fail(LBM_ERR_INVALID, "ny/block_y must be <= 65535 work-groups");
    lay.bx = bx; lay.by = by; lay.cpl = cpl; lay.bx4 = bx4; lay.by4 = by4; lay.flat = flat;
    return LBM_OK;
}

d3q19::Dims dims_of(int nx, int ny, int nz)
{
    d3q19::Dims d{};
    d.nx = nx; d.ny = ny; d.nz = nz;
    d.nxy = (uint32_t)nx * (uint32_t)ny;
    d.N = (uint32_t)((size_t)nx * ny * nz);
    return d;
}

// Porous geometry: at least this fraction of the fluid points have a solid
// neighbour. There the FP32 AB step gathers before the flag branches (sphere
// duct, 10%: 126.7 -> 114.1 us per step; 256^3 cavity, 2%: 3% slower) and
// the 16-bit AB step takes eight points per work-item when rows allow it
// (sphere duct 128 x 128 x 256: FP16 77.0 -> 69.1 us, BF16 79.4 -> 73.8 us;
// the plain 128-wide duct, 3%, is 1-6% faster with four). Bfloat16 steps
// taken while a body force is set still launch four (vec_shape).
constexpr double POROUS_MIN_NEAR_FRACTION = 0.08;
// Lattices without solid points up to this size step with one point per
// work-item when the width is automatic.
constexpr size_t SMALL_PERIODIC_MAX_POINTS = (size_t)1 << 18;
// Resident work-groups per compute unit of the FP32 multi-point AB step (one
// wave each): 256^3 cavity on MI355X, 426 us per step at the 12 that the
// kernel's registers allow, 412 us at 8, 415 us at 10, 438 us at 5.
constexpr int AUTO_GROUPS_PER_CU_F32 = 8;

}  // namespace

extern "C" {

lbm_status lbm_query_buffer_sizes(int nx, int ny, int nz, const lbm_options* opt_in, lbm_buffer_sizes* out)
{
    if (!out) return fail(LBM_ERR_INVALID, "out is NULL");
    lbm_options opt;
    if (opt_in) opt = *opt_in;
    else lbm_options_default(&opt);
    Layout lay;
    lbm_status st = resolve_layout(nx, ny, nz, opt, lay);
    if (st != LBM_OK) return st;
    const d3q19::Dims d = dims_of(nx, ny, nz);
    size_t nblk = 0;
    out->population_bytes = round256((size_t)Q * d.N * storage_bytes(opt.storage));
    out->population_arrays = opt.pattern == LBM_PATTERN_AB ? 2 : 1;
    out->adjoint_bytes = adjoint_bytes_of(d, opt.cells_per_lane != 1, nblk);
    out->state_bytes = state_bytes_of(d.N);
    return LBM_OK;
}

size_t lbm_trajectory_bytes(int nx, int ny, int nz, int T, int K)
{
    if (nx <= 0 || ny <= 0 || nz <= 0 || T < 0 || K <= 0) return 0;
    const unsigned long long N = (unsigned long long)nx * ny * nz;
    if (N >= (1ull << 30)) return 0;
    const size_t nck = T == 0 ? 1 : (size_t)((T + K - 1) / K);
    const size_t segK = (size_t)std::min(K, std::max(T, 1));
    return (nck + segK - 1) * round256(state_bytes_of((size_t)N));
}

lbm_status lbm_create_ex(int nx, int ny, int nz, float tau, const uint8_t* flags_host,
                         const lbm_options* opt_in, lbm_lattice** out)
{
    g_last_error.clear();
    if (!out) return fail(LBM_ERR_INVALID, "out is NULL");
    *out = nullptr;
    lbm_options opt;
    if (opt_in) opt = *opt_in;
    else lbm_options_default(&opt);
    Layout lay;
    lbm_status st0 = resolve_layout(nx, ny, nz, opt, lay);
    if (st0 != LBM_OK) return st0;
    if (!(tau > 0.5f) || !std::isfinite(tau)) return fail(LBM_ERR_INVALID, "tau must be finite and > 0.5 (got %g)", (double)tau);
    const unsigned long long N = (unsigned long long)nx * ny * nz;
    const int nbuf = opt.pattern == LBM_PATTERN_AB ? 2 : 1;
    const bool caller_f = opt.population_dev[0] || opt.population_dev[1];
    if (caller_f) {
        for (int b = 0; b < 2; ++b) {
            if (b < nbuf && !opt.population_dev[b])
                return fail(LBM_ERR_INVALID, "population_dev[%d] is NULL (the %s pattern needs %d arrays)", b,
                            nbuf == 2 ? "AB" : "AA", nbuf);
            if (b >= nbuf && opt.population_dev[b])
                return fail(LBM_ERR_INVALID, "population_dev[1] must be NULL for the AA pattern");
            if (b < nbuf && !aligned256(opt.population_dev[b]))
                return fail(LBM_ERR_INVALID, "population_dev[%d] must be 256-byte aligned", b);
        }
        if (nbuf == 2 && opt.population_dev[0] == opt.population_dev[1])
            return fail(LBM_ERR_INVALID, "population_dev[0] and [1] must be different buffers");
    }
    bool onsite = false;
    if (flags_host) {
        for (unsigned long long c = 0; c < N; ++c) {
            if (flags_host[c] > 4) return fail(LBM_ERR_INVALID, "flag value %u at point %llu (allowed 0..4)", flags_host[c], c);
            onsite = onsite || flags_host[c] >= 3;
        }
    }

    int dev = opt.device;
    if (dev < 0) {
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return fail(LBM_ERR_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    }
    DeviceGuard guard(dev);

    lbm_lattice* L = new (std::nothrow) lbm_lattice;
    if (!L) return fail(LBM_ERR_OOM, "host allocation failed");
    L->nx = nx; L->ny = ny; L->nz = nz; L->N = (size_t)N;
    L->dims = dims_of(nx, ny, nz);
    L->device = dev;
    L->storage = opt.storage;
    L->pattern = opt.pattern;
    L->bx = lay.bx; L->by = lay.by;
    L->stream = static_cast<hipStream_t>(opt.hip_stream);
    L->tau = tau;
    L->timing_cap = opt.timing_capacity;
    L->check_interval = opt.check_interval;
    L->cpl = lay.cpl;
    L->vec_ok = opt.cells_per_lane != 1;
    L->onsite = onsite;
    if (lay.cpl > 1) { L->bx4 = lay.bx4; L->by4 = lay.by4; L->flat = lay.flat; }

    lbm_status st = LBM_OK;
    const size_t fbytes = (size_t)Q * L->N * storage_bytes(L->storage);
    if (caller_f) {
        L->own_f = false;
        for (int b = 0; b < nbuf; ++b) L->d_f[b] = opt.population_dev[b];
    } else {
        for (int b = 0; b < nbuf && st == LBM_OK; ++b) st = dalloc(L, &L->d_f[b], fbytes, "populations");
    }
    if (st == LBM_OK) st = dalloc(L, &L->d_flags, L->N, "flags");
    if (st == LBM_OK) st = dalloc(L, &L->d_smask, L->N * sizeof(uint32_t), "neighbour masks");
    if (st == LBM_OK) st = dalloc(L, &L->d_mmask, L->N * sizeof(uint32_t), "neighbour masks");
    if (st == LBM_OK) st = dalloc(L, &L->d_check, 4 * sizeof(int), "check flag and counters");
    uint8_t* d_raw = nullptr;
    if (st == LBM_OK) st = dalloc(L, &d_raw, L->N, "raw flags");
    if (st == LBM_OK) {
        hipError_t e = flags_host ? hipMemcpyAsync(d_raw, flags_host, L->N, hipMemcpyHostToDevice, L->stream)
                                  : hipMemsetAsync(d_raw, 0, L->N, L->stream);
        st = hip_check(L, e, "flags upload");
    }
    if (st == LBM_OK) st = hip_check(L, hipMemsetAsync(L->d_check, 0, 4 * sizeof(int), L->stream), "check flag clear");
    if (st == LBM_OK)
        st = hip_check(L, lbmk::launch_mark_near_wall(d_raw, L->d_flags, L->d_smask, L->d_mmask, L->d_check,
                                                      reinterpret_cast<unsigned*>(L->d_check + 1), L->dims,
                                                      launch_of(L)), "mark_near_wall");
    int counts[3] = {0, 0, 0};   // bad on-site node, near-wall fluid points, fluid points
    if (st == LBM_OK)
        st = hip_check(L, hipMemcpyAsync(counts, L->d_check, sizeof counts, hipMemcpyDeviceToHost, L->stream),
                       "check flag read");
    // rest state in every array (solid points keep it forever)
    for (int b = 0; b < nbuf && st == LBM_OK; ++b)
        st = hip_check(L, lbmk::launch_init_eq(L->storage, L->d_f[b], nullptr, nullptr, L->dims, launch_of(L)), "init");
    if (st == LBM_OK && L->timing_cap > 0) {
        L->events.resize((size_t)L->timing_cap + 1, nullptr);
        for (auto& ev : L->events)
            if (st == LBM_OK) st = hip_check(L, hipEventCreate(&ev), "hipEventCreate");
    }
    if (st == LBM_OK) st = hip_check(L, hipStreamSynchronize(L->stream), "create sync");
    if (st == LBM_OK && counts[0])
        st = fail(LBM_ERR_INVALID, "an on-site velocity node (flag 3 or 4) has solid neighbours that do not form "
                                   "a box face, edge or corner");
    if (d_raw) dfree(L, d_raw, L->N);
    if (st != LBM_OK) {
        std::string msg = g_last_error;
        lbm_destroy(L);
        g_last_error = msg;
        return st;
    }
    const double near_fraction = counts[2] > 0 ? (double)(unsigned)counts[1] / (double)(unsigned)counts[2] : 0.0;
    const bool porous = near_fraction >= POROUS_MIN_NEAR_FRACTION;
    if (L->cpl > 1 && opt.cells_per_lane == 0 && (size_t)(unsigned)counts[2] == L->N && L->N <= SMALL_PERIODIC_MAX_POINTS) {
        // small box without solid points: one point per work-item. The vector
        // step's row ends then load their periodic x-neighbours separately,
        // and the grid holds too few waves to fill the GPU: on MI355X the
        // 32^3 periodic step ran 3.5 us against 6.5 us, 64^3 12% faster
        L->cpl = 1;
        L->flat = false;
    }
    if (porous && L->storage != LBM_STORAGE_F32 && L->cpl == 4 && opt.cells_per_lane == 0 && nx % 8 == 0) {
        // 16-bit storage on porous geometry: eight points per work-item
        lbm_options o8 = opt;
        o8.cells_per_lane = 8;
        Layout l8;
        if (resolve_layout(nx, ny, nz, o8, l8) == LBM_OK && l8.cpl == 8) {
            L->cpl = l8.cpl; L->bx4 = l8.bx4; L->by4 = l8.by4; L->flat = l8.flat;
        }
        g_last_error.clear();
    }
    if (L->storage == LBM_STORAGE_BF16 && L->cpl == 8 && opt.cells_per_lane == 0) {
        // the four-point launch taken while a body force is set
        lbm_options o4 = opt;
        o4.cells_per_lane = 4;
        Layout l4;
        if (resolve_layout(nx, ny, nz, o4, l4) == LBM_OK && l4.cpl == 4) {
            L->alt4 = true; L->alt_bx4 = l4.bx4; L->alt_by4 = l4.by4; L->alt_flat = l4.flat;
        }
        g_last_error.clear();
    }
    const bool early_ok = L->storage == LBM_STORAGE_F32 && L->pattern == LBM_PATTERN_AB && L->cpl > 1 && !L->onsite;
    L->early = early_ok && (opt.gather_mode == 2 ||
                            (opt.gather_mode == 0 && porous));
    // residency cap of the vector AB step
    int cap = opt.groups_per_cu;
    if (cap == 0)
        cap = (L->cpl > 1 && L->storage == LBM_STORAGE_F32 && !L->early && opt.block_x == 0 && opt.block_y == 0)
                  ? AUTO_GROUPS_PER_CU_F32 : -1;
    if (cap > 0 && L->cpl > 1) {
        int lds_cu = 0, lds_block = 0;
        hipError_t e = hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&lds_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        if (e != hipSuccess) {
            lbm_destroy(L);
            return fail(LBM_ERR_DEVICE, "LDS size query: %s", hipGetErrorString(e));
        }
        // the largest multiple of 512 bytes that still fits `cap` groups
        const unsigned sh = (unsigned)(lds_cu / cap) & ~511u;
        if (sh == 0 || (int)sh > lds_block || lds_cu / (int)sh != cap) {
            lbm_destroy(L);
            return fail(LBM_ERR_INVALID, "groups_per_cu = %d cannot be set with %d bytes of LDS per compute unit", cap,
                        lds_cu);
        }
        L->shmem4 = sh;
    }
    *out = L;
    return LBM_OK;
}

void lbm_destroy(lbm_lattice* L)
{
    if (!L) return;
    DeviceGuard guard(L->device);
    (void)hipStreamSynchronize(L->stream);
    drop_trajectory(L);
    drop_adjoint_buffers(L);
    const size_t fbytes = (size_t)Q * L->N * storage_bytes(L->storage);
    if (L->own_f) {
        dfree(L, L->d_f[0], fbytes);
        dfree(L, L->d_f[1], fbytes);
    }
    dfree(L, L->d_flags, L->N);
    dfree(L, L->d_smask, L->N * sizeof(uint32_t));
    dfree(L, L->d_mmask, L->N * sizeof(uint32_t));
    dfree(L, L->d_check, sizeof(int));
    dfree(L, L->d_force, 3 * L->N * sizeof(float));
    for (auto ev : L->events)
        if (ev) (void)hipEventDestroy(ev);
    if (L->order_ev) (void)hipEventDestroy(L->order_ev);
    delete L;
}

lbm_status lbm_get_info(const lbm_lattice* L, int* nx, int* ny, int* nz, int* storage, int* pattern)
{
    if (!L) return fail(LBM_ERR_INVALID, "lattice is NULL");
    if (nx) *nx = L->nx;
    if (ny) *ny = L->ny;
    if (nz) *nz = L->nz;
    if (storage) *storage = L->storage;
    if (pattern) *pattern = L->pattern;
    return LBM_OK;
}

size_t lbm_device_bytes(const lbm_lattice* L) { return L ? L->bytes : 0; }

lbm_status lbm_set_stream(lbm_lattice* L, void* s)
{
    lbm_status st = usable(L);
    if (st != LBM_OK) return st;
    hipStream_t ns = static_cast<hipStream_t>(s);
    if (ns == L->stream) return LBM_OK;
    DeviceGuard guard(L->device);
    // work already queued on the old stream comes before anything enqueued
    // on the new one
    if (!L->order_ev) HIPCHK(L, hipEventCreateWithFlags(&L->order_ev, hipEventDisableTiming));
    HIPCHK(L, hipEventRecord(L->order_ev, L->stream));
    HIPCHK(L, hipStreamWaitEvent(ns, L->order_ev, 0));
    L->stream = ns;
    return LBM_OK;
}

lbm_status lbm_set_trajectory_buffer(lbm_lattice* L, void* dev, size_t bytes)
{
    lbm_status st = usable(L);
    if (st != LBM_OK) return st;
    if (dev && !aligned256(dev)) return fail(LBM_ERR_INVALID, "trajectory buffer must be 256-byte aligned");
    DeviceGuard guard(L->device);
    HIPCHK(L, hipStreamSynchronize(L->stream));   // the old store may still be read
    drop_trajectory(L);
    L->traj_dev = dev;
    L->traj_bytes = dev ? bytes : 0;
    return LBM_OK;
}

lbm_status lbm_set_adjoint_buffer(lbm_lattice* L, void* dev, size_t bytes)
{
    lbm_status st = usable(L);
    if (st != LBM_OK) return st;
    size_t nblk = 0;
    const size_t need = adjoint_bytes_of(L->dims, L->vec_ok, nblk);
    if (dev && !aligned256(dev)) return fail(LBM_ERR_INVALID, "adjoint buffer must be 256-byte aligned");
    if (dev && bytes < need)
        return fail(LBM_ERR_INVALID, "adjoint buffer of %zu bytes is smaller than the %zu bytes needed", bytes, need);
    DeviceGuard guard(L->device);
    HIPCHK(L, hipStreamSynchronize(L->stream));
    drop_adjoint_buffers(L);
    L->adj_dev = dev;
    L->adj_bytes = dev ? bytes : 0;
    if (dev) {
        const size_t sbr = round256(state_bytes_of(L->N));
        char* base = static_cast<char*>(dev);
        L->d_adj[0] = reinterpret_cast<float*>(base);
        L->d_adj[1] = reinterpret_cast<float*>(base + sbr);
        L->d_taupart = reinterpret_cast<double*>(base + 2 * sbr);
        L->taupart_n = nblk;
    }
    return LBM_OK;
}

lbm_status lbm_step_kernel_name(lbm_lattice* L, char* buf, size_t cap)
{
    lbm_status st = usable(L);
    if (st != LBM_OK) return st;
    if (!buf || cap == 0) return fail(LBM_ERR_INVALID, "buffer is NULL or empty");
    DeviceGuard guard(L->device);
    const bool vector = L->pattern == LBM_PATTERN_AB && L->cpl > 1;
    const void* fn = nullptr;
    HIPCHK(L, lbmk::resolve_step_kernel(vector, L->storage, L->pattern, L->parity, vec_shape(L).cpl, true, force_mode(L),
                                        L->d_f[L->cur], L->d_f[L->cur ^ 1], L->d_flags, L->d_smask, L->d_mmask,
                                        L->d_force, step_args(L), vector ? launch4_of(L) : launch_of(L), L->onsite,
                                        &fn));
    const char* mangled = hipKernelNameRefByPtr(fn, L->stream);
    if (!mangled) return fail(LBM_ERR_DEVICE, "the runtime does not name the step kernel");
    int dst = -1;
    char* dem = abi::__cxa_demangle(mangled, nullptr, nullptr, &dst);
    const char* name = (dst == 0 && dem) ? dem : mangled;
    std::snprintf(buf, cap, "%s", name);
    std::free(dem);
    return LBM_OK;
}

lbm_status lbm_set_tau(lbm_lattice* L, float tau)
{
    lbm_status st = usable(L);
    if (st != LBM_OK) return st;
    if (!(tau > 0.5f) || !std::isfinite(tau)) return fail(LBM_ERR_INVALID, "tau must be finite and > 0.5 (got %g)", (double)tau);
    if (tau != L->tau) invalidate(L);
    L->tau = tau;
    return LBM_OK;
}

lbm_status lbm_set_wall_velocity(lbm_lattice* L, float ux, float uy, float uz)
{
    lbm_status st = usable(L);
    if (st != LBM_OK) return st;
    if (!std::isfinite(ux) || !std::isfinite(uy) || !std::isfinite(uz))
        return fail(LBM_ERR_INVALID, "wall velocity must be finite");
    if (std::sqrt((double)ux * ux + (double)uy * uy + (double)uz * uz) >= 0.3)
        return fail(LBM_ERR_INVALID, "|u_wall| must be < 0.3 (low Mach number)");
    L->uw[0] = ux; L->uw[1] = uy; L->uw[2] = uz;
    invalidate(L);
    return LBM_OK;
}

lbm_status lbm_set_force_uniform(lbm_lattice* L, float fx, float fy, float fz)
{
    lbm_status st = usable(L);
    if (st != LBM_OK) return st;
    if (!std::isfinite(fx) || !std::isfinite(fy) || !std::isfinite(fz))
        return fail(LBM_ERR_INVALID, "force must be finite");
    L->force[0] = fx; L->force[1] = fy; L->force[2] = fz;
    L->has_force_uniform = (fx != 0.0f || fy != 0.0f || fz != 0.0f);
    L->has_force_field = false;
    invalidate(L);
    return LBM_OK;
}

lbm_status lbm_set_force_field(lbm_lattice* L, const float* F_dev)
{
    lbm_status st = usable(L);
    if (st != LBM_OK) return st;
    DeviceGuard guard(L->device);
    invalidate(L);
    if (!F_dev) {
        L->has_force_field = false;
        return LBM_OK;
    }
    if (!L->d_force) {
        st = dalloc(L, &L->d_force, 3 * L->N * sizeof(float), "force field");
        if (st != LBM_OK) return st;
    }
    HIPCHK(L, hipMemcpyAsync(L->d_force, F_dev, 3 * L->N * sizeof(float), hipMemcpyDeviceToDevice, L->stream));
    L->has_force_field = true;
    L->has_force_uniform = false;
    L->force[0] = L->force[1] = L->force[2] = 0.0f;
    return LBM_OK;
}

lbm_status lbm_init_equilibrium(lbm_lattice* L, const float* rho, const float* u)
{
    lbm_status st = usable(L);
    if (st != LBM_OK) return st;
    DeviceGuard guard(L->device);
    HIPCHK(L, lbmk::launch_init_eq(L->storage, L->d_f[L->cur], rho, u, L->dims, launch_of(L)));
    L->parity = 0;
    invalidate(L);
    return LBM_OK;
}

lbm_status lbm_step(lbm_lattice* L, int n)
{
    if (!L) return fail(LBM_ERR_INVALID, "lattice is NULL");
    if (L->sticky) return fail(LBM_ERR_STATE, "lattice is in a failed state after a device error");
    if (n < 0) return fail(LBM_ERR_INVALID, "n must be >= 0 (got %d)", n);
    DeviceGuard guard(L->device);
    return run_steps(L, n, true);
}

lbm_status lbm_step_macros(lbm_lattice* L, int n, float* rho, float* u)
{
    if (!L) return fail(LBM_ERR_INVALID, "lattice is NULL");
    if (L->sticky) return fail(LBM_ERR_STATE, "lattice is in a failed state after a device error");
    if (n < 1) return fail(LBM_ERR_INVALID, "n must be >= 1 (got %d)", n);
    if (!rho || !u) return fail(LBM_ERR_INVALID, "rho and u must both be given");
    DeviceGuard guard(L->device);
    if (L->pattern == LBM_PATTERN_AB) return run_steps(L, n, true, rho, u);
    lbm_status st = run_steps(L, n, true);
    if (st != LBM_OK) return st;
    return lbm_macros(L, rho, u);
}

lbm_status lbm_debug_stream_only(lbm_lattice* L, int n)
{
    lbm_status st = usable(L);
    if (st != LBM_OK) return st;
    if (n < 0) return fail(LBM_ERR_INVALID, "n must be >= 0 (got %d)", n);
    DeviceGuard guard(L->device);
    return run_steps(L, n, false);
}

lbm_status lbm_macros(lbm_lattice* L, float* rho, float* u)
{
    lbm_status st = usable(L);
    if (st != LBM_OK) return st;
    if (!rho && !u) return fail(LBM_ERR_INVALID, "rho and u are both NULL");
    DeviceGuard guard(L->device);
    HIPCHK(L, lbmk::launch_macros(L->storage, L->parity, force_mode(L), L->d_f[L->cur], L->d_flags,
                                  L->d_force, rho, u, step_args(L), launch_of(L)));
    return LBM_OK;
}

lbm_status lbm_get_populations(lbm_lattice* L, float* f)
{
    lbm_status st = usable(L);
    if (st != LBM_OK) return st;
    if (!f) return fail(LBM_ERR_INVALID, "f is NULL");
    DeviceGuard guard(L->device);
    HIPCHK(L, lbmk::launch_get(L->storage, L->parity, L->d_f[L->cur], L->d_flags, f, L->dims, launch_of(L)));
    return LBM_OK;
}

lbm_status lbm_set_populations(lbm_lattice* L, const float* f)
{
    lbm_status st = usable(L);
    if (st != LBM_OK) return st;
    if (!f) return fail(LBM_ERR_INVALID, "f is NULL");
    DeviceGuard guard(L->device);
    HIPCHK(L, lbmk::launch_set(L->storage, L->d_f[L->cur], f, L->dims, launch_of(L)));
    L->parity = 0;
    invalidate(L);
    return LBM_OK;
}

lbm_status lbm_check_finite(lbm_lattice* L)
{
    lbm_status st = usable(L);
    if (st != LBM_OK) return st;
    DeviceGuard guard(L->device);
    HIPCHK(L, hipMemsetAsync(L->d_check, 0, sizeof(int), L->stream));
    HIPCHK(L, lbmk::launch_check_finite(L->storage, L->parity, L->d_f[L->cur], L->d_flags, L->d_check, L->dims,
                                        launch_of(L)));
    int h = 0;
    HIPCHK(L, hipMemcpyAsync(&h, L->d_check, sizeof(int), hipMemcpyDeviceToHost, L->stream));
    HIPCHK(L, hipStreamSynchronize(L->stream));
    if (h) return fail(LBM_ERR_NONFINITE, "non-finite population found after %lld steps", L->steps_done);
    return LBM_OK;
}

lbm_status lbm_sync(lbm_lattice* L)
{
    lbm_status st = usable(L);
    if (st != LBM_OK) return st;
    DeviceGuard guard(L->device);
    HIPCHK(L, hipStreamSynchronize(L->stream));
    return LBM_OK;
}

lbm_status lbm_step_times(lbm_lattice* L, float* ms, int cap, int* count)
{
    lbm_status st = usable(L);
    if (st != LBM_OK) return st;
    if (!count || (cap > 0 && !ms) || cap < 0) return fail(LBM_ERR_INVALID, "bad output arguments");
    *count = 0;
    if (L->timing_cap <= 0) return fail(LBM_ERR_STATE, "timing log not enabled (timing_capacity = 0)");
    DeviceGuard guard(L->device);
    HIPCHK(L, hipStreamSynchronize(L->stream));
    const long long R = (long long)L->events.size();   // ring slots
    const long long rec = L->ev_recorded;
    // the newest min(rec, R) events are valid; durations between consecutive ones
    const long long valid = std::min(rec, R);
    const long long ndur = valid > 0 ? valid - 1 : 0;
    const long long nout = std::min<long long>(ndur, cap);
    const long long first = rec - nout - 1;   // index of the event before the first duration
    for (long long k = 0; k < nout; ++k) {
        hipEvent_t a = L->events[(size_t)((first + k) % R)];
        hipEvent_t b = L->events[(size_t)((first + k + 1) % R)];
        float t = 0.0f;
        HIPCHK(L, hipEventElapsedTime(&t, a, b));
        ms[k] = t;
    }
    *count = (int)nout;
    L->ev_recorded = 0;
    return LBM_OK;
}

lbm_status lbm_copy_f32(const float* src, float* dst, size_t n, void* stream)
{
    if ((!src || !dst) && n) return fail(LBM_ERR_INVALID, "NULL buffer");
    if (n && (((uintptr_t)src | (uintptr_t)dst) & 15u)) return fail(LBM_ERR_INVALID, "buffers must be 16-byte aligned");
    hipError_t e = lbmk::launch_copy(src, dst, n, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(LBM_ERR_DEVICE, "copy: %s", hipGetErrorString(e));
    return LBM_OK;
}

lbm_status lbm_forward_checkpointed(lbm_lattice* L, int T, int K)
{
    lbm_status st = usable(L);
    if (st != LBM_OK) return st;
    if (T < 0 || K <= 0) return fail(LBM_ERR_INVALID, "need T >= 0 and K > 0 (got T=%d K=%d)", T, K);
    if (L->storage != LBM_STORAGE_F32 || L->pattern != LBM_PATTERN_AB)
        return fail(LBM_ERR_STATE, "the adjoint rollout needs F32 storage and the AB pattern");
    if (L->onsite) return fail(LBM_ERR_STATE, "the adjoint does not cover on-site velocity nodes");
    const size_t need = lbm_trajectory_bytes(L->nx, L->ny, L->nz, T, K);
    if (L->traj_dev && need > L->traj_bytes)
        return fail(LBM_ERR_INVALID, "the trajectory buffer holds %zu bytes; T = %d, K = %d needs %zu", L->traj_bytes,
                    T, K, need);
    DeviceGuard guard(L->device);
    drop_trajectory(L);
    const size_t sb = (size_t)Q * L->N * sizeof(float);
    const int nck = T == 0 ? 1 : (T + K - 1) / K;
    const int segK = std::min(K, std::max(T, 1));
    if (L->traj_dev) {
        // caller store: checkpoints at 256-byte-aligned state slots, then the
        // segment states back to back
        L->traj_owned = false;
        char* base = static_cast<char*>(L->traj_dev);
        const size_t sbr = round256(sb);
        for (int k = 0; k < nck; ++k) L->ckpt.push_back(reinterpret_cast<float*>(base + (size_t)k * sbr));
        if (segK > 1) {
            L->d_seg = reinterpret_cast<float*>(base + (size_t)nck * sbr);
            L->seg_cap = segK - 1;
        }
    } else {
        L->traj_owned = true;
        for (int k = 0; k < nck; ++k) {
            float* p = nullptr;
            st = dalloc(L, &p, sb, "checkpoint");
            if (st != LBM_OK) { drop_trajectory(L); return st; }
            L->ckpt.push_back(p);
        }
        if (segK > 1) {
            st = dalloc(L, &L->d_seg, sb * (size_t)(segK - 1), "segment store");
            if (st != LBM_OK) { drop_trajectory(L); return st; }
            L->seg_cap = segK - 1;
        }
    }
    for (int k = 0; k < nck; ++k) {
        HIPCHK(L, hipMemcpyAsync(L->ckpt[k], L->d_f[L->cur], sb, hipMemcpyDeviceToDevice, L->stream));
        const int len = std::min(K, T - k * K);
        if (len > 0) {
            st = run_steps(L, len, true);
            if (st != LBM_OK) { drop_trajectory(L); return st; }
        }
    }
    L->traj_T = T;
    L->traj_K = K;
    L->traj_version = L->version;
    return LBM_OK;
}

lbm_status lbm_adjoint(lbm_lattice* L, const float* g, float* gF, double* grad_tau)
{
    lbm_status st = usable(L);
    if (st != LBM_OK) return st;
    if (!g || !gF || !grad_tau) return fail(LBM_ERR_INVALID, "NULL argument");
    if (L->traj_T < 0 || L->traj_version != L->version)
        return fail(LBM_ERR_STATE, "no valid trajectory: call lbm_forward_checkpointed after the last change");
    DeviceGuard guard(L->device);
    const size_t sb = (size_t)Q * L->N * sizeof(float);
    bool vec = false;
    const lbmk::Launch LR = adjoint_launch(L->dims, L->vec_ok, L->stream, vec);
    const size_t nblk = (size_t)LR.grid.x * LR.grid.y * LR.grid.z;
    if (!L->adj_dev) {
        for (int b = 0; b < 2; ++b)
            if (!L->d_adj[b]) {
                st = dalloc(L, &L->d_adj[b], sb, "adjoint buffer");
                if (st != LBM_OK) return st;
            }
        if (L->taupart_n < nblk) {
            dfree(L, L->d_taupart, L->taupart_n * sizeof(double));
            L->d_taupart = nullptr;
            L->taupart_n = 0;
            st = dalloc(L, &L->d_taupart, nblk * sizeof(double), "tau partials");
            if (st != LBM_OK) return st;
            L->taupart_n = nblk;
        }
    }
    HIPCHK(L, hipMemsetAsync(L->d_taupart, 0, nblk * sizeof(double), L->stream));
    float* adj[2] = {L->d_adj[0], L->d_adj[1]};
    st = adjoint_sweep(L, g, gF, adj, L->d_taupart, LR, vec);
    if (st != LBM_OK) return st;
    std::vector<double> parts(nblk);
    HIPCHK(L, hipMemcpyAsync(parts.data(), L->d_taupart, nblk * sizeof(double), hipMemcpyDeviceToHost, L->stream));
    HIPCHK(L, hipStreamSynchronize(L->stream));
    double s = 0.0;
    for (double v : parts) s += v;
    *grad_tau = s;
    return LBM_OK;
}

}  // extern "C"

// ------------------------- allocation-free adjoint -------------------------
// lbm_adjoint_noalloc keeps its adjoint arrays, tau partials and tau sum in
// `scratch`, a file-scope device array that every GPU the library runs on
// holds for the life of the process. In host code the array's name is only a
// stand-in: its device address comes from hipGetSymbolAddress, once per
// device with that device current, and only that address is handed to
// kernels. Calls on one GPU share the array: overlapping calls race.
namespace {

constexpr size_t NOALLOC_MAX_POINTS = (size_t)1 << 18;   // a 64^3 lattice
constexpr size_t NOALLOC_STATE_BYTES = ((size_t)Q * NOALLOC_MAX_POINTS * sizeof(float) + 255) & ~(size_t)255;
constexpr size_t NOALLOC_PART_OFFSET = 2 * NOALLOC_STATE_BYTES;
constexpr size_t NOALLOC_SUM_OFFSET = NOALLOC_PART_OFFSET + NOALLOC_MAX_POINTS * sizeof(double);
constexpr size_t NOALLOC_SCRATCH_BYTES = NOALLOC_SUM_OFFSET + 256;   // 38.0 MiB + 2 MiB + 256 B

}  // namespace

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on device `dev` (current), looked up on the
// first call for that device.
lbm_status scratch_on(int dev, char** out)
{
    if (dev < 0 || dev >= MAX_DEVICES) return fail(LBM_ERR_DEVICE, "device ordinal %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(LBM_ERR_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = static_cast<char*>(g_scratch_ptr[dev]);
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_adjoint_noalloc(lbm_lattice* L, const float* g, float* gF, double* grad_tau)
{
    lbm_status st = usable(L);
    if (st != LBM_OK) return st;
    if (!g || !gF || !grad_tau) return fail(LBM_ERR_INVALID, "NULL argument");
    if (L->N > NOALLOC_MAX_POINTS)
        return fail(LBM_ERR_INVALID, "lbm_adjoint_noalloc handles at most %zu points (a 64^3 lattice); this lattice "
                                     "has %zu: use lbm_adjoint", NOALLOC_MAX_POINTS, L->N);
    if (L->traj_T < 0 || L->traj_version != L->version)
        return fail(LBM_ERR_STATE, "no valid trajectory: call lbm_forward_checkpointed after the last change");
    DeviceGuard guard(L->device);
    bool vec = false;
    const lbmk::Launch LR = adjoint_launch(L->dims, L->vec_ok, L->stream, vec);
    const size_t nblk = (size_t)LR.grid.x * LR.grid.y * LR.grid.z;
    if (nblk > NOALLOC_MAX_POINTS)   // at most one work-group per point
        return fail(LBM_ERR_INVALID, "%zu reverse-step work-groups exceed the scratch partials", nblk);
    char* base = nullptr;
    st = scratch_on(L->device, &base);
    if (st != LBM_OK) {
        L->sticky = true;
        return st;
    }
    float* adj[2] = {reinterpret_cast<float*>(base), reinterpret_cast<float*>(base + NOALLOC_STATE_BYTES)};
    double* part = reinterpret_cast<double*>(base + NOALLOC_PART_OFFSET);
    double* sum = reinterpret_cast<double*>(base + NOALLOC_SUM_OFFSET);
    // the partials accumulate over the reverse steps: clear this call's
    // (the previous call's contents stay in the array)
    HIPCHK(L, lbmk::launch_zero_f64(part, nblk, L->stream));
    st = adjoint_sweep(L, g, gF, adj, part, LR, vec);
    if (st != LBM_OK) return st;
    HIPCHK(L, lbmk::launch_sum_f64_ordered(part, nblk, sum, L->stream));
    double h = 0.0;
    HIPCHK(L, hipMemcpyAsync(&h, sum, sizeof(double), hipMemcpyDeviceToHost, L->stream));
    HIPCHK(L, hipStreamSynchronize(L->stream));
    *grad_tau = h;
    return LBM_OK;
}

}  // extern "C"

namespace {

// Seed plus reverse sweep over the recorded trajectory: adjoint arrays adj[0]
// and adj[1] (19 N floats each), tau partials `part` (one per reverse-step
// work-group, zeroed by the caller), reverse-step launch LR.
lbm_status adjoint_sweep(lbm_lattice* L, const float* g, float* gF, float* adj[2], double* part,
                         const lbmk::Launch& LR, bool vec)
{
    const lbmk::Launch LA = launch_of(L);
    const lbmk::StepArgs args = step_args(L);
    const int fm = force_mode(L);
    const float inv_tau2 = (float)(1.0 / ((double)L->tau * (double)L->tau));
    const int T = L->traj_T, K = L->traj_K;
    const int nck = (int)L->ckpt.size();

    // seed from the final state (the lattice's current array)
    HIPCHK(L, lbmk::launch_adjoint_seed(fm, static_cast<const float*>(L->d_f[L->cur]), L->d_flags, L->d_force, g,
                                        adj[0], gF, args, LA));
    int ab = 0;            // adj[ab] holds the adjoint input of the next reverse step
    bool direct = true;
    for (int k = nck - 1; k >= 0 && T > 0; --k) {
        const int t0 = k * K;
        const int len = std::min(K, T - t0);
        // recompute s^{t0+1} .. s^{t0+len-1} into the segment store
        auto state = [&](int j) -> float* { return j == 0 ? L->ckpt[k] : L->d_seg + (size_t)(j - 1) * Q * L->N; };
        for (int j = 1; j < len; ++j) {
            if (L->cpl > 1)
                HIPCHK(L, lbmk::launch_step_abv(LBM_STORAGE_F32, L->cpl, true, fm, state(j - 1), state(j), L->d_flags,
                                                L->d_smask, L->d_mmask, L->d_force, args, launch4_of(L)));
            else
                HIPCHK(L, lbmk::launch_step(LBM_STORAGE_F32, LBM_PATTERN_AB, 0, true, fm, state(j - 1), state(j),
                                            L->d_flags, L->d_smask, L->d_mmask, L->d_force, args, LA));
        }
        for (int j = len - 1; j >= 0; --j) {
            if (vec)
                HIPCHK(L, lbmk::launch_adjoint_stepv(2, direct, fm, state(j), adj[ab], adj[ab ^ 1], gF, part,
                                                     L->d_flags, L->d_smask, L->d_mmask, L->d_force, args, inv_tau2,
                                                     LR));
            else
                HIPCHK(L, lbmk::launch_adjoint_step(direct, fm, state(j), adj[ab], adj[ab ^ 1], gF, part, L->d_flags,
                                                    L->d_force, args, inv_tau2, LR));
            ab ^= 1;
            direct = false;
        }
    }
    return LBM_OK;
}

// n steps; with rho/u (AB pattern) the last step also stores its in-step
// rho and u.
lbm_status run_steps(lbm_lattice* L, int n, bool collide, float* rho, float* u)
{
    if (n == 0) return LBM_OK;
    const lbmk::StepArgs args = step_args(L);
    const lbmk::Launch LA = launch_of(L);
    const lbmk::Launch LA4 = L->cpl > 1 ? launch4_of(L) : LA;
    const int fm = collide ? force_mode(L) : lbmk::FORCE_NONE;
    const long long R = (long long)L->events.size();
    if (R > 0 && L->ev_recorded == 0) {
        HIPCHK(L, hipEventRecord(L->events[0], L->stream));
        L->ev_recorded = 1;
    }
    for (int s = 0; s < n; ++s) {
        float* mr = s == n - 1 ? rho : nullptr;
        float* mu = s == n - 1 ? u : nullptr;
        if (L->pattern == LBM_PATTERN_AB && L->cpl > 1) {
            HIPCHK(L, lbmk::launch_step_abv(L->storage, vec_shape(L).cpl, collide, fm, L->d_f[L->cur], L->d_f[L->cur ^ 1], L->d_flags,
                                            L->d_smask, L->d_mmask, L->d_force, args, LA4, mr, mu, L->onsite));
            L->cur ^= 1;
        } else if (L->pattern == LBM_PATTERN_AB) {
            HIPCHK(L, lbmk::launch_step(L->storage, 0, 0, collide, fm, L->d_f[L->cur], L->d_f[L->cur ^ 1], L->d_flags,
                                        L->d_smask, L->d_mmask, L->d_force, args, LA, mr, mu, L->onsite));
            L->cur ^= 1;
        } else {
            HIPCHK(L, lbmk::launch_step(L->storage, 1, L->parity, collide, fm, L->d_f[0], nullptr, L->d_flags,
                                        L->d_smask, L->d_mmask, L->d_force, args, LA, nullptr, nullptr,
                                        L->onsite));
            L->parity ^= 1;
        }
        ++L->steps_done;
        if (R > 0) {
            HIPCHK(L, hipEventRecord(L->events[(size_t)(L->ev_recorded % R)], L->stream));
            ++L->ev_recorded;
        }
        if (L->check_interval > 0 && L->steps_done % L->check_interval == 0) {
            lbm_status st = lbm_check_finite(L);
            if (st != LBM_OK) return st;
        }
    }
    invalidate(L);
    return LBM_OK;
}

}  // namespace

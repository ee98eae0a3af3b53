// Host-side launch interface of the gfx950 kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "d3q19.hpp"

namespace lbmk {

enum ForceMode { FORCE_NONE = 0, FORCE_UNIFORM = 1, FORCE_FIELD = 2 };

struct StepArgs {
    d3q19::Dims d;
    float omega;   // 1/tau
    float cF;      // 1 - 1/(2 tau)
    float Fx, Fy, Fz;           // uniform force (FORCE_UNIFORM)
    float mw[d3q19::Q];         // 6 w_i (e_i . u_wall), rho_wall = 1
    float uw[3];                // wall velocity (velocity of moving on-site nodes)
    uint32_t gx;                // vector AB step: > 0 = its grid is one-dimensional in x over
                                // the gx * ny point groups of a z-plane (gx = nx / vw groups
                                // per row, x fastest); 0 = two-dimensional (x groups, y)
    uint32_t early;             // FP32 vector AB step: issue the gather before the flag
                                // branches (porous geometry)
};

struct Launch {
    dim3 grid, block;
    hipStream_t stream;
    // Dynamic LDS reserved per work-group and never touched by the kernel:
    // caps the work-groups resident on a compute unit (its LDS / shmem).
    unsigned shmem = 0;
};

Launch make_launch(const d3q19::Dims& d, int bx, int by, hipStream_t s);

// One step. AB: reads `a`, writes `b`. AA: in place on `a`; parity 0 is the
// gather/scatter step, parity 1 the local step.
// AB only: rho/u non-null also stores the in-step rho [N] and u [3][N].
// onsite: the lattice has on-site velocity nodes (rebuilt when collide).
hipError_t launch_step(int storage, int pattern, int parity, bool collide, int force_mode,
                       void* a, void* b, const uint8_t* flags, const uint32_t* smask,
                       const uint32_t* mmask, const float* ffield, const StepArgs& args,
                       const Launch& L, float* rho = nullptr, float* u = nullptr, bool onsite = false);

// One AB step with vw consecutive x-points per work-item: vw = 4 (FP32,
// 16-byte accesses; or 16-bit storage, 8-byte accesses) or vw = 8 (16-bit
// storage, 16-byte accesses). Needs nx % vw == 0 and at most 256 work-items
// per work-group; the launch's grid counts groups of vw points along x.
bool vector_width_ok(int storage, int vw);
hipError_t launch_step_abv(int storage, int vw, bool collide, int force_mode, void* a, void* b,
                           const uint8_t* flags, const uint32_t* smask, const uint32_t* mmask,
                           const float* ffield, const StepArgs& args, const Launch& L,
                           float* rho = nullptr, float* u = nullptr, bool onsite = false);

// The kernel (host-side function pointer) that launch_step_abv (vector) or
// launch_step would launch with these arguments, without launching it.
hipError_t resolve_step_kernel(bool vector, int storage, int pattern, int parity, int vw, bool collide,
                               int force_mode, void* a, void* b, const uint8_t* flags, const uint32_t* smask,
                               const uint32_t* mmask, const float* ffield, const StepArgs& args, const Launch& L,
                               bool onsite, const void** kernel);

// flags_in holds the caller's values 0..4 (fluid, wall, moving wall, on-site
// node at rest, on-site node moving with u_w). flags_out = type bits (on-site
// nodes are fluid) plus NEAR_WALL / NEAR_MOVING on fluid cells next to a
// solid / moving-wall cell and ONSITE / ONSITE_MOVING; smask / mmask bit i
// set when x - e_i is solid / a moving wall. *bad |= 1 for an on-site node
// whose solid neighbours do not form a box face, edge or corner.
// counts[0] += fluid points with a solid neighbour, counts[1] += fluid points.
hipError_t launch_mark_near_wall(const uint8_t* flags_in, uint8_t* flags_out, uint32_t* smask,
                                 uint32_t* mmask, int* bad, unsigned* counts, const d3q19::Dims& d,
                                 const Launch& L);

// f = f^eq(rho, u) in the given storage (natural layout).
hipError_t launch_init_eq(int storage, void* f, const float* rho, const float* u,
                          const d3q19::Dims& d, const Launch& L);

// Plain populations of the current state (layout = 1: AA after an odd number
// of steps, 0 otherwise) into out [19][N] float.
hipError_t launch_get(int storage, int layout, const void* f, const uint8_t* flags, float* out,
                      const d3q19::Dims& d, const Launch& L);

// State from plain populations, natural layout.
hipError_t launch_set(int storage, void* f, const float* in, const d3q19::Dims& d,
                      const Launch& L);

// rho [N], u [3][N] from the current state.
hipError_t launch_macros(int storage, int layout, int force_mode, const void* f,
                         const uint8_t* flags, const float* ffield, float* rho, float* u,
                         const StepArgs& args, const Launch& L);

// *flag |= 1 if any stored population of a fluid cell is not finite.
hipError_t launch_check_finite(int storage, int layout, const void* f, const uint8_t* flags,
                               int* flag, const d3q19::Dims& d, const Launch& L);

hipError_t launch_copy(const float* src, float* dst, size_t n, hipStream_t s);

// ----------------------------- adjoint ------------------------------------
// Seed: a = dL/ds(T) from g = dL/du(T) on the state f (F32, natural layout);
// grad_F = -g/(2 rho) (overwritten; 0 at solid cells).
hipError_t launch_adjoint_seed(int force_mode, const float* f, const uint8_t* flags,
                               const float* ffield, const float* g, float* a, float* gF,
                               const StepArgs& args, const Launch& L);

// Reverse step t (at most 256 work-items per group): a^{t+1} from bin (direct = seed layout, else gathered
// through the transposed streaming), p from the pull gather of state s^t,
// bout = J_C(p)^T a^{t+1}; grad_F += dC/dF^T a; taupart[block] += dC/dtau . a.
hipError_t launch_adjoint_step(bool direct, int force_mode, const float* s, const float* bin,
                               float* bout, float* gF, double* taupart, const uint8_t* flags,
                               const float* ffield, const StepArgs& args, float inv_tau2,
                               const Launch& L);

// The same reverse step with vw = 2 or 4 consecutive x-points per work-item
// (nx % vw == 0, at most 256 work-items per group, grid counting groups).
hipError_t launch_adjoint_stepv(int vw, bool direct, int force_mode, const float* s, const float* bin,
                                float* bout, float* gF, double* taupart, const uint8_t* flags,
                                const uint32_t* smask, const uint32_t* mmask, const float* ffield,
                                const StepArgs& args, float inv_tau2, const Launch& L);

// p[0..n) = 0 (a kernel, not a memset). out[0] = sum of p[0..n) added in
// index order by one work-item.
hipError_t launch_zero_f64(double* p, size_t n, hipStream_t s);
hipError_t launch_sum_f64_ordered(const double* p, size_t n, double* out, hipStream_t s);

}  // namespace lbmk

// pmg_internal.hpp -- host-side interface between the C ABI (pmg_api.cpp)
// and the kernel launchers (pmg_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "pmg.h"
#include "pmg_device.hpp"

namespace pmg {

struct SetupArgs {
    const double* coords[MAX_LEVELS];   // caller's coordinates per level
    double* detmin;                     // [nlev][B]
    int* pivot;                         // [B] nonzero if a zero pivot was met
    double* cr64[MAX_LEVELS][3];        // FP64 line factors per level and axis
    float* cr32[MAX_LEVELS][3];         // FP32 copies (nullptr if unused)
    double* G64[MAX_LEVELS];
    float* G32[MAX_LEVELS];             // nullptr if unused
    double* mass;                       // finest level
    double* cinv64;                     // [B] 1 / A_0 (level 0, one interior node)
    float* cinv32;                      // [B] FP32 copy (nullptr if unused)
    double* X64[MAX_LEVELS];
    const double* rho[MAX_LEVELS];      // GLL weights (device)
    const double* D64[MAX_LEVELS];
    const double* DT64[MAX_LEVELS];
    int smoother;
};

struct SolveArgs {
    const double* b;
    double* x;
    double* V;          // [B][nv][N]
    double* Z;          // [B][restart][N]
    double* Hs;         // [B][hs]
    double* TR64;       // [B][DIM][N]
    pmg_info* info;     // [B]
    long long nv, hs;
    int restart, max_iter, krylov;
    double rtol;
};

// All launchers return a hipError_t value (hipSuccess on success).
hipError_t launch_setup(int dim, int p_fine, int nlev, int B, const SetupArgs& a,
                        pmg_info* info, hipStream_t s);
hipError_t launch_rhs(int dim, int p, int B, const Hier<double>& H64, const double* f,
                      const double* g, double* b, double* tmp, hipStream_t s);
hipError_t launch_lift(int dim, int p, int B, const double* w, const double* g, double* u,
                       hipStream_t s);
hipError_t launch_apply(int dim, int p, bool f32, int B, const void* H, const void* x,
                        void* y, hipStream_t s);
hipError_t launch_restrict(int dim, int p, bool f32, int B, const void* H, const void* rf,
                           void* rc, hipStream_t s);
hipError_t launch_prolong(int dim, int p, bool f32, int B, const void* H, const void* ec,
                          void* xf, hipStream_t s);
hipError_t launch_line_solve(int dim, int p, bool f32, int B, const void* H, int dir,
                             const void* r, void* z, hipStream_t s);
hipError_t launch_line_smooth(int dim, int p, bool f32, int B, const void* H, int dir,
                              const void* r, void* x, hipStream_t s);
hipError_t launch_cycle(int dim, int p, bool f32, int B, const void* H, const void* r,
                        void* y, hipStream_t s);
hipError_t launch_solve_f64(int dim, int p, bool f32, int B, const void* H, const SolveArgs& a,
                            hipStream_t s);
hipError_t launch_solve_f32(int dim, int p, bool f32, int B, const void* H, const SolveArgs& a,
                            hipStream_t s);
inline hipError_t launch_solve(int dim, int p, bool f32, int B, const void* H, const SolveArgs& a,
                               hipStream_t s)
{
    return f32 ? launch_solve_f32(dim, p, f32, B, H, a, s) : launch_solve_f64(dim, p, f32, B, H, a, s);
}
hipError_t launch_line_coefs(int dim, int p, int B, const Hier<double>& H64, int smoother,
                             int dir, double* lo, double* di, double* up, hipStream_t s);

}  // namespace pmg

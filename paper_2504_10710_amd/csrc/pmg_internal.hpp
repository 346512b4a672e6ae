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
    int* sstatus;                       // [B] setup status
    const int* slots;                   // nullable: workgroup -> problem index
    int nslots;                         // workgroups to launch (B without slots)
    double* cr64[MAX_LEVELS][3];        // FP64 line factors per level and axis
    float* cr32[MAX_LEVELS][3];         // FP32 copies (nullptr if unused)
    double* bd64[MAX_LEVELS][3];        // half-bandwidth-2 line rows (GLL band-2 smoother)
    float* bd32[MAX_LEVELS][3];         // FP32 copies (nullptr if unused)
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
    int K;                              // spectral elements per axis (1: one element)
    int l0;                             // coarsest present level
    double* Cc0;                        // K > 1: [B][ni][ni] exact inverse of level l0
};

// Resumable state of one problem's outer solve (kept in the workspace, so a
// solve can be split over several launches with identical arithmetic).
enum { ST_RUNNING = 1, ST_IDLE = 2 };
enum { PH_INIT = 0, PH_RESTART = 1, PH_ARNOLDI = 2 };
struct SolveState {
    int status;   // ST_RUNNING, ST_IDLE, or the final PMG_OK / PMG_E* code
    int it;       // outer iterations so far
    int j;        // FGMRES: position inside the current restart cycle
    int phase;    // PH_*
    double bn;    // ||b||
    double rz;    // PCG: (r, z); FCG: (p, q) of the current direction
};

struct SolveArgs {
    SolveState* st;     // [B] per-problem state
    const int* sstatus; // [B] setup status (PMG_OK, PMG_EGEOM, PMG_EPIVOT)
    const int* slots;   // nullable: workgroup -> problem index
    int budget;         // outer iterations allowed in this launch
    int fresh;          // 1: (re)start every problem from the setup status
    const double* b;
    double* x;
    double* V;          // [B][nv][N]
    double* Z;          // [B][restart][N]
    double* Hs;         // [B][hs]
    double* TR64;       // [B][DIM][N]
    double* EX64;       // [B][ng] FP64 element-local operand (element hierarchies), or null
    int elem;           // 1: the hierarchy has several elements per axis (element kernels)
    pmg_info* info;     // [B]
    long long nv, hs;
    int restart, max_iter, krylov;
    double rtol;
};

// All launchers return a hipError_t value (hipSuccess on success).
hipError_t launch_setup(int dim, int p_fine, int nlev, int B, const SetupArgs& a,
                        pmg_info* info, hipStream_t s);
// tmp: per-problem scratch of N doubles at tmp + b * tmp_stride
hipError_t launch_rhs(int dim, int p, int B, const Hier<double>* H64, const double* f,
                      const double* g, double* b, double* tmp, long long tmp_stride, hipStream_t s,
                      const int* slots = nullptr, int nslots = 0);
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
hipError_t launch_line_smooth(int dim, int p, bool f32, bool elem, int B, const void* H, int dir,
                              const void* r, void* x, hipStream_t s);
hipError_t launch_cycle(int dim, int p, bool f32, bool elem, int B, const void* H, const void* r,
                        void* y, hipStream_t s);
// dense matrices of the collapsed coarse cycle of level pc (collapse_lo(dim)
// or collapse_p(dim); the lower one first) for nb problems (all, or the
// listed slots); elem: the hierarchy has several elements per axis
hipError_t launch_collapse(int dim, int pc, bool f32, bool elem, int nb, const void* H, double* Cc,
                           const int* slots, hipStream_t s);
// grid = B workgroups (problem b = workgroup, or a.slots[workgroup])
hipError_t launch_solve_f64(int dim, int p, bool f32, int B, const void* H, const SolveArgs& a,
                            hipStream_t s);
hipError_t launch_solve_f32(int dim, int p, bool f32, int B, const void* H, const SolveArgs& a,
                            hipStream_t s);
// resident workgroups per CU of the solve kernel (0 if unknown)
int solve_blocks_per_cu_f64(int dim, int p);
int solve_blocks_per_cu_f32(int dim, int p);
inline hipError_t launch_solve(int dim, int p, bool f32, int B, const void* H, const SolveArgs& a,
                               hipStream_t s)
{
    return f32 ? launch_solve_f32(dim, p, f32, B, H, a, s) : launch_solve_f64(dim, p, f32, B, H, a, s);
}
hipError_t launch_pool_start(const int* slots, int n, const int* sstatus, SolveState* st,
                             pmg_info* info, hipStream_t s);
hipError_t launch_pool_idle(SolveState* st, int B, hipStream_t s);
hipError_t launch_pool_take(int dim, int p, int slot, const double* w, const double* g, double* u,
                            SolveState* st, hipStream_t s);
hipError_t launch_pool_take_many(int dim, int p, int n, const int* slots, double* const* outs,
                                 const double* w, const double* g, SolveState* st, hipStream_t s);
// one contiguous copy of n doubles; a batch of them runs as one launch
struct CopyJob {
    const double* src;
    double* dst;
    long long n;
};
hipError_t launch_copy_jobs(int n, const CopyJob* jobs, hipStream_t s);
hipError_t launch_line_coefs(int dim, int p, int B, const Hier<double>* H64, int smoother,
                             int dir, double* lo, double* di, double* up, hipStream_t s);

}  // namespace pmg

// pmg_solve_f64.hip -- instances of the solve kernel, FP64 inner cycle.
// room in LDS for the 2-D operator at p = 64 (x and F0 in FP64) and at
// p = 32 (every operand: x, F0, F1, G, D, D^T)
#define PMG_WORK_LDS_WORDS (8 * 33 * 33)
#include "pmg_solve.hpp"

namespace pmg {

hipError_t launch_solve_f64(int dim, int p, bool f32, int B, const void* H, const SolveArgs& a,
                        hipStream_t s)
{
    // the element instances (several elements per axis) are separate kernels
    if (a.elem)
        PMG_DISPATCH_P(dim, p, hipLaunchKernelGGL((k_solve<double, P_, D_, true>), dim3(B), dim3(NT),
                                                   0, s, (const Hier<double>*)H, a));
    else
        PMG_DISPATCH_P(dim, p, hipLaunchKernelGGL((k_solve<double, P_, D_, false>), dim3(B), dim3(NT),
                                                   0, s, (const Hier<double>*)H, a));
    return last();
}

int solve_blocks_per_cu_f64(int dim, int p)
{
    int nb = 0;
    PMG_DISPATCH_P(dim, p, (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(
                               &nb, k_solve<double, P_, D_, false>, NT, 0));
    return nb;
}

}  // namespace pmg

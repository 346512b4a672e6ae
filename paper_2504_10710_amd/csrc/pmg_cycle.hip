// pmg_cycle.hip -- one gamma-cycle application per problem.
// room in LDS for the 2-D operator at p = 64 (x and F0 in FP64) and at
// p = 32 (every operand: x, F0, F1, G, D, D^T)
#define PMG_WORK_LDS_WORDS (8 * 33 * 33)
#include <cmath>

#include "pmg_dispatch.hpp"

namespace pmg {

template <class T, int P, int DIM, bool E>
__global__ void __launch_bounds__(NT, 4) k_cycle(const Hier<T>* __restrict__ Hp, const T* __restrict__ r, T* __restrict__ y)
{
    const Hier<T>& H = *Hp;
    using S = Shape<P, DIM>;
    const long long b = blockIdx.x;
    gamma_cycle<T, P, DIM, collapse_p(DIM), E>(H, (int)b, r + b * S::N, y + b * S::N);
}

hipError_t launch_cycle(int dim, int p, bool f32, bool elem, int B, const void* H, const void* r,
                        void* y, hipStream_t s)
{
    if (elem)
        PMG_TYPED(f32, PMG_DISPATCH_P(dim, p, hipLaunchKernelGGL((k_cycle<T_, P_, D_, true>), dim3(B),
                                                                  dim3(NT), 0, s, (const Hier<T_>*)H,
                                                                  (const T_*)r, (T_*)y)));
    else
        PMG_TYPED(f32, PMG_DISPATCH_P(dim, p, hipLaunchKernelGGL((k_cycle<T_, P_, D_, false>), dim3(B),
                                                                  dim3(NT), 0, s, (const Hier<T_>*)H,
                                                                  (const T_*)r, (T_*)y)));
    return last();
}

// Build the dense matrix of the gamma-cycle of level PC (with every level
// below it) for each problem: column i = M^{-1} e_i for the i-th interior
// node, the cycle applied to unit vectors in the level's own right-hand side
// and iterate buffers, with the levels below PC applied by their matrices
// where those are already built (with several elements, E, the coarsest
// level's exact inverse among them).  One workgroup per problem (or per
// listed slot).
template <class T, int PC, int DIM, bool E>
__global__ void __launch_bounds__(NT, 4) k_collapse(const Hier<T>* __restrict__ Hp,
                                                    double* __restrict__ Cc,
                                                    const int* __restrict__ slots)
{
    const Hier<T>& H = *Hp;
    using S = Shape<PC, DIM>;
    constexpr int ni = ipow(PC - 1, DIM);
    const int b = slots ? slots[blockIdx.x] : (int)blockIdx.x;
    const LevelData<T>& L = H.lev[S::LEV];
    T* r = L.R + (long long)b * S::N;
    T* x = L.X + (long long)b * S::N;
    const auto rg = gmem(r);
    const auto xg = gmem((const T*)x);
    const auto C = gmem(Cc + (long long)b * ni * ni);
    for (int i = 0; i < ni; ++i) {
        const int qi = interior_node<PC, DIM>(i);
        for (int q = threadIdx.x; q < S::N; q += NT) rg[q] = q == qi ? T(1) : T(0);
        wg_barrier();
        gamma_cycle<T, PC, DIM, PC / 2, E>(H, b, r, x);
        for (int j = threadIdx.x; j < ni; j += NT) C[(long long)i * ni + j] = (double)xg[interior_node<PC, DIM>(j)];
        wg_barrier();
    }
}

template <bool E>
static hipError_t launch_collapse_e(int dim, int pc, bool f32, int nb, const void* H, double* Cc,
                                    const int* slots, hipStream_t s)
{
    if (dim == 2 && pc == collapse_lo(2)) {
        PMG_TYPED(f32, hipLaunchKernelGGL((k_collapse<T_, collapse_lo(2), 2, E>), dim3(nb), dim3(NT),
                                          0, s, (const Hier<T_>*)H, Cc, slots));
    } else if (dim == 2 && pc == collapse_p(2)) {
        PMG_TYPED(f32, hipLaunchKernelGGL((k_collapse<T_, collapse_p(2), 2, E>), dim3(nb), dim3(NT),
                                          0, s, (const Hier<T_>*)H, Cc, slots));
    } else if (dim == 3 && pc == collapse_lo(3)) {
        PMG_TYPED(f32, hipLaunchKernelGGL((k_collapse<T_, collapse_lo(3), 3, E>), dim3(nb), dim3(NT),
                                          0, s, (const Hier<T_>*)H, Cc, slots));
    } else if (dim == 3 && pc == collapse_p(3)) {
        PMG_TYPED(f32, hipLaunchKernelGGL((k_collapse<T_, collapse_p(3), 3, E>), dim3(nb), dim3(NT),
                                          0, s, (const Hier<T_>*)H, Cc, slots));
    } else {
        return hipErrorInvalidValue;
    }
    return last();
}

hipError_t launch_collapse(int dim, int pc, bool f32, bool elem, int nb, const void* H, double* Cc,
                           const int* slots, hipStream_t s)
{
    if (nb <= 0) return hipSuccess;
    return elem ? launch_collapse_e<true>(dim, pc, f32, nb, H, Cc, slots, s)
                : launch_collapse_e<false>(dim, pc, f32, nb, H, Cc, slots, s);
}

}  // namespace pmg

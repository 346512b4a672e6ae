// pmg_cycle.hip -- one gamma-cycle application per problem.
#include <cmath>

#include "pmg_dispatch.hpp"

namespace pmg {

template <class T, int P, int DIM>
__global__ void __launch_bounds__(NT, 4) k_cycle(const Hier<T>* __restrict__ Hp, const T* __restrict__ r, T* __restrict__ y)
{
    const Hier<T>& H = *Hp;
    using S = Shape<P, DIM>;
    const long long b = blockIdx.x;
    gamma_cycle<T, P, DIM>(H, (int)b, r + b * S::N, y + b * S::N);
}

hipError_t launch_cycle(int dim, int p, bool f32, int B, const void* H, const void* r, void* y,
                        hipStream_t s)
{
    PMG_TYPED(f32, PMG_DISPATCH_P(dim, p, hipLaunchKernelGGL((k_cycle<T_, P_, D_>), dim3(B),
                                                              dim3(NT), 0, s, (const Hier<T_>*)H,
                                                              (const T_*)r, (T_*)y)));
    return last();
}

}  // namespace pmg

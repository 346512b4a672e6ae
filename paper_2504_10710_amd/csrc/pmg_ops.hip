// pmg_ops.hip -- level operations as batched kernels (one problem per
// workgroup): operator, transfers, line solve, smoothing step.
#include <cmath>

#include "pmg_dispatch.hpp"

namespace pmg {

// ================================================================== level operations

template <class T, int P, int DIM>
__global__ void __launch_bounds__(NT) k_apply(const Hier<T>* __restrict__ Hp, const T* __restrict__ x, T* __restrict__ y)
{
    const Hier<T>& H = *Hp;
    using S = Shape<P, DIM>;
    const long long b = blockIdx.x;
    const LevelData<T>& L = H.lev[S::LEV];
    apply_any<T, P, DIM, false>(H.K, L.EX ? L.EX + b * L.ng : nullptr, L.G + b * S::NC * L.ng,
                                L.D, L.DT, L.TR + b * DIM * L.ng, x + b * S::N, nullptr,
                                y + b * S::N);
}

template <class T, int P, int DIM>
__global__ void __launch_bounds__(NT) k_restrict(const Hier<T>* __restrict__ Hp, const T* __restrict__ rf, T* __restrict__ rc)
{
    const Hier<T>& H = *Hp;
    using S = Shape<P, DIM>;
    using C = Shape<P / 2, DIM>;
    const long long b = blockIdx.x;
    const LevelData<T>& L = H.lev[S::LEV];
    restrict_level<T, P, DIM>(rf + b * S::N, rc + b * C::N, L.JR, L.JT, H.W1 + b * H.w1,
                              H.W2 ? H.W2 + b * H.w2 : nullptr);
}

template <class T, int P, int DIM>
__global__ void __launch_bounds__(NT) k_prolong(const Hier<T>* __restrict__ Hp, const T* __restrict__ ec, T* __restrict__ xf)
{
    const Hier<T>& H = *Hp;
    using S = Shape<P, DIM>;
    using C = Shape<P / 2, DIM>;
    const long long b = blockIdx.x;
    const LevelData<T>& L = H.lev[S::LEV];
    prolong_level<T, P, DIM>(ec + b * C::N, xf + b * S::N, L.J, L.JT, H.W1 + b * H.w1,
                             H.W2 ? H.W2 + b * H.w2 : nullptr);
}

template <class T, int P, int DIM>
__global__ void __launch_bounds__(NT, 8) k_line_solve(const Hier<T>* __restrict__ Hp, int dir, const T* __restrict__ r,
                                                   T* __restrict__ z)
{
    const Hier<T>& H = *Hp;
    using S = Shape<P, DIM>;
    const long long b = blockIdx.x;
    const LevelData<T>& L = H.lev[S::LEV];
    T* zb = z + b * S::N;
    const T* rb = r + b * S::N;
    if constexpr (wave_lines<P>()) {
        // lane-group lines read r and write z: one pass over each, and the
        // boundary of z set to zero (the lines cover every interior node)
        for (int q = threadIdx.x; q < S::N; q += NT)
            if (is_boundary<P, DIM>(q)) zb[q] = T(0);
        level_lines<T, P, DIM, false>(L, (int)b, dir, const_cast<T*>(rb), zb, T(0));
    } else {
        for (int q = threadIdx.x; q < S::N; q += NT) zb[q] = is_boundary<P, DIM>(q) ? T(0) : rb[q];
        wg_barrier();
        line_cr<T, P, DIM, false>(L.cr[dir] + b * 3 * S::CRW * S::NL, dir, zb, nullptr, T(0));
    }
}

template <class T, int P, int DIM, bool E>
__global__ void __launch_bounds__(NT) k_line_smooth(const Hier<T>* __restrict__ Hp, int dir, const T* __restrict__ r,
                                                    T* __restrict__ x)
{
    const Hier<T>& H = *Hp;
    using S = Shape<P, DIM>;
    const long long b = blockIdx.x;
    smooth_step<T, P, DIM, E>(H, (int)b, dir, r + b * S::N, x + b * S::N, false);
}

hipError_t launch_apply(int dim, int p, bool f32, int B, const void* H, const void* x, void* y,
                        hipStream_t s)
{
    PMG_TYPED(f32, PMG_DISPATCH_P(dim, p, hipLaunchKernelGGL((k_apply<T_, P_, D_>), dim3(B),
                                                              dim3(NT), 0, s, (const Hier<T_>*)H,
                                                              (const T_*)x, (T_*)y)));
    return last();
}

hipError_t launch_restrict(int dim, int p, bool f32, int B, const void* H, const void* rf,
                           void* rc, hipStream_t s)
{
    PMG_TYPED(f32, PMG_DISPATCH_P4(dim, p, hipLaunchKernelGGL((k_restrict<T_, P_, D_>), dim3(B),
                                                               dim3(NT), 0, s, (const Hier<T_>*)H,
                                                               (const T_*)rf, (T_*)rc)));
    return last();
}

hipError_t launch_prolong(int dim, int p, bool f32, int B, const void* H, const void* ec,
                          void* xf, hipStream_t s)
{
    PMG_TYPED(f32, PMG_DISPATCH_P4(dim, p, hipLaunchKernelGGL((k_prolong<T_, P_, D_>), dim3(B),
                                                               dim3(NT), 0, s, (const Hier<T_>*)H,
                                                               (const T_*)ec, (T_*)xf)));
    return last();
}

hipError_t launch_line_solve(int dim, int p, bool f32, int B, const void* H, int dir,
                             const void* r, void* z, hipStream_t s)
{
    PMG_TYPED(f32, PMG_DISPATCH_P(dim, p, hipLaunchKernelGGL((k_line_solve<T_, P_, D_>), dim3(B),
                                                              dim3(NT), 0, s, (const Hier<T_>*)H,
                                                              dir, (const T_*)r, (T_*)z)));
    return last();
}

hipError_t launch_line_smooth(int dim, int p, bool f32, bool elem, int B, const void* H, int dir,
                              const void* r, void* x, hipStream_t s)
{
    if (elem)
        PMG_TYPED(f32, PMG_DISPATCH_P(dim, p, hipLaunchKernelGGL((k_line_smooth<T_, P_, D_, true>),
                                                                  dim3(B), dim3(NT), 0, s,
                                                                  (const Hier<T_>*)H, dir,
                                                                  (const T_*)r, (T_*)x)));
    else
        PMG_TYPED(f32, PMG_DISPATCH_P(dim, p, hipLaunchKernelGGL((k_line_smooth<T_, P_, D_, false>),
                                                                  dim3(B), dim3(NT), 0, s,
                                                                  (const Hier<T_>*)H, dir,
                                                                  (const T_*)r, (T_*)x)));
    return last();
}

}  // namespace pmg

// pmg_solve.hpp -- outer Krylov solve kernel (one problem per workgroup).
#pragma once

#include <cmath>

#include "pmg_dispatch.hpp"

namespace pmg {

// ================================================================== outer Krylov

__device__ inline double wg_dot(const double* a, const double* b, int n, double* red)
{
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += NT) s += a[i] * b[i];
    return wg_sum(s, red);
}

// z = M^{-1} v with the gamma-cycle in T (FP64 in/out)
template <class T, int P, int DIM>
__device__ void precondition(const Hier<T>& H, int b, const double* v, double* z)
{
    using S = Shape<P, DIM>;
    if constexpr (sizeof(T) == sizeof(double)) {
        gamma_cycle<T, P, DIM>(H, b, (const T*)v, (T*)z);
    } else {
        const LevelData<T>& L = H.lev[S::LEV];
        T* r = L.R + (long long)b * S::N;
        T* x = L.X + (long long)b * S::N;
        for (int q = threadIdx.x; q < S::N; q += NT) r[q] = (T)v[q];
        wg_barrier();
        gamma_cycle<T, P, DIM>(H, b, r, x);
        for (int q = threadIdx.x; q < S::N; q += NT) z[q] = (double)x[q];
        wg_barrier();
    }
}

template <class T, int P, int DIM>
__device__ void apply64(const Hier<T>& H, const SolveArgs& A, int b, const double* x,
                        const double* r, double* out)
{
    using S = Shape<P, DIM>;
    const LevelData<T>& L = H.lev[S::LEV];
    if (r)
        apply_level<double, P, DIM, true>(L.G64 + (long long)b * S::NC * S::N, L.D64, L.DT64,
                                          A.TR64 + (long long)b * DIM * S::N, x, r, out);
    else
        apply_level<double, P, DIM, false>(L.G64 + (long long)b * S::NC * S::N, L.D64, L.DT64,
                                           A.TR64 + (long long)b * DIM * S::N, x, nullptr, out);
}

// Right-preconditioned FGMRES with modified Gram-Schmidt and restarts, PCG or
// flexible CG, one workgroup per problem; convergence is declared on the
// true residual ||b - A x|| <= rtol ||b||.
template <class T, int P, int DIM>
__global__ void __launch_bounds__(NT) k_solve(Hier<T> H, SolveArgs A)
{
    using S = Shape<P, DIM>;
    constexpr int N = S::N;
    __shared__ double red[NT];
    __shared__ double sh[4];
    const int b = blockIdx.x;
    const double* bb = A.b + (long long)b * N;
    double* x = A.x + (long long)b * N;
    double* V = A.V + (long long)b * A.nv * N;
    double* Z = A.Z + (long long)b * A.restart * N;
    double* Hs = A.Hs + (long long)b * A.hs;
    pmg_info* info = A.info + b;
    const int kr = A.restart;

    wg_zero(x, N);
    int status = info->status;
    int it = 0;
    double relres = NAN;
    wg_barrier();
    if (status != PMG_OK) {
        if (threadIdx.x == 0) { info->iterations = 0; info->relres = NAN; }
        return;
    }
    const double bn = sqrt(wg_dot(bb, bb, N, red));
    if (!(bn > 0.0)) {
        if (threadIdx.x == 0) {
            info->status = bn == 0.0 ? PMG_OK : PMG_ENAN;
            info->iterations = 0;
            info->relres = 0.0;
        }
        return;
    }
    const double tol = A.rtol * bn;
    status = PMG_ENOTCONV;

    if (A.krylov == PMG_FGMRES) {
        double* Hm = Hs;                         // (kr+1) x kr
        double* cs = Hs + (kr + 1) * kr;
        double* sn = cs + kr;
        double* gv = sn + kr;                    // kr + 1
        double* yv = gv + kr + 1;                // kr
        while (true) {
            apply64<T, P, DIM>(H, A, b, x, bb, V);
            const double beta = sqrt(wg_dot(V, V, N, red));
            relres = beta / bn;
            if (!isfinite(beta)) { status = PMG_ENAN; break; }
            if (beta <= tol) { status = PMG_OK; break; }
            if (it >= A.max_iter) break;
            for (int q = threadIdx.x; q < N; q += NT) V[q] /= beta;
            if (threadIdx.x == 0) {
                gv[0] = beta;
                for (int i = 1; i <= kr; ++i) gv[i] = 0.0;
            }
            int used = 0;
            bool fail = false;
            for (int j = 0; j < kr; ++j) {
                double* vj = V + (long long)j * N;
                double* zj = Z + (long long)j * N;
                double* w = V + (long long)(j + 1) * N;
                precondition<T, P, DIM>(H, b, vj, zj);
                apply64<T, P, DIM>(H, A, b, zj, nullptr, w);
                for (int i = 0; i <= j; ++i) {
                    const double* vi = V + (long long)i * N;
                    const double hij = wg_dot(w, vi, N, red);
                    for (int q = threadIdx.x; q < N; q += NT) w[q] -= hij * vi[q];
                    if (threadIdx.x == 0) Hm[i * kr + j] = hij;
                    wg_barrier();
                }
                const double hn = sqrt(wg_dot(w, w, N, red));
                if (hn > 0.0)
                    for (int q = threadIdx.x; q < N; q += NT) w[q] /= hn;
                if (threadIdx.x == 0) {
                    Hm[(j + 1) * kr + j] = hn;
                    for (int i = 0; i < j; ++i) {
                        const double t = cs[i] * Hm[i * kr + j] + sn[i] * Hm[(i + 1) * kr + j];
                        Hm[(i + 1) * kr + j] = -sn[i] * Hm[i * kr + j] + cs[i] * Hm[(i + 1) * kr + j];
                        Hm[i * kr + j] = t;
                    }
                    const double a = Hm[j * kr + j], c = Hm[(j + 1) * kr + j];
                    const double rr = sqrt(a * a + c * c);
                    double est = -1.0;
                    if (rr > 0.0 && isfinite(rr)) {
                        cs[j] = a / rr;
                        sn[j] = c / rr;
                        Hm[j * kr + j] = rr;
                        Hm[(j + 1) * kr + j] = 0.0;
                        gv[j + 1] = -sn[j] * gv[j];
                        gv[j] = cs[j] * gv[j];
                        est = fabs(gv[j + 1]);
                    }
                    sh[0] = est;
                    sh[1] = hn;
                }
                wg_barrier();
                const double est = sh[0], hnb = sh[1];
                wg_barrier();
                ++it;
                if (est < 0.0) { fail = true; break; }
                used = j + 1;
                if (!isfinite(est)) { fail = true; break; }
                if (est <= tol || hnb == 0.0 || it >= A.max_iter) break;
            }
            if (used > 0) {
                if (threadIdx.x == 0) {
                    for (int i = used - 1; i >= 0; --i) {
                        double s = gv[i];
                        for (int k = i + 1; k < used; ++k) s -= Hm[i * kr + k] * yv[k];
                        yv[i] = s / Hm[i * kr + i];
                    }
                }
                wg_barrier();
                for (int q = threadIdx.x; q < N; q += NT) {
                    double s = x[q];
                    for (int i = 0; i < used; ++i) s += yv[i] * Z[(long long)i * N + q];
                    x[q] = s;
                }
                wg_barrier();
            }
            if (fail) {
                apply64<T, P, DIM>(H, A, b, x, bb, V);
                relres = sqrt(wg_dot(V, V, N, red)) / bn;
                status = isfinite(relres) ? (relres <= A.rtol ? PMG_OK : PMG_EBREAKDOWN) : PMG_ENAN;
                break;
            }
        }
    } else {
        // CG family: V holds r, z, p, q, t
        double* r = V;
        double* z = V + N;
        double* p = V + 2LL * N;
        double* q = V + 3LL * N;
        double* t = V + 4LL * N;
        const bool flex = A.krylov == PMG_FCG;
        wg_copy(r, bb, N);
        wg_barrier();
        precondition<T, P, DIM>(H, b, r, z);
        wg_copy(p, z, N);
        wg_barrier();
        double rz = wg_dot(r, z, N, red);
        if (flex) apply64<T, P, DIM>(H, A, b, p, nullptr, q);
        relres = 1.0;
        while (true) {
            if (!flex) apply64<T, P, DIM>(H, A, b, p, nullptr, q);
            const double pq = wg_dot(p, q, N, red);
            if (!(pq > 0.0)) { status = isfinite(pq) ? PMG_EBREAKDOWN : PMG_ENAN; break; }
            const double al = (flex ? wg_dot(p, r, N, red) : rz) / pq;
            for (int i = threadIdx.x; i < N; i += NT) {
                x[i] += al * p[i];
                r[i] -= al * q[i];
            }
            wg_barrier();
            ++it;
            double rn = sqrt(wg_dot(r, r, N, red));
            if (!isfinite(rn)) { status = PMG_ENAN; break; }
            if (rn <= tol) {
                apply64<T, P, DIM>(H, A, b, x, bb, t);
                const double tn = sqrt(wg_dot(t, t, N, red));
                relres = tn / bn;
                if (tn <= tol) { status = PMG_OK; break; }
                wg_copy(r, t, N);
                wg_barrier();
            }
            relres = rn / bn;
            if (it >= A.max_iter) break;
            precondition<T, P, DIM>(H, b, r, z);
            if (flex) {
                const double be = -wg_dot(z, q, N, red) / pq;
                for (int i = threadIdx.x; i < N; i += NT) p[i] = z[i] + be * p[i];
                wg_barrier();
                apply64<T, P, DIM>(H, A, b, p, nullptr, q);
            } else {
                const double rz2 = wg_dot(r, z, N, red);
                const double be = rz2 / rz;
                rz = rz2;
                for (int i = threadIdx.x; i < N; i += NT) p[i] = z[i] + be * p[i];
                wg_barrier();
            }
        }
        if (status == PMG_ENOTCONV) {
            apply64<T, P, DIM>(H, A, b, x, bb, t);
            relres = sqrt(wg_dot(t, t, N, red)) / bn;
        }
    }
    if (threadIdx.x == 0) {
        info->status = status;
        info->iterations = it;
        info->relres = relres;
    }
}

}  // namespace pmg

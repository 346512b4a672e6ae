// pmg_solve.hpp -- outer Krylov solve (one problem per workgroup), resumable:
// the iteration state lives in the workspace, so one solve may run in one
// launch (pmg_solve) or be advanced a few iterations per launch (the serving
// pools) with exactly the same arithmetic.
#pragma once

#include <cmath>

#include "pmg_dispatch.hpp"

namespace pmg {

__device__ inline double wg_dot(const double* a_, const double* b_, int n, double* red)
{
    const auto a = gmem(a_);
    const auto b = gmem(b_);
    double s = 0.0;
#pragma unroll 4
    for (int i = threadIdx.x; i < n; i += NT) s += a[i] * b[i];
    return wg_sum(s, red);
}

// v /= d
__device__ inline void wg_scale_div(double* __restrict__ v_, double d, int n)
{
    const auto v = gmem(v_);
#pragma unroll 4
    for (int i = threadIdx.x; i < n; i += NT) v[i] = v[i] / d;
}

// z = M^{-1} v with the gamma-cycle in T (FP64 in/out)
template <class T, int P, int DIM, bool E>
__device__ void precondition(const Hier<T>& H, int b, const double* v, double* z)
{
    using S = Shape<P, DIM>;
    if constexpr (sizeof(T) == sizeof(double)) {
        gamma_cycle<T, P, DIM, collapse_p(DIM), E>(H, b, (const T*)v, (T*)z);
    } else {
        const LevelData<T>& L = H.lev[S::LEV];
        T* r = L.R + (long long)b * S::N;
        T* x = L.X + (long long)b * S::N;
        {
            const auto rg = gmem(r);
            const auto vg = gmem(v);
            for (int q = threadIdx.x; q < S::N; q += NT) rg[q] = (T)vg[q];
        }
        wg_barrier();
        gamma_cycle<T, P, DIM, collapse_p(DIM), E>(H, b, r, x);
        {
            const auto zg = gmem(z);
            const auto xg = gmem((const T*)x);
            for (int q = threadIdx.x; q < S::N; q += NT) zg[q] = (double)xg[q];
        }
        wg_barrier();
    }
}

template <class T, int P, int DIM, bool E>
__device__ void apply64(const Hier<T>& H, const SolveArgs& A, int b, const double* x,
                        const double* r, double* out)
{
    using S = Shape<P, DIM>;
    const LevelData<T>& L = H.lev[S::LEV];
    if constexpr (E) {
        // the FP64 element-local operand of an element hierarchy's finest level
        double* ex = A.EX64 ? A.EX64 + (long long)b * L.ng : nullptr;
        if (r)
            apply_elements_level<double, P, DIM, true>(H.K, L.G64 + (long long)b * S::NC * L.ng,
                                                       L.D64, L.DT64,
                                                       A.TR64 + (long long)b * DIM * L.ng, ex, x, r,
                                                       out);
        else
            apply_elements_level<double, P, DIM, false>(H.K, L.G64 + (long long)b * S::NC * L.ng,
                                                        L.D64, L.DT64,
                                                        A.TR64 + (long long)b * DIM * L.ng, ex, x,
                                                        nullptr, out);
    } else {
        if (r)
            apply_level<double, P, DIM, true>(L.G64 + (long long)b * S::NC * S::N, L.D64, L.DT64,
                                              A.TR64 + (long long)b * DIM * S::N, x, r, out);
        else
            apply_level<double, P, DIM, false>(L.G64 + (long long)b * S::NC * S::N, L.D64, L.DT64,
                                               A.TR64 + (long long)b * DIM * S::N, x, nullptr, out);
    }
}

// Modified Gram-Schmidt for column j of the Arnoldi process: for i = 0..j,
// h_i = <w, v_i> and w -= h_i v_i, in that order.  The subtraction of v_i
// and the partial products of the next inner product (with v_{i+1}, or
// <w, w> after the last one) share one pass over w, so each basis vector
// costs one pass and one reduction.  Returns ||w|| after orthogonalisation;
// H[i * ldh] = h_i.
// One pass of the column: w -= h v_i and this thread's part of <w, v_next>
// (or of <w, w> after the last basis vector).  The three vectors are distinct
// (restrict), so the loads of several elements can be issued together.
__device__ inline double mgs_pass(double* __restrict__ w_, const double* __restrict__ vi_,
                                  const double* __restrict__ vn_, double h, int N)
{
    const auto w = gmem(w_);
    const auto vi = gmem(vi_);
    const auto vn = gmem(vn_);
    double d = 0.0;
#pragma unroll 4
    for (int q = threadIdx.x; q < N; q += NT) {
        const double wq = w[q] - h * vi[q];
        w[q] = wq;
        d += wq * vn[q];
    }
    return d;
}

__device__ inline double mgs_pass_last(double* __restrict__ w_, const double* __restrict__ vi_,
                                       double h, int N)
{
    const auto w = gmem(w_);
    const auto vi = gmem(vi_);
    double d = 0.0;
#pragma unroll 4
    for (int q = threadIdx.x; q < N; q += NT) {
        const double wq = w[q] - h * vi[q];
        w[q] = wq;
        d += wq * wq;
    }
    return d;
}

__device__ inline double mgs_column(double* w_, const double* V_, long long N, int j, double* H,
                                    int ldh, double* red)
{
    const auto w = gmem(w_);
    const auto V = gmem(V_);
    double d = 0.0;
    for (long long q = threadIdx.x; q < N; q += NT) d += w[q] * V[q];
    double h = wg_sum(d, red);
    for (int i = 0; i <= j; ++i) {
        d = i < j ? mgs_pass(w_, V_ + i * N, V_ + (i + 1) * N, h, (int)N)
                  : mgs_pass_last(w_, V_ + i * N, h, (int)N);
        if (threadIdx.x == 0) H[i * ldh] = h;
        h = wg_sum(d, red);
    }
    return sqrt(h);
}

// Right-preconditioned flexible GMRES (Arnoldi by modified Gram-Schmidt),
// restarted every `restart` iterations; PCG; flexible CG.  Convergence is declared on the
// true residual ||b - A x|| <= rtol ||b||.  At most A.budget iterations are
// taken in this launch; the state is saved in A.st[b].
template <class T, int P, int DIM, bool E>
__global__ void __launch_bounds__(NT, 4) k_solve(const Hier<T>* __restrict__ Hp, SolveArgs A)
{
    const Hier<T>& H = *Hp;
    using S = Shape<P, DIM>;
    constexpr int N = S::N;
    __shared__ double red[NT];
    __shared__ double sh[4];
    const int b = A.slots ? A.slots[blockIdx.x] : (int)blockIdx.x;
    const double* bb = A.b + (long long)b * N;
    double* x = A.x + (long long)b * N;
    double* V = A.V + (long long)b * A.nv * N;
    double* Z = A.Z + (long long)b * A.restart * N;
    double* Hs = A.Hs + (long long)b * A.hs;
    pmg_info* info = A.info + b;
    SolveState* stp = A.st + b;
    const int kr = A.restart;

    SolveState st = *stp;
    if (A.fresh) {
        st.status = A.sstatus[b] == PMG_OK ? ST_RUNNING : A.sstatus[b];
        st.it = 0;
        st.j = 0;
        st.phase = PH_INIT;
        st.bn = 0.0;
        st.rz = 0.0;
    }
    if (st.status != ST_RUNNING) {
        if (A.fresh && threadIdx.x == 0) {
            *stp = st;
            info->status = st.status;
            info->iterations = 0;
            info->relres = NAN;
        }
        if (A.fresh) wg_zero(x, N);
        return;
    }
    double relres = info->relres;
    int budget = A.budget;
    const bool fgmres = A.krylov == PMG_FGMRES;
    const bool flex = A.krylov == PMG_FCG;

    if (st.phase == PH_INIT) {
        wg_zero(x, N);
        wg_barrier();
        st.bn = sqrt(wg_dot(bb, bb, N, red));
        if (!(st.bn > 0.0)) {
            st.status = st.bn == 0.0 ? PMG_OK : PMG_ENAN;
            relres = 0.0;
            goto done;
        }
        if (fgmres) {
            st.phase = PH_RESTART;
        } else {
            double* r = V;
            double* z = V + N;
            double* pp = V + 2LL * N;
            double* q = V + 3LL * N;
            wg_copy(r, bb, N);
            wg_barrier();
            precondition<T, P, DIM, E>(H, b, r, z);
            wg_copy(pp, z, N);
            wg_barrier();
            if (flex) {
                apply64<T, P, DIM, E>(H, A, b, pp, nullptr, q);
                st.rz = wg_dot(pp, q, N, red);
            } else {
                st.rz = wg_dot(r, z, N, red);
            }
            relres = 1.0;
            st.phase = PH_RESTART;
        }
    }

    if (fgmres) {
        double* Hm = Hs;                         // (kr+1) x kr
        double* cs = Hs + (kr + 1) * kr;
        double* sn = cs + kr;
        double* gv = sn + kr;                    // kr + 1
        double* yv = gv + kr + 1;                // kr
        const double tol = A.rtol * st.bn;
        for (;;) {
            if (st.phase == PH_RESTART) {
                apply64<T, P, DIM, E>(H, A, b, x, bb, V);
                const double beta = sqrt(wg_dot(V, V, N, red));
                relres = beta / st.bn;
                if (!isfinite(beta)) { st.status = PMG_ENAN; goto done; }
                if (beta <= tol) { st.status = PMG_OK; goto done; }
                if (st.it >= A.max_iter) { st.status = PMG_ENOTCONV; goto done; }
                wg_scale_div(V, beta, N);
                if (threadIdx.x == 0) {
                    gv[0] = beta;
                    for (int i = 1; i <= kr; ++i) gv[i] = 0.0;
                }
                wg_barrier();
                st.j = 0;
                st.phase = PH_ARNOLDI;
            }
            if (budget <= 0) break;
            // one Arnoldi step
            const int j = st.j;
            double* vj = V + (long long)j * N;
            double* zj = Z + (long long)j * N;
            double* w = V + (long long)(j + 1) * N;
            precondition<T, P, DIM, E>(H, b, vj, zj);
            apply64<T, P, DIM, E>(H, A, b, zj, nullptr, w);
            const double hn = mgs_column(w, V, N, j, Hm + j, kr, red);
            if (hn > 0.0) wg_scale_div(w, hn, N);
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
            ++st.it;
            --budget;
            const bool fail = !(est >= 0.0) || !isfinite(est);
            const int used = fail ? j : j + 1;
            st.j = j + 1;
            if (fail || est <= tol || hnb == 0.0 || st.it >= A.max_iter || st.j == kr) {
                // end of the restart cycle: x += Z y with H y = g
                if (used > 0) {
                    if (threadIdx.x == 0) {
                        for (int i = used - 1; i >= 0; --i) {
                            double s = gv[i];
                            for (int k = i + 1; k < used; ++k) s -= Hm[i * kr + k] * yv[k];
                            yv[i] = s / Hm[i * kr + i];
                        }
                    }
                    wg_barrier();
                    const auto xg = gmem(x);
                    const auto Zg = gmem((const double*)Z);
                    for (int q = threadIdx.x; q < N; q += NT) {
                        double s = xg[q];
                        for (int i = 0; i < used; ++i) s += yv[i] * Zg[(long long)i * N + q];
                        xg[q] = s;
                    }
                    wg_barrier();
                }
                st.phase = PH_RESTART;
                if (fail) {
                    apply64<T, P, DIM, E>(H, A, b, x, bb, V);
                    relres = sqrt(wg_dot(V, V, N, red)) / st.bn;
                    st.status = isfinite(relres) ? (relres <= A.rtol ? PMG_OK : PMG_EBREAKDOWN) : PMG_ENAN;
                    goto done;
                }
            }
        }
    } else {
        // CG family: V holds r, z, p, q, t
        double* r = V;
        double* z = V + N;
        double* pp = V + 2LL * N;
        double* q = V + 3LL * N;
        double* t = V + 4LL * N;
        const double tol = A.rtol * st.bn;
        while (budget > 0) {
            if (!flex) apply64<T, P, DIM, E>(H, A, b, pp, nullptr, q);
            const double pq = flex ? st.rz : wg_dot(pp, q, N, red);
            if (!(pq > 0.0)) { st.status = isfinite(pq) ? PMG_EBREAKDOWN : PMG_ENAN; goto done; }
            const double al = (flex ? wg_dot(pp, r, N, red) : st.rz) / pq;
            {
                const auto xg = gmem(x), rg = gmem(r);
                const auto pg = gmem((const double*)pp), qg = gmem((const double*)q);
                for (int i = threadIdx.x; i < N; i += NT) {
                    xg[i] += al * pg[i];
                    rg[i] -= al * qg[i];
                }
            }
            wg_barrier();
            ++st.it;
            --budget;
            const double rn = sqrt(wg_dot(r, r, N, red));
            if (!isfinite(rn)) { st.status = PMG_ENAN; goto done; }
            relres = rn / st.bn;
            if (rn <= tol) {
                apply64<T, P, DIM, E>(H, A, b, x, bb, t);
                const double tn = sqrt(wg_dot(t, t, N, red));
                relres = tn / st.bn;
                if (tn <= tol) { st.status = PMG_OK; goto done; }
                wg_copy(r, t, N);
                wg_barrier();
            }
            if (st.it >= A.max_iter) {
                apply64<T, P, DIM, E>(H, A, b, x, bb, t);
                relres = sqrt(wg_dot(t, t, N, red)) / st.bn;
                st.status = PMG_ENOTCONV;
                goto done;
            }
            precondition<T, P, DIM, E>(H, b, r, z);
            if (flex) {
                const double be = -wg_dot(z, q, N, red) / pq;
                const auto pg = gmem(pp);
                const auto zg = gmem((const double*)z);
                for (int i = threadIdx.x; i < N; i += NT) pg[i] = zg[i] + be * pg[i];
                wg_barrier();
                apply64<T, P, DIM, E>(H, A, b, pp, nullptr, q);
                st.rz = wg_dot(pp, q, N, red);
            } else {
                const double rz2 = wg_dot(r, z, N, red);
                const double be = rz2 / st.rz;
                st.rz = rz2;
                const auto pg = gmem(pp);
                const auto zg = gmem((const double*)z);
                for (int i = threadIdx.x; i < N; i += NT) pg[i] = zg[i] + be * pg[i];
                wg_barrier();
            }
        }
    }
done:
    if (threadIdx.x == 0) {
        *stp = st;
        info->relres = relres;
        info->iterations = st.it;
        info->status = st.status;
    }
}

}  // namespace pmg

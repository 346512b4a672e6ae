// pmg_device.hpp -- device-side building blocks of the gfx950 p-multigrid
// gamma-cycle with cyclic-reduction line smoothers (arXiv 2504.10710).
//
// Execution model: one workgroup of NT threads owns one problem of a batch
// and runs every operation of that problem cooperatively; workgroup barriers
// separate dependent phases.  Problems never share a workgroup, so results
// do not depend on what else is in the batch.  All level data lives in the
// caller's workspace in HBM; the per-problem working set of the smaller
// levels stays in L2.
//
// Layouts (per problem, all levels):
//   vectors     N = (p+1)^dim nodes, first axis fastest
//   G           ncomp arrays of N: 2-D (G00, G11, G01), 3-D (G00, G11, G22,
//               G01, G02, G12): weighted inverse metric of the mapping
//   line data   per axis: 3 words x CRW x NL, where NL = (p-1)^(dim-1)
//               lines, CRW = sum over cyclic-reduction levels of the level's
//               unknown count; word (slot, w) of a line at (slot*3 + w)*NL +
//               line (line index fastest, one thread per line), except for
//               p <= 128: line-major (line*CRW + slot)*3 + w, one lane group
//               per line, holding only the raw rows of level 0 (operators
//               built on the fly)
#pragma once

#include <hip/hip_runtime.h>

namespace pmg {

constexpr int NT = 512;          // threads per workgroup (one problem each)
constexpr int MAX_LEVELS = 9;
// smallest degree whose operator and transfers run on the matrix cores
// (16x16 tiles over rows and columns 1..p); below it the vector units.  The
// 2-D operator and transfers start at p = 16, where their operands are
// staged in LDS.
constexpr int MFMA_MIN_P = 32;
constexpr int MFMA_MIN_P2 = 16;

__host__ __device__ constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }
__host__ __device__ constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

// Number of unknowns summed over the cyclic-reduction levels of a line of n
// unknowns (n = 2^q - 1: levels of 2^(q-k) - 1 unknowns, k = 0..q-1).
__host__ __device__ constexpr int cr_words(int n) { return n <= 1 ? n : n + cr_words(n / 2); }

template <int P, int DIM>
struct Shape {
    static constexpr int n1 = P + 1;
    static constexpr int N = ipow(n1, DIM);
    static constexpr int n = P - 1;
    static constexpr int NL = ipow(n, DIM - 1);
    static constexpr int NC = DIM == 2 ? 3 : 6;
    static constexpr int CRW = cr_words(n);
    static constexpr int LEV = ilog2(P) - 1;   // level index (p = 2 is level 0)
};

// index of G_ab in the packed component list
__host__ __device__ constexpr int gidx(int dim, int a, int b)
{
    return a == b ? a : (dim == 2 ? 2 : (a + b == 1 ? 3 : (a + b == 2 ? 4 : 5)));
}

template <class T>
struct LevelData {
    const double* G64;   // [B][NC][N] FP64 geometric factors
    const T* G;          // [B][NC][N] in T (aliases G64 for T = double)
    const double* mass;  // [B][N] finest level only
    const double* X64;   // [B][DIM][N] physical node coordinates
    const T* cr[3];      // [B][3][CRW][NL] cyclic-reduction factors per axis
    const T* bd[3];      // [B][NL][n][5] half-bandwidth-2 line rows per axis (entries at
                         // offsets -2..2 along the line, zero outside it), or null
    T* X;                // [B][N] level iterate
    T* R;                // [B][N] level right-hand side
    T* Tm;               // [B][N] residual / line-solve buffer
    T* TR;               // [B][DIM][N] apply fluxes
    T* EX;               // [B][ng] K > 1: element-local operand and output of the element
                         // operator on the matrix cores (element degree >= 16), or null
    const T* D;          // [n1][n1]  D[i][j] = pi_j'(xi_i)
    const T* DT;         // [n1][n1]  transpose
    const T* J;          // [n1][n1c] prolongation from the next coarser level
    const T* JT;         // [n1c][n1]
    const T* JR;         // [n1][n1c] restriction to the next coarser level, transposed:
                         // R = JR^T (x) JR^T [(x) JR^T]; JR = J for R = P^T, JR[i][j] =
                         // pi^f_i(xi^c_j) (fine basis at the coarse nodes) for interpolation
    const double* D64;
    const double* DT64;
    long long ng;        // per-problem nodes of G and TR: N, or for K elements per
                         // axis the K^dim (p/K + 1)^dim element nodes
};

template <class T>
struct Hier {
    LevelData<T> lev[MAX_LEVELS];
    const T* cinv;       // [B] 1 / A_0 of the one interior node of level 0
    const double* cinv64;   // the same in FP64 (the coarsest solve stays FP64)
    const double* Cc[MAX_LEVELS];   // [B][ni][ni] the gamma-cycle of that level (with the
                         // levels below it) as a dense matrix over its ni interior
                         // nodes, column after column; null where not collapsed
    T* W1;               // [B][w1] transfer temporaries
    T* W2;               // [B][w2]
    long long w1, w2;    // per-problem sizes of W1, W2
    int nlev, gamma, m;
    int K;               // spectral elements per axis (1: one element)
    T alpha;
};

// ------------------------------------------------------------------ utilities

__device__ inline void wg_barrier() { __syncthreads(); }

// The workspace pointers reach device code through structures in memory, so
// the compiler cannot prove that they address global memory and would emit
// flat accesses, which are waited for together with LDS traffic.  Hot code
// converts them once with gmem() so that loads and stores are global ones.
template <class T>
__device__ inline __attribute__((address_space(1))) T* gmem(T* p)
{
    return (__attribute__((address_space(1))) T*)p;
}
template <class T>
__device__ inline __attribute__((address_space(1))) T* gmem(__attribute__((address_space(1))) T* p)
{
    return p;
}

// LDS pointers pass through unchanged (operands staged in LDS)
template <class T>
__device__ inline __attribute__((address_space(3))) T* gmem(__attribute__((address_space(3))) T* p)
{
    return p;
}

// One LDS work buffer per kernel, shared by the phases of a workgroup that
// stage data on chip (strided line strips, the collapsed solve's right-hand
// side, the operands and fluxes of the 2-D operator at p <= 64); every phase
// ends with a barrier before the next one writes it.  Its size is set per
// compilation unit: the one-launch solve and cycle kernels take room for the
// p = 32 operator's eight fields of 33^2 FP64 words (70 KB, which also holds
// two p = 64 fields; still two workgroups per CU), the single-operation
// kernels the line strip only.
#ifndef PMG_WORK_LDS_WORDS
#define PMG_WORK_LDS_WORDS (127 * 17)
#endif
__device__ inline void* work_lds()
{
    __shared__ double buf[PMG_WORK_LDS_WORDS];
    return buf;
}

template <class T>
__device__ inline void wg_copy(T* __restrict__ dst_, const T* __restrict__ src_, int n)
{
    const auto dst = gmem(dst_);
    const auto src = gmem(src_);
    for (int i = threadIdx.x; i < n; i += NT) dst[i] = src[i];
}

template <class T>
__device__ inline void wg_zero(T* dst_, int n)
{
    const auto dst = gmem(dst_);
    for (int i = threadIdx.x; i < n; i += NT) dst[i] = T(0);
}

// Deterministic workgroup reductions: every thread first folds its own
// elements in a fixed order, then a fixed binary tree over the NT partial
// results in LDS (red: NT doubles).  The result does not depend on timing or
// on other workgroups.
__device__ inline double wg_sum(double v, double* red)
{
    red[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__device__ inline double wg_min(double v, double* red)
{
    red[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

template <int P, int DIM>
__device__ inline bool is_boundary(int q)
{
    constexpr int n1 = P + 1;
    int c0 = q % n1, c1 = (q / n1) % n1;
    bool bd = c0 == 0 || c0 == P || c1 == 0 || c1 == P;
    if (DIM == 3) {
        int c2 = q / (n1 * n1);
        bd = bd || c2 == 0 || c2 == P;
    }
    return bd;
}

// ------------------------------------------------------------------ operator

// ------------------------------------------------------------------ MFMA tiles

// 16x16x4 matrix-core step: A fragment lane l holds A[l % 16][l / 16], B fragment
// B[l / 16][l % 16]; accumulator register v of lane l holds C[row(l, v)][l % 16]
// with row = 4 (l / 16) + v for FP32 and (l / 16) + 4 v for FP64 (measured).
template <class T>
struct Mfma;
template <>
struct Mfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    __device__ static inline v4 op(double a, double b, v4 c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static inline int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <>
struct Mfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    __device__ static inline v4 op(float a, float b, v4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static inline int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// Two independent 16x16 matrix-core products on one wave, accumulated over
// k = 0 .. K-1: c0 += A0 B0 and c1 += A1 B1.  a0 / a1 point at the lane's A
// element (row r + lane % 16, column lane / 16), b0 / b1 at its B element
// (row lane / 16, column c + lane % 16); SA* and SB* are the element strides
// between consecutive k.  The operand loads of the next PF k-steps are issued
// before the current matrix-core steps so that their latency overlaps the
// matrix core; the k tail past the last multiple of 4 contributes zero.
template <class T, int K, int SA0, int SB0, int SA1, int SB1, class PA0, class PB0, class PA1,
          class PB1>
__device__ inline void mfma2(PA0 a0_, PB0 b0_, PA1 a1_, PB1 b1_,
                             typename Mfma<T>::v4& c0, typename Mfma<T>::v4& c1)
{
    const auto a0 = gmem(a0_);
    const auto b0 = gmem(b0_);
    const auto a1 = gmem(a1_);
    const auto b1 = gmem(b1_);
    constexpr int KS = K / 4;
    constexpr int PF = 2;
    T x0[PF], y0[PF], x1[PF], y1[PF];
#pragma unroll
    for (int u = 0; u < PF; ++u)
        if (u < KS) {
            x0[u] = a0[4 * u * SA0];
            y0[u] = b0[4 * u * SB0];
            x1[u] = a1[4 * u * SA1];
            y1[u] = b1[4 * u * SB1];
        }
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        const int u = s % PF;
        const T p0 = x0[u], q0 = y0[u], p1 = x1[u], q1 = y1[u];
        if (s + PF < KS) {
            x0[u] = a0[4 * (s + PF) * SA0];
            y0[u] = b0[4 * (s + PF) * SB0];
            x1[u] = a1[4 * (s + PF) * SA1];
            y1[u] = b1[4 * (s + PF) * SB1];
        }
        c0 = Mfma<T>::op(p0, q0, c0);
        c1 = Mfma<T>::op(p1, q1, c1);
    }
    if constexpr (K % 4 != 0) {
        const int kq = (threadIdx.x & 63) >> 4;
        const bool in = 4 * KS + kq < K;
        const int kk = (in ? 4 * KS + kq : K - 1) - kq;   // stays inside the row / column
        T p0 = a0[kk * SA0], q0 = b0[kk * SB0], p1 = a1[kk * SA1], q1 = b1[kk * SB1];
        if (!in) { p0 = T(0); q0 = T(0); p1 = T(0); q1 = T(0); }
        c0 = Mfma<T>::op(p0, q0, c0);
        c1 = Mfma<T>::op(p1, q1, c1);
    }
}

// C (M x N, row-major) = A B (MODE 0), += A B (MODE 1), or = A B with the
// boundary rows and columns set to zero (MODE 2), for row-major A (M x K,
// leading dimension LDA) and B (K x N, LDB).  ATR: A is given by its
// transpose (K x M, row-major, leading dimension LDA), which the 16 lanes of
// a k-step read as 16 consecutive words.  NS > 1: NS products C_s = A B_s
// with B_s = B + s SB and C_s = C + s SC (one A), and MODE 2 also zeroes the
// first and last slab (the boundary faces of a 3-D box).  Each wave computes
// a 16 x 32 block as two 16x16 tiles that share their A rows; rows and
// columns past M, N are clamped in the loads and never stored.
template <class T, int M, int N, int K, int LDA, int LDB, int MODE, bool ATR = false, int NS = 1,
          int SB = 0, int SC = 0, class PA, class PB, class PC>
__device__ void wg_gemm(PA __restrict__ A, PB __restrict__ B_, PC __restrict__ C_)
{
    const auto C = gmem(C_);
    constexpr int TM = (M + 15) / 16, TN2 = (N + 31) / 32;
    using V4 = typename Mfma<T>::v4;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, kq = lane >> 4;
    for (int t = wave; t < NS * TM * TN2; t += NT / 64) {
        const int sl = t / (TM * TN2), tt = t % (TM * TN2);
        const int r0 = (tt / TN2) * 16, c0 = (tt % TN2) * 32;
        const int ar = min(r0 + lr, M - 1);
        const int bc0 = min(c0 + lr, N - 1), bc1 = min(c0 + 16 + lr, N - 1);
        const auto B = B_ + (long long)sl * SB;
        const auto Cs = C + (long long)sl * SC;
        V4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
        constexpr int SA = ATR ? LDA : 1;
        const auto ap = ATR ? A + kq * LDA + ar : A + ar * LDA + kq;
        mfma2<T, K, SA, LDB, SA, LDB>(ap, B + kq * LDB + bc0, ap, B + kq * LDB + bc1, acc0, acc1);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int i = c0 + 16 * h + lr;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int j = r0 + Mfma<T>::row(lane, v);
                const T a = h ? acc1[v] : acc0[v];
                if (j < M && i < N) {
                    if (MODE == 1)
                        Cs[j * N + i] += a;
                    else if (MODE == 2)
                        Cs[j * N + i] = (j == 0 || j == M - 1 || i == 0 || i == N - 1 ||
                                         (NS > 1 && (sl == 0 || sl == NS - 1)))
                                            ? T(0)
                                            : a;
                    else
                        Cs[j * N + i] = a;
                }
            }
        }
    }
    wg_barrier();
}

// Register-blocked form of mfma2 for BR x BC tiles per product: c0[i][j] +=
// A0_i B0_j and c1[i][j] += A1_i B1_j over k = 0 .. K-1, where A_i are the
// row strips 16 i apart (row stride LDA*, k stride KA*) and B_j the column
// strips 16 j apart (row-major, leading dimension LDB*, stride LDB* in k).
// A row-major A has LDA = its leading dimension and KA = 1; an A read from
// its stored transpose has LDA = 1 and KA = the transpose's leading
// dimension, so that the 16 lanes of a k-step read 16 consecutive words.
// Pointers as in mfma2 (the lane's element of the first strip).  Each
// operand fragment feeds BR or BC matrix-core steps, so a block needs
// BR + BC loads per product and k-step instead of 2 BR BC.  c0 and c1 may be
// the same array (both products then accumulate into it).  NP = 1 computes
// only the first product (a1, b1, c1 unused).
template <class T, int K, int LDA0, int LDB0, int LDA1, int LDB1, int BR, int BC, int NP = 2,
          int KA0 = 1, int KA1 = 1, class PA0, class PB0, class PA1, class PB1>
__device__ inline void mfma_blocks(PA0 a0_, PB0 b0_, PA1 a1_, PB1 b1_,
                                   typename Mfma<T>::v4 (&c0)[BR][BC],
                                   typename Mfma<T>::v4 (&c1)[BR][BC])
{
    static_assert(NP == 1 || NP == 2, "one or two products");
    const auto a0 = gmem(a0_);
    const auto b0 = gmem(b0_);
    const auto a1 = gmem(a1_);
    const auto b1 = gmem(b1_);
    constexpr int KS = K / 4;
    constexpr int PF = 2;
    T xa0[PF][BR], xb0[PF][BC], xa1[PF][BR], xb1[PF][BC];
#pragma unroll
    for (int u = 0; u < PF; ++u)
        if (u < KS) {
#pragma unroll
            for (int i = 0; i < BR; ++i) {
                xa0[u][i] = a0[i * 16 * LDA0 + 4 * u * KA0];
                if constexpr (NP == 2) xa1[u][i] = a1[i * 16 * LDA1 + 4 * u * KA1];
            }
#pragma unroll
            for (int j = 0; j < BC; ++j) {
                xb0[u][j] = b0[j * 16 + 4 * u * LDB0];
                if constexpr (NP == 2) xb1[u][j] = b1[j * 16 + 4 * u * LDB1];
            }
        }
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        const int u = s % PF;
        T pa0[BR], pb0[BC], pa1[BR], pb1[BC];
#pragma unroll
        for (int i = 0; i < BR; ++i) {
            pa0[i] = xa0[u][i];
            if constexpr (NP == 2) pa1[i] = xa1[u][i];
        }
#pragma unroll
        for (int j = 0; j < BC; ++j) {
            pb0[j] = xb0[u][j];
            if constexpr (NP == 2) pb1[j] = xb1[u][j];
        }
        if (s + PF < KS) {
#pragma unroll
            for (int i = 0; i < BR; ++i) {
                xa0[u][i] = a0[i * 16 * LDA0 + 4 * (s + PF) * KA0];
                if constexpr (NP == 2) xa1[u][i] = a1[i * 16 * LDA1 + 4 * (s + PF) * KA1];
            }
#pragma unroll
            for (int j = 0; j < BC; ++j) {
                xb0[u][j] = b0[j * 16 + 4 * (s + PF) * LDB0];
                if constexpr (NP == 2) xb1[u][j] = b1[j * 16 + 4 * (s + PF) * LDB1];
            }
        }
#pragma unroll
        for (int i = 0; i < BR; ++i)
#pragma unroll
            for (int j = 0; j < BC; ++j) c0[i][j] = Mfma<T>::op(pa0[i], pb0[j], c0[i][j]);
        if constexpr (NP == 2) {
#pragma unroll
            for (int i = 0; i < BR; ++i)
#pragma unroll
                for (int j = 0; j < BC; ++j) c1[i][j] = Mfma<T>::op(pa1[i], pb1[j], c1[i][j]);
        }
    }
    if constexpr (K % 4 != 0) {
        const int kq = (threadIdx.x & 63) >> 4;
        const bool in = 4 * KS + kq < K;
        const int kk = (in ? 4 * KS + kq : K - 1) - kq;   // stays inside the row / column
        T pa0[BR], pb0[BC], pa1[BR], pb1[BC];
#pragma unroll
        for (int i = 0; i < BR; ++i) {
            pa0[i] = in ? a0[i * 16 * LDA0 + kk * KA0] : T(0);
            if constexpr (NP == 2) pa1[i] = in ? a1[i * 16 * LDA1 + kk * KA1] : T(0);
        }
#pragma unroll
        for (int j = 0; j < BC; ++j) {
            pb0[j] = in ? b0[j * 16 + kk * LDB0] : T(0);
            if constexpr (NP == 2) pb1[j] = in ? b1[j * 16 + kk * LDB1] : T(0);
        }
#pragma unroll
        for (int i = 0; i < BR; ++i)
#pragma unroll
            for (int j = 0; j < BC; ++j) c0[i][j] = Mfma<T>::op(pa0[i], pb0[j], c0[i][j]);
        if constexpr (NP == 2) {
#pragma unroll
            for (int i = 0; i < BR; ++i)
#pragma unroll
                for (int j = 0; j < BC; ++j) c1[i][j] = Mfma<T>::op(pa1[i], pb1[j], c1[i][j]);
        }
    }
}

// 2-D A x on matrix cores.  Pass 1: the reference gradients x D^T and D x at
// the nodes with both indices in 1..P, one wave per block of BLK x BLK
// 16x16 tiles (both gradients of the block), combined into the fluxes at
// once; row 0 and column 0 on the vector units.  Pass 2: F0 D + D^T F1 on
// the same blocks, both products accumulating into one set of tiles; the
// boundary rows and columns are zero.  Where the work buffer holds them
// (p <= 64), x and F0 (and F1 where three fields fit) live in LDS: x is
// read once from memory and the flux round trip stays on chip; the
// arithmetic is the same.
// The two passes of apply2d_mfma on operands given by their own pointers
// (LDS or global): G the geometric factors, D / DT the derivative matrix and
// its transpose, xs the operand of the first pass, xb the operand of the
// boundary gradients (in D's memory), f0 / f1 the fluxes (F1SEP false: F1
// follows F0 at f0 + N, one base pointer, which is how the global form is
// compiled best).
template <class T, int P, bool RESID, bool F1SEP, class PG, class PD, class PX, class PB, class PF0,
          class PF1>
__device__ inline void apply2d_mfma_passes(PG __restrict__ G, PD __restrict__ D,
                                           PD __restrict__ DT, PX __restrict__ xs,
                                           PB __restrict__ xb, PF0 __restrict__ f0,
                                           PF1 __restrict__ f1, const T* __restrict__ r_,
                                           T* __restrict__ out_)
{
    const auto r = gmem(r_);
    const auto out = gmem(out_);
    // tiles per block side: 2 x 2 blocks at p >= 128; at p = 64 single tiles
    // keep all eight waves busy and the function under fewer registers to
    // save and restore per call (measured faster inside the cycle)
    constexpr int BLK = P >= 128 ? 2 : 1;
    constexpr int n1 = P + 1, N = n1 * n1, NB = P / (16 * BLK);
    using V4 = typename Mfma<T>::v4;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, kq = lane >> 4;
    // p = 128 (4 x 4 blocks, two rounds of eight): each round's two block
    // rows of the row-major operand (64 full rows, x in pass 1, F0 in pass
    // 2) are staged in the LDS work buffer where it holds them, so that the
    // four waves sharing a row strip read it from LDS instead of L2 / memory
    constexpr int LDSW = PMG_WORK_LDS_WORDS * (int)(sizeof(double) / sizeof(T));
    constexpr bool STRIPS = BLK == 2 && NB == 4 && 64 * n1 <= LDSW;
    static_assert(!STRIPS || NB * NB == 2 * (NT / 64), "two rounds of one block per wave");
    const auto sl = (__attribute__((address_space(3))) T*)work_lds();
    for (int t = wave; t < NB * NB; t += NT / 64) {
        const int r0 = 1 + (t / NB) * 16 * BLK, c0 = 1 + (t % NB) * 16 * BLK;
        const int row0 = 1 + (t / (2 * NB)) * 64;        // first staged row of this round
        if constexpr (STRIPS) {
            if (t >= NT / 64) wg_barrier();               // the first round's reads are done
            for (int e = threadIdx.x; e < 64 * n1; e += NT) sl[e] = xs[row0 * n1 + e];
            wg_barrier();
        }
        V4 ur[BLK][BLK], us[BLK][BLK];
#pragma unroll
        for (int i = 0; i < BLK; ++i)
#pragma unroll
            for (int j = 0; j < BLK; ++j) {
                ur[i][j] = V4{0, 0, 0, 0};
                us[i][j] = V4{0, 0, 0, 0};
            }
        // single tiles: the tile's geometric factors are loaded before the
        // products, their latency hidden behind them
        constexpr bool PREG = BLK == 1;
        T gp[PREG ? 4 : 1][3];
        if constexpr (PREG) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int q = (r0 + Mfma<T>::row(lane, v)) * n1 + c0 + lr;
                gp[v][0] = G[q];
                gp[v][1] = G[N + q];
                gp[v][2] = G[2 * N + q];
            }
        }
        if constexpr (STRIPS)
            mfma_blocks<T, n1, n1, n1, 1, n1, BLK, BLK, 2, 1, n1>(sl + (r0 - row0 + lr) * n1 + kq,
                                                                  DT + kq * n1 + c0 + lr,
                                                                  DT + kq * n1 + r0 + lr,
                                                                  xs + kq * n1 + c0 + lr, ur, us);
        else
            mfma_blocks<T, n1, n1, n1, 1, n1, BLK, BLK, 2, 1, n1>(xs + (r0 + lr) * n1 + kq,
                                                                  DT + kq * n1 + c0 + lr,
                                                                  DT + kq * n1 + r0 + lr,
                                                                  xs + kq * n1 + c0 + lr, ur, us);
#pragma unroll
        for (int i = 0; i < BLK; ++i)
#pragma unroll
            for (int j = 0; j < BLK; ++j) {
                const int col = c0 + 16 * j + lr;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int q = (r0 + 16 * i + Mfma<T>::row(lane, v)) * n1 + col;
                    const T g00 = PREG ? gp[v][0] : G[q], g11 = PREG ? gp[v][1] : G[N + q],
                            g01 = PREG ? gp[v][2] : G[2 * N + q];
                    f0[q] = g00 * ur[i][j][v] + g01 * us[i][j][v];
                    if constexpr (F1SEP)
                        f1[q] = g01 * ur[i][j][v] + g11 * us[i][j][v];
                    else
                        f0[N + q] = g01 * ur[i][j][v] + g11 * us[i][j][v];
                }
            }
    }
    // Index 0 of the gradients on the vector units.  The second pass reads
    // only F1 on row 0 (columns 1..P) and F0 on column 0 (rows 1..P), so
    // those 2P fluxes are formed (the corner's are never read).  Each of
    // their 4P dot products (ur and us of a node) is split over KS lanes
    // that take every KS-th term, summed by a fixed butterfly, so that every
    // thread of the workgroup carries a short chain of loads.
    {
        constexpr int NODES = 2 * P;
        constexpr int KS = NT >= 16 * NODES ? 8 : NT >= 8 * NODES ? 4 : NT >= 4 * NODES ? 2 : 1;
        constexpr int KT = (n1 + KS - 1) / KS;       // terms per lane
        constexpr int TASKS = NODES * 2 * KS;        // node-major, then ur / us, then k-part
        static_assert(64 % (2 * KS) == 0 && NT % (2 * KS) == 0, "a node's lanes share a wave");
        for (int t = threadIdx.x; t < TASKS; t += NT) {
            const int node = t / (2 * KS), a = (t / KS) & 1, part = t % KS;
            const bool row = node < P;                // row 0, column node + 1
            const int at = row ? 0 : (node - P + 1) * n1;   // first factor's row
            const int bt = row ? node + 1 : 0;              // second factor's column
            // ur = sum_k x[at + k] DT[k][bt], us = sum_k D[at + k] x[k][bt]
            const auto A = a == 0 ? xb : D;
            const auto Bm = a == 0 ? DT : xb;
            T acc = 0;
#pragma unroll 16
            for (int u = 0; u < KT; ++u) {
                const int k = part + u * KS;
                if (KT * KS == n1 || k < n1) acc += A[at + k] * Bm[k * n1 + bt];
            }
#pragma unroll
            for (int o = KS / 2; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
            const T other = __shfl_xor(acc, KS, 64);
            if (a == 0 && part == 0) {
                const T ur = acc, us = other;
                const int q = at + bt;
                if (row) {   // F1 = g01 ur + g11 us
                    if constexpr (F1SEP)
                        f1[q] = G[2 * N + q] * ur + G[N + q] * us;
                    else
                        f0[N + q] = G[2 * N + q] * ur + G[N + q] * us;
                } else {     // F0 = g00 ur + g01 us
                    f0[q] = G[q] * ur + G[2 * N + q] * us;
                }
            }
        }
    }
    wg_barrier();
    for (int t = wave; t < NB * NB; t += NT / 64) {
        const int r0 = 1 + (t / NB) * 16 * BLK, c0 = 1 + (t % NB) * 16 * BLK;
        const int row0 = 1 + (t / (2 * NB)) * 64;
        if constexpr (STRIPS) {
            if (t >= NT / 64) wg_barrier();
            for (int e = threadIdx.x; e < 64 * n1; e += NT) sl[e] = f0[row0 * n1 + e];
            wg_barrier();
        }
        V4 y[BLK][BLK];
#pragma unroll
        for (int i = 0; i < BLK; ++i)
#pragma unroll
            for (int j = 0; j < BLK; ++j) y[i][j] = V4{0, 0, 0, 0};
        // single tiles: the residual's right-hand side is loaded before the
        // products, its latency hidden behind them
        constexpr bool PRE = RESID && BLK == 1;
        T rv[4];
        if constexpr (PRE) {
#pragma unroll
            for (int v = 0; v < 4; ++v) rv[v] = r[(r0 + Mfma<T>::row(lane, v)) * n1 + c0 + lr];
        }
        // sum_k F0[j][k] D[k][i] and sum_k D^T[j][k] F1[k][i]
        if constexpr (STRIPS && !F1SEP)
            mfma_blocks<T, n1, n1, n1, 1, n1, BLK, BLK, 2, 1, n1>(sl + (r0 - row0 + lr) * n1 + kq,
                                                                  D + kq * n1 + c0 + lr,
                                                                  D + kq * n1 + r0 + lr,
                                                                  f0 + N + kq * n1 + c0 + lr, y, y);
        else if constexpr (F1SEP)
            mfma_blocks<T, n1, n1, n1, 1, n1, BLK, BLK, 2, 1, n1>(f0 + (r0 + lr) * n1 + kq,
                                                                  D + kq * n1 + c0 + lr,
                                                                  D + kq * n1 + r0 + lr,
                                                                  f1 + kq * n1 + c0 + lr, y, y);
        else
            mfma_blocks<T, n1, n1, n1, 1, n1, BLK, BLK, 2, 1, n1>(f0 + (r0 + lr) * n1 + kq,
                                                                  D + kq * n1 + c0 + lr,
                                                                  D + kq * n1 + r0 + lr,
                                                                  f0 + N + kq * n1 + c0 + lr, y, y);
#pragma unroll
        for (int i = 0; i < BLK; ++i)
#pragma unroll
            for (int jj = 0; jj < BLK; ++jj) {
                const int col = c0 + 16 * jj + lr;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = r0 + 16 * i + Mfma<T>::row(lane, v);
                    const int q = row * n1 + col;
                    const T rq = RESID ? (PRE ? rv[v] : r[q]) : T(0);
                    out[q] = (col == P || row == P) ? T(0) : (RESID ? rq - y[i][jj][v] : y[i][jj][v]);
                }
            }
    }
    for (int e = threadIdx.x; e < 2 * P + 1; e += NT) out[e <= P ? e : (e - P) * n1] = T(0);
    wg_barrier();
}

template <class T, int P, bool RESID>
__device__ void apply2d_mfma(const T* __restrict__ G_, const T* __restrict__ D_,
                             const T* __restrict__ DT_, T* __restrict__ TR_,
                             const T* __restrict__ x_, const T* __restrict__ r_, T* __restrict__ out_)
{
    static_assert(P % 16 == 0, "tiles cover rows 1..P");
    constexpr int N = (P + 1) * (P + 1);
    constexpr int LDSW = PMG_WORK_LDS_WORDS * (int)(sizeof(double) / sizeof(T));   // in T words
    constexpr bool ALL = P <= 64 && 8 * N <= LDSW;   // x, F0, F1, G, D, D^T in LDS
    constexpr bool XL = P <= 64 && 2 * N <= LDSW;    // x and F0 in LDS
    constexpr bool F1L = XL && 3 * N <= LDSW;        // F1 as well
    const auto TR = gmem(TR_);
    const auto x = gmem(x_);
    const auto G = gmem(G_);
    const auto D = gmem(D_);
    const auto DT = gmem(DT_);
    const auto wl = (__attribute__((address_space(3))) T*)work_lds();
    if constexpr (ALL) {
        // every operand in one round trip; then only the residual's
        // right-hand side and the result touch memory
        for (int q = threadIdx.x; q < N; q += NT) {
            wl[q] = x[q];
            wl[3 * N + q] = G[q];
            wl[4 * N + q] = G[N + q];
            wl[5 * N + q] = G[2 * N + q];
            wl[6 * N + q] = D[q];
            wl[7 * N + q] = DT[q];
        }
        wg_barrier();
        apply2d_mfma_passes<T, P, RESID, true>(wl + 3 * N, wl + 6 * N, wl + 7 * N, wl, wl, wl + N,
                                               wl + 2 * N, r_, out_);
    } else if constexpr (XL) {
        for (int q = threadIdx.x; q < N; q += NT) wl[q] = x[q];
        wg_barrier();
        if constexpr (F1L)
            apply2d_mfma_passes<T, P, RESID, true>(G, D, DT, wl, x, wl + N, wl + 2 * N, r_, out_);
        else
            apply2d_mfma_passes<T, P, RESID, true>(G, D, DT, wl, x, wl + N, TR + N, r_, out_);
    } else {
        apply2d_mfma_passes<T, P, RESID, false>(G, D, DT, x, x, TR, TR, r_, out_);
    }
}

// 3-D A x on matrix cores, node q = i + n1 j + n1^2 k.  The four passes are
// 16x16-tile products over index ranges 1..P (blocks of BLK x BLK tiles per
// wave); index 0 of the gradients is filled on the vector units and the
// output's boundary faces are zero.
//   1a  g2(k, i) = sum_m D[k][m] x(i, j, m)        for each j   -> TR2
//   1b  g0(j, i) = sum_m x(m, j, k) D[i][m],
//       g1(j, i) = sum_m D[j][m] x(i, m, k)        for each k;
//       fluxes f_a = sum_b G_ab g_b at once        -> TR0, TR1, TR2
//   2a  y(k, i)  = sum_m D[m][k] f2(i, j, m)       for interior j -> out
//   2b  y(j, i) += sum_m f0(m, j, k) D[m][i] + D[m][j] f1(i, m, k)
//                                                 for interior k -> out
template <class T, int P, bool RESID>
__device__ void apply3d_mfma(const T* __restrict__ G_, const T* __restrict__ D_,
                             const T* __restrict__ DT_, T* __restrict__ TR_,
                             const T* __restrict__ x_, const T* __restrict__ r_, T* __restrict__ out_)
{
    const auto G = gmem(G_);
    const auto D = gmem(D_);
    const auto DT = gmem(DT_);
    const auto TR = gmem(TR_);
    const auto x = gmem(x_);
    const auto r = gmem(r_);
    const auto out = gmem(out_);
    static_assert(P % 16 == 0, "tiles cover indices 1..P");
    constexpr int BLK = P >= 64 ? 2 : 1;
    constexpr int n1 = P + 1, S2 = n1 * n1, N = S2 * n1, NB = P / (16 * BLK), NBB = NB * NB;
    using V4 = typename Mfma<T>::v4;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, kq = lane >> 4;
    const auto F0 = TR, F1 = TR + N, F2 = TR + 2 * N;

    // ---- 1a: z-gradient into F2
    for (int t = wave; t < n1 * NBB; t += NT / 64) {
        const int j = t / NBB, bb = t % NBB;
        const int r0 = 1 + (bb / NB) * 16 * BLK, c0 = 1 + (bb % NB) * 16 * BLK;   // k, i
        V4 acc[BLK][BLK];
#pragma unroll
        for (int a = 0; a < BLK; ++a)
#pragma unroll
            for (int b = 0; b < BLK; ++b) acc[a][b] = V4{0, 0, 0, 0};
        const auto bp = x + n1 * j + kq * S2 + c0 + lr;
        mfma_blocks<T, n1, 1, S2, 1, S2, BLK, BLK, 1, n1, n1>(DT + kq * n1 + r0 + lr, bp, DT, bp,
                                                              acc, acc);
#pragma unroll
        for (int a = 0; a < BLK; ++a)
#pragma unroll
            for (int b = 0; b < BLK; ++b) {
                const int i = c0 + 16 * b + lr;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int k = r0 + 16 * a + Mfma<T>::row(lane, v);
                    F2[i + n1 * j + S2 * k] = acc[a][b][v];
                }
            }
    }
    for (int e = threadIdx.x; e < n1 * (2 * P + 1); e += NT) {
        const int j = e / (2 * P + 1), tt = e % (2 * P + 1);
        const int k = tt <= P ? 0 : tt - P, i = tt <= P ? tt : 0;
        T g2 = 0;
#pragma unroll 8
        for (int m = 0; m < n1; ++m) g2 += D[k * n1 + m] * x[i + n1 * j + S2 * m];
        F2[i + n1 * j + S2 * k] = g2;
    }
    wg_barrier();

    // ---- 1b: x- and y-gradients per z-slab, fluxes
    for (int t = wave; t < n1 * NBB; t += NT / 64) {
        const int k = t / NBB, bb = t % NBB;
        const int r0 = 1 + (bb / NB) * 16 * BLK, c0 = 1 + (bb % NB) * 16 * BLK;   // j, i
        const auto xk = x + S2 * k;
        V4 g0[BLK][BLK], g1[BLK][BLK];
#pragma unroll
        for (int a = 0; a < BLK; ++a)
#pragma unroll
            for (int b = 0; b < BLK; ++b) {
                g0[a][b] = V4{0, 0, 0, 0};
                g1[a][b] = V4{0, 0, 0, 0};
            }
        mfma_blocks<T, n1, n1, n1, 1, n1, BLK, BLK, 2, 1, n1>(xk + (r0 + lr) * n1 + kq,
                                                              DT + kq * n1 + c0 + lr,
                                                              DT + kq * n1 + r0 + lr,
                                                              xk + kq * n1 + c0 + lr, g0, g1);
#pragma unroll
        for (int a = 0; a < BLK; ++a)
#pragma unroll
            for (int b = 0; b < BLK; ++b) {
                const int i = c0 + 16 * b + lr;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int q = i + n1 * (r0 + 16 * a + Mfma<T>::row(lane, v)) + S2 * k;
                    const T u0 = g0[a][b][v], u1 = g1[a][b][v], u2 = F2[q];
                    const T G00 = G[q], G11 = G[N + q], G22 = G[2 * N + q];
                    const T G01 = G[3 * N + q], G02 = G[4 * N + q], G12 = G[5 * N + q];
                    F0[q] = G00 * u0 + G01 * u1 + G02 * u2;
                    F1[q] = G01 * u0 + G11 * u1 + G12 * u2;
                    F2[q] = G02 * u0 + G12 * u1 + G22 * u2;
                }
            }
    }
    for (int e = threadIdx.x; e < n1 * (2 * P + 1); e += NT) {
        const int k = e / (2 * P + 1), tt = e % (2 * P + 1);
        const int j = tt <= P ? 0 : tt - P, i = tt <= P ? tt : 0;
        T u0 = 0, u1 = 0;
#pragma unroll 8
        for (int m = 0; m < n1; ++m) {
            u0 += x[m + n1 * j + S2 * k] * DT[m * n1 + i];
            u1 += D[j * n1 + m] * x[i + n1 * m + S2 * k];
        }
        const int q = i + n1 * j + S2 * k;
        const T u2 = F2[q];
        const T G00 = G[q], G11 = G[N + q], G22 = G[2 * N + q];
        const T G01 = G[3 * N + q], G02 = G[4 * N + q], G12 = G[5 * N + q];
        F0[q] = G00 * u0 + G01 * u1 + G02 * u2;
        F1[q] = G01 * u0 + G11 * u1 + G12 * u2;
        F2[q] = G02 * u0 + G12 * u1 + G22 * u2;
    }
    wg_barrier();

    // ---- 2a: z-part of the divergence on interior y-rows
    for (int t = wave; t < (P - 1) * NBB; t += NT / 64) {
        const int j = 1 + t / NBB, bb = t % NBB;
        const int r0 = 1 + (bb / NB) * 16 * BLK, c0 = 1 + (bb % NB) * 16 * BLK;   // k, i
        V4 acc[BLK][BLK];
#pragma unroll
        for (int a = 0; a < BLK; ++a)
#pragma unroll
            for (int b = 0; b < BLK; ++b) acc[a][b] = V4{0, 0, 0, 0};
        const auto bp = F2 + n1 * j + kq * S2 + c0 + lr;
        mfma_blocks<T, n1, 1, S2, 1, S2, BLK, BLK, 1, n1, n1>(D + kq * n1 + r0 + lr, bp, D, bp,
                                                              acc, acc);
#pragma unroll
        for (int a = 0; a < BLK; ++a)
#pragma unroll
            for (int b = 0; b < BLK; ++b) {
                const int i = c0 + 16 * b + lr;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int k = r0 + 16 * a + Mfma<T>::row(lane, v);
                    if (i < P && k < P) out[i + n1 * j + S2 * k] = acc[a][b][v];
                }
            }
    }
    wg_barrier();

    // ---- 2b: x- and y-parts on interior z-slabs, residual
    for (int t = wave; t < (P - 1) * NBB; t += NT / 64) {
        const int k = 1 + t / NBB, bb = t % NBB;
        const int r0 = 1 + (bb / NB) * 16 * BLK, c0 = 1 + (bb % NB) * 16 * BLK;   // j, i
        V4 y[BLK][BLK];
#pragma unroll
        for (int a = 0; a < BLK; ++a)
#pragma unroll
            for (int b = 0; b < BLK; ++b) y[a][b] = V4{0, 0, 0, 0};
        const auto f0k = F0 + S2 * k, f1k = F1 + S2 * k;
        mfma_blocks<T, n1, n1, n1, 1, n1, BLK, BLK, 2, 1, n1>(f0k + (r0 + lr) * n1 + kq,
                                                              D + kq * n1 + c0 + lr,
                                                              D + kq * n1 + r0 + lr,
                                                              f1k + kq * n1 + c0 + lr, y, y);
#pragma unroll
        for (int a = 0; a < BLK; ++a)
#pragma unroll
            for (int b = 0; b < BLK; ++b) {
                const int i = c0 + 16 * b + lr;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int j = r0 + 16 * a + Mfma<T>::row(lane, v);
                    if (i < P && j < P) {
                        const int q = i + n1 * j + S2 * k;
                        const T yy = y[a][b][v] + out[q];
                        out[q] = RESID ? r[q] - yy : yy;
                    }
                }
            }
    }
    // boundary faces
    for (int e = threadIdx.x; e < 6 * S2; e += NT) {
        const int f = e / S2, a = e % S2, u = a % n1, w = a / n1, c = (f & 1) ? P : 0;
        const int q = f < 2 ? c + n1 * u + S2 * w : (f < 4 ? u + n1 * c + S2 * w : u + n1 * w + S2 * c);
        out[q] = T(0);
    }
    wg_barrier();
}

// ------------------------------------------------------------------ several elements

// Levels made of K x K spectral elements of degree pe = P / K on the
// composite node grid of degree P (interface nodes shared, the one-element
// vector layout): the operator is the sum of the element operators
// (direct stiffness summation), each the one-element sum factorisation of
// eq. discreteBilinear with the element's own GLL rule, derivative matrix D
// (ne1 x ne1, ne1 = pe + 1) and geometric factors G (per element e: G00,
// G11, G01 arrays of NE = ne1^2 element nodes at G + 3 NE e, elements in
// lexicographic order).  Pass 1: per element node, the two reference
// gradients and the fluxes into TR (per element: 2 NE).  Pass 2: per global
// node, the sum over the elements holding it (one inside an element, two
// on an edge, four at a corner, in element order) of D^T of their fluxes.
// The element operator's two passes on operands given by their own
// pointers (LDS or global): G the element factors, D the element D, x the
// composite operand, TR the element fluxes.
template <class T, int P, bool RESID, class PG, class PD, class PX, class PT>
__device__ inline void apply2d_elements_passes(int K, PG __restrict__ G, PD __restrict__ D,
                                               PT __restrict__ TR, PX __restrict__ x,
                                               const T* __restrict__ r_, T* __restrict__ out_)
{
    const auto r = gmem(r_);
    const auto out = gmem(out_);
    constexpr int n1 = P + 1, N = n1 * n1;
    const int pe = P / K, ne1 = pe + 1, NE = ne1 * ne1;
    for (int t = threadIdx.x; t < K * K * NE; t += NT) {
        const int e = t / NE, lq = t - e * NE;
        const int i = lq % ne1, j = lq / ne1;
        const int gx = (e % K) * pe, gy = (e / K) * pe;
        T g0 = 0, g1 = 0;
#pragma unroll 4
        for (int k = 0; k < ne1; ++k) {
            g0 += D[i * ne1 + k] * x[(gx + k) + (gy + j) * n1];
            g1 += D[j * ne1 + k] * x[(gx + i) + (gy + k) * n1];
        }
        const auto Ge = G + (long long)3 * NE * e;
        const T g00 = Ge[lq], g11 = Ge[NE + lq], g01 = Ge[2 * NE + lq];
        TR[(long long)2 * NE * e + lq] = g00 * g0 + g01 * g1;
        TR[(long long)2 * NE * e + NE + lq] = g01 * g0 + g11 * g1;
    }
    wg_barrier();
    for (int q = threadIdx.x; q < N; q += NT) {
        const int I = q % n1, J = q / n1;
        if (I == 0 || I == P || J == 0 || J == P) {
            out[q] = T(0);
            continue;
        }
        const int ex1 = I / pe, ey1 = J / pe;
        const int ex0 = I % pe == 0 ? ex1 - 1 : ex1, ey0 = J % pe == 0 ? ey1 - 1 : ey1;
        T y = 0;
        for (int ey = ey0; ey <= ey1 && ey < K; ++ey)
            for (int ex = ex0; ex <= ex1 && ex < K; ++ex) {
                const int e = ex + K * ey, i = I - ex * pe, j = J - ey * pe;
                const auto f = TR + (long long)2 * NE * e;
#pragma unroll 4
                for (int k = 0; k < ne1; ++k)
                    y += D[k * ne1 + i] * f[k + j * ne1] + D[k * ne1 + j] * f[NE + i + k * ne1];
            }
        out[q] = RESID ? r[q] - y : y;
    }
    wg_barrier();
}

template <class T, int P, bool RESID>
__device__ void apply2d_elements(int K, const T* __restrict__ G_, const T* __restrict__ D_,
                                 T* __restrict__ TR_, const T* __restrict__ x_,
                                 const T* __restrict__ r_, T* __restrict__ out_)
{
    constexpr int n1 = P + 1, N = n1 * n1;
    const int pe = P / K, ne1 = pe + 1, NE = ne1 * ne1, NG = 3 * K * K * NE, NTR = 2 * K * K * NE;
    constexpr int LDSW = PMG_WORK_LDS_WORDS * (int)(sizeof(double) / sizeof(T));
    // x, the element factors and fluxes and D staged in the LDS work buffer
    // where they fit (one memory round trip in; 4 x 4 elements up to
    // composite degree 32 in the one-launch kernels)
    if (N + NG + NTR + NE <= LDSW) {
        const auto wl = (__attribute__((address_space(3))) T*)work_lds();
        const auto G = gmem(G_);
        const auto D = gmem(D_);
        const auto x = gmem(x_);
        const auto lx = wl, lg = wl + N, ltr = wl + N + NG, ld = wl + N + NG + NTR;
        for (int q = threadIdx.x; q < N; q += NT) lx[q] = x[q];
        for (int q = threadIdx.x; q < NG; q += NT) lg[q] = G[q];
        for (int q = threadIdx.x; q < NE; q += NT) ld[q] = D[q];
        wg_barrier();
        apply2d_elements_passes<T, P, RESID>(K, lg, ld, ltr, lx, r_, out_);
    } else {
        apply2d_elements_passes<T, P, RESID>(K, gmem(G_), gmem(D_), gmem(TR_), gmem(x_), r_, out_);
    }
}

// The same in 3-D (K^3 elements of degree pe, per element G00, G11, G22,
// G01, G02, G12 arrays of NE = ne1^3 element nodes, fluxes 3 NE): pass 1 the
// three reference gradients and the fluxes per element node, pass 2 per
// global node the sum over the (up to eight) elements holding it.
template <class T, int P, bool RESID>
__device__ void apply3d_elements(int K, const T* __restrict__ G_, const T* __restrict__ D_,
                                 T* __restrict__ TR_, const T* __restrict__ x_,
                                 const T* __restrict__ r_, T* __restrict__ out_)
{
    const auto G = gmem(G_);
    const auto D = gmem(D_);
    const auto TR = gmem(TR_);
    const auto x = gmem(x_);
    const auto r = gmem(r_);
    const auto out = gmem(out_);
    constexpr int n1 = P + 1, N = n1 * n1 * n1;
    const int pe = P / K, ne1 = pe + 1, NE = ne1 * ne1 * ne1;
    const int gst[3] = {1, n1, n1 * n1};
    const int est[3] = {1, ne1, ne1 * ne1};
    for (int t = threadIdx.x; t < K * K * K * NE; t += NT) {
        const int e = t / NE, lq = t - e * NE;
        const int c[3] = {lq % ne1, (lq / ne1) % ne1, lq / (ne1 * ne1)};
        const int eo[3] = {(e % K) * pe, ((e / K) % K) * pe, (e / (K * K)) * pe};
        const int g0 = (eo[0] + c[0]) + (eo[1] + c[1]) * n1 + (eo[2] + c[2]) * n1 * n1;
        T g[3];
        for (int a = 0; a < 3; ++a) {
            const int gb = g0 - c[a] * gst[a];
            T sum = 0;
            for (int k = 0; k < ne1; ++k) sum += D[c[a] * ne1 + k] * x[gb + k * gst[a]];
            g[a] = sum;
        }
        const auto Ge = G + 6LL * NE * e;
        const T g00 = Ge[lq], g11 = Ge[NE + lq], g22 = Ge[2 * NE + lq];
        const T g01 = Ge[3 * NE + lq], g02 = Ge[4 * NE + lq], g12 = Ge[5 * NE + lq];
        const auto f = TR + 3LL * NE * e;
        f[lq] = g00 * g[0] + g01 * g[1] + g02 * g[2];
        f[NE + lq] = g01 * g[0] + g11 * g[1] + g12 * g[2];
        f[2 * NE + lq] = g02 * g[0] + g12 * g[1] + g22 * g[2];
    }
    wg_barrier();
    for (int q = threadIdx.x; q < N; q += NT) {
        const int I[3] = {q % n1, (q / n1) % n1, q / (n1 * n1)};
        if (I[0] == 0 || I[0] == P || I[1] == 0 || I[1] == P || I[2] == 0 || I[2] == P) {
            out[q] = T(0);
            continue;
        }
        int e0[3], e1[3];
        for (int a = 0; a < 3; ++a) {
            e1[a] = I[a] / pe;
            e0[a] = I[a] % pe == 0 ? e1[a] - 1 : e1[a];
        }
        T y = 0;
        for (int ez = e0[2]; ez <= e1[2]; ++ez)
            for (int ey = e0[1]; ey <= e1[1]; ++ey)
                for (int ex = e0[0]; ex <= e1[0]; ++ex) {
                    const int e = ex + K * (ey + K * ez);
                    const int c[3] = {I[0] - ex * pe, I[1] - ey * pe, I[2] - ez * pe};
                    const int lq = c[0] + c[1] * ne1 + c[2] * ne1 * ne1;
                    const auto f = TR + 3LL * NE * e;
                    for (int a = 0; a < 3; ++a) {
                        const int lb = lq - c[a] * est[a];
                        for (int k = 0; k < ne1; ++k)
                            y += D[k * ne1 + c[a]] * f[(long long)a * NE + lb + k * est[a]];
                    }
                }
        out[q] = RESID ? r[q] - y : y;
    }
    wg_barrier();
}

// The element operator on the matrix cores (element degree PE = P / K, a
// multiple of 16): the elements' nodal values are first copied into the
// element-local array EX (interface nodes once per element); each element is
// then the one-element sum factorisation of apply2d_mfma on its own tiles
// (rows and columns 1..PE on 16x16 tiles, row and column 0 on the vector
// units), with the full element output (no boundary rows dropped) written
// back into EX; finally each global node sums the outputs of the elements
// holding it, in element order.  Tiles of all elements are shared out over
// the waves.
template <class T, int P, int PE, bool RESID>
__device__ void apply2d_elements_mfma(const T* __restrict__ G_, const T* __restrict__ D_,
                                      const T* __restrict__ DT_, T* __restrict__ TR_,
                                      T* __restrict__ EX_, const T* __restrict__ x_,
                                      const T* __restrict__ r_, T* __restrict__ out_)
{
    static_assert(PE % 16 == 0 && P % PE == 0, "element tiles cover rows 1..PE");
    const auto G = gmem(G_);
    const auto D = gmem(D_);
    const auto DT = gmem(DT_);
    const auto TR = gmem(TR_);
    const auto EX = gmem(EX_);
    const auto x = gmem(x_);
    const auto r = gmem(r_);
    const auto out = gmem(out_);
    constexpr int K = P / PE, n1 = P + 1, N = n1 * n1;
    constexpr int ne1 = PE + 1, NE = ne1 * ne1, NEL = K * K;
    constexpr int BLK = PE >= 64 ? 2 : 1, NB = PE / (16 * BLK), NT2 = NB * NB;
    using V4 = typename Mfma<T>::v4;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, kq = lane >> 4;
    for (int t = threadIdx.x; t < NEL * NE; t += NT) {
        const int e = t / NE, lq = t - e * NE;
        EX[t] = x[((e % K) * PE + lq % ne1) + ((e / K) * PE + lq / ne1) * n1];
    }
    wg_barrier();
    // pass 1: reference gradients and fluxes of every element node
    for (int t = wave; t < NEL * NT2; t += NT / 64) {
        const int e = t / NT2, tb = t - e * NT2;
        const int r0 = 1 + (tb / NB) * 16 * BLK, c0 = 1 + (tb % NB) * 16 * BLK;
        const auto xe = EX + (long long)NE * e;
        const auto Ge = G + 3LL * NE * e;
        const auto Fe = TR + 2LL * NE * e;
        V4 ur[BLK][BLK], us[BLK][BLK];
#pragma unroll
        for (int i = 0; i < BLK; ++i)
#pragma unroll
            for (int j = 0; j < BLK; ++j) {
                ur[i][j] = V4{0, 0, 0, 0};
                us[i][j] = V4{0, 0, 0, 0};
            }
        mfma_blocks<T, ne1, ne1, ne1, 1, ne1, BLK, BLK, 2, 1, ne1>(xe + (r0 + lr) * ne1 + kq,
                                                                    DT + kq * ne1 + c0 + lr,
                                                                    DT + kq * ne1 + r0 + lr,
                                                                    xe + kq * ne1 + c0 + lr, ur, us);
#pragma unroll
        for (int i = 0; i < BLK; ++i)
#pragma unroll
            for (int j = 0; j < BLK; ++j) {
                const int col = c0 + 16 * j + lr;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int q = (r0 + 16 * i + Mfma<T>::row(lane, v)) * ne1 + col;
                    const T g00 = Ge[q], g11 = Ge[NE + q], g01 = Ge[2 * NE + q];
                    Fe[q] = g00 * ur[i][j][v] + g01 * us[i][j][v];
                    Fe[NE + q] = g01 * ur[i][j][v] + g11 * us[i][j][v];
                }
            }
    }
    for (int t = threadIdx.x; t < NEL * (2 * PE + 1); t += NT) {
        const int e = t / (2 * PE + 1), k2 = t - e * (2 * PE + 1);
        const int j = k2 <= PE ? 0 : k2 - PE, i = k2 <= PE ? k2 : 0;
        const auto xe = EX + (long long)NE * e;
        T ur = 0, us = 0;
#pragma unroll 8
        for (int k = 0; k < ne1; ++k) {   // loads of eight terms in flight
            ur += xe[j * ne1 + k] * DT[k * ne1 + i];
            us += D[j * ne1 + k] * xe[k * ne1 + i];
        }
        const int q = j * ne1 + i;
        const auto Ge = G + 3LL * NE * e;
        const auto Fe = TR + 2LL * NE * e;
        const T g00 = Ge[q], g11 = Ge[NE + q], g01 = Ge[2 * NE + q];
        Fe[q] = g00 * ur + g01 * us;
        Fe[NE + q] = g01 * ur + g11 * us;
    }
    wg_barrier();
    // pass 2: every element's full output (its values are no longer needed)
    for (int t = wave; t < NEL * NT2; t += NT / 64) {
        const int e = t / NT2, tb = t - e * NT2;
        const int r0 = 1 + (tb / NB) * 16 * BLK, c0 = 1 + (tb % NB) * 16 * BLK;
        const auto Fe = TR + 2LL * NE * e;
        const auto ye = EX + (long long)NE * e;
        V4 y[BLK][BLK];
#pragma unroll
        for (int i = 0; i < BLK; ++i)
#pragma unroll
            for (int j = 0; j < BLK; ++j) y[i][j] = V4{0, 0, 0, 0};
        mfma_blocks<T, ne1, ne1, ne1, 1, ne1, BLK, BLK, 2, 1, ne1>(Fe + (r0 + lr) * ne1 + kq,
                                                                    D + kq * ne1 + c0 + lr,
                                                                    D + kq * ne1 + r0 + lr,
                                                                    Fe + NE + kq * ne1 + c0 + lr, y, y);
#pragma unroll
        for (int i = 0; i < BLK; ++i)
#pragma unroll
            for (int jj = 0; jj < BLK; ++jj) {
                const int col = c0 + 16 * jj + lr;
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    ye[(r0 + 16 * i + Mfma<T>::row(lane, v)) * ne1 + col] = y[i][jj][v];
            }
    }
    for (int t = threadIdx.x; t < NEL * (2 * PE + 1); t += NT) {
        const int e = t / (2 * PE + 1), k2 = t - e * (2 * PE + 1);
        const int j = k2 <= PE ? 0 : k2 - PE, i = k2 <= PE ? k2 : 0;
        const auto Fe = TR + 2LL * NE * e;
        T y = 0;
#pragma unroll 8
        for (int k = 0; k < ne1; ++k) y += Fe[j * ne1 + k] * D[k * ne1 + i] + D[k * ne1 + j] * Fe[NE + k * ne1 + i];
        EX[(long long)NE * e + j * ne1 + i] = y;
    }
    wg_barrier();
    // assembly: each interior global node sums the elements holding it
    for (int q = threadIdx.x; q < N; q += NT) {
        const int I = q % n1, J = q / n1;
        if (I == 0 || I == P || J == 0 || J == P) {
            out[q] = T(0);
            continue;
        }
        const int ex1 = I / PE, ey1 = J / PE;
        const int ex0 = I % PE == 0 ? ex1 - 1 : ex1, ey0 = J % PE == 0 ? ey1 - 1 : ey1;
        T y = 0;
        for (int ey = ey0; ey <= ey1; ++ey)
            for (int ex = ex0; ex <= ex1; ++ex)
                y += EX[(long long)NE * (ex + K * ey) + (I - ex * PE) + (J - ey * PE) * ne1];
        out[q] = RESID ? r[q] - y : y;
    }
    wg_barrier();
}

// Matrix-free A x of eq. discreteBilinear by sum factorisation: reference
// gradients g_b = D along axis b, fluxes f_a = sum_b G_ab g_b at every node,
// then (A x)(n) = sum_a sum_k D[k][n_a] f_a(n with axis a <- k) on interior
// rows.  RESID: out = r - A x.  out has zero boundary rows.
// The operator of a level of K^dim elements (K > 1), out of line so that the
// one-element operator's code and registers stay as they are: element degree
// P / K >= 16 (2-D) on the matrix cores, else the vector units.
template <class T, int P, int DIM, bool RESID>
__device__ __attribute__((noinline)) void apply_elements_level(
    int K, const T* __restrict__ G_, const T* __restrict__ D_, const T* __restrict__ DT_,
    T* __restrict__ TR_, T* __restrict__ EX_, const T* __restrict__ x_, const T* __restrict__ r_,
    T* __restrict__ out_)
{
    if constexpr (DIM == 2) {
        if constexpr (P / 2 >= 16 && (P / 2) % 16 == 0) {
            if (K == 2 && EX_) {
                apply2d_elements_mfma<T, P, P / 2, RESID>(G_, D_, DT_, TR_, EX_, x_, r_, out_);
                return;
            }
        }
        if constexpr (P / 4 >= 16 && (P / 4) % 16 == 0) {
            if (K == 4 && EX_) {
                apply2d_elements_mfma<T, P, P / 4, RESID>(G_, D_, DT_, TR_, EX_, x_, r_, out_);
                return;
            }
        }
        if constexpr (P / 8 >= 16 && (P / 8) % 16 == 0) {
            if (K == 8 && EX_) {
                apply2d_elements_mfma<T, P, P / 8, RESID>(G_, D_, DT_, TR_, EX_, x_, r_, out_);
                return;
            }
        }
        apply2d_elements<T, P, RESID>(K, G_, D_, TR_, x_, r_, out_);
    } else {
        apply3d_elements<T, P, RESID>(K, G_, D_, TR_, x_, r_, out_);
    }
}

// The vector-unit operator (levels below the matrix-core tiles) on
// operands given by their own pointers (LDS or global): G the geometric
// factors, D / DT, x, TR the fluxes.
template <class T, int P, int DIM, bool RESID, class PG, class PD, class PX, class PT>
__device__ inline void apply_vector(PG __restrict__ G, PD __restrict__ D, PD __restrict__ DT,
                                    PX __restrict__ x, PT __restrict__ TR,
                                    const T* __restrict__ r_, T* __restrict__ out_)
{
    const auto r = gmem(r_);
    const auto out = gmem(out_);
    using S = Shape<P, DIM>;
    constexpr int n1 = S::n1, N = S::N;
    for (int q = threadIdx.x; q < N; q += NT) {
        int c[3] = {q % n1, (q / n1) % n1, DIM == 3 ? q / (n1 * n1) : 0};
        T g[DIM];
        {
            const auto xr = x + (q - c[0]);
            T s = 0;
#pragma unroll 8
            for (int k = 0; k < n1; ++k) s += DT[k * n1 + c[0]] * xr[k];
            g[0] = s;
        }
#pragma unroll
        for (int a = 1; a < DIM; ++a) {
            const int st = a == 1 ? n1 : n1 * n1;
            const auto xr = x + (q - c[a] * st);
            const auto Dr = D + c[a] * n1;
            T s = 0;
#pragma unroll 8
            for (int k = 0; k < n1; ++k) s += Dr[k] * xr[k * st];
            g[a] = s;
        }
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            T f = 0;
#pragma unroll
            for (int b = 0; b < DIM; ++b) f += G[gidx(DIM, a, b) * N + q] * g[b];
            TR[a * N + q] = f;
        }
    }
    wg_barrier();
    for (int q = threadIdx.x; q < N; q += NT) {
        if (is_boundary<P, DIM>(q)) {
            out[q] = T(0);
            continue;
        }
        int c[3] = {q % n1, (q / n1) % n1, DIM == 3 ? q / (n1 * n1) : 0};
        T y = 0;
        {
            const auto fr = TR + (q - c[0]);
#pragma unroll 8
            for (int k = 0; k < n1; ++k) y += D[k * n1 + c[0]] * fr[k];
        }
#pragma unroll
        for (int a = 1; a < DIM; ++a) {
            const int st = a == 1 ? n1 : n1 * n1;
            const auto fr = TR + a * N + (q - c[a] * st);
#pragma unroll 8
            for (int k = 0; k < n1; ++k) y += D[k * n1 + c[a]] * fr[k * st];
        }
        out[q] = RESID ? r[q] - y : y;
    }
    wg_barrier();
}

template <class T, int P, int DIM, bool RESID>
__device__ __attribute__((noinline)) void apply_level(const T* __restrict__ G_,
                                                      const T* __restrict__ D_,
                                                      const T* __restrict__ DT_, T* __restrict__ TR_,
                                                      const T* __restrict__ x_,
                                                      const T* __restrict__ r_, T* __restrict__ out_)
{
    if constexpr (DIM == 2 && P >= MFMA_MIN_P2) {
        apply2d_mfma<T, P, RESID>(G_, D_, DT_, TR_, x_, r_, out_);
        return;
    }
    if constexpr (DIM == 3 && P >= MFMA_MIN_P) {
        apply3d_mfma<T, P, RESID>(G_, D_, DT_, TR_, x_, r_, out_);
        return;
    }
    using S = Shape<P, DIM>;
    constexpr int N = S::N, n1 = S::n1;
    // every operand staged in the LDS work buffer where it fits (2-D and
    // 3-D p <= 8 in the one-launch kernels): one memory round trip in
    constexpr int LDSW = PMG_WORK_LDS_WORDS * (int)(sizeof(double) / sizeof(T));
    constexpr int NG = S::NC * N, NTR = DIM * N, ND = n1 * n1;
    if constexpr (N + NG + NTR + 2 * ND <= LDSW) {
        const auto wl = (__attribute__((address_space(3))) T*)work_lds();
        const auto G = gmem(G_);
        const auto D = gmem(D_);
        const auto DT = gmem(DT_);
        const auto x = gmem(x_);
        const auto lx = wl, lg = wl + N, ltr = wl + N + NG, ld = wl + N + NG + NTR, ldt = ld + ND;
        for (int q = threadIdx.x; q < N; q += NT) lx[q] = x[q];
        for (int q = threadIdx.x; q < NG; q += NT) lg[q] = G[q];
        for (int q = threadIdx.x; q < ND; q += NT) {
            ld[q] = D[q];
            ldt[q] = DT[q];
        }
        wg_barrier();
        apply_vector<T, P, DIM, RESID>(lg, ld, ldt, lx, ltr, r_, out_);
    } else {
        apply_vector<T, P, DIM, RESID>(gmem(G_), gmem(D_), gmem(DT_), gmem(x_), gmem(TR_), r_,
                                       out_);
    }
}

// A x of a level of one element (apply_level) or of K^dim elements
// (apply_elements_level); the branch sits at the call site so that each
// operator keeps its own code and registers.
template <class T, int P, int DIM, bool RESID>
__device__ __attribute__((always_inline)) inline void apply_any(
    int K, T* EX, const T* __restrict__ G, const T* __restrict__ D, const T* __restrict__ DT,
    T* __restrict__ TR, const T* __restrict__ x, const T* __restrict__ r, T* __restrict__ out)
{
    if constexpr (P >= 4) {
        if (K > 1) {
            apply_elements_level<T, P, DIM, RESID>(K, G, D, DT, TR, EX, x, r, out);
            return;
        }
    }
    apply_level<T, P, DIM, RESID>(G, D, DT, TR, x, r, out);
}

// ------------------------------------------------------------------ line solver

// node index of position s (0-based, interior) on line `line` along axis dir
template <int P, int DIM>
__device__ inline void line_base(int dir, int line, int& base, int& st)
{
    constexpr int n1 = P + 1, n = P - 1;
    if (DIM == 2) {
        int o = line + 1;
        base = dir == 0 ? o * n1 : o;
        st = dir == 0 ? 1 : n1;
    } else {
        int o1 = line % n + 1, o2 = line / n + 1;
        if (dir == 0) { base = o1 * n1 + o2 * n1 * n1; st = 1; }
        else if (dir == 1) { base = o1 + o2 * n1 * n1; st = n1; }
        else { base = o1 + o2 * n1; st = n1 * n1; }
    }
}

// Lines along the first axis (p <= 128) are solved one line per group of
// (n+1)/2 lanes (a whole wave at p = 128) with the cyclic-reduction operators
// built on the fly (Prop. "line-solver cost", matrix-free variant, Remark on
// its memory footprint): only the line's tridiagonal (l, a, u) is stored
// ([line][position][3], contiguous).  Lane u holds positions 2u (an F point
// of level 0) and 2u+1 (a C point, which is also where every coarser level
// keeps its unknowns: level-k unknown t lives in lane (t+1) 2^(k-1) - 1).
// Going down, each F point turns its row into (1/a, l/a, u/a) and each C point
// forms its row of the coarse matrix D - C A^{-1} B (stencil of the proof of
// Prop. "line coarse space") from its F neighbours' values, exchanged with
// cross-lane shuffles; every lane keeps the (l/a, u/a) of the two F points it
// owns (level 0 and the level where its C unknown becomes F) for the way up.
// The whole hierarchy lives in registers: O(n) memory and O(n) work per line,
// instead of the paper's O(n^2) for the on-the-fly variant.
template <int P>
__host__ __device__ constexpr bool wave_lines() { return P >= 2 && P <= 128; }

// The two tridiagonal rows lane u of a line's lane group holds (positions
// 2u and 2u+1), loaded ahead of the solve so that the next line's loads can
// be in flight while the current one is reduced.
template <class T>
struct CrRows {
    T lF, aF, uF, cl, ca, cu;
};
template <class T, class PC>
__device__ inline CrRows<T> cr_rows(PC c, int u, bool has1)
{
    CrRows<T> w;
    w.lF = c[(2 * u) * 3 + 0];
    w.aF = c[(2 * u) * 3 + 1];
    w.uF = c[(2 * u) * 3 + 2];
    w.cl = has1 ? c[(2 * u + 1) * 3 + 0] : T(0);
    w.ca = has1 ? c[(2 * u + 1) * 3 + 1] : T(1);
    w.cu = has1 ? c[(2 * u + 1) * 3 + 2] : T(0);
    return w;
}

// Solve one line held by a lane group of W lanes (lane u: e0 = position 2u,
// e1 = position 2u+1) with its tridiagonal rows c[s*3 + {0,1,2}] = (l, a, u),
// given as the lane's two rows (cr_rows).
template <class T, int n, int W>
__device__ inline void cr_wave_solve_rows(const CrRows<T>& rw, int u, bool has1, T& e0, T& e1)
{
    constexpr int NK = ilog2(n + 1);
    const T lF = rw.lF, aF = rw.aF, uF = rw.uF;
    T cl = rw.cl, ca = rw.ca, cu = rw.cu;
    // level 0 down: F solve, then C residual and C's coarse row
    const T iF = T(1) / aF;
    const T pl0 = lF * iF, pu0 = uF * iF;
    e0 *= iF;
    {
        const T xr = __shfl(e0, u + 1, W), plr = __shfl(pl0, u + 1, W), pur = __shfl(pu0, u + 1, W);
        if (has1) {
            e1 -= cl * e0 + cu * xr;
            const T na = ca - cl * pu0 - cu * plr;
            const T nl = -cl * pl0, nu = -cu * pur;
            cl = nl;
            ca = na;
            cu = nu;
        }
    }
    T plF = T(0), puF = T(0);   // row of this lane's C unknown where it becomes F
#pragma unroll
    for (int k = 1; k < NK; ++k) {
        const int nk = ((n + 1) >> k) - 1;
        const int hs = 1 << (k - 1);
        const bool on = ((u + 1) % hs == 0) && ((u + 1) / hs - 1 < nk);
        const int t = (u + 1) / hs - 1;
        if (nk == 1) {
            if (on) e1 /= ca;
        } else {
            if (on && (t & 1) == 0) {
                const T ia = T(1) / ca;
                plF = cl * ia;
                puF = cu * ia;
                e1 *= ia;
            }
            const T lf = __shfl(e1, u - hs, W), rg = __shfl(e1, u + hs, W);
            const T pul = __shfl(puF, u - hs, W), pll = __shfl(plF, u - hs, W);
            const T plr = __shfl(plF, u + hs, W), pur = __shfl(puF, u + hs, W);
            if (on && (t & 1) == 1) {
                e1 -= cl * lf + cu * rg;
                const T na = ca - cl * pul - cu * plr;
                const T nl = -cl * pll, nu = -cu * pur;
                cl = nl;
                ca = na;
                cu = nu;
            }
        }
    }
#pragma unroll
    for (int k = NK - 2; k >= 1; --k) {
        const int nk = ((n + 1) >> k) - 1;
        const int hs = 1 << (k - 1);
        const T lf = __shfl(e1, u - hs, W), rg = __shfl(e1, u + hs, W);
        const bool on = ((u + 1) % hs == 0) && ((u + 1) / hs - 1 < nk);
        const int t = (u + 1) / hs - 1;
        if (on && (t & 1) == 0) {
            T v = e1;
            if (t >= 1) v -= plF * lf;
            if (t + 1 < nk) v -= puF * rg;
            e1 = v;
        }
    }
    {
        const T lf = __shfl(e1, u - 1, W);
        T v = e0;
        if (u >= 1) v -= pl0 * lf;
        if (has1) v -= pu0 * e1;
        e0 = v;
    }
}

template <class T, int n, int W, class PC>
__device__ inline void cr_wave_solve(PC c, int u, bool has1, T& e0, T& e1)
{
    cr_wave_solve_rows<T, n, W>(cr_rows<T>(c, u, has1), u, has1, e0, e1);
}

// Block cyclic reduction of one line whose matrix has half-bandwidth 2, as a
// block-tridiagonal matrix of 2x2 blocks (Def. block-tridiagonal matrix;
// unknowns 2u and 2u+1 form block u, an odd line length is padded with one
// decoupled unknown), solved by the direct multigrid of Thm. "Two-level
// direct solver" with block operators, level after level (Cor. "Direct
// multigrid solver").  Lane u of a group of W = (n+1)/2 lanes holds block u
// (positions 2u, 2u+1: the same data placement as cr_wave_solve).  At level
// k the blocks still present sit in lanes (t+1) 2^k - 1, t = 0, 1, ...; the F
// blocks (t even) form A^{-1} L, A^{-1} U and A^{-1} g and keep them for the
// way up; each C block forms its row of D - C A^{-1} B and its right-hand
// side from its F neighbours' (stencil of the proof of Prop. "line coarse
// space"), received by cross-lane shuffles.  c[s*5 + k + 2] = entry (s, s+k).
template <class T, int n, int W, class PC>
__device__ inline void bcr_wave_solve(PC c, int u, bool has1, T& e0, T& e1)
{
    constexpr int NB = (n + 1) / 2;
    constexpr int NK = ilog2(NB);
    static_assert((1 << NK) == NB, "a power-of-two number of blocks");
    const int s0 = 2 * u, s1 = 2 * u + 1;
    auto E = [&](int s, int k) -> T { return c[s * 5 + k + 2]; };
    // A, L (block u-1), U (block u+1) of this lane's block row; out-of-line
    // entries are stored as zero, the padding row is an identity row
    T a00 = E(s0, 0), a01 = E(s0, 1), a10 = has1 ? E(s1, -1) : T(0), a11 = has1 ? E(s1, 0) : T(1);
    T l00 = E(s0, -2), l01 = E(s0, -1), l10 = T(0), l11 = has1 ? E(s1, -2) : T(0);
    T u00 = E(s0, 2), u01 = T(0), u10 = has1 ? E(s1, 1) : T(0), u11 = has1 ? E(s1, 2) : T(0);
    T g0 = e0, g1 = has1 ? e1 : T(0);
    T p00 = 0, p01 = 0, p10 = 0, p11 = 0;   // A^{-1} L of the level where this block is F
    T q00 = 0, q01 = 0, q10 = 0, q11 = 0;   // A^{-1} U
    T y0 = 0, y1 = 0;                       // A^{-1} g
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        const int hs = 1 << k, nbk = NB >> k;
        const bool on = (u + 1) % hs == 0;
        const int t = (u + 1) / hs - 1;
        if (on && (t & 1) == 0) {
            const T id = T(1) / (a00 * a11 - a01 * a10);
            const T i00 = a11 * id, i01 = -a01 * id, i10 = -a10 * id, i11 = a00 * id;
            p00 = i00 * l00 + i01 * l10; p01 = i00 * l01 + i01 * l11;
            p10 = i10 * l00 + i11 * l10; p11 = i10 * l01 + i11 * l11;
            q00 = i00 * u00 + i01 * u10; q01 = i00 * u01 + i01 * u11;
            q10 = i10 * u00 + i11 * u10; q11 = i10 * u01 + i11 * u11;
            y0 = i00 * g0 + i01 * g1;
            y1 = i10 * g0 + i11 * g1;
        }
        // from the F block on the left (u - hs) and on the right (u + hs)
        const int ul = u - hs, ur = u + hs;
        const T Lp00 = __shfl(p00, ul, W), Lp01 = __shfl(p01, ul, W), Lp10 = __shfl(p10, ul, W),
                Lp11 = __shfl(p11, ul, W);
        const T Lq00 = __shfl(q00, ul, W), Lq01 = __shfl(q01, ul, W), Lq10 = __shfl(q10, ul, W),
                Lq11 = __shfl(q11, ul, W);
        const T Ly0 = __shfl(y0, ul, W), Ly1 = __shfl(y1, ul, W);
        const T Rp00 = __shfl(p00, ur, W), Rp01 = __shfl(p01, ur, W), Rp10 = __shfl(p10, ur, W),
                Rp11 = __shfl(p11, ur, W);
        const T Rq00 = __shfl(q00, ur, W), Rq01 = __shfl(q01, ur, W), Rq10 = __shfl(q10, ur, W),
                Rq11 = __shfl(q11, ur, W);
        const T Ry0 = __shfl(y0, ur, W), Ry1 = __shfl(y1, ur, W);
        if (on && (t & 1) == 1) {
            const bool hasR = t + 1 < nbk;
            // right-hand side and diagonal block of D - C A^{-1} B
            g0 -= l00 * Ly0 + l01 * Ly1;
            g1 -= l10 * Ly0 + l11 * Ly1;
            a00 -= l00 * Lq00 + l01 * Lq10; a01 -= l00 * Lq01 + l01 * Lq11;
            a10 -= l10 * Lq00 + l11 * Lq10; a11 -= l10 * Lq01 + l11 * Lq11;
            T n00 = -(l00 * Lp00 + l01 * Lp10), n01 = -(l00 * Lp01 + l01 * Lp11);
            T n10 = -(l10 * Lp00 + l11 * Lp10), n11 = -(l10 * Lp01 + l11 * Lp11);
            T m00 = 0, m01 = 0, m10 = 0, m11 = 0;
            if (hasR) {
                g0 -= u00 * Ry0 + u01 * Ry1;
                g1 -= u10 * Ry0 + u11 * Ry1;
                a00 -= u00 * Rp00 + u01 * Rp10; a01 -= u00 * Rp01 + u01 * Rp11;
                a10 -= u10 * Rp00 + u11 * Rp10; a11 -= u10 * Rp01 + u11 * Rp11;
                m00 = -(u00 * Rq00 + u01 * Rq10); m01 = -(u00 * Rq01 + u01 * Rq11);
                m10 = -(u10 * Rq00 + u11 * Rq10); m11 = -(u10 * Rq01 + u11 * Rq11);
            }
            l00 = n00; l01 = n01; l10 = n10; l11 = n11;
            u00 = m00; u01 = m01; u10 = m10; u11 = m11;
        }
    }
    // the one block left (lane NB - 1) is solved directly
    T x0 = T(0), x1 = T(0);
    if (u == NB - 1) {
        const T id = T(1) / (a00 * a11 - a01 * a10);
        x0 = (a11 * g0 - a01 * g1) * id;
        x1 = (a00 * g1 - a10 * g0) * id;
    }
#pragma unroll
    for (int k = NK - 1; k >= 0; --k) {
        const int hs = 1 << k, nbk = NB >> k;
        const bool on = (u + 1) % hs == 0;
        const int t = (u + 1) / hs - 1;
        const T xl0 = __shfl(x0, u - hs, W), xl1 = __shfl(x1, u - hs, W);
        const T xr0 = __shfl(x0, u + hs, W), xr1 = __shfl(x1, u + hs, W);
        if (on && (t & 1) == 0) {
            // y = A^{-1} g - A^{-1} L x_left - A^{-1} U x_right  (x + P e)
            T v0 = y0, v1 = y1;
            if (t >= 1) {
                v0 -= p00 * xl0 + p01 * xl1;
                v1 -= p10 * xl0 + p11 * xl1;
            }
            if (t + 1 < nbk) {
                v0 -= q00 * xr0 + q01 * xr1;
                v1 -= q10 * xr0 + q11 * xr1;
            }
            x0 = v0;
            x1 = v1;
        }
    }
    e0 = x0;
    e1 = has1 ? x1 : T(0);
}

// One lane-group solve of line lc: scalar cyclic reduction on the
// tridiagonal rows (3 CRW words per line), or block cyclic reduction on the
// half-bandwidth-2 rows (5 n words per line).
template <class T, int n, int W, int CRW, bool BAND, class PC>
__device__ inline void wave_line_solve(PC cr, int lc, int u, bool has1, T& e0, T& e1)
{
    if constexpr (BAND)
        bcr_wave_solve<T, n, W>(cr + (long long)lc * 5 * n, u, has1, e0, e1);
    else
        cr_wave_solve<T, n, W>(cr + (long long)lc * 3 * CRW, u, has1, e0, e1);
}

template <class T, int P, int DIM, bool FUSED, bool BAND = false>
__device__ void line_cr_wave(const T* __restrict__ cr_, T* __restrict__ g_, T* __restrict__ x_,
                             T alpha, bool assign)
{
    const auto cr = gmem(cr_);
    const auto g = gmem(g_);
    const auto x = gmem(x_);
    using S = Shape<P, DIM>;
    constexpr int n = S::n, NL = S::NL, CRW = S::CRW;
    constexpr int W = (n + 1) / 2 > 0 ? (n + 1) / 2 : 1;   // lanes per line
    constexpr int LPW = 64 / W;                              // lines per wave
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int u = lane % W, sub = lane / W;
    const bool has1 = 2 * u + 1 < n;
    constexpr int STEP = (NT / 64) * LPW;
    if constexpr (!BAND) {
        // software-pipelined: a line's rows, right-hand side and (fused) x
        // are loaded together, one line ahead of its reduction
        const bool rdx = FUSED && !assign;
        auto load = [&](int line0, CrRows<T>& rw, T& e0, T& e1, T& x0, T& x1) {
            const int line = line0 + sub;
            const int lc = line < NL ? line : NL - 1;
            int base, st;
            line_base<P, DIM>(0, lc, base, st);
            rw = cr_rows<T>(cr + (long long)lc * 3 * CRW, u, has1);
            e0 = g[base + 2 * u + 1];
            e1 = has1 ? g[base + 2 * u + 2] : T(0);
            x0 = rdx ? x[base + 2 * u + 1] : T(0);
            x1 = rdx && has1 ? x[base + 2 * u + 2] : T(0);
        };
        CrRows<T> rn;
        T e0n, e1n, x0n, x1n;
        int line0 = wave * LPW;
        if (line0 < NL) load(line0, rn, e0n, e1n, x0n, x1n);
        for (; line0 < NL; line0 += STEP) {
            const CrRows<T> rw = rn;
            T e0 = e0n, e1 = e1n;
            const T x0 = x0n, x1 = x1n;
            if (line0 + STEP < NL) load(line0 + STEP, rn, e0n, e1n, x0n, x1n);
            const int line = line0 + sub;
            cr_wave_solve_rows<T, n, W>(rw, u, has1, e0, e1);
            if (line < NL) {
                int base, st;
                line_base<P, DIM>(0, line, base, st);
                const int q0 = base + 2 * u + 1;
                if (FUSED) {
                    x[q0] = x0 + alpha * e0;
                    if (has1) x[q0 + 1] = x1 + alpha * e1;
                } else {
                    const auto z = x_ ? x : g;
                    z[q0] = e0;
                    if (has1) z[q0 + 1] = e1;
                }
            }
        }
        wg_barrier();
        return;
    }
    for (int line0 = wave * LPW; line0 < NL; line0 += STEP) {
        const int line = line0 + sub;
        const bool act = line < NL;
        const int lc = act ? line : NL - 1;
        int base, st;
        line_base<P, DIM>(0, lc, base, st);
        T e0 = g[base + 2 * u + 1];
        T e1 = has1 ? g[base + 2 * u + 2] : T(0);
        wave_line_solve<T, n, W, CRW, BAND>(cr, lc, u, has1, e0, e1);
        if (act) {
            if (FUSED) {
                const int q0 = base + 2 * u + 1;
                x[q0] = (assign ? T(0) : x[q0]) + alpha * e0;
                if (has1) x[q0 + 1] = (assign ? T(0) : x[q0 + 1]) + alpha * e1;
            } else {
                const auto z = x_ ? x : g;
                z[base + 2 * u + 1] = e0;
                if (has1) z[base + 2 * u + 2] = e1;
            }
        }
    }
    wg_barrier();
}

// LDS strip of the strided line solves: up to 16 lines of 127 unknowns or
// 32 of 63, padded rows.
constexpr int LINE_STRIP_WORDS = 127 * 17;

// Lines along the second axis (and the third in 3-D), strided in memory, in
// strips of SW adjacent lines (consecutive first-axis positions at one value
// of the remaining coordinate): the strip's right-hand sides are read row by
// row (coalesced) into LDS, each line is solved by a lane group as above,
// and the solutions go back row by row.  Line index = (i-1) + n (o-1) for
// first-axis position i and outer coordinate o, as everywhere else; the
// lines' tridiagonals are stored line-major like the first axis'.
template <class T, int P, int DIM, bool FUSED, bool BAND = false>
__device__ void line_cr_wave_strided(const T* __restrict__ cr_, int dir, T* __restrict__ g_,
                                     T* __restrict__ x_, T alpha, bool assign)
{
    const auto cr = gmem(cr_);
    const auto g = gmem(g_);
    const auto x = gmem(x_);
    using S = Shape<P, DIM>;
    constexpr int n1 = S::n1, n = S::n, CRW = S::CRW;
    constexpr int W = (n + 1) / 2 > 0 ? (n + 1) / 2 : 1;
    constexpr int LPW = 64 / W;
    // lines per strip: 64 long lines where the work buffer holds them (fewer
    // barriers, 512-byte row segments), else 16; 32 short ones
    constexpr int SW = n > 63 ? (n * 65 * (int)sizeof(T) <= 8 * PMG_WORK_LDS_WORDS ? 64 : 16) : 32;
    constexpr int LD = SW + 1;                               // LDS row
    constexpr int NO = DIM == 2 ? 1 : n;                     // values of the outer coordinate
    static_assert(n * LD * sizeof(T) <= sizeof(double) * PMG_WORK_LDS_WORDS, "strip fits");
    static_assert(LINE_STRIP_WORDS <= PMG_WORK_LDS_WORDS, "the work buffer holds a strip");
    const auto strip = (__attribute__((address_space(3))) T*)work_lds();
    const int RS = dir == 1 ? n1 : n1 * n1;                  // stride along the line
    const int OS = DIM == 2 ? 0 : (dir == 1 ? n1 * n1 : n1); // stride of the outer coordinate
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int u = lane % W, sub = lane / W;
    const bool has1 = 2 * u + 1 < n;
    constexpr int STEP = (NT / 64) * LPW;
    // the rows of the line a lane group solves (the same line index as the
    // loop below), loaded one line ahead; the first ones while the strip's
    // right-hand sides arrive
    auto rows_of = [&](int s0, int l0, int o) {
        const int sc = min(s0 + sub, SW - 1);
        const int lc = min(l0 + sc, n - 1) + n * o;
        return cr_rows<T>(cr + (long long)lc * 3 * CRW, u, has1);
    };
    for (int o = 0; o < NO; ++o) {
        const int ob = DIM == 2 ? 0 : (o + 1) * OS;
        for (int l0 = 0; l0 < n; l0 += SW) {
            CrRows<T> rn;
            if constexpr (!BAND)
                if (wave * LPW < SW) rn = rows_of(wave * LPW, l0, o);
            for (int e = threadIdx.x; e < n * SW; e += NT) {
                const int r = e / SW, ci = e % SW, i = l0 + ci;
                strip[r * LD + ci] = i < n ? g[ob + (r + 1) * RS + i + 1] : T(0);
            }
            wg_barrier();
            for (int s0 = wave * LPW; s0 < SW; s0 += STEP) {
                const int sl = s0 + sub;                   // line within the strip
                const int sc = min(sl, SW - 1);            // lane groups past the strip
                const int lc = min(l0 + sc, n - 1) + n * o;   // compute on a copy, store nothing
                T e0 = strip[(2 * u) * LD + sc];
                T e1 = has1 ? strip[(2 * u + 1) * LD + sc] : T(0);
                if constexpr (BAND) {
                    wave_line_solve<T, n, W, CRW, BAND>(cr, lc, u, has1, e0, e1);
                } else {
                    const CrRows<T> rw = rn;
                    if (s0 + STEP < SW) rn = rows_of(s0 + STEP, l0, o);
                    cr_wave_solve_rows<T, n, W>(rw, u, has1, e0, e1);
                }
                if (sl < SW) {
                    strip[(2 * u) * LD + sl] = e0;
                    if (has1) strip[(2 * u + 1) * LD + sl] = e1;
                }
            }
            wg_barrier();
            for (int e = threadIdx.x; e < n * SW; e += NT) {
                const int r = e / SW, ci = e % SW, i = l0 + ci;
                if (i < n) {
                    const int q = ob + (r + 1) * RS + i + 1;
                    if (FUSED)
                        x[q] = (assign ? T(0) : x[q]) + alpha * strip[r * LD + ci];
                    else
                        (x_ ? x : g)[q] = strip[r * LD + ci];
                }
            }
            wg_barrier();
        }
    }
}

// Cyclic reduction as a direct multigrid (Thm. "Two-level direct solver",
// Cor. "Direct multigrid solver"), one thread per line, in place on g.
// Level k of a line of n = 2^q - 1 unknowns holds the unknowns at 1-based
// positions t * 2^k; F points are t odd, C points t even (Def. odd-even
// reordering).  Factors per level slot: F (1/a, -l/a, -u/a) = (S^{-1}, rows
// of P); C (l, a, u) of that level's matrix, whose Schur complement
// D - C A^{-1} B is the next level.
//   down: x_F = g_F / a_F;  g_C -= l_C x_{C-1} + u_C x_{C+1}   (R (g - M x))
//   coarsest: x = g / a
//   up:   y_F = x_F - (l_F e_{F-1} + u_F e_{F+1}) / a_F         (x + P e)
// FUSED: instead of storing z, x += alpha z (x = alpha z with assign, lane
// groups only: x is then not read).  Not fused, lines solved by
// lane groups (wave_lines) store z into x when x is given (g is then only
// read), else in place; the thread-per-line form is in place only.
template <class T, int P, int DIM, bool FUSED, bool BAND = false>
__device__ __attribute__((noinline)) void line_cr(const T* __restrict__ cr_, int dir,
                                                  T* __restrict__ g_, T* __restrict__ x_, T alpha,
                                                  bool assign = false)
{
    if constexpr (wave_lines<P>()) {
        if (dir == 0) {
            line_cr_wave<T, P, DIM, FUSED, BAND>(cr_, g_, x_, alpha, assign);
            return;
        }
        line_cr_wave_strided<T, P, DIM, FUSED, BAND>(cr_, dir, g_, x_, alpha, assign);
        return;
    }
    if constexpr (BAND) return;   // half-bandwidth-2 lines only up to p = 128 (host-checked)
    const auto cr = gmem(cr_);
    const auto g = gmem(g_);
    const auto x = gmem(x_);
    using S = Shape<P, DIM>;
    constexpr int n = S::n, NL = S::NL;
    constexpr int NK = ilog2(n + 1);   // number of CR levels
    for (int line = threadIdx.x; line < NL; line += NT) {
        int base, st;
        line_base<P, DIM>(dir, line, base, st);
        auto node = [&](int s) { return base + (s + 1) * st; };
        auto W = [&](int slot, int w) -> T { return cr[(slot * 3 + w) * NL + line]; };
        int off = 0;
#pragma unroll
        for (int k = 0; k < NK - 1; ++k) {
            const int nk = (n + 1) / (1 << k) - 1;
#pragma unroll 8
            for (int t = 0; t < nk; t += 2) {
                int s = ((t + 1) << k) - 1;
                g[node(s)] *= W(off + t, 0);
            }
#pragma unroll 8
            for (int t = 1; t < nk; t += 2) {
                int s = ((t + 1) << k) - 1;
                int sl = (t << k) - 1, sr = ((t + 2) << k) - 1;
                g[node(s)] -= W(off + t, 0) * g[node(sl)] + W(off + t, 2) * g[node(sr)];
            }
            off += nk;
        }
        {
            int s = (1 << (NK - 1)) - 1;
            g[node(s)] *= W(off, 0);
        }
#pragma unroll
        for (int k = NK - 2; k >= 0; --k) {
            const int nk = (n + 1) / (1 << k) - 1;
            off -= nk;
            if (FUSED && k == 0) {
#pragma unroll 8
                for (int t = 0; t < nk; ++t) {
                    int s = t;
                    T v;
                    if ((t & 1) == 0) {
                        v = g[node(s)];
                        if (t >= 1) v += W(off + t, 1) * g[node(s - 1)];
                        if (t + 1 < nk) v += W(off + t, 2) * g[node(s + 1)];
                    } else {
                        v = g[node(s)];
                    }
                    x[node(s)] += alpha * v;
                }
            } else {
#pragma unroll 8
                for (int t = 0; t < nk; t += 2) {
                    int s = ((t + 1) << k) - 1;
                    T v = g[node(s)];
                    if (t >= 1) v += W(off + t, 1) * g[node((t << k) - 1)];
                    if (t + 1 < nk) v += W(off + t, 2) * g[node(((t + 2) << k) - 1)];
                    g[node(s)] = v;
                }
            }
        }
        if (FUSED && NK == 1) x[node(0)] += alpha * g[node(0)];
    }
    wg_barrier();
}

// ------------------------------------------------------------------ transfers

// One axis of the restriction R = (J x J [x J])^T: out(.., o_a, ..) =
// sum_t J[t][o_a] in(.., t, ..), in has extent n1f along a, out n1c.
template <class T>
__device__ void restrict_axis(const T* __restrict__ in_, T* __restrict__ out_, int e0, int e1,
                              int e2, int a, int n1f, int n1c, const T* __restrict__ J_,
                              bool zero_boundary)
{
    const auto in = gmem(in_);
    const auto out = gmem(out_);
    const auto J = gmem(J_);
    int eo[3] = {e0, e1, e2};
    eo[a] = n1c;
    int ei[3] = {e0, e1, e2};
    ei[a] = n1f;
    const int tot = eo[0] * eo[1] * eo[2];
    const int sti = a == 0 ? 1 : (a == 1 ? ei[0] : ei[0] * ei[1]);
    for (int q = threadIdx.x; q < tot; q += NT) {
        int o0 = q % eo[0], o1 = (q / eo[0]) % eo[1], o2 = q / (eo[0] * eo[1]);
        int oa = a == 0 ? o0 : (a == 1 ? o1 : o2);
        if (zero_boundary) {
            bool bd = o0 == 0 || o0 == eo[0] - 1 || o1 == 0 || o1 == eo[1] - 1 ||
                      (eo[2] > 1 && (o2 == 0 || o2 == eo[2] - 1));
            if (bd) { out[q] = T(0); continue; }
        }
        int ii[3] = {o0, o1, o2};
        ii[a] = 0;
        const auto src = in + ii[0] + ei[0] * (ii[1] + ei[1] * ii[2]);
        T s = 0;
        for (int t = 0; t < n1f; ++t) s += J[t * n1c + oa] * src[t * sti];
        out[q] = s;
    }
    wg_barrier();
}

// One axis of the prolongation P = J x J [x J]: out(.., o_a, ..) =
// sum_t J[o_a][t] in(.., t, ..), in has extent n1c along a, out n1f.
template <class T, bool ADD>
__device__ void prolong_axis(const T* __restrict__ in_, T* __restrict__ out_, int e0, int e1,
                             int e2, int a, int n1f, int n1c, const T* __restrict__ J_,
                             const T* __restrict__ JT_)
{
    const auto in = gmem(in_);
    const auto out = gmem(out_);
    const auto J = gmem(J_);
    const auto JT = gmem(JT_);
    int eo[3] = {e0, e1, e2};
    eo[a] = n1f;
    int ei[3] = {e0, e1, e2};
    ei[a] = n1c;
    const int tot = eo[0] * eo[1] * eo[2];
    const int sti = a == 0 ? 1 : (a == 1 ? ei[0] : ei[0] * ei[1]);
    for (int q = threadIdx.x; q < tot; q += NT) {
        int o0 = q % eo[0], o1 = (q / eo[0]) % eo[1], o2 = q / (eo[0] * eo[1]);
        int ii[3] = {o0, o1, o2};
        ii[a] = 0;
        const auto src = in + ii[0] + ei[0] * (ii[1] + ei[1] * ii[2]);
        T s = 0;
        if (a == 0) {
            for (int t = 0; t < n1c; ++t) s += JT[t * n1f + o0] * src[t * sti];
        } else {
            int oa = a == 1 ? o1 : o2;
            for (int t = 0; t < n1c; ++t) s += J[oa * n1c + t] * src[t * sti];
        }
        if (ADD) out[q] += s; else out[q] = s;
    }
    wg_barrier();
}

// rc = R_l rf with zero coarse boundary (Sec. 3.3).  R is the tensor product
// of the transpose of the 1-D table passed as J: the prolongation J itself
// for R = P^T, or the fine basis at the coarse nodes for the interpolation
// reading of the same section.
template <class T, int P, int DIM>
__device__ __attribute__((noinline)) void restrict_level(const T* rf, T* rc, const T* J,
                                                         const T* JT, T* w1, T* w2)
{
    constexpr int n1f = P + 1, n1c = P / 2 + 1;
    constexpr int LDSW = PMG_WORK_LDS_WORDS * (int)(sizeof(double) / sizeof(T));
    if constexpr (DIM == 2 && P >= MFMA_MIN_P2) {
        // W1 = rf J (n1f x n1c); rc = J^T W1 with zero boundary; W1 in the
        // LDS work buffer where it fits (p <= 128 in the solve kernels)
        (void)w2;
        if constexpr (n1f * n1c <= LDSW) {
            const auto wl = (__attribute__((address_space(3))) T*)work_lds();
            wg_gemm<T, n1f, n1c, n1f, n1f, n1c, 0>(rf, J, wl);
            wg_gemm<T, n1c, n1c, n1f, n1c, n1c, 2, true>(J, wl, rc);
        } else {
            wg_gemm<T, n1f, n1c, n1f, n1f, n1c, 0>(rf, J, w1);
            wg_gemm<T, n1c, n1c, n1f, n1c, n1c, 2, true>(J, w1, rc);
        }
        return;
    }
    if constexpr (DIM == 3 && P >= MFMA_MIN_P) {
        // third axis:  W1 = J^T RF, RF as n1f x n1f^2       -> [k'][j][i]
        // first axis:  W2 = W1 J, W1 as (n1c n1f) x n1f      -> [k'][j][i']
        // second axis: rc_k' = J^T W2_k' for every slab k', boundary faces zero
        wg_gemm<T, n1c, n1f * n1f, n1f, n1c, n1f * n1f, 0, true>(J, rf, w1);
        wg_gemm<T, n1c * n1f, n1c, n1f, n1f, n1c, 0>(w1, J, w2);
        wg_gemm<T, n1c, n1c, n1f, n1c, n1c, 2, true, n1c, n1f * n1c, n1c * n1c>(J, w2, rc);
        return;
    }
    if (DIM == 2) {
        restrict_axis<T>(rf, w1, n1f, n1f, 1, 0, n1f, n1c, J, false);
        restrict_axis<T>(w1, rc, n1c, n1f, 1, 1, n1f, n1c, J, true);
    } else {
        restrict_axis<T>(rf, w1, n1f, n1f, n1f, 0, n1f, n1c, J, false);
        restrict_axis<T>(w1, w2, n1c, n1f, n1f, 1, n1f, n1c, J, false);
        restrict_axis<T>(w2, rc, n1c, n1c, n1f, 2, n1f, n1c, J, true);
    }
}

// xf += P_l ec
template <class T, int P, int DIM>
__device__ __attribute__((noinline)) void prolong_level(const T* ec, T* xf, const T* J, const T* JT, T* w1, T* w2)
{
    constexpr int n1f = P + 1, n1c = P / 2 + 1;
    constexpr int LDSW = PMG_WORK_LDS_WORDS * (int)(sizeof(double) / sizeof(T));
    if constexpr (DIM == 2 && P >= MFMA_MIN_P2) {
        // W1 = ec J^T (n1c x n1f); xf += J W1; W1 in LDS where it fits
        (void)w2;
        if constexpr (n1c * n1f <= LDSW) {
            const auto wl = (__attribute__((address_space(3))) T*)work_lds();
            wg_gemm<T, n1c, n1f, n1c, n1c, n1f, 0>(ec, JT, wl);
            wg_gemm<T, n1f, n1f, n1c, n1f, n1f, 1, true>(JT, wl, xf);
        } else {
            wg_gemm<T, n1c, n1f, n1c, n1c, n1f, 0>(ec, JT, w1);
            wg_gemm<T, n1f, n1f, n1c, n1f, n1f, 1, true>(JT, w1, xf);
        }
        return;
    }
    if constexpr (DIM == 3 && P >= MFMA_MIN_P) {
        // third axis:  W1 = J EC, EC as n1c x n1c^2           -> [k][j'][i']
        // first axis:  W2 = W1 J^T, W1 as (n1f n1c) x n1c     -> [k][j'][i]
        // second axis: xf_k += J W2_k for every slab k
        wg_gemm<T, n1f, n1c * n1c, n1c, n1f, n1c * n1c, 0, true>(JT, ec, w1);
        wg_gemm<T, n1f * n1c, n1f, n1c, n1c, n1f, 0>(w1, JT, w2);
        wg_gemm<T, n1f, n1f, n1c, n1f, n1f, 1, true, n1f, n1c * n1f, n1f * n1f>(JT, w2, xf);
        return;
    }
    if (DIM == 2) {
        prolong_axis<T, false>(ec, w1, n1c, n1c, 1, 0, n1f, n1c, J, JT);
        prolong_axis<T, true>(w1, xf, n1f, n1c, 1, 1, n1f, n1c, J, JT);
    } else {
        prolong_axis<T, false>(ec, w1, n1c, n1c, n1c, 0, n1f, n1c, J, JT);
        prolong_axis<T, false>(w1, w2, n1f, n1c, n1c, 1, n1f, n1c, J, JT);
        prolong_axis<T, true>(w2, xf, n1f, n1f, n1c, 2, n1f, n1c, J, JT);
    }
}

// ------------------------------------------------------------------ gamma-cycle

template <class T, int P, int DIM>
__device__ inline const LevelData<T>& lvl(const Hier<T>& H)
{
    return H.lev[Shape<P, DIM>::LEV];
}

// The line solve of level P along axis dir on the level's line systems:
// half-bandwidth-2 rows by block cyclic reduction when the hierarchy has
// them, else the tridiagonal rows by scalar cyclic reduction.
template <class T, int P, int DIM, bool FUSED>
__device__ inline void level_lines(const LevelData<T>& L, int b, int dir, T* g, T* x, T alpha,
                                   bool assign = false)
{
    using S = Shape<P, DIM>;
    if constexpr (wave_lines<P>()) {
        if (L.bd[dir]) {
            line_cr<T, P, DIM, FUSED, true>(L.bd[dir] + (long long)b * 5 * S::n * S::NL, dir, g, x,
                                            alpha, assign);
            return;
        }
    }
    line_cr<T, P, DIM, FUSED>(L.cr[dir] + (long long)b * 3 * S::CRW * S::NL, dir, g, x, alpha,
                              assign);
}

// x += alpha B_dir^{-1} (r - A x)   (Alg. 2 smoothing step)
// E: the hierarchy has several elements per axis (H.K > 1); the one-element
// instances (E = false) carry no element code.
template <class T, int P, int DIM, bool E = false>
__device__ void smooth_step(const Hier<T>& H, int b, int dir, const T* r, T* x, bool x_is_zero)
{
    using S = Shape<P, DIM>;
    const LevelData<T>& L = lvl<T, P, DIM>(H);
    T* tmp = L.Tm + (long long)b * S::N;
    if (x_is_zero && wave_lines<P>()) {
        // the residual is r itself; lane-group lines only read their
        // right-hand side, so they take it from r without a copy, and they
        // assign x = alpha z on the interior (x's boundary is already zero)
        level_lines<T, P, DIM, true>(L, b, dir, const_cast<T*>(r), x, H.alpha, true);
        return;
    }
    if (x_is_zero) {
        wg_copy(tmp, r, S::N);   // the thread-per-line form works in place
        wg_barrier();
    } else {
        if constexpr (E)
            apply_elements_level<T, P, DIM, true>(H.K, L.G + (long long)b * S::NC * L.ng, L.D,
                                                  L.DT, L.TR + (long long)b * DIM * L.ng,
                                                  L.EX ? L.EX + (long long)b * L.ng : nullptr, x, r,
                                                  tmp);
        else
            apply_level<T, P, DIM, true>(L.G + (long long)b * S::NC * S::N, L.D, L.DT,
                                         L.TR + (long long)b * DIM * S::N, x, r, tmp);
    }
    level_lines<T, P, DIM, true>(L, b, dir, tmp, x, H.alpha);
}

// Levels whose gamma-cycle (with everything below it) is applied as one
// dense matrix: the cycle is linear in its right-hand side (Alg. 2 is a
// fixed sequence of linear steps), so M_c^{-1} r = C r with C = M_c^{-1}
// built once per problem at setup from the cycle itself (k_collapse): first
// the lower level from the recursive cycle, then the upper one from the
// cycle that uses the lower matrix.  2-D: p = 8 and 16 (49 and 225 interior
// nodes); 3-D: p = 4 and 8 (27 and 343).
__host__ __device__ constexpr int collapse_p(int dim) { return dim == 2 ? 16 : 8; }
__host__ __device__ constexpr int collapse_lo(int dim) { return collapse_p(dim) / 2; }

// node index of interior node number i (interior nodes in lexicographic order)
template <int P, int DIM>
__device__ inline int interior_node(int i)
{
    constexpr int n = P - 1, n1 = P + 1;
    const int i0 = i % n + 1, i1 = (i / n) % n + 1;
    return DIM == 2 ? i0 + n1 * i1 : i0 + n1 * i1 + n1 * n1 * (i / (n * n) + 1);
}

// x = C r on the interior of level P (FP64 arithmetic whatever T), zero
// boundary.  r's interior is staged in LDS (the work buffer); each entry of C r is split over KS lanes
// that take consecutive chunks of its terms (coalesced loads of C's rows),
// and the chunks are added in a fixed order.  Out of line and small: the
// function needs no callee-saved registers.
template <class T, int P, int DIM>
__device__ __attribute__((noinline)) void collapsed_solve(const double* C_, const T* r_, T* x_)
{
    using S = Shape<P, DIM>;
    constexpr int ni = ipow(P - 1, DIM);
    constexpr int KS = 2 * ni <= NT ? 2 : 1;          // lanes per entry
    constexpr int KL = (ni + KS - 1) / KS;            // terms per lane
    static_assert(3 * ni <= PMG_WORK_LDS_WORDS, "r and the partial sums fit the work buffer");
    const auto C = gmem(C_);
    const auto r = gmem(r_);
    const auto x = gmem(x_);
    const auto rl = (__attribute__((address_space(3))) double*)work_lds();
    for (int i = threadIdx.x; i < ni; i += NT) rl[i] = (double)r[interior_node<P, DIM>(i)];
    for (int q = threadIdx.x; q < S::N; q += NT)
        if (is_boundary<P, DIM>(q)) x[q] = T(0);
    wg_barrier();
    for (int t = threadIdx.x; t < KS * ni; t += NT) {
        const int part = t / ni, j = t - part * ni;
        const int i0 = part * KL, i1 = i0 + KL < ni ? i0 + KL : ni;
        double s = 0.0;
        if constexpr (KL >= 64) {   // long rows: sixteen loads in flight
#pragma unroll 16
            for (int i = i0; i < i1; ++i) s += C[(long long)i * ni + j] * rl[i];
        } else {
#pragma unroll 8
            for (int i = i0; i < i1; ++i) s += C[(long long)i * ni + j] * rl[i];
        }
        if (KS == 1)
            x[interior_node<P, DIM>(j)] = T(s);
        else if (part == 1)
            rl[ni + j] = s;
        else
            rl[2 * ni + j] = s;
    }
    if constexpr (KS > 1) {
        wg_barrier();
        for (int j = threadIdx.x; j < ni; j += NT)
            x[interior_node<P, DIM>(j)] = T(rl[2 * ni + j] + rl[ni + j]);
    }
    wg_barrier();
}

template <class T, int P, int DIM, int CMAX, bool E>
__device__ __attribute__((noinline)) void gamma_cycle(const Hier<T>& H, int b, const T* r, T* x);

// The coarse level's M^{-1} r of a coarse-grid correction: a level the
// hierarchy holds a dense matrix for is applied here, in the caller, which
// saves that level's out-of-line call and the registers it saves and
// restores (27 visits per fine cycle at gamma = 3); others recurse.
template <class T, int P, int DIM, int CMAX, bool E>
__device__ __attribute__((always_inline)) inline void coarse_correction(const Hier<T>& H, int b,
                                                                         const T* r, T* x)
{
    using S = Shape<P, DIM>;
    if constexpr (P <= CMAX && (P >= collapse_lo(DIM) || (E && P >= 4))) {
        if (H.Cc[S::LEV]) {
            constexpr int ni = ipow(P - 1, DIM);
            collapsed_solve<T, P, DIM>(H.Cc[S::LEV] + (long long)b * ni * ni, r, x);
            return;
        }
    }
    gamma_cycle<T, P, DIM, CMAX, E>(H, b, r, x);
}

// x = M_l^{-1} r (Alg. 2).  Readings: pre-smoothing m steps per axis in axis
// order, then gamma passes of {coarse correction of the current iterate,
// m post-smoothing steps per axis in reverse axis order}; level 0 (p = 2,
// one interior node) is solved exactly.  Levels of degree <= CMAX that the
// hierarchy holds a dense matrix for are applied as that matrix.
template <class T, int P, int DIM, int CMAX = collapse_p(DIM), bool E = false>
__device__ __attribute__((noinline)) void gamma_cycle(const Hier<T>& H, int b, const T* r, T* x)
{
    using S = Shape<P, DIM>;
    const LevelData<T>& L = lvl<T, P, DIM>(H);
    // (also the coarsest level of K x K elements, degree 2K: its exact inverse)
    if constexpr (P <= CMAX && (P >= collapse_lo(DIM) || (E && P >= 4))) {
        if (H.Cc[S::LEV]) {
            constexpr int ni = ipow(P - 1, DIM);
            collapsed_solve<T, P, DIM>(H.Cc[S::LEV] + (long long)b * ni * ni, r, x);
            return;
        }
    }
    if constexpr (P == 2) {
        // one interior node: M_0^{-1} = A_0^{-1} is a division, done in FP64
        // whatever the cycle's type (one product with the FP64 1 / A_0)
        constexpr int c = DIM == 2 ? 4 : 13;
        const double ia = H.cinv64[b];
        const auto xg = gmem(x);
        const auto rg = gmem(r);
        for (int q = threadIdx.x; q < S::N; q += NT) xg[q] = q == c ? T((double)rg[c] * ia) : T(0);
        wg_barrier();
    } else {
        using C = Shape<P / 2, DIM>;
        const LevelData<T>& Lc = lvl<T, P / 2, DIM>(H);
        T* rc = Lc.R + (long long)b * C::N;
        T* xc = Lc.X + (long long)b * C::N;
        T* tmp = L.Tm + (long long)b * S::N;
        T* w1 = H.W1 + (long long)b * H.w1;
        T* w2 = H.W2 ? H.W2 + (long long)b * H.w2 : nullptr;
        if (wave_lines<P>() && H.m > 0) {
            // the first smoothing step assigns every interior node
            const auto xg = gmem(x);
            for (int q = threadIdx.x; q < S::N; q += NT)
                if (is_boundary<P, DIM>(q)) xg[q] = T(0);
        } else {
            wg_zero(x, S::N);
        }
        wg_barrier();
        bool zero = true;
        for (int dir = 0; dir < DIM; ++dir)
            for (int s = 0; s < H.m; ++s) {
                smooth_step<T, P, DIM, E>(H, b, dir, r, x, zero);
                zero = false;
            }
        for (int g = 0; g < H.gamma; ++g) {
            if constexpr (E)
                apply_elements_level<T, P, DIM, true>(H.K, L.G + (long long)b * S::NC * L.ng, L.D,
                                                      L.DT, L.TR + (long long)b * DIM * L.ng,
                                                      L.EX ? L.EX + (long long)b * L.ng : nullptr,
                                                      x, r, tmp);
            else
                apply_level<T, P, DIM, true>(L.G + (long long)b * S::NC * S::N, L.D, L.DT,
                                             L.TR + (long long)b * DIM * S::N, x, r, tmp);
            restrict_level<T, P, DIM>(tmp, rc, L.JR, L.JT, w1, w2);
            coarse_correction<T, P / 2, DIM, CMAX, E>(H, b, rc, xc);
            prolong_level<T, P, DIM>(xc, x, L.J, L.JT, w1, w2);
            for (int dir = DIM - 1; dir >= 0; --dir)
                for (int s = 0; s < H.m; ++s) smooth_step<T, P, DIM, E>(H, b, dir, r, x, false);
        }
    }
}

}  // namespace pmg

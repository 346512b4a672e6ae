// pmg_setup.hip -- setup kernels (geometry, line tridiagonals and their
// cyclic-reduction factors), Dirichlet lifting, line-coefficient export.
//
// Every kernel of the library runs one problem of the batch per workgroup
// (grid = B, block = NT threads) and calls the device building blocks of
// pmg_device.hpp.  Setup kernels run in FP64.
#include <cmath>

#include "pmg_dispatch.hpp"

namespace pmg {

// ================================================================== setup

// Geometry of the mapped element (eq. DiscreteSpace, eq. discreteBilinear):
// isoparametric Jacobian dx_c/dxi_a = D applied along axis a to the nodal
// coordinates, phi = rho x rho (x rho) * det J, G_ab = phi * sum_c
// (dxi_a/dx_c)(dxi_b/dx_c), mass = phi.
template <int P, int DIM>
__global__ void __launch_bounds__(NT) k_geom(const double* __restrict__ coords,
                                             const double* __restrict__ rho,
                                             const double* __restrict__ D_,
                                             const double* __restrict__ DT_,
                                             double* __restrict__ G, float* __restrict__ G32,
                                             double* __restrict__ mass, double* __restrict__ X64,
                                             double* __restrict__ detmin, const int* slots,
                                             int* pivot)
{
    using S = Shape<P, DIM>;
    constexpr int n1 = S::n1, N = S::N, NC = S::NC;
    __shared__ double red[NT];
    const long long b = slots ? slots[blockIdx.x] : blockIdx.x;
    if (pivot && threadIdx.x == 0) pivot[b] = 0;
    const auto X = gmem(coords + b * DIM * N);
    const auto D = gmem(D_);
    const auto DT = gmem(DT_);
    const auto Gb = gmem(G + b * NC * N);
    const auto G32b = G32 ? gmem(G32 + b * NC * N) : nullptr;
    const auto massb = mass ? gmem(mass + b * N) : nullptr;
    const auto Xo = gmem(X64 + b * DIM * N);
    double dmin = INFINITY;
    // everything after the Jacobian is pointwise: Jm[comp][a] = dx_comp/dxi_a at node q
    auto point = [&](int q, const int (&c)[3], const double (&Jm)[3][3]) {
        double det, inv[3][3];
        if (DIM == 2) {
            det = Jm[0][0] * Jm[1][1] - Jm[0][1] * Jm[1][0];
            double id = 1.0 / det;
            inv[0][0] = Jm[1][1] * id;
            inv[0][1] = -Jm[0][1] * id;
            inv[1][0] = -Jm[1][0] * id;
            inv[1][1] = Jm[0][0] * id;
        } else {
            // cofactors: inv[a][comp] = cof[comp][a] / det
            double c00 = Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1];
            double c01 = Jm[1][2] * Jm[2][0] - Jm[1][0] * Jm[2][2];
            double c02 = Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0];
            det = Jm[0][0] * c00 + Jm[0][1] * c01 + Jm[0][2] * c02;
            double id = 1.0 / det;
            inv[0][0] = c00 * id;
            inv[1][0] = c01 * id;
            inv[2][0] = c02 * id;
            inv[0][1] = (Jm[0][2] * Jm[2][1] - Jm[0][1] * Jm[2][2]) * id;
            inv[1][1] = (Jm[0][0] * Jm[2][2] - Jm[0][2] * Jm[2][0]) * id;
            inv[2][1] = (Jm[0][1] * Jm[2][0] - Jm[0][0] * Jm[2][1]) * id;
            inv[0][2] = (Jm[0][1] * Jm[1][2] - Jm[0][2] * Jm[1][1]) * id;
            inv[1][2] = (Jm[0][2] * Jm[1][0] - Jm[0][0] * Jm[1][2]) * id;
            inv[2][2] = (Jm[0][0] * Jm[1][1] - Jm[0][1] * Jm[1][0]) * id;
        }
        dmin = fmin(dmin, det);
        double w = rho[c[0]] * rho[c[1]] * (DIM == 3 ? rho[c[2]] : 1.0);
        double phi = w * det;
        for (int a = 0; a < DIM; ++a)
            for (int bb = a; bb < DIM; ++bb) {
                double s = 0.0;
                for (int comp = 0; comp < DIM; ++comp) s += inv[a][comp] * inv[bb][comp];
                int gi = gidx(DIM, a, bb);
                Gb[gi * N + q] = phi * s;
                if (G32b) G32b[gi * N + q] = (float)(phi * s);
            }
        if (massb) massb[q] = phi;
        for (int comp = 0; comp < DIM; ++comp) Xo[comp * N + q] = X[comp * N + q];
    };
    // Jacobian by plain dot products (every node, or the first row and column)
    auto valu = [&](int q) {
        int c[3] = {q % n1, (q / n1) % n1, DIM == 3 ? q / (n1 * n1) : 0};
        double Jm[3][3] = {};
        for (int comp = 0; comp < DIM; ++comp) {
            const auto Xc = X + comp * N;
            for (int a = 0; a < DIM; ++a) {
                const int st = a == 0 ? 1 : (a == 1 ? n1 : n1 * n1);
                const auto xr = Xc + (q - c[a] * st);
                double s = 0.0;
                if (a == 0)
                    for (int k = 0; k < n1; ++k) s += DT[k * n1 + c[0]] * xr[k];
                else
                    for (int k = 0; k < n1; ++k) s += D[c[a] * n1 + k] * xr[k * st];
                Jm[comp][a] = s;
            }
        }
        point(q, c, Jm);
    };
    if constexpr (DIM == 2 && P >= MFMA_MIN_P) {
        // the four derivatives x D^T, D x, y D^T, D y on matrix-core tiles
        // over rows and columns 1..P; row 0 and column 0 on the vector units
        using V4 = Mfma<double>::v4;
        constexpr int NB = P / 16;
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const int lr = lane & 15, kq = lane >> 4;
        for (int t = wave; t < NB * NB; t += NT / 64) {
            const int r0 = 1 + (t / NB) * 16, c0 = 1 + (t % NB) * 16;
            V4 xr[1][1] = {{V4{0, 0, 0, 0}}}, xs[1][1] = {{V4{0, 0, 0, 0}}};
            V4 yr[1][1] = {{V4{0, 0, 0, 0}}}, ys[1][1] = {{V4{0, 0, 0, 0}}};
            mfma_blocks<double, n1, n1, n1, n1, n1, 1, 1>(X + (r0 + lr) * n1 + kq, DT + kq * n1 + c0 + lr,
                                                          D + (r0 + lr) * n1 + kq, X + kq * n1 + c0 + lr,
                                                          xr, xs);
            mfma_blocks<double, n1, n1, n1, n1, n1, 1, 1>(X + N + (r0 + lr) * n1 + kq,
                                                          DT + kq * n1 + c0 + lr, D + (r0 + lr) * n1 + kq,
                                                          X + N + kq * n1 + c0 + lr, yr, ys);
            const int i = c0 + lr;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int j = r0 + Mfma<double>::row(lane, v);
                const int c[3] = {i, j, 0};
                const double Jm[3][3] = {{xr[0][0][v], xs[0][0][v], 0.0},
                                         {yr[0][0][v], ys[0][0][v], 0.0},
                                         {0.0, 0.0, 0.0}};
                point(j * n1 + i, c, Jm);
            }
        }
        for (int e = threadIdx.x; e < 2 * P + 1; e += NT) valu(e <= P ? e : (e - P) * n1);
    } else {
        for (int q = threadIdx.x; q < N; q += NT) valu(q);
    }
    double m = wg_min(dmin, red);
    if (threadIdx.x == 0) detmin[b] = m;
}

// Entry of the bilinear finite-element stiffness on the quadrilaterals of
// neighbouring GLL nodes (FEM line preconditioners, Sec. 3.1): sum over the
// elements having both nodes as corners of the 2x2-Gauss integral of
// grad(phi_a).grad(phi_b) on the element's bilinear map.
template <int P>
__device__ double fem_entry_2d(const double* __restrict__ X, int i, int j, int i2, int j2)
{
    constexpr int n1 = P + 1, N = n1 * n1;
    const double h = 0.5 / sqrt(3.0);
    const double gq[2] = {0.5 - h, 0.5 + h};
    double s = 0.0;
    for (int ex = (i > i2 ? i : i2) - 1; ex <= (i < i2 ? i : i2); ++ex)
        for (int ey = (j > j2 ? j : j2) - 1; ey <= (j < j2 ? j : j2); ++ey) {
            if (ex < 0 || ey < 0 || ex >= P || ey >= P) continue;
            double cx[4], cy[4];
            for (int v = 0; v < 4; ++v) {
                int q = (ex + (v & 1)) + n1 * (ey + (v >> 1));
                cx[v] = X[q];
                cy[v] = X[N + q];
            }
            const int va = (i - ex) + 2 * (j - ey), vb = (i2 - ex) + 2 * (j2 - ey);
            for (int gx = 0; gx < 2; ++gx)
                for (int gy = 0; gy < 2; ++gy) {
                    const double u = gq[gx], v = gq[gy];
                    // d/du and d/dv of the corner functions (1-u)(1-v), u(1-v), (1-u)v, uv
                    const double du[4] = {-(1 - v), 1 - v, -v, v};
                    const double dv[4] = {-(1 - u), -u, 1 - u, u};
                    double xu = 0, xv = 0, yu = 0, yv = 0;
                    for (int c = 0; c < 4; ++c) {
                        xu += du[c] * cx[c];
                        xv += dv[c] * cx[c];
                        yu += du[c] * cy[c];
                        yv += dv[c] * cy[c];
                    }
                    const double det = xu * yv - xv * yu;
                    const double ax = (yv * du[va] - yu * dv[va]) / det;
                    const double ay = (-xv * du[va] + xu * dv[va]) / det;
                    const double bx = (yv * du[vb] - yu * dv[vb]) / det;
                    const double by = (-xv * du[vb] + xu * dv[vb]) / det;
                    s += 0.25 * fabs(det) * (ax * bx + ay * by);
                }
        }
    return s;
}

// 3-D analogue: trilinear elements on the hexahedra of neighbouring GLL
// nodes, 2x2x2 Gauss rule on each element's trilinear map; nodes c and c2
// differ by at most one position per axis.
template <int P>
__device__ double fem_entry_3d(const double* __restrict__ X, const int* c, const int* c2)
{
    constexpr int n1 = P + 1, N = n1 * n1 * n1;
    const double h = 0.5 / sqrt(3.0);
    const double gq[2] = {0.5 - h, 0.5 + h};
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = (c[a] > c2[a] ? c[a] : c2[a]) - 1;
        hi[a] = c[a] < c2[a] ? c[a] : c2[a];
    }
    double s = 0.0;
    for (int e2 = lo[2]; e2 <= hi[2]; ++e2)
        for (int e1 = lo[1]; e1 <= hi[1]; ++e1)
            for (int e0 = lo[0]; e0 <= hi[0]; ++e0) {
                if (e0 < 0 || e1 < 0 || e2 < 0 || e0 >= P || e1 >= P || e2 >= P) continue;
                double cx[8][3];
                for (int v = 0; v < 8; ++v) {
                    const int q = (e0 + (v & 1)) + n1 * (e1 + ((v >> 1) & 1)) +
                                  n1 * n1 * (e2 + ((v >> 2) & 1));
                    for (int k = 0; k < 3; ++k) cx[v][k] = X[k * N + q];
                }
                const int va = (c[0] - e0) + 2 * (c[1] - e1) + 4 * (c[2] - e2);
                const int vb = (c2[0] - e0) + 2 * (c2[1] - e1) + 4 * (c2[2] - e2);
                for (int gi = 0; gi < 8; ++gi) {
                    const double u[3] = {gq[gi & 1], gq[(gi >> 1) & 1], gq[(gi >> 2) & 1]};
                    // gradient (d/du0, d/du1, d/du2) of the corner function v
                    auto grad = [&](int v, double* g) {
                        double f[3], df[3];
                        for (int k = 0; k < 3; ++k) {
                            const int bit = (v >> k) & 1;
                            f[k] = bit ? u[k] : 1.0 - u[k];
                            df[k] = bit ? 1.0 : -1.0;
                        }
                        g[0] = df[0] * f[1] * f[2];
                        g[1] = f[0] * df[1] * f[2];
                        g[2] = f[0] * f[1] * df[2];
                    };
                    double Jm[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // Jm[comp][ref axis]
                    for (int v = 0; v < 8; ++v) {
                        double g[3];
                        grad(v, g);
                        for (int k = 0; k < 3; ++k)
                            for (int a = 0; a < 3; ++a) Jm[k][a] += cx[v][k] * g[a];
                    }
                    const double c00 = Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1];
                    const double c01 = Jm[1][2] * Jm[2][0] - Jm[1][0] * Jm[2][2];
                    const double c02 = Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0];
                    const double det = Jm[0][0] * c00 + Jm[0][1] * c01 + Jm[0][2] * c02;
                    double inv[3][3];  // inv[a][comp] = d u_a / d x_comp
                    inv[0][0] = c00 / det;
                    inv[1][0] = c01 / det;
                    inv[2][0] = c02 / det;
                    inv[0][1] = (Jm[0][2] * Jm[2][1] - Jm[0][1] * Jm[2][2]) / det;
                    inv[1][1] = (Jm[0][0] * Jm[2][2] - Jm[0][2] * Jm[2][0]) / det;
                    inv[2][1] = (Jm[0][1] * Jm[2][0] - Jm[0][0] * Jm[2][1]) / det;
                    inv[0][2] = (Jm[0][1] * Jm[1][2] - Jm[0][2] * Jm[1][1]) / det;
                    inv[1][2] = (Jm[0][2] * Jm[1][0] - Jm[0][0] * Jm[1][2]) / det;
                    inv[2][2] = (Jm[0][0] * Jm[1][1] - Jm[0][1] * Jm[1][0]) / det;
                    double ga[3], gb[3], pa[3] = {0, 0, 0}, pb[3] = {0, 0, 0};
                    grad(va, ga);
                    grad(vb, gb);
                    for (int k = 0; k < 3; ++k)
                        for (int a = 0; a < 3; ++a) {
                            pa[k] += inv[a][k] * ga[a];
                            pb[k] += inv[a][k] * gb[a];
                        }
                    s += 0.125 * fabs(det) * (pa[0] * pb[0] + pa[1] * pb[1] + pa[2] * pb[2]);
                }
            }
    return s;
}

// All line couplings of interior node c at once for the trilinear FEM
// matrix: out = {a, l_0, u_0, l_1, u_1, l_2, u_2}, the diagonal entry and the
// entries coupling c to c - e_k and c + e_k.  Same element integrals as
// fem_entry_3d, but each element's Gauss-point geometry is computed once for
// the seven entries (the elements are visited in the same order).
template <int P>
__device__ void fem_node_3d(const double* __restrict__ X, const int* c, double* out)
{
    constexpr int n1 = P + 1, N = n1 * n1 * n1;
    const double h = 0.5 / sqrt(3.0);
    const double gq[2] = {0.5 - h, 0.5 + h};
    for (int i = 0; i < 7; ++i) out[i] = 0.0;
    for (int e2 = c[2] - 1; e2 <= c[2]; ++e2)
        for (int e1 = c[1] - 1; e1 <= c[1]; ++e1)
            for (int e0 = c[0] - 1; e0 <= c[0]; ++e0) {
                if (e0 < 0 || e1 < 0 || e2 < 0 || e0 >= P || e1 >= P || e2 >= P) continue;
                double cx[8][3];
                for (int v = 0; v < 8; ++v) {
                    const int q = (e0 + (v & 1)) + n1 * (e1 + ((v >> 1) & 1)) +
                                  n1 * n1 * (e2 + ((v >> 2) & 1));
                    for (int k = 0; k < 3; ++k) cx[v][k] = X[k * N + q];
                }
                const int va = (c[0] - e0) + 2 * (c[1] - e1) + 4 * (c[2] - e2);
                for (int gi = 0; gi < 8; ++gi) {
                    const double u[3] = {gq[gi & 1], gq[(gi >> 1) & 1], gq[(gi >> 2) & 1]};
                    auto grad = [&](int v, double* g) {
                        double f[3], df[3];
                        for (int k = 0; k < 3; ++k) {
                            const int bit = (v >> k) & 1;
                            f[k] = bit ? u[k] : 1.0 - u[k];
                            df[k] = bit ? 1.0 : -1.0;
                        }
                        g[0] = df[0] * f[1] * f[2];
                        g[1] = f[0] * df[1] * f[2];
                        g[2] = f[0] * f[1] * df[2];
                    };
                    double Jm[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // Jm[comp][ref axis]
                    for (int v = 0; v < 8; ++v) {
                        double g[3];
                        grad(v, g);
                        for (int k = 0; k < 3; ++k)
                            for (int a = 0; a < 3; ++a) Jm[k][a] += cx[v][k] * g[a];
                    }
                    const double c00 = Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1];
                    const double c01 = Jm[1][2] * Jm[2][0] - Jm[1][0] * Jm[2][2];
                    const double c02 = Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0];
                    const double det = Jm[0][0] * c00 + Jm[0][1] * c01 + Jm[0][2] * c02;
                    double inv[3][3];  // inv[a][comp] = d u_a / d x_comp
                    inv[0][0] = c00 / det;
                    inv[1][0] = c01 / det;
                    inv[2][0] = c02 / det;
                    inv[0][1] = (Jm[0][2] * Jm[2][1] - Jm[0][1] * Jm[2][2]) / det;
                    inv[1][1] = (Jm[0][0] * Jm[2][2] - Jm[0][2] * Jm[2][0]) / det;
                    inv[2][1] = (Jm[0][1] * Jm[2][0] - Jm[0][0] * Jm[2][1]) / det;
                    inv[0][2] = (Jm[0][1] * Jm[1][2] - Jm[0][2] * Jm[1][1]) / det;
                    inv[1][2] = (Jm[0][2] * Jm[1][0] - Jm[0][0] * Jm[1][2]) / det;
                    inv[2][2] = (Jm[0][0] * Jm[1][1] - Jm[0][1] * Jm[1][0]) / det;
                    const double w = 0.125 * fabs(det);
                    auto phys = [&](int v, double* pg) {
                        double gg[3];
                        grad(v, gg);
                        for (int k = 0; k < 3; ++k) pg[k] = 0.0;
                        for (int k = 0; k < 3; ++k)
                            for (int a = 0; a < 3; ++a) pg[k] += inv[a][k] * gg[a];
                    };
                    double pa[3];
                    phys(va, pa);
                    out[0] += w * (pa[0] * pa[0] + pa[1] * pa[1] + pa[2] * pa[2]);
                    for (int a = 0; a < 3; ++a) {
                        const int bit = (va >> a) & 1;   // 1: c - e_a is a corner, 0: c + e_a
                        double pb[3];
                        phys(va ^ (1 << a), pb);
                        out[1 + 2 * a + (bit ? 0 : 1)] += w * (pa[0] * pb[0] + pa[1] * pb[1] + pa[2] * pb[2]);
                    }
                }
            }
}

// Entry of A_p (eq. discreteBilinear) between node q (multi-index c) and its
// neighbour along axis dir (offset dd = -1, 0 or +1 along that axis), read off
// the tensor-product structure: the G_dd term along the line, plus the
// cross terms weighted by the diagonal entries D[c_b][c_b] of the other axes
// (which vanish at interior GLL nodes up to rounding).
template <int P, int DIM>
__device__ double gll_entry(const double* __restrict__ Gb, const double* __restrict__ D, int q,
                            const int* c, int dir, int dd)
{
    constexpr int n1 = P + 1, N = Shape<P, DIM>::N;
    auto st = [](int a) { return a == 0 ? 1 : (a == 1 ? n1 : n1 * n1); };
    double s = 0.0;
    if (dd == 0) {
        for (int a = 0; a < DIM; ++a) {
            const double* Ga = Gb + gidx(DIM, a, a) * N + (q - c[a] * st(a));
            for (int k = 0; k < n1; ++k) {
                double d = D[k * n1 + c[a]];
                s += d * d * Ga[k * st(a)];
            }
        }
        for (int a = 0; a < DIM; ++a)
            for (int b = 0; b < DIM; ++b)
                if (a != b) s += Gb[gidx(DIM, a, b) * N + q] * D[c[a] * n1 + c[a]] * D[c[b] * n1 + c[b]];
    } else {
        const int cd = c[dir], ce = c[dir] + dd;
        const int q2 = q + dd * st(dir);
        const double* Gd = Gb + gidx(DIM, dir, dir) * N + (q - cd * st(dir));
        for (int k = 0; k < n1; ++k) s += D[k * n1 + cd] * D[k * n1 + ce] * Gd[k * st(dir)];
        for (int b = 0; b < DIM; ++b) {
            if (b == dir) continue;
            const double dbb = D[c[b] * n1 + c[b]];
            s += dbb * (Gb[gidx(DIM, dir, b) * N + q2] * D[ce * n1 + cd] +
                        Gb[gidx(DIM, dir, b) * N + q] * D[cd * n1 + ce]);
        }
    }
    return s;
}

// Entry A[r, c] (composite nodes r = (r0, r1), c = (c0, c1)) of the assembled
// operator of K x K elements of degree P / K (2-D): the one-element
// quadrature formula of eq. discreteBilinear on each element holding both
// nodes (element factors Gb: per element G00, G11, G01 arrays of NE element
// nodes; D the element's derivative matrix), summed in element order; zero
// when no element holds both.
template <int P>
__device__ double elements_entry2d(int K, const double* __restrict__ Gb_, const double* __restrict__ D_,
                                   const int* r, const int* c)
{
    const auto Gb = gmem(Gb_);
    const auto D = gmem(D_);
    const int pe = P / K, ne1 = pe + 1, NE = ne1 * ne1;
    auto lo_of = [&](int I) { return (I % pe == 0 && I > 0) ? I / pe - 1 : min(I / pe, K - 1); };
    auto hi_of = [&](int I) { return min(I / pe, K - 1); };
    const int ex0 = max(lo_of(r[0]), lo_of(c[0])), ex1 = min(hi_of(r[0]), hi_of(c[0]));
    const int ey0 = max(lo_of(r[1]), lo_of(c[1])), ey1 = min(hi_of(r[1]), hi_of(c[1]));
    double v = 0.0;
    for (int ey = ey0; ey <= ey1; ++ey)
        for (int ex = ex0; ex <= ex1; ++ex) {
            const int e = ex + K * ey;
            const int lr[2] = {r[0] - ex * pe, r[1] - ey * pe};
            const int lc[2] = {c[0] - ex * pe, c[1] - ey * pe};
            const auto Ge = Gb + 3LL * NE * e;
            for (int a = 0; a < 2; ++a)
                for (int k = 0; k < ne1; ++k) {
                    int qc[2] = {lr[0], lr[1]};
                    qc[a] = k;
                    const double da = D[k * ne1 + lr[a]];
                    const int q = qc[0] + ne1 * qc[1];
                    for (int bb = 0; bb < 2; ++bb)
                        if (qc[1 - bb] == lc[1 - bb])
                            v += Ge[gidx(2, a, bb) * NE + q] * da * D[qc[bb] * ne1 + lc[bb]];
                }
        }
    return v;
}

// The same in 3-D: K^3 elements, per element the six arrays G00, G11, G22,
// G01, G02, G12 of NE = ne1^3 element nodes.
template <int P>
__device__ double elements_entry3d(int K, const double* __restrict__ Gb_, const double* __restrict__ D_,
                                   const int* r, const int* c)
{
    const auto Gb = gmem(Gb_);
    const auto D = gmem(D_);
    const int pe = P / K, ne1 = pe + 1, NE = ne1 * ne1 * ne1;
    auto lo_of = [&](int I) { return (I % pe == 0 && I > 0) ? I / pe - 1 : min(I / pe, K - 1); };
    auto hi_of = [&](int I) { return min(I / pe, K - 1); };
    int e0[3], e1[3];
    for (int a = 0; a < 3; ++a) {
        e0[a] = max(lo_of(r[a]), lo_of(c[a]));
        e1[a] = min(hi_of(r[a]), hi_of(c[a]));
    }
    double v = 0.0;
    for (int ez = e0[2]; ez <= e1[2]; ++ez)
        for (int ey = e0[1]; ey <= e1[1]; ++ey)
            for (int ex = e0[0]; ex <= e1[0]; ++ex) {
                const int e = ex + K * (ey + K * ez);
                const int eo[3] = {ex * pe, ey * pe, ez * pe};
                int lr[3], lc[3];
                for (int a = 0; a < 3; ++a) {
                    lr[a] = r[a] - eo[a];
                    lc[a] = c[a] - eo[a];
                }
                const auto Ge = Gb + 6LL * NE * e;
                for (int a = 0; a < 3; ++a)
                    for (int k = 0; k < ne1; ++k) {
                        int qc[3] = {lr[0], lr[1], lr[2]};
                        qc[a] = k;
                        const double da = D[k * ne1 + lr[a]];
                        const int q = qc[0] + ne1 * (qc[1] + ne1 * qc[2]);
                        for (int bb = 0; bb < 3; ++bb) {
                            bool match = true;
                            for (int f = 0; f < 3; ++f)
                                if (f != bb && qc[f] != lc[f]) match = false;
                            if (match) v += Ge[gidx(3, a, bb) * NE + q] * da * D[qc[bb] * ne1 + lc[bb]];
                        }
                    }
            }
    return v;
}

// per-problem offset of a level's geometric factors: N nodes, or the
// K^2 (P/K + 1)^2 element nodes of K x K elements
template <int P, int DIM>
__host__ __device__ inline long long geom_nodes(int K)
{
    if (K <= 1) return Shape<P, DIM>::N;
    const long long ne1 = P / K + 1;
    return DIM == 2 ? (long long)K * K * ne1 * ne1 : (long long)K * K * K * ne1 * ne1 * ne1;
}

template <int P, int DIM>
__device__ void line_raw(const double* Gb, const double* Xb, const double* D, int smoother,
                         int dir, int line, int s, double& l, double& a, double& u, int K = 1)
{
    constexpr int n1 = P + 1, n = P - 1;
    int base, st;
    line_base<P, DIM>(dir, line, base, st);
    const int q = base + (s + 1) * st;
    int c[3] = {q % n1, (q / n1) % n1, DIM == 3 ? q / (n1 * n1) : 0};
    if constexpr (DIM == 2) {
        if (K > 1 && smoother != PMG_SMOOTHER_FEM) {
            // GLL rows of the assembled operator of several elements
            int cl[2] = {c[0], c[1]}, cu[2] = {c[0], c[1]};
            cl[dir] -= 1;
            cu[dir] += 1;
            a = elements_entry2d<P>(K, Gb, D, c, c);
            l = s > 0 ? elements_entry2d<P>(K, Gb, D, c, cl) : 0.0;
            u = s < n - 1 ? elements_entry2d<P>(K, Gb, D, c, cu) : 0.0;
            return;
        }
    } else {
        if (K > 1 && smoother != PMG_SMOOTHER_FEM) {
            int cl[3] = {c[0], c[1], c[2]}, cu[3] = {c[0], c[1], c[2]};
            cl[dir] -= 1;
            cu[dir] += 1;
            a = elements_entry3d<P>(K, Gb, D, c, c);
            l = s > 0 ? elements_entry3d<P>(K, Gb, D, c, cl) : 0.0;
            u = s < n - 1 ? elements_entry3d<P>(K, Gb, D, c, cu) : 0.0;
            return;
        }
    }
    if (smoother == PMG_SMOOTHER_FEM && DIM == 2) {
        const int di = dir == 0 ? 1 : 0, dj = dir == 0 ? 0 : 1;
        a = fem_entry_2d<P>(Xb, c[0], c[1], c[0], c[1]);
        l = s > 0 ? fem_entry_2d<P>(Xb, c[0], c[1], c[0] - di, c[1] - dj) : 0.0;
        u = s < n - 1 ? fem_entry_2d<P>(Xb, c[0], c[1], c[0] + di, c[1] + dj) : 0.0;
    } else if (smoother == PMG_SMOOTHER_FEM) {
        int cl[3] = {c[0], c[1], c[2]}, cu[3] = {c[0], c[1], c[2]};
        cl[dir] -= 1;
        cu[dir] += 1;
        a = fem_entry_3d<P>(Xb, c, c);
        l = s > 0 ? fem_entry_3d<P>(Xb, c, cl) : 0.0;
        u = s < n - 1 ? fem_entry_3d<P>(Xb, c, cu) : 0.0;
    } else {
        a = gll_entry<P, DIM>(Gb, D, q, c, dir, 0);
        l = s > 0 ? gll_entry<P, DIM>(Gb, D, q, c, dir, -1) : 0.0;
        u = s < n - 1 ? gll_entry<P, DIM>(Gb, D, q, c, dir, +1) : 0.0;
    }
}

// Line tridiagonals and their cyclic-reduction factors, one thread per line.
// Level-k slots first receive the raw (l, a, u) of the level-k matrix; the
// coarse matrix D - C A^{-1} B of Prop. "line coarse space" (stencil of its
// proof) fills the level-(k+1) slots; then the F slots are turned into
// (1/a, -l/a, -u/a).  For p <= 128 the lines are solved by lane groups and
// keep their level-0 rows raw (their solver builds the operators on the
// fly); all pivots are still checked here.  All in FP64, cast to FP32 when
// requested.
template <int P, int DIM>
__global__ void __launch_bounds__(NT) k_lines(const double* __restrict__ G,
                                              const double* __restrict__ X64,
                                              const double* __restrict__ D, int smoother,
                                              double* cr0, double* cr1, double* cr2, float* f0,
                                              float* f1, float* f2, int* pivot,
                                              double* cinv64, float* cinv32, const int* slots,
                                              double* bd0, double* bd1, double* bd2, float* bf0,
                                              float* bf1, float* bf2, int K)
{
    using S = Shape<P, DIM>;
    constexpr int n = S::n, NL = S::NL, CRW = S::CRW, N = S::N, NC = S::NC;
    const long long b = slots ? slots[blockIdx.x] : blockIdx.x;
    const double* Gb = G + b * NC * geom_nodes<P, DIM>(K);
    const double* Xb = X64 + b * DIM * N;
    int bad = 0;
    auto crp = [&](int dir) { return (dir == 0 ? cr0 : (dir == 1 ? cr1 : cr2)) + b * 3 * CRW * NL; };
    auto idx = [&](int dir, int line, int slot, int w) -> long long {
        const bool lm = wave_lines<P>();   // line-major, raw level 0
        return lm ? ((long long)line * CRW + slot) * 3 + w : (long long)(slot * 3 + w) * NL + line;
    };
    if (bd0) {
        // half-bandwidth-2 line rows of the GLL operator: entries (s, s+k),
        // k = -2..2, of every line of every axis (zero outside the line),
        // then every block-CR level's 2x2 pivots checked by a solve with a
        // right-hand side of ones
        if constexpr (wave_lines<P>()) {
            auto bdp = [&](int dir) { return (dir == 0 ? bd0 : (dir == 1 ? bd1 : bd2)) + b * 5 * n * NL; };
            for (int e = threadIdx.x; e < DIM * NL * n * 5; e += NT) {
                const int dir = e / (NL * n * 5), line = (e / (n * 5)) % NL, sq = (e / 5) % n;
                const int k = e % 5 - 2;
                int base, st;
                line_base<P, DIM>(dir, line, base, st);
                const int q = base + (sq + 1) * st;
                const int c[3] = {q % (P + 1), (q / (P + 1)) % (P + 1), DIM == 3 ? q / ((P + 1) * (P + 1)) : 0};
                double v = 0.0;
                if (sq + k >= 0 && sq + k < n) {
                    if (DIM == 2 && K > 1) {
                        int c2[2] = {c[0], c[1]};
                        c2[dir] += k;
                        v = elements_entry2d<P>(K, Gb, D, c, c2);
                    } else if (K > 1) {
                        int c2[3] = {c[0], c[1], c[2]};
                        c2[dir] += k;
                        v = elements_entry3d<P>(K, Gb, D, c, c2);
                    } else {
                        v = gll_entry<P, DIM>(Gb, D, q, c, dir, k);
                    }
                }
                bdp(dir)[((long long)line * n + sq) * 5 + k + 2] = v;
            }
            wg_barrier();
            constexpr int W = (n + 1) / 2 > 0 ? (n + 1) / 2 : 1;
            constexpr int LPW = 64 / W;
            const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
            const int u = lane % W, sub = lane / W;
            const bool has1 = 2 * u + 1 < n;
            for (int dir = 0; dir < DIM; ++dir) {
                const auto bd = gmem((const double*)bdp(dir));
                for (int line0 = wave * LPW; line0 < NL; line0 += (NT / 64) * LPW) {
                    const int line = line0 + sub;
                    const int lc = line < NL ? line : NL - 1;
                    double e0 = 1.0, e1 = has1 ? 1.0 : 0.0;
                    bcr_wave_solve<double, n, W>(bd + (long long)lc * 5 * n, u, has1, e0, e1);
                    if (line < NL && !(isfinite(e0) && isfinite(e1))) bad = 1;
                }
                float* bf = dir == 0 ? bf0 : (dir == 1 ? bf1 : bf2);
                if (bf) {
                    const auto bfb = gmem(bf + b * 5 * n * NL);
                    for (int e = threadIdx.x; e < NL * 5 * n; e += NT) bfb[e] = (float)bd[e];
                }
            }
        }
    } else {
    // 1. the raw tridiagonals of every line of every axis, one entry per work
    //    item (3-D FEM: one interior node per work item, all axes at once)
    if constexpr (DIM == 3) {
        if (smoother == PMG_SMOOTHER_FEM) {
            for (int e = threadIdx.x; e < n * n * n; e += NT) {
                const int c[3] = {e % n + 1, (e / n) % n + 1, e / (n * n) + 1};
                double v[7];
                fem_node_3d<P>(Xb, c, v);
                for (int dir = 0; dir < 3; ++dir) {
                    const int o1 = dir == 0 ? c[1] : c[0], o2 = dir == 2 ? c[1] : c[2];
                    const int line = (o1 - 1) + n * (o2 - 1), sq = c[dir] - 1;
                    double* cr = crp(dir);
                    cr[idx(dir, line, sq, 0)] = sq > 0 ? v[1 + 2 * dir] : 0.0;
                    cr[idx(dir, line, sq, 1)] = v[0];
                    cr[idx(dir, line, sq, 2)] = sq < n - 1 ? v[2 + 2 * dir] : 0.0;
                }
            }
        }
    }
    for (int e = threadIdx.x; e < DIM * NL * n; e += NT) {
        if (DIM == 3 && smoother == PMG_SMOOTHER_FEM) break;
        const int dir = e / (NL * n), line = (e / n) % NL, sq = e % n;
        double l, a, u;
        line_raw<P, DIM>(Gb, Xb, D, smoother, dir, line, sq, l, a, u, K);
        double* cr = crp(dir);
        cr[idx(dir, line, sq, 0)] = l;
        cr[idx(dir, line, sq, 1)] = a;
        cr[idx(dir, line, sq, 2)] = u;
    }
    wg_barrier();
    if constexpr (wave_lines<P>()) {
        // 2'. lane-group lines keep only their raw rows: the solver builds
        //     every CR level from them.  Every level's pivots are checked by
        //     solving each line with a right-hand side of ones (a zero or
        //     non-finite pivot makes the solution non-finite), and the FP32
        //     copy is of the raw rows alone.
        constexpr int W = (n + 1) / 2 > 0 ? (n + 1) / 2 : 1;   // lanes per line
        constexpr int LPW = 64 / W;
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        const int u = lane % W, sub = lane / W;
        const bool has1 = 2 * u + 1 < n;
        for (int dir = 0; dir < DIM; ++dir) {
            const auto cr = gmem((const double*)crp(dir));
            for (int line0 = wave * LPW; line0 < NL; line0 += (NT / 64) * LPW) {
                const int line = line0 + sub;
                const int lc = line < NL ? line : NL - 1;
                double e0 = 1.0, e1 = has1 ? 1.0 : 0.0;
                cr_wave_solve<double, n, W>(cr + (long long)lc * 3 * CRW, u, has1, e0, e1);
                if (line < NL && !(isfinite(e0) && isfinite(e1))) bad = 1;
            }
            float* cf = dir == 0 ? f0 : (dir == 1 ? f1 : f2);
            if (cf) {
                const auto cfb = gmem(cf + b * 3 * CRW * NL);
                for (int e = threadIdx.x; e < NL * 3 * n; e += NT) {
                    const long long o = (long long)(e / (3 * n)) * 3 * CRW + e % (3 * n);
                    cfb[o] = (float)cr[o];
                }
            }
        }
    } else {
    // 2. cyclic-reduction factors, one line per thread over all axes
    for (int e = threadIdx.x; e < DIM * NL; e += NT) {
        const int dir = e / NL, line = e % NL;
        double* cr = crp(dir);
        float* cf = dir == 0 ? f0 : (dir == 1 ? f1 : f2);
        auto W = [&](int slot, int w) -> double& { return cr[idx(dir, line, slot, w)]; };
        {
            int off = 0, nk = n;
            while (nk > 1) {
                const int nc = nk / 2;
                for (int t = 1; t < nk; t += 2) {
                    const double lc = W(off + t, 0), ac = W(off + t, 1), uc = W(off + t, 2);
                    const double lL = W(off + t - 1, 0), aL = W(off + t - 1, 1), uL = W(off + t - 1, 2);
                    const double lR = W(off + t + 1, 0), aR = W(off + t + 1, 1), uR = W(off + t + 1, 2);
                    const int sc = off + nk + (t - 1) / 2;
                    W(sc, 0) = -lc * lL / aL;
                    W(sc, 1) = ac - lc * uL / aL - uc * lR / aR;
                    W(sc, 2) = -uc * uR / aR;
                }
                for (int t = 0; t < nk; t += 2) {
                    const double a = W(off + t, 1);
                    if (a == 0.0 || !isfinite(a)) bad = 1;
                    // first-axis lines in the wave layout keep level 0 raw:
                    // their solver builds every level's operators on the fly
                    if (off == 0 && wave_lines<P>()) continue;
                    const double ia = 1.0 / a;
                    const double l = W(off + t, 0), u = W(off + t, 2);
                    W(off + t, 0) = ia;
                    W(off + t, 1) = -l * ia;
                    W(off + t, 2) = -u * ia;
                }
                off += nk;
                nk = nc;
            }
            {
                const double a = W(off, 1);
                if (a == 0.0 || !isfinite(a)) bad = 1;
                if (!(off == 0 && wave_lines<P>())) {
                    W(off, 0) = 1.0 / a;
                    W(off, 1) = 0.0;
                    W(off, 2) = 0.0;
                }
            }
            if (cf) {
                float* cfb = cf + b * 3 * CRW * NL;
                for (int slot = 0; slot < CRW; ++slot)
                    for (int w = 0; w < 3; ++w) cfb[idx(dir, line, slot, w)] = (float)W(slot, w);
            }
        }
    }
    }
    }   // tridiagonal line systems
    if (P == 2 && threadIdx.x == 0) {
        // level 0: the exact coarse solve uses A_0 itself (eq. discreteBilinear),
        // whatever line systems the smoother uses
        constexpr int c = DIM == 2 ? 4 : 13;
        const int cc[3] = {1, 1, 1};
        const double a0 = gll_entry<P, DIM>(Gb, D, c, cc, 0, 0);
        if (a0 == 0.0 || !isfinite(a0)) bad = 1;
        cinv64[b] = 1.0 / a0;
        if (cinv32) cinv32[b] = (float)(1.0 / a0);
    }
    if (bad) atomicOr(pivot + b, 1);
}

// Geometry of a level of K x K elements (2-D): per element node, the
// Jacobian of the mapping by the element's derivative matrix on the element
// block of the composite coordinates, then G = rho_i rho_j det J J^{-1}
// J^{-T} (element layout, as in the one-element kernel); per global node,
// the assembled mass (the element weights rho_i rho_j det J of every
// element holding the node, in element order).
template <int P>
__global__ void __launch_bounds__(NT) k_geom_elements(int K, const double* __restrict__ coords,
                                                      const double* __restrict__ rho_,
                                                      const double* __restrict__ D_,
                                                      double* __restrict__ G, float* __restrict__ G32,
                                                      double* __restrict__ mass,
                                                      double* __restrict__ X64,
                                                      double* __restrict__ detmin,
                                                      const int* slots, int* pivot)
{
    constexpr int n1 = P + 1, N = n1 * n1;
    const int pe = P / K, ne1 = pe + 1, NE = ne1 * ne1, NEt = K * K * NE;
    __shared__ double red[NT];
    const long long b = slots ? slots[blockIdx.x] : blockIdx.x;
    if (pivot && threadIdx.x == 0) pivot[b] = 0;
    const auto X = gmem(coords + b * 2 * N);
    const auto D = gmem(D_);
    const auto rho = gmem(rho_);
    const auto Gb = gmem(G + b * 3 * NEt);
    const auto G32b = G32 ? gmem(G32 + b * 3 * NEt) : nullptr;
    const auto Xo = gmem(X64 + b * 2 * N);
    for (int q = threadIdx.x; q < 2 * N; q += NT) Xo[q] = X[q];
    // det J and J at element node (i, j) of element (ex, ey)
    auto jac = [&](int ex, int ey, int i, int j, double (&Jm)[2][2]) {
        const int gx = ex * pe, gy = ey * pe;
        for (int comp = 0; comp < 2; ++comp) {
            const auto Xc = X + comp * N;
            double s0 = 0.0, s1 = 0.0;
            for (int k = 0; k < ne1; ++k) {
                s0 += D[i * ne1 + k] * Xc[(gx + k) + (gy + j) * n1];
                s1 += D[j * ne1 + k] * Xc[(gx + i) + (gy + k) * n1];
            }
            Jm[comp][0] = s0;
            Jm[comp][1] = s1;
        }
        return Jm[0][0] * Jm[1][1] - Jm[0][1] * Jm[1][0];
    };
    double dmin = INFINITY;
    for (int t = threadIdx.x; t < NEt; t += NT) {
        const int e = t / NE, lq = t - e * NE, i = lq % ne1, j = lq / ne1;
        double Jm[2][2];
        const double det = jac(e % K, e / K, i, j, Jm);
        dmin = fmin(dmin, det);
        const double id = 1.0 / det;
        const double inv[2][2] = {{Jm[1][1] * id, -Jm[0][1] * id}, {-Jm[1][0] * id, Jm[0][0] * id}};
        const double phi = rho[i] * rho[j] * det;
        for (int a = 0; a < 2; ++a)
            for (int c = a; c < 2; ++c) {
                const double v = phi * (inv[a][0] * inv[c][0] + inv[a][1] * inv[c][1]);
                const int gi = gidx(2, a, c);
                Gb[(long long)3 * NE * e + gi * NE + lq] = v;
                if (G32b) G32b[(long long)3 * NE * e + gi * NE + lq] = (float)v;
            }
    }
    if (mass) {
        const auto massb = gmem(mass + b * N);
        for (int q = threadIdx.x; q < N; q += NT) {
            const int I = q % n1, J = q / n1;
            const int ex1 = min(I / pe, K - 1), ey1 = min(J / pe, K - 1);
            const int ex0 = (I % pe == 0 && I > 0) ? I / pe - 1 : ex1;
            const int ey0 = (J % pe == 0 && J > 0) ? J / pe - 1 : ey1;
            double m = 0.0;
            for (int ey = ey0; ey <= ey1; ++ey)
                for (int ex = ex0; ex <= ex1; ++ex) {
                    double Jm[2][2];
                    const int i = I - ex * pe, j = J - ey * pe;
                    m += rho[i] * rho[j] * jac(ex, ey, i, j, Jm);
                }
            massb[q] = m;
        }
    }
    const double mn = wg_min(dmin, red);
    if (threadIdx.x == 0) detmin[b] = mn;
}

// Geometry of a level of K^3 elements (3-D): the one-element formulas per
// element node (Jacobian by the element's D on the element block of the
// composite coordinates, adjugate inverse), G in the six-array element layout;
// the assembled mass per global node (the weights of the elements holding it,
// in element order).
template <int P>
__global__ void __launch_bounds__(NT) k_geom_elements3d(int K, const double* __restrict__ coords,
                                                        const double* __restrict__ rho_,
                                                        const double* __restrict__ D_,
                                                        double* __restrict__ G, float* __restrict__ G32,
                                                        double* __restrict__ mass,
                                                        double* __restrict__ X64,
                                                        double* __restrict__ detmin,
                                                        const int* slots, int* pivot)
{
    constexpr int n1 = P + 1, N = n1 * n1 * n1;
    const int pe = P / K, ne1 = pe + 1, NE = ne1 * ne1 * ne1, NEt = K * K * K * NE;
    __shared__ double red[NT];
    const long long b = slots ? slots[blockIdx.x] : blockIdx.x;
    if (pivot && threadIdx.x == 0) pivot[b] = 0;
    const auto X = gmem(coords + b * 3 * N);
    const auto D = gmem(D_);
    const auto rho = gmem(rho_);
    const auto Gb = gmem(G + b * 6 * NEt);
    const auto G32b = G32 ? gmem(G32 + b * 6 * NEt) : nullptr;
    const auto Xo = gmem(X64 + b * 3 * N);
    for (int q = threadIdx.x; q < 3 * N; q += NT) Xo[q] = X[q];
    const int gst[3] = {1, n1, n1 * n1};
    // Jacobian Jm[comp][a] at element node c of the element at offset eo
    auto jac = [&](const int (&eo)[3], const int (&c)[3], double (&Jm)[3][3]) {
        const int g0 = (eo[0] + c[0]) + (eo[1] + c[1]) * n1 + (eo[2] + c[2]) * n1 * n1;
        for (int comp = 0; comp < 3; ++comp) {
            const auto Xc = X + comp * N;
            for (int a = 0; a < 3; ++a) {
                const int gb = g0 - c[a] * gst[a];
                double sum = 0.0;
                for (int k = 0; k < ne1; ++k) sum += D[c[a] * ne1 + k] * Xc[gb + k * gst[a]];
                Jm[comp][a] = sum;
            }
        }
        const double c00 = Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1];
        const double c01 = Jm[1][2] * Jm[2][0] - Jm[1][0] * Jm[2][2];
        const double c02 = Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0];
        return Jm[0][0] * c00 + Jm[0][1] * c01 + Jm[0][2] * c02;
    };
    double dmin = INFINITY;
    for (int t = threadIdx.x; t < NEt; t += NT) {
        const int e = t / NE, lq = t - e * NE;
        const int c[3] = {lq % ne1, (lq / ne1) % ne1, lq / (ne1 * ne1)};
        const int eo[3] = {(e % K) * pe, ((e / K) % K) * pe, (e / (K * K)) * pe};
        double Jm[3][3];
        const double det = jac(eo, c, Jm);
        dmin = fmin(dmin, det);
        const double id = 1.0 / det;
        double inv[3][3];   // inv[a][comp] = d xi_a / d x_comp
        inv[0][0] = (Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1]) * id;
        inv[1][0] = (Jm[1][2] * Jm[2][0] - Jm[1][0] * Jm[2][2]) * id;
        inv[2][0] = (Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0]) * id;
        inv[0][1] = (Jm[0][2] * Jm[2][1] - Jm[0][1] * Jm[2][2]) * id;
        inv[1][1] = (Jm[0][0] * Jm[2][2] - Jm[0][2] * Jm[2][0]) * id;
        inv[2][1] = (Jm[0][1] * Jm[2][0] - Jm[0][0] * Jm[2][1]) * id;
        inv[0][2] = (Jm[0][1] * Jm[1][2] - Jm[0][2] * Jm[1][1]) * id;
        inv[1][2] = (Jm[0][2] * Jm[1][0] - Jm[0][0] * Jm[1][2]) * id;
        inv[2][2] = (Jm[0][0] * Jm[1][1] - Jm[0][1] * Jm[1][0]) * id;
        const double phi = rho[c[0]] * rho[c[1]] * rho[c[2]] * det;
        for (int a = 0; a < 3; ++a)
            for (int bb = a; bb < 3; ++bb) {
                const double v = phi * (inv[a][0] * inv[bb][0] + inv[a][1] * inv[bb][1] +
                                        inv[a][2] * inv[bb][2]);
                const int gi = gidx(3, a, bb);
                Gb[6LL * NE * e + gi * NE + lq] = v;
                if (G32b) G32b[6LL * NE * e + gi * NE + lq] = (float)v;
            }
    }
    if (mass) {
        const auto massb = gmem(mass + b * N);
        for (int q = threadIdx.x; q < N; q += NT) {
            const int I[3] = {q % n1, (q / n1) % n1, q / (n1 * n1)};
            int e0[3], e1[3];
            for (int a = 0; a < 3; ++a) {
                e1[a] = min(I[a] / pe, K - 1);
                e0[a] = (I[a] % pe == 0 && I[a] > 0) ? I[a] / pe - 1 : e1[a];
            }
            double m = 0.0;
            for (int ez = e0[2]; ez <= e1[2]; ++ez)
                for (int ey = e0[1]; ey <= e1[1]; ++ey)
                    for (int ex = e0[0]; ex <= e1[0]; ++ex) {
                        const int eo[3] = {ex * pe, ey * pe, ez * pe};
                        const int c[3] = {I[0] - eo[0], I[1] - eo[1], I[2] - eo[2]};
                        double Jm[3][3];
                        m += rho[c[0]] * rho[c[1]] * rho[c[2]] * jac(eo, c, Jm);
                    }
            massb[q] = m;
        }
    }
    const double mn = wg_min(dmin, red);
    if (threadIdx.x == 0) detmin[b] = mn;
}

// Exact solve on the coarsest level of K x K elements (degree P = 2K, ni =
// (P-1)^2 interior nodes): the interior matrix of the assembled operator,
// entry by entry (the element quadrature sums of eq. discreteBilinear over
// the elements holding both nodes), then its inverse by Gauss-Jordan
// elimination in place (symmetric positive definite: no pivoting; a pivot
// that is not positive flags the problem), stored for collapsed_solve as
// C[i ni + j] = (A^{-1})[j][i].
template <int P, int DIM>
__global__ void __launch_bounds__(NT) k_elements_coarse(int K, const double* __restrict__ G,
                                                        const double* __restrict__ D_,
                                                        double* __restrict__ Cc, const int* slots,
                                                        int* pivot)
{
    constexpr int n = P - 1, ni = DIM == 2 ? n * n : n * n * n;
    const long long b = slots ? slots[blockIdx.x] : blockIdx.x;
    const auto A = gmem(Cc + b * (long long)ni * ni);
    const double* Gb = G + b * (DIM == 2 ? 3LL : 6LL) * geom_nodes<P, DIM>(K);
    for (int t = threadIdx.x; t < ni * ni; t += NT) {
        const int row = t / ni, col = t - row * ni;
        if constexpr (DIM == 2) {
            const int r[2] = {row % n + 1, row / n + 1}, c[2] = {col % n + 1, col / n + 1};
            A[t] = elements_entry2d<P>(K, Gb, D_, r, c);
        } else {
            const int r[3] = {row % n + 1, (row / n) % n + 1, row / (n * n) + 1};
            const int c[3] = {col % n + 1, (col / n) % n + 1, col / (n * n) + 1};
            A[t] = elements_entry3d<P>(K, Gb, D_, r, c);
        }
    }
    wg_barrier();
    bool bad = false;
    for (int k = 0; k < ni; ++k) {
        const double akk = A[(long long)k * ni + k];
        bad = bad || !(akk > 0.0);
        const double pk = 1.0 / akk;
        for (int t = threadIdx.x; t < ni * ni; t += NT) {
            const int i = t / ni, j = t - i * ni;
            if (i != k && j != k) A[t] -= A[(long long)i * ni + k] * A[(long long)k * ni + j] * pk;
        }
        wg_barrier();
        for (int t = threadIdx.x; t < ni; t += NT) {
            if (t != k) {
                A[(long long)k * ni + t] *= pk;
                A[(long long)t * ni + k] *= -pk;
            }
        }
        if (threadIdx.x == 0) A[(long long)k * ni + k] = pk;
        wg_barrier();
    }
    // transpose in place: C[i ni + j] = (A^{-1})[j][i]
    for (int t = threadIdx.x; t < ni * ni; t += NT) {
        const int i = t / ni, j = t - i * ni;
        if (i < j) {
            const double u = A[t], w = A[(long long)j * ni + i];
            A[t] = w;
            A[(long long)j * ni + i] = u;
        }
    }
    if (bad && threadIdx.x == 0) pivot[b] = 1;
    wg_barrier();
}

__global__ void k_setup_finish(const double* __restrict__ detmin, const int* __restrict__ pivot,
                               int l0, int nlev, int B, int n, const int* slots,
                               pmg_info* __restrict__ info, int* sstatus)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int b = slots ? slots[i] : i;
    double m = INFINITY;
    for (int l = l0; l < nlev; ++l) m = fmin(m, detmin[(long long)l * B + b]);
    pmg_info r;
    r.min_detj = m;
    r.iterations = 0;
    r.relres = NAN;
    r.status = !(m > 0.0) ? PMG_EGEOM : (pivot[b] ? PMG_EPIVOT : PMG_OK);
    info[b] = r;
    sstatus[b] = r.status;
}

// ================================================================== RHS

// b = M f - A v on interior nodes, 0 on the boundary (Sec. 2.3)
template <int P, int DIM>
__global__ void __launch_bounds__(NT) k_rhs(const Hier<double>* __restrict__ Hp, const double* __restrict__ f,
                                            const double* __restrict__ g, double* __restrict__ bo,
                                            double* __restrict__ tmp, long long tmp_stride,
                                            const int* slots)
{
    const Hier<double>& H = *Hp;
    using S = Shape<P, DIM>;
    constexpr int N = S::N;
    const long long b = slots ? slots[blockIdx.x] : blockIdx.x;
    const LevelData<double>& L = H.lev[S::LEV];
    double* v = tmp + b * tmp_stride;   // the problem's own scratch
    for (int q = threadIdx.x; q < N; q += NT) v[q] = is_boundary<P, DIM>(q) ? g[b * N + q] : 0.0;
    wg_barrier();
    double* out = bo + b * N;
    apply_any<double, P, DIM, false>(H.K, L.EX ? L.EX + b * L.ng : nullptr, L.G64 + b * S::NC * L.ng,
                                     L.D64, L.DT64, L.TR + b * DIM * L.ng, v, nullptr, out);
    for (int q = threadIdx.x; q < N; q += NT)
        out[q] = is_boundary<P, DIM>(q) ? 0.0 : L.mass[b * N + q] * f[b * N + q] - out[q];
}

template <int P, int DIM>
__global__ void __launch_bounds__(NT) k_lift(const double* __restrict__ w,
                                             const double* __restrict__ g, double* u)
{
    constexpr int N = Shape<P, DIM>::N;
    const long long b = blockIdx.x;
    for (int q = threadIdx.x; q < N; q += NT)
        u[b * N + q] = is_boundary<P, DIM>(q) ? g[b * N + q] : w[b * N + q];
}

template <int P, int DIM>
__global__ void __launch_bounds__(NT) k_line_coefs(const Hier<double>* __restrict__ Hp, int smoother, int dir,
                                                   double* lo, double* di, double* up)
{
    const Hier<double>& H = *Hp;
    using S = Shape<P, DIM>;
    constexpr int n = S::n, NL = S::NL;
    const long long b = blockIdx.x;
    const LevelData<double>& L = H.lev[S::LEV];
    const double* Gb = L.G64 + b * S::NC * L.ng;
    const double* Xb = L.X64 + b * DIM * S::N;
    const long long o = b * (long long)NL * n;
    for (int k = threadIdx.x; k < NL * n; k += NT) {
        int line = k / n, s = k % n;
        double l, a, u;
        line_raw<P, DIM>(Gb, Xb, L.D64, smoother, dir, line, s, l, a, u, H.K);
        lo[o + k] = l;
        di[o + k] = a;
        up[o + k] = u;
    }
}


// ================================================================== serving pools

// Mark the listed slots as fresh solves (their setup status decides).
__global__ void k_pool_start(const int* __restrict__ slots, int n, const int* __restrict__ sstatus,
                             SolveState* __restrict__ st, pmg_info* __restrict__ info)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int b = slots[i];
    SolveState s;
    s.status = sstatus[b] == PMG_OK ? ST_RUNNING : sstatus[b];
    s.it = 0;
    s.j = 0;
    s.phase = PH_INIT;
    s.bn = 0.0;
    s.rz = 0.0;
    st[b] = s;
    info[b].status = s.status;
    info[b].iterations = 0;
    info[b].relres = NAN;
}

__global__ void k_pool_idle(SolveState* __restrict__ st, int B)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    st[b].status = ST_IDLE;
}

// u = w inside, g on the boundary, for one slot; the slot becomes idle.
template <int P, int DIM>
__global__ void __launch_bounds__(NT) k_pool_take(int slot, const double* __restrict__ w,
                                                  const double* __restrict__ g,
                                                  double* __restrict__ u, SolveState* st)
{
    constexpr int N = Shape<P, DIM>::N;
    const long long b = slot;
    for (int q = threadIdx.x; q < N; q += NT)
        u[q] = is_boundary<P, DIM>(q) ? g[b * N + q] : w[b * N + q];
    if (threadIdx.x == 0) st[b].status = ST_IDLE;
}

// The same for n slots at once: workgroup i lifts slot slots[i] into outs[i].
template <int P, int DIM>
__global__ void __launch_bounds__(NT) k_pool_take_many(const int* __restrict__ slots,
                                                       double* const* __restrict__ outs,
                                                       const double* __restrict__ w,
                                                       const double* __restrict__ g, SolveState* st)
{
    constexpr int N = Shape<P, DIM>::N;
    const long long b = slots[blockIdx.x];
    double* u = outs[blockIdx.x];
    for (int q = threadIdx.x; q < N; q += NT)
        u[q] = is_boundary<P, DIM>(q) ? g[b * N + q] : w[b * N + q];
    if (threadIdx.x == 0) st[b].status = ST_IDLE;
}

hipError_t launch_setup(int dim, int p_fine, int nlev, int B, const SetupArgs& a, pmg_info* info,
                        hipStream_t s)
{
    hipError_t e;
    const int nb = a.slots ? a.nslots : B;
    if (nb <= 0) return hipSuccess;
    for (int l = a.l0; l < nlev; ++l) {
        const int p = 2 << l;
        double* mass = (p == p_fine) ? a.mass : nullptr;
        if (a.K > 1 && dim == 2) {
            PMG_DISPATCH_P2D(p, hipLaunchKernelGGL((k_geom_elements<P_>), dim3(nb), dim3(NT), 0, s,
                                                   a.K, a.coords[l], a.rho[l], a.D64[l], a.G64[l],
                                                   a.G32[l], mass, a.X64[l],
                                                   a.detmin + (long long)l * B, a.slots,
                                                   l == a.l0 ? a.pivot : nullptr));
        } else if (a.K > 1) {
            PMG_DISPATCH_P3D(p, hipLaunchKernelGGL((k_geom_elements3d<P_>), dim3(nb), dim3(NT), 0, s,
                                                   a.K, a.coords[l], a.rho[l], a.D64[l], a.G64[l],
                                                   a.G32[l], mass, a.X64[l],
                                                   a.detmin + (long long)l * B, a.slots,
                                                   l == a.l0 ? a.pivot : nullptr));
        } else {
            PMG_DISPATCH_P(dim, p, hipLaunchKernelGGL((k_geom<P_, D_>), dim3(nb), dim3(NT), 0, s,
                                                       a.coords[l], a.rho[l], a.D64[l], a.DT64[l],
                                                       a.G64[l], a.G32[l], mass, a.X64[l],
                                                       a.detmin + (long long)l * B, a.slots,
                                                       l == 0 ? a.pivot : nullptr));
        }
        if ((e = last()) != hipSuccess) return e;
        PMG_DISPATCH_P(dim, p, hipLaunchKernelGGL((k_lines<P_, D_>), dim3(nb), dim3(NT), 0, s,
                                                   a.G64[l], a.X64[l], a.D64[l], a.smoother,
                                                   a.cr64[l][0], a.cr64[l][1], a.cr64[l][2],
                                                   a.cr32[l][0], a.cr32[l][1], a.cr32[l][2],
                                                   a.pivot, a.cinv64, a.cinv32, a.slots,
                                                   a.bd64[l][0], a.bd64[l][1], a.bd64[l][2],
                                                   a.bd32[l][0], a.bd32[l][1], a.bd32[l][2], a.K));
        if ((e = last()) != hipSuccess) return e;
    }
    if (a.K > 1) {
        // the coarsest level's exact inverse (degree 2K), after its geometry
        const int p0 = 2 << a.l0;
        switch (dim * 100 + p0) {
#define PMG_COARSE(DM, PC)                                                                      \
    case DM * 100 + PC:                                                                         \
        hipLaunchKernelGGL((k_elements_coarse<PC, DM>), dim3(nb), dim3(NT), 0, s, a.K,          \
                           a.G64[a.l0], a.D64[a.l0], a.Cc0, a.slots, a.pivot);                  \
        break;
            PMG_COARSE(2, 4)
            PMG_COARSE(2, 8)
            PMG_COARSE(2, 16)
            PMG_COARSE(3, 4)
            PMG_COARSE(3, 8)
#undef PMG_COARSE
        default: return hipErrorInvalidValue;
        }
        if ((e = last()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_setup_finish, dim3((nb + 255) / 256), dim3(256), 0, s, a.detmin, a.pivot,
                       a.l0, nlev, B, nb, a.slots, info, a.sstatus);
    return last();
}

hipError_t launch_rhs(int dim, int p, int B, const Hier<double>* H64, const double* f,
                      const double* g, double* b, double* tmp, long long tmp_stride, hipStream_t s,
                      const int* slots, int nslots)
{
    const int nb = slots ? nslots : B;
    if (nb <= 0) return hipSuccess;
    PMG_DISPATCH_P(dim, p, hipLaunchKernelGGL((k_rhs<P_, D_>), dim3(nb), dim3(NT), 0, s, H64, f,
                                               g, b, tmp, tmp_stride, slots));
    return last();
}

hipError_t launch_lift(int dim, int p, int B, const double* w, const double* g, double* u,
                       hipStream_t s)
{
    PMG_DISPATCH_P(dim, p, hipLaunchKernelGGL((k_lift<P_, D_>), dim3(B), dim3(NT), 0, s, w, g, u));
    return last();
}

hipError_t launch_line_coefs(int dim, int p, int B, const Hier<double>* H64, int smoother, int dir,
                             double* lo, double* di, double* up, hipStream_t s)
{
    PMG_DISPATCH_P(dim, p, hipLaunchKernelGGL((k_line_coefs<P_, D_>), dim3(B), dim3(NT), 0, s,
                                               H64, smoother, dir, lo, di, up));
    return last();
}

hipError_t launch_pool_start(const int* slots, int n, const int* sstatus, SolveState* st,
                             pmg_info* info, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pool_start, dim3((n + 255) / 256), dim3(256), 0, s, slots, n, sstatus, st, info);
    return last();
}

hipError_t launch_pool_idle(SolveState* st, int B, hipStream_t s)
{
    hipLaunchKernelGGL(k_pool_idle, dim3((B + 255) / 256), dim3(256), 0, s, st, B);
    return last();
}

hipError_t launch_pool_take(int dim, int p, int slot, const double* w, const double* g, double* u,
                            SolveState* st, hipStream_t s)
{
    PMG_DISPATCH_P(dim, p, hipLaunchKernelGGL((k_pool_take<P_, D_>), dim3(1), dim3(NT), 0, s, slot,
                                               w, g, u, st));
    return last();
}

// Workgroup i performs copy job i.
__global__ void __launch_bounds__(NT) k_copy_jobs(const CopyJob* __restrict__ jobs)
{
    const CopyJob j = jobs[blockIdx.x];
    const auto src = gmem(j.src);
    const auto dst = gmem(j.dst);
    for (long long q = threadIdx.x; q < j.n; q += NT) dst[q] = src[q];
}

hipError_t launch_copy_jobs(int n, const CopyJob* jobs, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_jobs, dim3(n), dim3(NT), 0, s, jobs);
    return last();
}

hipError_t launch_pool_take_many(int dim, int p, int n, const int* slots, double* const* outs,
                                 const double* w, const double* g, SolveState* st, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    PMG_DISPATCH_P(dim, p, hipLaunchKernelGGL((k_pool_take_many<P_, D_>), dim3(n), dim3(NT), 0, s,
                                               slots, outs, w, g, st));
    return last();
}

}  // namespace pmg

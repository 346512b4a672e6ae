/*
 * pmg_oracle.h -- plain, slow, FP64 CPU oracle for the p-multigrid gamma-cycle
 * with cyclic-reduction line smoothers of Lucero Lorca, Rosenberg, Jankov,
 * McCoid and Gander, "On an efficient line smoother for the p-multigrid
 * gamma-cycle" (arXiv 2504.10710).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library.
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no code, header, table or helper with the GPU
 * path, and the GPU path never calls it.
 *
 * Every routine follows a definition of the paper in the paper's order and
 * notation, with no blocking, fusion or reordering beyond what the
 * definition states.  Readings of passages that are silent, ambiguous or
 * garbled are stated where they are used.
 *
 * Conventions
 *   - Node (i0,i1[,i2]) of a level of degree p has index
 *     i0 + (p+1)*i1 (+ (p+1)^2*i2): lexicographic, first axis fastest
 *     (Sec. 3.1, Fig. 4 node ordering).
 *   - Vectors are full node arrays; boundary entries of residuals and
 *     corrections are zero (Dirichlet elimination, Sec. 2.3).
 *   - Levels are numbered 0 (coarsest) .. nlev-1 (finest), as in Sec. 3.3.
 *   - Dense matrices are row-major.
 */
#ifndef PMG_ORACLE_H
#define PMG_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* ---- one-dimensional GLL building blocks (Sec. 2.2) ---- */

/* GLL nodes xi[0..p] and weights rho[0..p] of order p (Def. GLL quadrature
 * rule).  Returns 0, or -1 if p < 1 or Newton fails to converge. */
int or_gll(int p, double* xi, double* rho);

/* Legendre polynomial L_p and its derivative at x (three-term recurrence). */
void or_legendre(int p, double x, double* L, double* dL);

/* D[i*(p+1)+j] = pi_j'(xi_i), derivative of the j-th Lagrange basis
 * polynomial of Def. GLL interpolation basis at node i. */
void or_deriv(int p, const double* xi, double* D);

/* J[i*(pc+1)+j] = pi^c_j(xf_i): coarse basis j evaluated at fine node i
 * (the 1-D prolongation of Sec. 3.3). */
void or_interp(int pc, const double* xic, int nf, const double* xf, double* J);

/* ---- line solvers (Sec. 3.2) ---- */

/* Tridiagonal M with sub-diagonal l[i] (couples i to i-1), diagonal a[i]
 * and super-diagonal u[i] (couples i to i+1), i = 0..n-1; l[0] and u[n-1]
 * are ignored.  Solves M y = g by the direct multigrid of Thm. "Two-level
 * direct solver" applied recursively (Cor. "Direct multigrid solver").
 * Returns 0, or -1 on a zero pivot. */
int or_cr_solve(int n, const double* l, const double* a, const double* u,
                const double* g, double* y);

/* Same matrix, classical Thomas elimination (pin only). */
int or_thomas(int n, const double* l, const double* a, const double* u,
              const double* g, double* y);

/* Dense LU with partial pivoting: solves A y = g in place (A n x n
 * row-major is overwritten, g is overwritten by y).  Pin only. */
int or_dense_solve(int n, double* A, double* g);

/* One level of the two-level solver (Alg. 1 with the operators of
 * Thm. "Two-level direct solver"), exposed for pins: returns the coarse
 * matrix M0 = D - C A^{-1} B of Prop. "line coarse space" as a
 * tridiagonal (l0, a0, u0) of size n/2 (integer division). */
void or_cr_coarse(int n, const double* l, const double* a, const double* u,
                  double* l0, double* a0, double* u0);

/* Block-tridiagonal M (Def. block-tridiagonal matrix) of nb blocks of size
 * m x m: Lb, Ab, Ub hold nb row-major m x m blocks each (Lb[0] and Ub[nb-1]
 * are ignored).  Solves M y = g by the direct multigrid of Thm. "Two-level
 * direct solver" with block operators (S^{-1} = blockdiag(A_F^{-1}), P with
 * F rows -A_F^{-1}(L_F, U_F), R = P^T, M0 = D - C A^{-1} B as in the proof
 * of Prop. "line coarse space"), applied recursively; one block is a dense
 * solve.  g and y hold nb*m values.  Returns 0, or -1 on a singular block. */
int or_bcr_solve(int nb, int m, const double* Lb, const double* Ab, const double* Ub,
                 const double* g, double* y);

/* One level of the block solver, exposed for pins: the coarse blocks of
 * M0 = D - C A^{-1} B (nb/2 blocks, integer division). */
int or_bcr_coarse(int nb, int m, const double* Lb, const double* Ab, const double* Ub,
                  double* L0, double* A0, double* U0);

/* ---- the hierarchy: discretisation, smoother, gamma-cycle ---- */

/* Line systems of the smoother (Def. line preconditioners). */
#define OR_SMOOTHER_GLL 0       /* [A_l]^(1) on the line: tridiagonal, scalar CR */
#define OR_SMOOTHER_FEM 1       /* bilinear / trilinear FEM matrix on the GLL mesh */
#define OR_SMOOTHER_GLL_BAND2 2 /* [A_l]^(2) on the line: 2x2-block tridiagonal, block CR */
#define OR_SMOOTHER_GLL_FULL 3  /* the whole line block R A_l P (dense LU) */

/* Restriction of Sec. 3.3. */
#define OR_RESTRICT_TRANSPOSE 0 /* R_l = P_l^T */
#define OR_RESTRICT_INTERP 1    /* R_l = interpolation of the fine polynomial at the coarse nodes */

typedef struct or_hier or_hier;

/* dim = 2 or 3; p[0..nlev-1] ascending degrees (p[0] is the coarsest level);
 * coords[l] holds dim*N_l doubles (all first coordinates, then all second,
 * ...), the physical positions of the level-l GLL nodes.  smoother is one
 * of OR_SMOOTHER_*, restriction one of OR_RESTRICT_*.
 * Returns NULL on bad arguments, non-positive Jacobian, or a failed coarse
 * factorisation. */
or_hier* or_hier_create(int dim, int nlev, const int* p,
                        const double* const* coords,
                        int gamma, int m, double alpha, int smoother, int restriction);
void or_hier_destroy(or_hier* h);

/* The same hierarchy on K^dim spectral elements (K per axis; the paper's
 * closing outlook, multi-element hp-multigrid): the reference square (cube)
 * is split into K equal parts per axis, each an element of degree p[l] / K
 * (>= 2) with its own GLL rule; interface nodes are shared (continuous
 * basis), the operator and the mass are assembled from the element ones,
 * and the transfers interpolate element by element.  p[l] is the degree of
 * the level's composite grid (K * element degree; p[l] + 1 nodes per axis)
 * and coords[l] its node positions, so every vector keeps the one-element
 * layout.  K = 1 is or_hier_create. */
or_hier* or_hier_create_elements(int dim, int K, int nlev, const int* p,
                                 const double* const* coords, int gamma, int m, double alpha,
                                 int smoother, int restriction);
/* K of the hierarchy */
int or_elements(const or_hier* h);
/* Element geometric factors of level l of an element hierarchy (K > 1):
 * element e (lexicographic, first axis fastest) at G + e*dim*dim*NE, NE =
 * (p/K + 1)^dim, arrays ordered as in or_geom.  Returns the number of
 * doubles, or -1 for K = 1. */
int or_geom_elements(const or_hier* h, int l, double* G);

/* Number of nodes of level l. */
int or_nodes(const or_hier* h, int l);

/* Geometric factors of level l: G has dim*dim arrays of N doubles
 * (G[(a*dim+b)*N + q]; all zero for an element hierarchy, see
 * or_geom_elements), mass has N doubles (assembled over elements).
 * Returns minimum det J. */
double or_geom(const or_hier* h, int l, double* G, double* mass);

/* y = A_l x restricted to interior rows (boundary rows set to 0).  x is a
 * full node array (its boundary entries are used as given). */
void or_apply(const or_hier* h, int l, const double* x, double* y);

/* y = A_l x on every row, boundary rows included (pins only). */
void or_apply_all(const or_hier* h, int l, const double* x, double* y);

/* Entry A_l[row, col] straight from the quadrature sum of eq.
 * discreteBilinear (node indices). */
double or_entry(const or_hier* h, int l, int row, int col);

/* Entry A~_l[row, col] of the bilinear (2-D) or trilinear (3-D)
 * finite-element stiffness on the GLL node mesh (FEM line preconditioners,
 * Sec. 3.1). */
double or_fem_entry(const or_hier* h, int l, int row, int col);

/* Dense interior matrix of level l (n_int x n_int, interior nodes in
 * lexicographic order); n_int returned.  Pass A == NULL to get the size. */
int or_dense_interior(const or_hier* h, int l, double* A);

/* Dirichlet lifting on the finest level (Sec. 2.3):
 * b = M f - A v on the interior, 0 on the boundary, where v is g on the
 * boundary nodes and 0 inside. */
void or_rhs(const or_hier* h, const double* f, const double* g, double* b);

/* rc = R_l rf (level l -> l-1), R_l = P_l^T or the interpolation of the
 * fine polynomial at the coarse nodes (the hierarchy's restriction mode);
 * coarse boundary set to 0. */
void or_restrict(const or_hier* h, int l, const double* rf, double* rc);
/* xf += P_l ec (level l-1 -> l). */
void or_prolong_add(const or_hier* h, int l, const double* ec, double* xf);

/* Tridiagonals of the line systems of level l along axis dir:
 * (p-1)^(dim-1) lines, each of n = p-1 interior unknowns, stored line after
 * line; lines are ordered by the remaining interior indices, lexicographic.
 * Arrays have (p-1)^dim entries. */
void or_line_coefs(const or_hier* h, int l, int dir,
                   double* lo, double* di, double* up);

/* Banded line systems of the OR_SMOOTHER_GLL_BAND2 smoother: for every line
 * (ordered as in or_line_coefs) and position s = 0..n-1, the entries
 * [A_l]_{s, s+k} for k = -2..2 (zero outside the line), 5 per position:
 * band[(line*n + s)*5 + k + 2].  Returns -1 if the hierarchy has another
 * smoother. */
int or_line_band(const or_hier* h, int l, int dir, double* band);

/* z = B_{l,dir}^{-1} r (block-Jacobi over lines, each line by or_cr_solve,
 * or_bcr_solve or a dense solve, by smoother); boundary entries of z are 0. */
int or_line_solve(const or_hier* h, int l, int dir, const double* r, double* z);

/* One smoothing step x <- x + alpha B_{l,dir}^{-1} (r - A_l x). */
int or_smooth(const or_hier* h, int l, int dir, const double* r, double* x);

/* y = M_l^{-1} r, the gamma-cycle of Alg. 2. */
int or_cycle(const or_hier* h, int l, const double* r, double* y);

/* Outer solvers on the finest level, zero initial guess, relative residual
 * tolerance rtol on ||b - A x||_2 / ||b||_2.  hist (may be NULL) receives
 * up to maxit+1 relative residual estimates.  Return 0 converged,
 * 1 not converged, -1 breakdown. */
int or_fgmres(const or_hier* h, const double* b, double* x, double rtol,
              int maxit, int restart, double* hist, int* iters);
int or_pcg(const or_hier* h, const double* b, double* x, double rtol,
           int maxit, double* hist, int* iters);
int or_fcg(const or_hier* h, const double* b, double* x, double rtol,
           int maxit, double* hist, int* iters);

/* Level visit counters of the last or_cycle / outer solve (pins of the
 * cost proposition): visits[l] = number of times level l was entered. */
void or_visits(const or_hier* h, long long* visits);
void or_reset_visits(or_hier* h);

#ifdef __cplusplus
}
#endif
#endif

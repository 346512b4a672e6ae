/*
 * pmg.h -- C ABI of libpmg, an MI355X (gfx950) implementation of the
 * p-multigrid gamma-cycle with cyclic-reduction line smoothers of
 * Lucero Lorca, Rosenberg, Jankov, McCoid and Gander, "On an efficient line
 * smoother for the p-multigrid gamma-cycle" (arXiv 2504.10710), used as the
 * preconditioner of an outer Krylov solve of the GLL spectral Poisson
 * problem on one mapped element.
 *
 * Conventions shared by every call
 *   - Batches.  A handle describes B independent problems of one shape
 *     (dimension, finest degree, hierarchy).  Every device array holds the B
 *     problems back to back, problem b at offset b * (per-problem size).
 *   - Nodes.  Level l has degree p_l = p_coarse * 2^l (p_coarse = 2), n1 =
 *     p_l + 1 nodes per axis and N_l = n1^dim nodes; node (i0, i1[, i2]) has
 *     index i0 + n1*i1 (+ n1^2*i2), first axis fastest (lexicographic order of
 *     Sec. 3.1).  Vectors are full node arrays; residuals and corrections
 *     carry zeros on boundary nodes (Dirichlet elimination, Sec. 2.3).
 *   - Memory.  The caller owns all device memory and streams.  The library
 *     never allocates device memory: pmg_workspace_bytes() reports the size
 *     of the one workspace the caller passes to pmg_setup(); host-side
 *     handles are the only thing the library allocates (freed by
 *     pmg_destroy()).
 *   - Streams.  Device work is enqueued asynchronously on the given stream
 *     (NULL = default stream); no call synchronises unless documented.
 *   - Errors.  Every call returns PMG_OK (0) or a negative PMG_E* code and
 *     never throws.  pmg_last_error() returns a thread-local message for the
 *     last failure.  Errors found by kernels (det J <= 0, zero pivots, no
 *     convergence, NaN) are reported per problem in the pmg_info array.
 *   - Precision.  prec = PMG_F64 operates on double arrays, PMG_F32 on float
 *     arrays (the mixed-precision inner path); a handle built with
 *     inner_prec = PMG_F64 supports PMG_F64 calls only.
 */
#ifndef PMG_H
#define PMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* pmg_stream_t; /* hipStream_t */

enum {
    PMG_OK = 0,
    PMG_EINVAL = -1,     /* bad argument or unsupported shape */
    PMG_ENOMEM = -2,     /* workspace too small */
    PMG_EDEVICE = -3,    /* HIP runtime error */
    PMG_EGEOM = -4,      /* det J <= 0 somewhere (per-problem status) */
    PMG_ENAN = -5,       /* NaN or Inf in a residual (per-problem status) */
    PMG_EBREAKDOWN = -6, /* Krylov breakdown before convergence */
    PMG_ENOTCONV = -7,   /* max_iter reached */
    PMG_EPIVOT = -8      /* zero pivot in a line factorisation */
};

enum { PMG_F64 = 0, PMG_F32 = 1 };
enum { PMG_SMOOTHER_GLL = 0, PMG_SMOOTHER_FEM = 1, PMG_SMOOTHER_GLL_BAND2 = 2 };
enum { PMG_FGMRES = 0, PMG_PCG = 1, PMG_FCG = 2 };
enum { PMG_RESTRICT_TRANSPOSE = 0, PMG_RESTRICT_INTERP = 1 };

#define PMG_MAX_LEVELS 9

/* Problem and method description.
 *   dim        2 or 3
 *   p_fine     finest degree: a power of two, 4..256 (2-D) or 4..64 (3-D);
 *              levels halve down to p = 2 (one interior node, solved exactly:
 *              M_0^{-1} = A_0^{-1} in Alg. 2)
 *   batch      B >= 1 problems
 *   gamma, m, alpha   gamma-cycle parameters of Alg. 2 (gamma >= 1 coarse
 *              corrections per visit, m smoothing steps per axis, relaxation
 *              alpha > 0).  The cycle is linear in its right-hand side, so
 *              a coarse level of degree 8 or 16 (2-D; 4 or 8 in 3-D) entered
 *              gamma^depth >= ni / 16 times per cycle (ni its interior
 *              nodes) is applied as the dense FP64 matrix of its own cycle,
 *              built at setup (workspace regions "Cc[l]"); the result is
 *              the recursive cycle's up to rounding.
 *   smoother   PMG_SMOOTHER_GLL: tridiagonal part of A_p along each line
 *              (Def. line preconditioners with half-bandwidth 1);
 *              PMG_SMOOTHER_FEM: tridiagonal line systems of the bilinear
 *              (2-D) / trilinear (3-D) finite-element matrix on the GLL
 *              node mesh;
 *              PMG_SMOOTHER_GLL_BAND2: the part of A_p within half-bandwidth 2
 *              along each line (Def. Axelsson incomplete bandwidth
 *              preconditioner with bandwidth 2), a block-tridiagonal matrix
 *              of 2x2 blocks solved by block cyclic reduction (Thm. two-level
 *              direct solver with m = 2); p_fine <= 128
 *   inner_prec PMG_F64, or PMG_F32 for an FP32 gamma-cycle inside FP64
 *              Krylov (geometric factors and the outer solve stay FP64)
 *   krylov     PMG_FGMRES (right-preconditioned, modified Gram-Schmidt,
 *              restarted), PMG_PCG, PMG_FCG (flexible CG)
 *   restart    FGMRES restart length (1..64)
 *   max_iter   iteration cap of the outer solve
 *   rtol       stop when ||b - A x||_2 <= rtol ||b||_2 (true residual)
 *   restriction  R_l of Sec. 3.3, which the section gives two ways:
 *              PMG_RESTRICT_INTERP, the interpolation of the fine polynomial
 *              at the coarse GLL nodes (the reading that reproduces the
 *              iteration counts of Table 1), or PMG_RESTRICT_TRANSPOSE,
 *              R_l = P_l^T (a stronger, Galerkin-consistent preconditioner:
 *              fewer iterations, not the method behind Table 1).  Coarse
 *              boundary rows are zero either way; P_l is the interpolation
 *              of the coarse polynomial at the fine nodes in both.
 *   elements   K spectral elements per axis (0 or 1: the one element of the
 *              paper; 2, 4 or 8 in 2-D, 2 or 4 in 3-D: the multi-element
 *              hp-multigrid of the paper's closing outlook, any line
 *              smoother).  The square (cube) is split into K^dim equal
 *              parts of the reference square (cube), each an element of
 *              degree p_l / K with its own GLL rule; an
 *              interface node is shared by the elements that meet there
 *              (continuous basis), the operator and the mass are the sums
 *              of the element ones, and the transfers interpolate element
 *              by element.  p_fine is the degree of the composite node grid
 *              (K times the finest element degree, which must be >= 4):
 *              vectors keep the one-element layout of p_fine + 1 nodes per
 *              axis.  The levels halve the element degree down to 2, so the
 *              coarsest level has degree 2K (level index log2(2K) - 1; the
 *              levels below it are absent) and is solved exactly with the
 *              inverse of its (2K-1)^dim x (2K-1)^dim interior matrix, built at
 *              setup in FP64.  In 2-D the levels of composite degree 8 and
 *              16 above it are collapsed into dense matrices by the rule
 *              given under gamma (built at setup from the element cycle).
 *              Line systems run along the composite grid lines across
 *              element interfaces (GLL rows: entries of the assembled
 *              operator; FEM rows: the composite node mesh). */
typedef struct {
    int dim;
    int p_fine;
    int batch;
    int gamma;
    int m;
    double alpha;
    int smoother;
    int inner_prec;
    int krylov;
    int restart;
    int max_iter;
    double rtol;
    int restriction;
    int elements;
} pmg_desc;

/* Per-problem result of the device solve (written by pmg_solve). */
typedef struct {
    int status;       /* PMG_OK or a negative PMG_E* code; 1 while a pooled solve
                         is still running */
    int iterations;   /* outer Krylov iterations */
    double relres;    /* final true relative residual ||b - A x|| / ||b|| (FP64) */
    double min_detj;  /* minimum Jacobian determinant over all levels (setup) */
} pmg_info;

typedef struct pmg_handle pmg_handle;

/* Thread-local text of the last error. */
const char* pmg_last_error(void);

/* Number of levels of a description (p_fine = 2^L * 2 gives L + 1), and
 * the index of its coarsest present level (0, or log2(2K) - 1 for K
 * elements per axis; first_level may be NULL). */
int pmg_num_levels(const pmg_desc* desc, int* n_levels);
int pmg_first_level(const pmg_desc* desc, int* first_level);

/* GLL nodes xi[0..p] and weights rho[0..p] of order p (Def. GLL quadrature
 * rule), and D[i*(p+1)+j] = pi_j'(xi_i) (derivative of the Lagrange basis of
 * Def. GLL interpolation basis).  Host arrays; D may be NULL.  FP64. */
int pmg_gll(int p, double* xi, double* rho, double* D);

/* J[i*(p_c+1)+j] = pi^c_j(xi^f_i): the 1-D prolongation from degree p_c to
 * degree p_f (Sec. 3.3, interpolation between GLL bases).  Host array of
 * (p_f+1)*(p_c+1) doubles. */
int pmg_interp(int p_c, int p_f, double* J);

/* Bytes of device workspace pmg_setup needs for this description. */
int pmg_workspace_bytes(const pmg_desc* desc, size_t* bytes);

/* One named region of a workspace: byte offset from the workspace start and
 * size in bytes (each region starts on a 256-byte boundary). */
typedef struct {
    char name[24];
    size_t offset;
    size_t bytes;
} pmg_region;

/* The layout pmg_setup gives the workspace of this description, in address
 * order: *n_regions receives the number of regions, of which the first
 * max_regions are written to the host array regions (may be NULL when
 * max_regions is 0).  Host-only; for memory accounting and inspection.
 * Per-level regions are named "X[l]" and so on; Krylov regions "V", "Z",
 * "Hs", "TR64", "state". */
int pmg_workspace_layout(const pmg_desc* desc, pmg_region* regions, int max_regions,
                         int* n_regions);

/* Build the hierarchy on the device (geometry of eq. DiscreteSpace and eq.
 * discreteBilinear for every level, line tridiagonals and their
 * cyclic-reduction factors, Sec. 3.2).
 *   d_coords[l]  level-l physical node positions: B x dim x N_l doubles
 *                (all first coordinates of a problem, then all second, ...)
 *                at the level's GLL nodes (the composite grid's nodes for
 *                K elements per axis); read during the call's stream work.
 *                Entries of absent levels (below the first level) are
 *                ignored and may be NULL.
 *   d_ws         caller-owned device workspace of ws_bytes >= the size from
 *                pmg_workspace_bytes; must stay valid until pmg_destroy
 *   d_info       B pmg_info records (device), min_detj and status filled
 * On return *out holds a host handle.  Problems with det J <= 0 or a zero
 * pivot get status PMG_EGEOM / PMG_EPIVOT in d_info. */
int pmg_setup(const pmg_desc* desc, const double* const* d_coords, void* d_ws,
              size_t ws_bytes, pmg_info* d_info, pmg_stream_t stream, pmg_handle** out);

/* Dirichlet lifting of Sec. 2.3 on the finest level:
 * d_b = M f - A v on interior nodes, 0 on boundary nodes, where v is d_g on
 * boundary nodes and 0 inside.  d_f, d_g, d_b: B x N doubles. */
int pmg_rhs(pmg_handle* h, const double* d_f, const double* d_g, double* d_b,
            pmg_stream_t stream);

/* d_u = d_w on interior nodes and d_g on boundary nodes (u = w + v, Sec. 2.3).
 * May be called in place (d_u == d_w). */
int pmg_lift(pmg_handle* h, const double* d_w, const double* d_g, double* d_u,
             pmg_stream_t stream);

/* d_y = A_l d_x on interior rows, 0 on boundary rows (matrix-free sum
 * factorisation of eq. discreteBilinear).  B x N_l arrays of the given
 * precision. */
int pmg_apply(pmg_handle* h, int level, int prec, const void* d_x, void* d_y,
              pmg_stream_t stream);

/* d_rc = R_l d_rf (level l -> l-1, R_l = P_l^T, Sec. 3.3); coarse boundary
 * entries set to 0.  level >= 1. */
int pmg_restrict(pmg_handle* h, int level, int prec, const void* d_rf, void* d_rc,
                 pmg_stream_t stream);

/* d_xf += P_l d_ec (level l-1 -> l, tensor product of the 1-D
 * interpolation).  level >= 1. */
int pmg_prolong_add(pmg_handle* h, int level, int prec, const void* d_ec, void* d_xf,
                    pmg_stream_t stream);

/* d_z = B_{l,dir}^{-1} d_r: every interior line along axis dir solved by the
 * cyclic reduction of Thm. "Two-level direct solver" / Cor. "Direct
 * multigrid solver" (block Jacobi over lines, Def. line preconditioners);
 * boundary entries of d_z are 0.  d_r and d_z must not overlap. */
int pmg_line_solve(pmg_handle* h, int level, int dir, int prec, const void* d_r,
                   void* d_z, pmg_stream_t stream);

/* One smoothing step of Alg. 2: d_x += alpha B_{l,dir}^{-1} (d_r - A_l d_x). */
int pmg_line_smooth(pmg_handle* h, int level, int dir, int prec, const void* d_r,
                    void* d_x, pmg_stream_t stream);

/* d_y = M_L^{-1} d_r, one gamma-cycle of Alg. 2 from the finest level
 * (B x N arrays of the given precision). */
int pmg_gamma_cycle(pmg_handle* h, int prec, const void* d_r, void* d_y,
                    pmg_stream_t stream);

/* Outer solve A w = b on the finest level (FP64, zero initial guess),
 * preconditioned by the gamma-cycle; d_x receives w (zero boundary), d_info
 * per-problem status, iterations and true relative residual.  The whole
 * iteration runs on the device, one workgroup per problem. */
int pmg_solve(pmg_handle* h, const double* d_b, double* d_x, pmg_info* d_info,
              pmg_stream_t stream);

/* Bytes of the fixed device array behind pmg_solve_noalloc (per GPU). */
#define PMG_SCRATCH_BYTES ((size_t)64 << 20)

/* pmg_solve for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, arithmetic and results as pmg_solve (bit for bit), but the
 * solve's Krylov scratch (the FGMRES basis V and Z, Hessenberg and Givens
 * data, the FP64 flux buffer of the outer operator and the per-problem solve
 * state; the CG variants use the first five vectors of V) comes from a fixed
 * array of PMG_SCRATCH_BYTES inside the library instead of the handle's
 * workspace.  The call allocates nothing (no hipMalloc, no library
 * allocation); the array is reserved on each GPU the library runs on when
 * its code is loaded there and held until the process ends.  It needs
 *   B * 8 * N * (max(restart + 1, 5) + restart + dim)
 *   + B * 8 * ((restart + 1) * restart + 4 * restart + 1) + B * 32
 * bytes (each of the five regions rounded up to 256 bytes), N the finest
 * level's node count; larger batches return PMG_ENOMEM with a message and
 * launch nothing.  Every call on one GPU uses the same array: calls that
 * overlap on one GPU (other streams, other threads) race and must be
 * serialised by the caller; nothing in the array needs to start at zero
 * (every word is written before it is read), and it keeps the last call's
 * contents. */
int pmg_solve_noalloc(pmg_handle* h, const double* d_b, double* d_x, pmg_info* d_info,
                      pmg_stream_t stream);

/* Per-level line-system tridiagonals (lower, diagonal, upper) of axis dir,
 * (p_l-1)^dim doubles each per problem, line after line as described for the
 * oracle-independent layout: lines ordered by the remaining interior
 * indices (first remaining axis fastest), p_l - 1 entries per line.  For
 * inspection and tests; FP64. */
int pmg_line_coefs(pmg_handle* h, int level, int dir, double* d_lo, double* d_di,
                   double* d_up, pmg_stream_t stream);

/* Half-bandwidth-2 line rows of a PMG_SMOOTHER_GLL_BAND2 handle, level l,
 * axis dir: d_band holds B x (p_l-1)^(dim-1) x (p_l-1) x 5 doubles, for each
 * line (ordered as in pmg_line_coefs) and position s the entries (s, s+k),
 * k = -2..2, of A_l along the line (zero outside it).  FP64; for inspection
 * and tests.  PMG_EINVAL for handles with other smoothers. */
int pmg_line_band(pmg_handle* h, int level, int dir, double* d_band, pmg_stream_t stream);

/* Geometric factors of level l: d_G B x ncomp x N_l doubles (ncomp = 3 in
 * 2-D: G_00, G_11, G_01; 6 in 3-D: G_00, G_11, G_22, G_01, G_02, G_12) and
 * d_mass B x N_l doubles (may be NULL).  K elements per axis: d_G holds per
 * problem the K^dim elements in lexicographic order (first axis fastest),
 * each ncomp x (p_l/K + 1)^dim doubles at its element nodes, and the mass is
 * the assembled one at the composite nodes. */
int pmg_geom(pmg_handle* h, int level, double* d_G, double* d_mass, pmg_stream_t stream);

/* Release the host handle (the workspace stays the caller's). */
int pmg_destroy(pmg_handle* h);

/* ------------------------------------------------------------------------
 * Serving: solve pools and a continuous-batching server.
 *
 * A pool holds desc->batch solve slots of one shape.  Requests are admitted
 * into free slots one batch at a time (their setup and right-hand side are
 * built for those slots only); pmg_pool_step then advances every running
 * slot by iters_per_step outer iterations in one launch (captured once into a
 * HIP graph and replayed).  Each slot's Krylov and multigrid state stays in
 * the workspace between steps, and a pooled solve performs exactly the
 * arithmetic of pmg_solve on the same problem, so its result does not depend
 * on how it was batched or split into steps.  Only FGMRES and the CG
 * variants of pmg_solve are available (the same code).
 * ------------------------------------------------------------------------ */
typedef struct pmg_pool pmg_pool;

/* Workspace bytes of a pool of desc->batch slots (includes per-slot input
 * staging, right-hand side, solution and info). */
int pmg_pool_workspace_bytes(const pmg_desc* desc, size_t* bytes);

/* Create a pool in the caller's workspace; every slot starts idle.  With a
 * non-null `stream` the step (one launch of the resumable solve) is captured
 * into a graph on it here, so that steps only replay it; iters_per_step >= 1. */
int pmg_pool_create(const pmg_desc* desc, int iters_per_step, void* d_ws, size_t ws_bytes,
                    pmg_stream_t stream, pmg_pool** out);

/* Admit n requests into the idle slots slots[0..n-1] (host array).  Request i
 * provides d_coords[i*n_levels + l] (level-l coordinates, dim x N_l doubles,
 * layout of pmg_setup), d_f[i] and d_g[i] (finest-level N doubles: source
 * and Dirichlet data).  The inputs are copied into the slot before the call's
 * stream work completes; the caller may reuse them afterwards. */
int pmg_pool_admit(pmg_pool* pool, int n, const int* slots, const double* const* d_coords,
                   const double* const* d_f, const double* const* d_g, pmg_stream_t stream);

/* Advance every running slot by up to iters_per_step outer iterations. */
int pmg_pool_step(pmg_pool* pool, pmg_stream_t stream);

/* Synchronise the stream and copy every slot's state to the host:
 * slot_status[s] = 1 running, 2 idle, 0 converged, < 0 failed (PMG_E*);
 * info (may be NULL) receives the per-slot pmg_info. */
int pmg_pool_poll(pmg_pool* pool, int* slot_status, pmg_info* info, pmg_stream_t stream);

/* Write the finished solution of `slot` (Dirichlet data on the boundary,
 * u = w + v of Sec. 2.3) to d_u (N doubles) and make the slot idle. */
int pmg_pool_take(pmg_pool* pool, int slot, double* d_u, pmg_stream_t stream);

int pmg_pool_destroy(pmg_pool* pool);

/* A server owns one pool per shape class and admits queued requests in
 * arrival order whenever a slot of their class is free and the summed
 * footprint (per-slot workspace bytes) of the admitted, unfinished requests
 * stays within budget_bytes.  Each class runs on its own (caller's) stream and
 * advances independently: pmg_server_step retires the finished requests of
 * every class whose previous step has completed (waiting up to about 2 ms for
 * one if none has), admits queued requests into idle classes, and launches
 * the next step of every idle class with running slots, then returns without
 * waiting for those steps.  Fast classes are therefore not held by slow ones,
 * and the classes' kernels overlap on the device.  Admissions and launches
 * are issued class by class in decreasing per-slot footprint, so the longest
 * solves start first, and a class is admitted into only while the classes of
 * larger footprint run fewer requests than the device holds solve
 * workgroups at once (CUs x resident workgroups per CU): the heaviest work
 * fills the device by itself and lighter classes use what it leaves free.
 * The finished requests of a class are lifted into their d_u by one launch.
 * Call it repeatedly. */
#define PMG_SERVER_MAX_CLASSES 8
typedef struct {
    int n_classes;
    pmg_desc classes[PMG_SERVER_MAX_CLASSES]; /* .batch = slots of the class */
    int iters_per_step;
    size_t budget_bytes;
} pmg_server_desc;

typedef struct {
    int queued, running, finished;
    size_t bytes_in_use;
    long long steps;
} pmg_server_stats;

typedef struct pmg_server pmg_server;

int pmg_server_workspace_bytes(const pmg_server_desc* desc, size_t* bytes);
/* streams: n_classes caller-owned streams, class c runs on streams[c] (the
 * same stream may serve several classes, which then do not overlap); they
 * must outlive the server, which neither creates nor destroys streams. */
int pmg_server_create(const pmg_server_desc* desc, void* d_ws, size_t ws_bytes,
                      const pmg_stream_t* streams, pmg_server** out);
/* Queue a request of class cls.  d_coords holds n_levels pointers (level
 * order, coarsest first); the device inputs must stay valid until the request
 * is admitted (its step).  The solution is written to d_u (N doubles). */
int pmg_server_submit(pmg_server* srv, int cls, const double* const* d_coords,
                      const double* d_f, const double* d_g, double* d_u, long long* ticket);
/* One scheduling step; *n_done (may be NULL) receives the requests retired. */
int pmg_server_step(pmg_server* srv, int* n_done);
/* 1 if the request has finished (info filled, d_u written), 0 if pending. */
int pmg_server_poll(pmg_server* srv, long long ticket, pmg_info* info);
/* Move up to max tickets of requests retired since the previous drain, in
 * retirement order, into tickets[] (host array of max entries); *n receives
 * how many.  Entries not moved stay for the next call.  Lets a caller find
 * its finished requests without polling every open ticket. */
int pmg_server_drain(pmg_server* srv, long long* tickets, int max, int* n);
int pmg_server_stats_get(pmg_server* srv, pmg_server_stats* stats);
int pmg_server_destroy(pmg_server* srv);

#ifdef __cplusplus
}
#endif
#endif

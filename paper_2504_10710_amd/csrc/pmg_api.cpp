// pmg_api.cpp -- the C ABI of libpmg (include/pmg.h): argument checks,
// workspace layout, host-side 1-D GLL tables, kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <mutex>
#include <thread>
#include <vector>

#include "pmg_internal.hpp"

using namespace pmg;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* where)
{
    return fail(PMG_EDEVICE, "%s: %s", where, hipGetErrorString(e));
}

// ---------------------------------------------------------------- 1-D GLL tables

// Legendre L_n(x) and L_{n-1}(x) by the three-term recurrence.
void legendre2(int n, double x, double& Ln, double& Lnm1)
{
    double a = 1.0, b = x;
    if (n == 0) { Ln = 1.0; Lnm1 = 0.0; return; }
    for (int k = 2; k <= n; ++k) {
        double c = ((2.0 * k - 1.0) * x * b - (k - 1.0) * a) / k;
        a = b;
        b = c;
    }
    Ln = b;
    Lnm1 = a;
}

// GLL nodes by the Lobatto fixed-point Newton iteration
//   x <- x - (x L_p(x) - L_{p-1}(x)) / ((p + 1) L_p(x)),
// whose fixed points are the zeros of (1 - x^2) L_p'(x), started from the
// Chebyshev-Gauss-Lobatto points; weights 2 / (p (p+1) L_p(x)^2).
bool gll_nodes(int p, std::vector<double>& xi, std::vector<double>& rho)
{
    xi.assign(p + 1, 0.0);
    rho.assign(p + 1, 0.0);
    for (int j = 0; j <= p; ++j) {
        double x = -std::cos(M_PI * j / p);
        if (j == 0 || j == p) {
            xi[j] = x < 0 ? -1.0 : 1.0;
            continue;
        }
        bool ok = false;
        for (int it = 0; it < 200; ++it) {
            double Lp, Lm;
            legendre2(p, x, Lp, Lm);
            double dx = (x * Lp - Lm) / ((p + 1.0) * Lp);
            x -= dx;
            if (std::fabs(dx) <= 2e-16 * (1.0 + std::fabs(x))) { ok = true; break; }
        }
        if (!ok) return false;
        xi[j] = x;
    }
    // exact symmetry of the node set
    for (int j = 0; j < (p + 1) / 2; ++j) {
        double v = 0.5 * (xi[p - j] - xi[j]);
        xi[j] = -v;
        xi[p - j] = v;
    }
    if (p % 2 == 0) xi[p / 2] = 0.0;
    for (int j = 0; j <= p; ++j) {
        double Lp, Lm;
        legendre2(p, xi[j], Lp, Lm);
        rho[j] = 2.0 / (p * (p + 1.0) * Lp * Lp);
    }
    return true;
}

// GLL differentiation matrix: closed-form off-diagonals
// D_ij = L_p(xi_i) / (L_p(xi_j) (xi_i - xi_j)), i != j, and each diagonal
// entry the negative sum of its row's off-diagonals, D_ii = -sum_{j!=i} D_ij,
// so that D differentiates constants to zero in floating point as well
// (the "negative sum trick" of Baltensperger and Trummer, SIAM J. Sci.
// Comput. 24 (2003); the exact diagonal is -p(p+1)/4, 0, ..., 0, p(p+1)/4).
void gll_deriv(int p, const std::vector<double>& xi, std::vector<double>& D)
{
    int n1 = p + 1;
    std::vector<double> L(n1);
    for (int i = 0; i < n1; ++i) {
        double a, b;
        legendre2(p, xi[i], a, b);
        L[i] = a;
    }
    D.assign(n1 * n1, 0.0);
    for (int i = 0; i < n1; ++i) {
        double s = 0.0;
        for (int j = 0; j < n1; ++j) {
            if (i == j) continue;
            double v = L[i] / (L[j] * (xi[i] - xi[j]));
            D[i * n1 + j] = v;
            s += v;
        }
        D[i * n1 + i] = -s;
    }
}

// Barycentric Lagrange interpolation from the coarse GLL nodes xc to the
// points xf: J[i][j] = (w_j / (xf_i - xc_j)) / sum_k (w_k / (xf_i - xc_k)),
// w_j = 1 / prod_{k != j} (xc_j - xc_k); exact rows where xf_i is a node.
void bary_interp(const std::vector<double>& xc, const std::vector<double>& xf,
                 std::vector<double>& J)
{
    int nc = (int)xc.size(), nf = (int)xf.size();
    std::vector<double> w(nc, 1.0);
    for (int j = 0; j < nc; ++j)
        for (int k = 0; k < nc; ++k)
            if (k != j) w[j] /= (xc[j] - xc[k]);
    J.assign(nf * nc, 0.0);
    for (int i = 0; i < nf; ++i) {
        int hit = -1;
        for (int j = 0; j < nc; ++j)
            if (xf[i] == xc[j]) hit = j;
        if (hit >= 0) { J[i * nc + hit] = 1.0; continue; }
        double den = 0.0;
        for (int j = 0; j < nc; ++j) den += w[j] / (xf[i] - xc[j]);
        for (int j = 0; j < nc; ++j) J[i * nc + j] = (w[j] / (xf[i] - xc[j])) / den;
    }
}

// ---------------------------------------------------------------- layout

struct Layout {
    size_t off = 0;
    std::vector<pmg_region>* rec = nullptr;   // optional record of the named regions
    size_t take(size_t bytes)
    {
        size_t o = (off + 255) & ~size_t(255);
        off = o + bytes;
        return o;
    }
    size_t take(const char* name, int level, size_t bytes)
    {
        size_t o = take(bytes);
        if (rec) {
            pmg_region r;
            memset(&r, 0, sizeof(r));
            if (level >= 0)
                snprintf(r.name, sizeof(r.name), "%s[%d]", name, level);
            else
                snprintf(r.name, sizeof(r.name), "%s", name);
            r.offset = o;
            r.bytes = bytes;
            rec->push_back(r);
        }
        return o;
    }
};

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int check_desc(const pmg_desc* d)
{
    if (!d) return fail(PMG_EINVAL, "desc is NULL");
    if (d->dim != 2 && d->dim != 3) return fail(PMG_EINVAL, "dim must be 2 or 3 (got %d)", d->dim);
    int pmax = d->dim == 2 ? 256 : 64;
    if (!is_pow2(d->p_fine) || d->p_fine < 4 || d->p_fine > pmax)
        return fail(PMG_EINVAL, "p_fine must be a power of two in [4, %d] (got %d)", pmax, d->p_fine);
    if (d->batch < 1) return fail(PMG_EINVAL, "batch must be >= 1");
    if (d->gamma < 1 || d->gamma > 16) return fail(PMG_EINVAL, "gamma must be in [1, 16]");
    if (d->m < 0 || d->m > 8) return fail(PMG_EINVAL, "m must be in [0, 8]");
    if (!(d->alpha > 0.0) || !std::isfinite(d->alpha)) return fail(PMG_EINVAL, "alpha must be > 0");
    if (d->smoother != PMG_SMOOTHER_GLL && d->smoother != PMG_SMOOTHER_FEM &&
        d->smoother != PMG_SMOOTHER_GLL_BAND2)
        return fail(PMG_EINVAL, "unknown smoother %d", d->smoother);
    if (d->smoother == PMG_SMOOTHER_GLL_BAND2 && d->p_fine > 128)
        return fail(PMG_EINVAL, "half-bandwidth-2 line systems are supported up to p = 128 (got %d)",
                    d->p_fine);
    if (d->inner_prec != PMG_F64 && d->inner_prec != PMG_F32)
        return fail(PMG_EINVAL, "unknown inner precision %d", d->inner_prec);
    if (d->krylov != PMG_FGMRES && d->krylov != PMG_PCG && d->krylov != PMG_FCG)
        return fail(PMG_EINVAL, "unknown Krylov method %d", d->krylov);
    if (d->restart < 1 || d->restart > 64) return fail(PMG_EINVAL, "restart must be in [1, 64]");
    if (d->max_iter < 1) return fail(PMG_EINVAL, "max_iter must be >= 1");
    if (!(d->rtol > 0.0)) return fail(PMG_EINVAL, "rtol must be > 0");
    if (d->restriction != PMG_RESTRICT_TRANSPOSE && d->restriction != PMG_RESTRICT_INTERP)
        return fail(PMG_EINVAL, "unknown restriction %d", d->restriction);
    if (d->elements < 0 || d->elements > 8 || (d->elements > 1 && !is_pow2(d->elements)))
        return fail(PMG_EINVAL, "elements must be 0, 1, 2, 4 or 8 (got %d)", d->elements);
    if (d->elements > 1) {
        if (d->dim == 3 && d->elements > 4)
            return fail(PMG_EINVAL, "3-D supports up to 4 elements per axis (the coarsest level's "
                                    "exact inverse grows as (2K-1)^6)");
        if (d->p_fine / d->elements < 4)
            return fail(PMG_EINVAL, "the finest element degree p_fine / elements must be >= 4 "
                                    "(got %d / %d)", d->p_fine, d->elements);
    }
    return PMG_OK;
}

// elements per axis and the index of the coarsest present level (degree 2K)
int elems_of(const pmg_desc& d) { return d.elements > 1 ? d.elements : 1; }
int first_level_of(const pmg_desc& d) { return ilog2(2 * elems_of(d)) - 1; }

struct LevelShape {
    int p, n1, N, n, NL, NC, CRW;
};

LevelShape level_shape(int dim, int l)
{
    LevelShape s;
    s.p = 2 << l;
    s.n1 = s.p + 1;
    s.N = dim == 2 ? s.n1 * s.n1 : s.n1 * s.n1 * s.n1;
    s.n = s.p - 1;
    s.NL = dim == 2 ? s.n : s.n * s.n;
    s.NC = dim == 2 ? 3 : 6;
    s.CRW = cr_words(s.n);
    return s;
}

}  // namespace

struct pmg_handle {
    pmg_desc d;
    int nlev;
    int K = 1;    // elements per axis
    int l0 = 0;   // coarsest present level (degree 2K)
    bool f32;
    size_t ws_bytes;
    char* ws;
    // offsets
    size_t o_rho[MAX_LEVELS], o_D64[MAX_LEVELS], o_DT64[MAX_LEVELS], o_J64[MAX_LEVELS],
        o_JT64[MAX_LEVELS];
    size_t o_D32[MAX_LEVELS], o_DT32[MAX_LEVELS], o_J32[MAX_LEVELS], o_JT32[MAX_LEVELS];
    size_t o_JR64[MAX_LEVELS], o_JR32[MAX_LEVELS];
    size_t o_G64[MAX_LEVELS], o_G32[MAX_LEVELS], o_X64[MAX_LEVELS];
    size_t o_cr64[MAX_LEVELS][3], o_cr32[MAX_LEVELS][3];
    size_t o_bd64[MAX_LEVELS][3], o_bd32[MAX_LEVELS][3];   // band-2 line rows (0: none)
    size_t o_X[MAX_LEVELS], o_R[MAX_LEVELS], o_Tm[MAX_LEVELS], o_TR[MAX_LEVELS];
    size_t o_EX[MAX_LEVELS];   // element-local operand / output (K > 1), 0: none
    size_t o_EX64;             // its FP64 form on the finest level (K > 1), 0: none
    size_t o_mass, o_W1, o_W2, o_TR64, o_V, o_Z, o_Hs, o_detmin, o_pivot, o_cinv64, o_cinv32;
    size_t o_sstatus, o_state, o_hier64, o_hier32;
    size_t o_Cc[MAX_LEVELS];   // collapsed coarse cycles, B x ni x ni doubles (0: none)
    // serving pools only: per-slot input staging, right-hand side, solution,
    // info, and the slot list of an admission
    bool pool = false;
    size_t o_in_coords[MAX_LEVELS], o_in_f, o_in_g, o_b, o_x, o_info, o_slots;
    size_t o_take_slots, o_take_outs;   // slot and destination lists of a batched lift
    size_t o_jobs;                      // copy jobs of an admission (inputs into slots)
    long long w1, w2, nv, hs;
    size_t total;
    // host copies of the tables uploaded at setup (kept alive for async copies)
    std::vector<double> h64;
    std::vector<float> h32;
    Hier<double> H64;
    Hier<float> H32;
};

namespace {

void describe(pmg_handle* h, const pmg_desc* desc)
{
    h->d = *desc;
    h->nlev = ilog2(desc->p_fine);
    h->K = elems_of(*desc);
    h->l0 = first_level_of(*desc);
    h->f32 = desc->inner_prec == PMG_F32;
}

// element nodes of level l of a K-element handle (per problem: K^dim
// elements of (p_l/K + 1)^dim nodes); N_l for one element
long long elem_nodes(const pmg_handle* h, int l)
{
    const LevelShape s = level_shape(h->d.dim, l);
    if (h->K == 1) return s.N;
    const long long ne1 = s.p / h->K + 1;
    return h->d.dim == 2 ? (long long)h->K * h->K * ne1 * ne1
                         : (long long)h->K * h->K * h->K * ne1 * ne1 * ne1;
}

void plan(pmg_handle* h, std::vector<pmg_region>* rec = nullptr)
{
    const pmg_desc& d = h->d;
    const int dim = d.dim, B = d.batch;
    const size_t tsz = h->f32 ? sizeof(float) : sizeof(double);
    Layout L;
    L.rec = rec;
    long long w = 0;
    for (int l = 0; l < MAX_LEVELS; ++l) {
        h->o_rho[l] = h->o_D64[l] = h->o_DT64[l] = h->o_D32[l] = h->o_DT32[l] = 0;
        h->o_J64[l] = h->o_JT64[l] = h->o_J32[l] = h->o_JT32[l] = h->o_JR64[l] = h->o_JR32[l] = 0;
        h->o_G64[l] = h->o_G32[l] = h->o_X64[l] = h->o_X[l] = h->o_R[l] = h->o_Tm[l] = h->o_TR[l] = 0;
        h->o_EX[l] = 0;
        h->o_Cc[l] = 0;
        for (int a = 0; a < 3; ++a)
            h->o_cr64[l][a] = h->o_cr32[l][a] = h->o_bd64[l][a] = h->o_bd32[l][a] = 0;
    }
    for (int l = h->l0; l < h->nlev; ++l) {
        LevelShape s = level_shape(dim, l);
        h->o_rho[l] = L.take("rho", l, sizeof(double) * s.n1);
        h->o_D64[l] = L.take("D64", l, sizeof(double) * s.n1 * s.n1);
        h->o_DT64[l] = L.take("DT64", l, sizeof(double) * s.n1 * s.n1);
        h->o_D32[l] = L.take("D32", l, sizeof(float) * s.n1 * s.n1);
        h->o_DT32[l] = L.take("DT32", l, sizeof(float) * s.n1 * s.n1);
        if (l > h->l0) {
            int n1c = s.p / 2 + 1;
            h->o_J64[l] = L.take("J64", l, sizeof(double) * s.n1 * n1c);
            h->o_JT64[l] = L.take("JT64", l, sizeof(double) * s.n1 * n1c);
            h->o_J32[l] = L.take("J32", l, sizeof(float) * s.n1 * n1c);
            h->o_JT32[l] = L.take("JT32", l, sizeof(float) * s.n1 * n1c);
            h->o_JR64[l] = L.take("JR64", l, sizeof(double) * s.n1 * n1c);
            h->o_JR32[l] = L.take("JR32", l, sizeof(float) * s.n1 * n1c);
            long long ww = (long long)(dim == 2 ? s.n1 : s.n1 * s.n1) * n1c;
            if (ww > w) w = ww;
        } else {
            h->o_J64[l] = h->o_JT64[l] = h->o_J32[l] = h->o_JT32[l] = 0;
            h->o_JR64[l] = h->o_JR32[l] = 0;
        }
    }
    for (int l = h->l0; l < h->nlev; ++l) {
        LevelShape s = level_shape(dim, l);
        const long long NE = elem_nodes(h, l);   // geometric factors and fluxes per element node
        h->o_G64[l] = L.take("G64", l, sizeof(double) * (size_t)B * s.NC * NE);
        h->o_G32[l] = h->f32 ? L.take("G32", l, sizeof(float) * (size_t)B * s.NC * NE) : 0;
        h->o_X64[l] = L.take("X64", l, sizeof(double) * (size_t)B * dim * s.N);
        for (int a = 0; a < 3; ++a) {
            h->o_cr64[l][a] = a < dim ? L.take(a == 0 ? "cr64x" : (a == 1 ? "cr64y" : "cr64z"), l, sizeof(double) * (size_t)B * 3 * s.CRW * s.NL) : 0;
            h->o_cr32[l][a] =
                (a < dim && h->f32) ? L.take(a == 0 ? "cr32x" : (a == 1 ? "cr32y" : "cr32z"), l, sizeof(float) * (size_t)B * 3 * s.CRW * s.NL) : 0;
        }
        const bool band = d.smoother == PMG_SMOOTHER_GLL_BAND2;
        for (int a = 0; a < 3; ++a) {
            h->o_bd64[l][a] = (band && a < dim)
                ? L.take(a == 0 ? "bd64x" : (a == 1 ? "bd64y" : "bd64z"), l,
                         sizeof(double) * (size_t)B * 5 * s.n * s.NL) : 0;
            h->o_bd32[l][a] = (band && a < dim && h->f32)
                ? L.take(a == 0 ? "bd32x" : (a == 1 ? "bd32y" : "bd32z"), l,
                         sizeof(float) * (size_t)B * 5 * s.n * s.NL) : 0;
        }
        h->o_X[l] = L.take("X", l, tsz * (size_t)B * s.N);
        h->o_R[l] = L.take("R", l, tsz * (size_t)B * s.N);
        h->o_Tm[l] = L.take("Tm", l, tsz * (size_t)B * s.N);
        h->o_TR[l] = L.take("TR", l, tsz * (size_t)B * dim * NE);
        h->o_EX[l] = h->K > 1 ? L.take("EX", l, tsz * (size_t)B * NE) : 0;
    }
    LevelShape f = level_shape(dim, h->nlev - 1);
    h->w1 = h->w2 = w;
    h->o_mass = L.take("mass", -1, sizeof(double) * (size_t)B * f.N);
    h->o_W1 = L.take("W1", -1, tsz * (size_t)B * w);
    h->o_W2 = dim == 3 ? L.take("W2", -1, tsz * (size_t)B * w) : 0;
    h->o_TR64 = L.take("TR64", -1, sizeof(double) * (size_t)B * dim * elem_nodes(h, h->nlev - 1));
    h->o_EX64 = h->K == 1 ? 0
        : (h->f32 ? L.take("EX64", -1, sizeof(double) * (size_t)B * elem_nodes(h, h->nlev - 1))
                  : h->o_EX[h->nlev - 1]);
    const int kr = d.restart;
    h->nv = kr + 1 > 5 ? kr + 1 : 5;
    h->hs = (long long)(kr + 1) * kr + 4LL * kr + 1;
    h->o_V = L.take("V", -1, sizeof(double) * (size_t)B * h->nv * f.N);
    h->o_Z = L.take("Z", -1, sizeof(double) * (size_t)B * kr * f.N);
    h->o_Hs = L.take("Hs", -1, sizeof(double) * (size_t)B * h->hs);
    h->o_detmin = L.take("detmin", -1, sizeof(double) * (size_t)B * h->nlev);
    h->o_pivot = L.take("pivot", -1, sizeof(int) * (size_t)B);
    h->o_cinv64 = L.take("cinv64", -1, sizeof(double) * (size_t)B);
    h->o_cinv32 = L.take("cinv32", -1, sizeof(float) * (size_t)B);
    h->o_sstatus = L.take("sstatus", -1, sizeof(int) * (size_t)B);
    h->o_state = L.take("state", -1, sizeof(SolveState) * (size_t)B);
    // A coarse level is collapsed when its matrix pays for itself: building
    // it costs about ni cycles of that level, and every visit afterwards
    // saves about one; a level is entered gamma^depth times per cycle, so
    // with solves of about 16 iterations or more the build is repaid when
    // gamma^depth >= ni / 16.
    for (int l = h->l0; l < h->nlev; ++l) {
        const int pl = 2 << l;
        const long long ni = dim == 2 ? (pl - 1) * (pl - 1) : (pl - 1) * (pl - 1) * (pl - 1);
        double visits = 1.0;
        for (int k = l; k < h->nlev - 1; ++k) visits *= d.gamma;
        // several elements: the coarsest level holds its exact inverse, and
        // in 2-D the levels above it are collapsed by the same rule as one
        // element's
        const bool rule = (pl == collapse_lo(dim) || pl == collapse_p(dim)) && d.p_fine > pl &&
                          16.0 * visits >= (double)ni;
        const bool coll = h->K > 1 ? (l == h->l0 || (dim == 2 && rule)) : rule;
        h->o_Cc[l] = coll ? L.take("Cc", l, sizeof(double) * (size_t)B * ni * ni) : 0;
    }
    h->o_hier64 = L.take("hier64", -1, sizeof(Hier<double>));
    h->o_hier32 = L.take("hier32", -1, sizeof(Hier<float>));
    if (h->pool) {
        for (int l = 0; l < MAX_LEVELS; ++l) h->o_in_coords[l] = 0;
        for (int l = h->l0; l < h->nlev; ++l) {
            LevelShape s = level_shape(dim, l);
            h->o_in_coords[l] = L.take("in_coords", l, sizeof(double) * (size_t)B * dim * s.N);
        }
        h->o_in_f = L.take("in_f", -1, sizeof(double) * (size_t)B * f.N);
        h->o_in_g = L.take("in_g", -1, sizeof(double) * (size_t)B * f.N);
        h->o_b = L.take("b", -1, sizeof(double) * (size_t)B * f.N);
        h->o_x = L.take("x", -1, sizeof(double) * (size_t)B * f.N);
        h->o_info = L.take("info", -1, sizeof(pmg_info) * (size_t)B);
        h->o_slots = L.take("slots", -1, sizeof(int) * (size_t)B);
        h->o_take_slots = L.take("take_slots", -1, sizeof(int) * (size_t)B);
        h->o_take_outs = L.take("take_outs", -1, sizeof(double*) * (size_t)B);
        h->o_jobs = L.take("jobs", -1, sizeof(CopyJob) * (size_t)B * (h->nlev + 2));
    }
    h->total = L.take(0) + 256;
}

template <class T>
void fill_hier(pmg_handle* h, Hier<T>& H, bool is32)
{
    memset(&H, 0, sizeof(H));
    char* ws = h->ws;
    const int dim = h->d.dim;
    for (int l = h->l0; l < h->nlev; ++l) {
        LevelData<T>& L = H.lev[l];
        L.G64 = (const double*)(ws + h->o_G64[l]);
        L.G = is32 ? (const T*)(ws + h->o_G32[l]) : (const T*)(ws + h->o_G64[l]);
        L.mass = (l == h->nlev - 1) ? (const double*)(ws + h->o_mass) : nullptr;
        L.X64 = (const double*)(ws + h->o_X64[l]);
        for (int a = 0; a < dim; ++a) {
            L.cr[a] = is32 ? (const T*)(ws + h->o_cr32[l][a]) : (const T*)(ws + h->o_cr64[l][a]);
            const size_t ob = is32 ? h->o_bd32[l][a] : h->o_bd64[l][a];
            L.bd[a] = ob ? (const T*)(ws + ob) : nullptr;
        }
        L.X = (T*)(ws + h->o_X[l]);
        L.R = (T*)(ws + h->o_R[l]);
        L.Tm = (T*)(ws + h->o_Tm[l]);
        L.TR = (T*)(ws + h->o_TR[l]);
        L.EX = h->o_EX[l] ? (T*)(ws + h->o_EX[l]) : nullptr;
        L.D = (const T*)(ws + (is32 ? h->o_D32[l] : h->o_D64[l]));
        L.DT = (const T*)(ws + (is32 ? h->o_DT32[l] : h->o_DT64[l]));
        if (l > h->l0) {
            L.J = (const T*)(ws + (is32 ? h->o_J32[l] : h->o_J64[l]));
            L.JT = (const T*)(ws + (is32 ? h->o_JT32[l] : h->o_JT64[l]));
            L.JR = (const T*)(ws + (is32 ? h->o_JR32[l] : h->o_JR64[l]));
        }
        L.D64 = (const double*)(ws + h->o_D64[l]);
        L.DT64 = (const double*)(ws + h->o_DT64[l]);
        L.ng = elem_nodes(h, l);
    }
    H.cinv = (const T*)(ws + (is32 ? h->o_cinv32 : h->o_cinv64));
    H.cinv64 = (const double*)(ws + h->o_cinv64);
    for (int l = 0; l < h->nlev; ++l) H.Cc[l] = h->o_Cc[l] ? (const double*)(ws + h->o_Cc[l]) : nullptr;
    H.W1 = (T*)(ws + h->o_W1);
    H.W2 = dim == 3 ? (T*)(ws + h->o_W2) : nullptr;
    H.w1 = h->w1;
    H.w2 = h->w2;
    H.nlev = h->nlev;
    H.K = h->K;
    H.gamma = h->d.gamma;
    H.m = h->d.m;
    H.alpha = (T)h->d.alpha;
}

}  // namespace

extern "C" {

const char* pmg_last_error(void) { return g_err.c_str(); }

int pmg_num_levels(const pmg_desc* desc, int* n_levels)
{
    int rc = check_desc(desc);
    if (rc) return rc;
    if (!n_levels) return fail(PMG_EINVAL, "n_levels is NULL");
    *n_levels = ilog2(desc->p_fine);
    return PMG_OK;
}

int pmg_first_level(const pmg_desc* desc, int* first_level)
{
    int rc = check_desc(desc);
    if (rc) return rc;
    if (!first_level) return fail(PMG_EINVAL, "first_level is NULL");
    *first_level = first_level_of(*desc);
    return PMG_OK;
}

int pmg_gll(int p, double* xi, double* rho, double* D)
{
    if (p < 1 || p > 1024) return fail(PMG_EINVAL, "p must be in [1, 1024]");
    if (!xi || !rho) return fail(PMG_EINVAL, "xi and rho must not be NULL");
    std::vector<double> x, r, Dm;
    if (!gll_nodes(p, x, r)) return fail(PMG_EINVAL, "GLL Newton iteration failed for p = %d", p);
    memcpy(xi, x.data(), sizeof(double) * (p + 1));
    memcpy(rho, r.data(), sizeof(double) * (p + 1));
    if (D) {
        gll_deriv(p, x, Dm);
        memcpy(D, Dm.data(), sizeof(double) * (p + 1) * (p + 1));
    }
    return PMG_OK;
}

int pmg_interp(int p_c, int p_f, double* J)
{
    if (p_c < 1 || p_f < 1 || p_c > 1024 || p_f > 1024) return fail(PMG_EINVAL, "bad degrees");
    if (!J) return fail(PMG_EINVAL, "J is NULL");
    std::vector<double> xc, rc, xf, rf, Jm;
    if (!gll_nodes(p_c, xc, rc) || !gll_nodes(p_f, xf, rf))
        return fail(PMG_EINVAL, "GLL Newton iteration failed");
    bary_interp(xc, xf, Jm);
    memcpy(J, Jm.data(), sizeof(double) * (p_f + 1) * (p_c + 1));
    return PMG_OK;
}

int pmg_workspace_bytes(const pmg_desc* desc, size_t* bytes)
{
    int rc = check_desc(desc);
    if (rc) return rc;
    if (!bytes) return fail(PMG_EINVAL, "bytes is NULL");
    pmg_handle tmp;
    describe(&tmp, desc);
    plan(&tmp);
    *bytes = tmp.total;
    return PMG_OK;
}

int pmg_workspace_layout(const pmg_desc* desc, pmg_region* regions, int max_regions,
                         int* n_regions)
{
    int rc = check_desc(desc);
    if (rc) return rc;
    if (!n_regions || max_regions < 0 || (max_regions > 0 && !regions))
        return fail(PMG_EINVAL, "bad region buffer");
    pmg_handle tmp;
    describe(&tmp, desc);
    std::vector<pmg_region> rec;
    plan(&tmp, &rec);
    *n_regions = (int)rec.size();
    for (int i = 0; i < (int)rec.size() && i < max_regions; ++i) regions[i] = rec[i];
    return PMG_OK;
}

static const void* hier_of(pmg_handle* h, bool f32);

static int init_handle(const pmg_desc* desc, void* d_ws, size_t ws_bytes, bool pool,
                       hipStream_t s, pmg_handle** out)
{
    int rc = check_desc(desc);
    if (rc) return rc;
    if (!d_ws || !out) return fail(PMG_EINVAL, "NULL argument");
    pmg_handle* h = new pmg_handle();
    describe(h, desc);
    h->pool = pool;
    plan(h);
    if (ws_bytes < h->total) {
        size_t need = h->total;
        delete h;
        return fail(PMG_ENOMEM, "workspace too small: %zu < %zu bytes", ws_bytes, need);
    }
    h->ws = (char*)d_ws;
    h->ws_bytes = ws_bytes;
    const int dim = desc->dim;

    // host tables -> one staging buffer per precision, uploaded in one copy each.
    // Per level: the GLL rule and derivative matrix of the level's element
    // (the whole level for one element), and the 1-D transfers of the level's
    // composite grid, element block by element block.
    const size_t tab_end = h->o_G64[h->l0];
    h->h64.assign(tab_end / sizeof(double) + 1, 0.0);
    h->h32.assign(tab_end / sizeof(float) + 1, 0.0f);
    std::vector<std::vector<double>> xis(h->nlev);
    const int K = h->K;
    for (int l = h->l0; l < h->nlev; ++l) {
        LevelShape sh = level_shape(dim, l);
        const int pe = sh.p / K, ne1 = pe + 1;
        std::vector<double> rho, D;
        if (!gll_nodes(pe, xis[l], rho)) {
            delete h;
            return fail(PMG_EINVAL, "GLL Newton iteration failed for p = %d", pe);
        }
        gll_deriv(pe, xis[l], D);
        double* t64 = h->h64.data();
        float* t32 = h->h32.data();
        for (int i = 0; i < ne1; ++i) t64[h->o_rho[l] / 8 + i] = rho[i];
        for (int i = 0; i < ne1; ++i)
            for (int j = 0; j < ne1; ++j) {
                double v = D[i * ne1 + j];
                t64[h->o_D64[l] / 8 + i * ne1 + j] = v;
                t64[h->o_DT64[l] / 8 + j * ne1 + i] = v;
                t32[h->o_D32[l] / 4 + i * ne1 + j] = (float)v;
                t32[h->o_DT32[l] / 4 + j * ne1 + i] = (float)v;
            }
        if (l > h->l0) {
            // element blocks: Jl[i][j] = pi^c_j(xi^f_i); for the interpolation
            // reading Ql[j][i] = pi^f_i(xi^c_j), the fine basis at the coarse
            // nodes.  The composite tables put element e's block at rows
            // e pe .., columns e pc ..; an interface row is written by both
            // elements with the same values (the bases interpolate).
            const int pc = pe / 2, n1c = sh.p / 2 + 1;
            std::vector<double> Jl, Ql;
            bary_interp(xis[l - 1], xis[l], Jl);
            if (desc->restriction == PMG_RESTRICT_INTERP) bary_interp(xis[l], xis[l - 1], Ql);
            for (int e = 0; e < K; ++e)
                for (int i = 0; i < ne1; ++i)
                    for (int j = 0; j <= pc; ++j) {
                        const int I = e * pe + i, Jc = e * pc + j;
                        const double v = Jl[i * (pc + 1) + j];
                        // restriction table JR ([n1][n1c], R = JR^T per axis)
                        const double vr = desc->restriction == PMG_RESTRICT_INTERP ? Ql[j * ne1 + i] : v;
                        t64[h->o_J64[l] / 8 + I * n1c + Jc] = v;
                        t64[h->o_JT64[l] / 8 + Jc * sh.n1 + I] = v;
                        t32[h->o_J32[l] / 4 + I * n1c + Jc] = (float)v;
                        t32[h->o_JT32[l] / 4 + Jc * sh.n1 + I] = (float)v;
                        t64[h->o_JR64[l] / 8 + I * n1c + Jc] = vr;
                        t32[h->o_JR32[l] / 4 + I * n1c + Jc] = (float)vr;
                    }
        }
    }
    // The FP64 and FP32 tables interleave in [0, o_G64[l0]); upload the FP64
    // table regions from h64 and the FP32 regions from h32.
    hipError_t e;
    auto up64 = [&](size_t off, size_t n) {
        return hipMemcpyAsync(h->ws + off, h->h64.data() + off / 8, n * 8, hipMemcpyHostToDevice, s);
    };
    auto up32 = [&](size_t off, size_t n) {
        return hipMemcpyAsync(h->ws + off, h->h32.data() + off / 4, n * 4, hipMemcpyHostToDevice, s);
    };
    for (int l = h->l0; l < h->nlev; ++l) {
        LevelShape sh = level_shape(dim, l);
        const size_t ne1 = sh.p / K + 1, nn = ne1 * ne1;
        if ((e = up64(h->o_rho[l], ne1)) != hipSuccess ||
            (e = up64(h->o_D64[l], nn)) != hipSuccess || (e = up64(h->o_DT64[l], nn)) != hipSuccess ||
            (e = up32(h->o_D32[l], nn)) != hipSuccess || (e = up32(h->o_DT32[l], nn)) != hipSuccess) {
            delete h;
            return hip_fail(e, "table upload");
        }
        if (l > h->l0) {
            size_t nj = (size_t)sh.n1 * (sh.p / 2 + 1);
            if ((e = up64(h->o_J64[l], nj)) != hipSuccess || (e = up64(h->o_JT64[l], nj)) != hipSuccess ||
                (e = up32(h->o_J32[l], nj)) != hipSuccess || (e = up32(h->o_JT32[l], nj)) != hipSuccess ||
                (e = up64(h->o_JR64[l], nj)) != hipSuccess || (e = up32(h->o_JR32[l], nj)) != hipSuccess) {
                delete h;
                return hip_fail(e, "table upload");
            }
        }
    }
    fill_hier<double>(h, h->H64, false);
    fill_hier<float>(h, h->H32, true);
    // FP64 views used by the FP64-only operations of an FP32 handle
    h->H64.lev[h->nlev - 1].TR = (double*)(h->ws + h->o_TR64);
    h->H64.lev[h->nlev - 1].EX = h->o_EX64 ? (double*)(h->ws + h->o_EX64) : nullptr;
    // kernels read the hierarchy description from device memory
    if ((e = hipMemcpyAsync(h->ws + h->o_hier64, &h->H64, sizeof(Hier<double>), hipMemcpyHostToDevice,
                            s)) != hipSuccess ||
        (e = hipMemcpyAsync(h->ws + h->o_hier32, &h->H32, sizeof(Hier<float>), hipMemcpyHostToDevice,
                            s)) != hipSuccess) {
        delete h;
        return hip_fail(e, "hierarchy upload");
    }
    *out = h;
    return PMG_OK;
}

static void setup_args(pmg_handle* h, SetupArgs& a)
{
    const int dim = h->d.dim;
    memset(&a, 0, sizeof(a));
    a.K = h->K;
    a.l0 = h->l0;
    a.Cc0 = h->K > 1 ? (double*)(h->ws + h->o_Cc[h->l0]) : nullptr;
    for (int l = h->l0; l < h->nlev; ++l) {
        for (int k = 0; k < 3; ++k) {
            a.cr64[l][k] = k < dim ? (double*)(h->ws + h->o_cr64[l][k]) : nullptr;
            a.cr32[l][k] = (k < dim && h->f32) ? (float*)(h->ws + h->o_cr32[l][k]) : nullptr;
            a.bd64[l][k] = (k < dim && h->o_bd64[l][k]) ? (double*)(h->ws + h->o_bd64[l][k]) : nullptr;
            a.bd32[l][k] = (k < dim && h->o_bd32[l][k]) ? (float*)(h->ws + h->o_bd32[l][k]) : nullptr;
        }
        a.G64[l] = (double*)(h->ws + h->o_G64[l]);
        a.G32[l] = h->f32 ? (float*)(h->ws + h->o_G32[l]) : nullptr;
        a.X64[l] = (double*)(h->ws + h->o_X64[l]);
        a.rho[l] = (const double*)(h->ws + h->o_rho[l]);
        a.D64[l] = (const double*)(h->ws + h->o_D64[l]);
        a.DT64[l] = (const double*)(h->ws + h->o_DT64[l]);
    }
    a.mass = (double*)(h->ws + h->o_mass);
    a.detmin = (double*)(h->ws + h->o_detmin);
    a.pivot = (int*)(h->ws + h->o_pivot);
    a.sstatus = (int*)(h->ws + h->o_sstatus);
    a.cinv64 = (double*)(h->ws + h->o_cinv64);
    a.cinv32 = (float*)(h->ws + h->o_cinv32);
    a.smoother = h->d.smoother;
}

int pmg_setup(const pmg_desc* desc, const double* const* d_coords, void* d_ws, size_t ws_bytes,
              pmg_info* d_info, pmg_stream_t stream, pmg_handle** out)
{
    if (!d_coords || !d_info || !out) return fail(PMG_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    pmg_handle* h = nullptr;
    int rc = init_handle(desc, d_ws, ws_bytes, false, s, &h);
    if (rc) return rc;
    for (int l = h->l0; l < h->nlev; ++l)
        if (!d_coords[l]) {
            delete h;
            return fail(PMG_EINVAL, "coordinates of level %d are NULL", l);
        }
    SetupArgs a;
    setup_args(h, a);
    for (int l = h->l0; l < h->nlev; ++l) a.coords[l] = d_coords[l];
    hipError_t e = launch_setup(h->d.dim, h->d.p_fine, h->nlev, h->d.batch, a, d_info, s);
    // lower level first; above the coarsest level's exact inverse with elements
    for (int l = h->K > 1 ? h->l0 + 1 : 0; l < h->nlev && e == hipSuccess; ++l)
        if (h->o_Cc[l])
            e = launch_collapse(h->d.dim, 2 << l, h->f32, h->K > 1, h->d.batch,
                                hier_of(h, h->f32), (double*)(h->ws + h->o_Cc[l]), nullptr, s);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "setup kernels");
    }
    *out = h;
    return PMG_OK;
}

static int check_h(pmg_handle* h)
{
    if (!h) return fail(PMG_EINVAL, "handle is NULL");
    return PMG_OK;
}

static int check_prec(pmg_handle* h, int prec, bool* f32)
{
    if (prec != PMG_F64 && prec != PMG_F32) return fail(PMG_EINVAL, "unknown precision %d", prec);
    if ((prec == PMG_F32) != h->f32)
        return fail(PMG_EINVAL, "precision %s does not match the handle's inner precision",
                    prec == PMG_F32 ? "F32" : "F64");
    *f32 = prec == PMG_F32;
    return PMG_OK;
}

static const void* hier_of(pmg_handle* h, bool f32)
{
    return (const void*)(h->ws + (f32 ? h->o_hier32 : h->o_hier64));
}

static const Hier<double>* hier64_dev(pmg_handle* h)
{
    return (const Hier<double>*)(h->ws + h->o_hier64);
}

int pmg_rhs(pmg_handle* h, const double* d_f, const double* d_g, double* d_b, pmg_stream_t stream)
{
    int rc = check_h(h);
    if (rc) return rc;
    if (!d_f || !d_g || !d_b) return fail(PMG_EINVAL, "NULL argument");
    const long long vstride = h->nv * (long long)level_shape(h->d.dim, h->nlev - 1).N;
    hipError_t e = launch_rhs(h->d.dim, h->d.p_fine, h->d.batch, hier64_dev(h), d_f, d_g, d_b,
                              (double*)(h->ws + h->o_V), vstride, (hipStream_t)stream);
    return e == hipSuccess ? PMG_OK : hip_fail(e, "pmg_rhs");
}

int pmg_lift(pmg_handle* h, const double* d_w, const double* d_g, double* d_u, pmg_stream_t stream)
{
    int rc = check_h(h);
    if (rc) return rc;
    if (!d_w || !d_g || !d_u) return fail(PMG_EINVAL, "NULL argument");
    hipError_t e = launch_lift(h->d.dim, h->d.p_fine, h->d.batch, d_w, d_g, d_u, (hipStream_t)stream);
    return e == hipSuccess ? PMG_OK : hip_fail(e, "pmg_lift");
}

static int check_level(pmg_handle* h, int level, int lo)
{
    lo += h->l0;   // levels below the first present one do not exist
    if (level < lo || level >= h->nlev)
        return fail(PMG_EINVAL, "level %d out of range [%d, %d]", level, lo, h->nlev - 1);
    return PMG_OK;
}

int pmg_apply(pmg_handle* h, int level, int prec, const void* d_x, void* d_y, pmg_stream_t stream)
{
    bool f32;
    int rc;
    if ((rc = check_h(h)) || (rc = check_level(h, level, 0)) || (rc = check_prec(h, prec, &f32)))
        return rc;
    if (!d_x || !d_y) return fail(PMG_EINVAL, "NULL argument");
    hipError_t e = launch_apply(h->d.dim, 2 << level, f32, h->d.batch, hier_of(h, f32), d_x, d_y,
                                (hipStream_t)stream);
    return e == hipSuccess ? PMG_OK : hip_fail(e, "pmg_apply");
}

int pmg_restrict(pmg_handle* h, int level, int prec, const void* d_rf, void* d_rc, pmg_stream_t stream)
{
    bool f32;
    int rc;
    if ((rc = check_h(h)) || (rc = check_level(h, level, 1)) || (rc = check_prec(h, prec, &f32)))
        return rc;
    if (!d_rf || !d_rc) return fail(PMG_EINVAL, "NULL argument");
    hipError_t e = launch_restrict(h->d.dim, 2 << level, f32, h->d.batch, hier_of(h, f32), d_rf,
                                   d_rc, (hipStream_t)stream);
    return e == hipSuccess ? PMG_OK : hip_fail(e, "pmg_restrict");
}

int pmg_prolong_add(pmg_handle* h, int level, int prec, const void* d_ec, void* d_xf,
                    pmg_stream_t stream)
{
    bool f32;
    int rc;
    if ((rc = check_h(h)) || (rc = check_level(h, level, 1)) || (rc = check_prec(h, prec, &f32)))
        return rc;
    if (!d_ec || !d_xf) return fail(PMG_EINVAL, "NULL argument");
    hipError_t e = launch_prolong(h->d.dim, 2 << level, f32, h->d.batch, hier_of(h, f32), d_ec,
                                  d_xf, (hipStream_t)stream);
    return e == hipSuccess ? PMG_OK : hip_fail(e, "pmg_prolong_add");
}

int pmg_line_solve(pmg_handle* h, int level, int dir, int prec, const void* d_r, void* d_z,
                   pmg_stream_t stream)
{
    bool f32;
    int rc;
    if ((rc = check_h(h)) || (rc = check_level(h, level, 0)) || (rc = check_prec(h, prec, &f32)))
        return rc;
    if (dir < 0 || dir >= h->d.dim) return fail(PMG_EINVAL, "dir %d out of range", dir);
    if (!d_r || !d_z) return fail(PMG_EINVAL, "NULL argument");
    hipError_t e = launch_line_solve(h->d.dim, 2 << level, f32, h->d.batch, hier_of(h, f32), dir,
                                     d_r, d_z, (hipStream_t)stream);
    return e == hipSuccess ? PMG_OK : hip_fail(e, "pmg_line_solve");
}

int pmg_line_smooth(pmg_handle* h, int level, int dir, int prec, const void* d_r, void* d_x,
                    pmg_stream_t stream)
{
    bool f32;
    int rc;
    if ((rc = check_h(h)) || (rc = check_level(h, level, 0)) || (rc = check_prec(h, prec, &f32)))
        return rc;
    if (dir < 0 || dir >= h->d.dim) return fail(PMG_EINVAL, "dir %d out of range", dir);
    if (!d_r || !d_x) return fail(PMG_EINVAL, "NULL argument");
    hipError_t e = launch_line_smooth(h->d.dim, 2 << level, f32, h->K > 1, h->d.batch, hier_of(h, f32), dir,
                                      d_r, d_x, (hipStream_t)stream);
    return e == hipSuccess ? PMG_OK : hip_fail(e, "pmg_line_smooth");
}

int pmg_gamma_cycle(pmg_handle* h, int prec, const void* d_r, void* d_y, pmg_stream_t stream)
{
    bool f32;
    int rc;
    if ((rc = check_h(h)) || (rc = check_prec(h, prec, &f32))) return rc;
    if (!d_r || !d_y) return fail(PMG_EINVAL, "NULL argument");
    hipError_t e = launch_cycle(h->d.dim, h->d.p_fine, f32, h->K > 1, h->d.batch, hier_of(h, f32), d_r, d_y,
                                (hipStream_t)stream);
    return e == hipSuccess ? PMG_OK : hip_fail(e, "pmg_gamma_cycle");
}

int pmg_solve(pmg_handle* h, const double* d_b, double* d_x, pmg_info* d_info, pmg_stream_t stream)
{
    int rc = check_h(h);
    if (rc) return rc;
    if (!d_b || !d_x || !d_info) return fail(PMG_EINVAL, "NULL argument");
    SolveArgs a;
    a.b = d_b;
    a.x = d_x;
    a.V = (double*)(h->ws + h->o_V);
    a.Z = (double*)(h->ws + h->o_Z);
    a.Hs = (double*)(h->ws + h->o_Hs);
    a.TR64 = (double*)(h->ws + h->o_TR64);
    a.EX64 = h->o_EX64 ? (double*)(h->ws + h->o_EX64) : nullptr;
    a.elem = h->K > 1;
    a.info = d_info;
    a.nv = h->nv;
    a.hs = h->hs;
    a.restart = h->d.restart;
    a.max_iter = h->d.max_iter;
    a.krylov = h->d.krylov;
    a.rtol = h->d.rtol;
    a.st = (SolveState*)(h->ws + h->o_state);
    a.sstatus = (const int*)(h->ws + h->o_sstatus);
    a.slots = nullptr;
    a.budget = h->d.max_iter;
    a.fresh = 1;
    hipError_t e = launch_solve(h->d.dim, h->d.p_fine, h->f32, h->d.batch, hier_of(h, h->f32), a,
                                (hipStream_t)stream);
    return e == hipSuccess ? PMG_OK : hip_fail(e, "pmg_solve");
}

}  // extern "C"

// ---------------------------------------------------------------- solve without allocation

// The Krylov scratch of pmg_solve_noalloc: one fixed device array per GPU,
// reserved when the library's code object is loaded on that GPU and held
// until the process ends.  In host code `scratch` names a host-side shadow,
// not device memory: the device address is looked up once per device with
// hipGetSymbolAddress and only that address is used from then on.
static __device__ __align__(256) unsigned char scratch[PMG_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_device_ptr(void** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "pmg_solve_noalloc: hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(PMG_EDEVICE, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_fail(e, "pmg_solve_noalloc: hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return PMG_OK;
}

}  // namespace

extern "C" {

int pmg_solve_noalloc(pmg_handle* h, const double* d_b, double* d_x, pmg_info* d_info,
                      pmg_stream_t stream)
{
    int rc = check_h(h);
    if (rc) return rc;
    if (!d_b || !d_x || !d_info) return fail(PMG_EINVAL, "NULL argument");
    // the same regions pmg_solve takes from the handle's workspace, laid out
    // in the scratch array: V, Z, Hessenberg/Givens, FP64 fluxes, solve state
    const int dim = h->d.dim;
    const long long B = h->d.batch;
    const long long N = level_shape(dim, h->nlev - 1).N;
    Layout L;
    const size_t oV = L.take(sizeof(double) * (size_t)(B * h->nv * N));
    const size_t oZ = L.take(sizeof(double) * (size_t)(B * h->d.restart * N));
    const size_t oHs = L.take(sizeof(double) * (size_t)(B * h->hs));
    const long long NG = h->H64.lev[h->nlev - 1].ng;   // element nodes of the finest level
    const size_t oTR = L.take(sizeof(double) * (size_t)(B * dim * NG));
    const size_t oEX = h->K > 1 ? L.take(sizeof(double) * (size_t)(B * NG)) : 0;
    const size_t oSt = L.take(sizeof(SolveState) * (size_t)B);
    const size_t need = L.take(0);
    if (need > PMG_SCRATCH_BYTES)
        return fail(PMG_ENOMEM,
                    "pmg_solve_noalloc: this batch needs %zu bytes of Krylov scratch, more than "
                    "the library's fixed %zu (use a smaller batch or restart length, or pmg_solve)",
                    need, (size_t)PMG_SCRATCH_BYTES);
    void* base = nullptr;
    if ((rc = scratch_device_ptr(&base))) return rc;
    char* sp = (char*)base;
    SolveArgs a;
    a.b = d_b;
    a.x = d_x;
    a.V = (double*)(sp + oV);
    a.Z = (double*)(sp + oZ);
    a.Hs = (double*)(sp + oHs);
    a.TR64 = (double*)(sp + oTR);
    a.EX64 = h->K > 1 ? (double*)(sp + oEX) : nullptr;
    a.elem = h->K > 1;
    a.info = d_info;
    a.nv = h->nv;
    a.hs = h->hs;
    a.restart = h->d.restart;
    a.max_iter = h->d.max_iter;
    a.krylov = h->d.krylov;
    a.rtol = h->d.rtol;
    a.st = (SolveState*)(sp + oSt);   // written in full by the launch (fresh = 1)
    a.sstatus = (const int*)(h->ws + h->o_sstatus);
    a.slots = nullptr;
    a.budget = h->d.max_iter;
    a.fresh = 1;
    hipError_t e = launch_solve(dim, h->d.p_fine, h->f32, h->d.batch, hier_of(h, h->f32), a,
                                (hipStream_t)stream);
    return e == hipSuccess ? PMG_OK : hip_fail(e, "pmg_solve_noalloc");
}

int pmg_line_coefs(pmg_handle* h, int level, int dir, double* d_lo, double* d_di, double* d_up,
                   pmg_stream_t stream)
{
    int rc;
    if ((rc = check_h(h)) || (rc = check_level(h, level, 0))) return rc;
    if (dir < 0 || dir >= h->d.dim) return fail(PMG_EINVAL, "dir %d out of range", dir);
    if (!d_lo || !d_di || !d_up) return fail(PMG_EINVAL, "NULL argument");
    if (h->d.smoother == PMG_SMOOTHER_GLL_BAND2)
        return fail(PMG_EINVAL, "the handle's line systems are banded: use pmg_line_band");
    hipError_t e = launch_line_coefs(h->d.dim, 2 << level, h->d.batch, hier64_dev(h), h->d.smoother, dir,
                                     d_lo, d_di, d_up, (hipStream_t)stream);
    return e == hipSuccess ? PMG_OK : hip_fail(e, "pmg_line_coefs");
}

int pmg_line_band(pmg_handle* h, int level, int dir, double* d_band, pmg_stream_t stream)
{
    int rc;
    if ((rc = check_h(h)) || (rc = check_level(h, level, 0))) return rc;
    if (dir < 0 || dir >= h->d.dim) return fail(PMG_EINVAL, "dir %d out of range", dir);
    if (!d_band) return fail(PMG_EINVAL, "NULL argument");
    if (!h->o_bd64[level][dir])
        return fail(PMG_EINVAL, "the handle's smoother has no half-bandwidth-2 line systems");
    LevelShape sh = level_shape(h->d.dim, level);
    hipError_t e = hipMemcpyAsync(d_band, h->ws + h->o_bd64[level][dir],
                                  sizeof(double) * (size_t)h->d.batch * 5 * sh.n * sh.NL,
                                  hipMemcpyDeviceToDevice, (hipStream_t)stream);
    return e == hipSuccess ? PMG_OK : hip_fail(e, "pmg_line_band");
}

int pmg_geom(pmg_handle* h, int level, double* d_G, double* d_mass, pmg_stream_t stream)
{
    int rc;
    if ((rc = check_h(h)) || (rc = check_level(h, level, 0))) return rc;
    if (!d_G) return fail(PMG_EINVAL, "d_G is NULL");
    LevelShape sh = level_shape(h->d.dim, level);
    hipStream_t s = (hipStream_t)stream;
    size_t nG = sizeof(double) * (size_t)h->d.batch * sh.NC * elem_nodes(h, level);
    hipError_t e = hipMemcpyAsync(d_G, h->ws + h->o_G64[level], nG, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && d_mass) {
        if (level != h->nlev - 1) return fail(PMG_EINVAL, "mass is stored for the finest level only");
        e = hipMemcpyAsync(d_mass, h->ws + h->o_mass, sizeof(double) * (size_t)h->d.batch * sh.N,
                           hipMemcpyDeviceToDevice, s);
    }
    return e == hipSuccess ? PMG_OK : hip_fail(e, "pmg_geom");
}

int pmg_destroy(pmg_handle* h)
{
    delete h;
    return PMG_OK;
}


// ------------------------------------------------------------------ pools

struct pmg_pool {
    pmg_handle* h = nullptr;
    int iters = 1;
    CopyJob* hjobs = nullptr;   // pinned staging of an admission's copy jobs
    int* hslots = nullptr;      // pinned staging of an admission's slot list
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t graph_stream = nullptr;
};

static SolveArgs pool_solve_args(pmg_pool* P)
{
    pmg_handle* h = P->h;
    SolveArgs a;
    a.b = (const double*)(h->ws + h->o_b);
    a.x = (double*)(h->ws + h->o_x);
    a.V = (double*)(h->ws + h->o_V);
    a.Z = (double*)(h->ws + h->o_Z);
    a.Hs = (double*)(h->ws + h->o_Hs);
    a.TR64 = (double*)(h->ws + h->o_TR64);
    a.EX64 = h->o_EX64 ? (double*)(h->ws + h->o_EX64) : nullptr;
    a.elem = h->K > 1;
    a.info = (pmg_info*)(h->ws + h->o_info);
    a.nv = h->nv;
    a.hs = h->hs;
    a.restart = h->d.restart;
    a.max_iter = h->d.max_iter;
    a.krylov = h->d.krylov;
    a.rtol = h->d.rtol;
    a.st = (SolveState*)(h->ws + h->o_state);
    a.sstatus = (const int*)(h->ws + h->o_sstatus);
    a.slots = nullptr;
    a.budget = P->iters;
    a.fresh = 0;
    return a;
}

int pmg_pool_workspace_bytes(const pmg_desc* desc, size_t* bytes)
{
    int rc = check_desc(desc);
    if (rc) return rc;
    if (!bytes) return fail(PMG_EINVAL, "bytes is NULL");
    pmg_handle tmp;
    describe(&tmp, desc);
    tmp.pool = true;
    plan(&tmp);
    *bytes = tmp.total;
    return PMG_OK;
}

static void pool_capture(pmg_pool* P, hipStream_t s);

int pmg_pool_create(const pmg_desc* desc, int iters_per_step, void* d_ws, size_t ws_bytes,
                    pmg_stream_t stream, pmg_pool** out)
{
    if (!out) return fail(PMG_EINVAL, "out is NULL");
    if (iters_per_step < 1) return fail(PMG_EINVAL, "iters_per_step must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    pmg_handle* h = nullptr;
    int rc = init_handle(desc, d_ws, ws_bytes, true, s, &h);
    if (rc) return rc;
    hipError_t e = launch_pool_idle((SolveState*)(h->ws + h->o_state), desc->batch, s);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "pool init");
    }
    pmg_pool* P = new pmg_pool();
    P->h = h;
    P->iters = iters_per_step;
    const size_t njobs = (size_t)desc->batch * (h->nlev + 2);
    if ((e = hipHostMalloc((void**)&P->hjobs, sizeof(CopyJob) * njobs, hipHostMallocDefault)) !=
            hipSuccess ||
        (e = hipHostMalloc((void**)&P->hslots, sizeof(int) * desc->batch, hipHostMallocDefault)) !=
            hipSuccess) {
        pmg_pool_destroy(P);
        return hip_fail(e, "pool staging");
    }
    // the step graph is captured now, so that the first step of a serving
    // loop does not pay for its instantiation
    if (s) pool_capture(P, s);
    *out = P;
    return PMG_OK;
}

int pmg_pool_admit(pmg_pool* P, int n, const int* slots, const double* const* d_coords,
                   const double* const* d_f, const double* const* d_g, pmg_stream_t stream)
{
    if (!P) return fail(PMG_EINVAL, "pool is NULL");
    pmg_handle* h = P->h;
    const int B = h->d.batch, dim = h->d.dim;
    if (n == 0) return PMG_OK;
    if (n < 0 || n > B || !slots || !d_coords || !d_f || !d_g)
        return fail(PMG_EINVAL, "bad admission arguments");
    hipStream_t s = (hipStream_t)stream;
    const int N = level_shape(dim, h->nlev - 1).N;
    // the copies of every admitted request (coordinates per level, f, g)
    // into their slots' staging, as one launch of copy jobs; the pinned
    // staging is free again because every admission ends with a
    // synchronisation of its stream
    int nj = 0;
    for (int i = 0; i < n; ++i) {
        const int b = slots[i];
        if (b < 0 || b >= B) return fail(PMG_EINVAL, "slot %d out of range", b);
        for (int l = h->l0; l < h->nlev; ++l) {
            const long long cnt = (long long)dim * level_shape(dim, l).N;
            const double* src = d_coords[(size_t)i * h->nlev + l];
            if (!src) return fail(PMG_EINVAL, "NULL coordinates");
            P->hjobs[nj++] = {src, (double*)(h->ws + h->o_in_coords[l]) + cnt * b, cnt};
        }
        if (!d_f[i] || !d_g[i]) return fail(PMG_EINVAL, "NULL right-hand side or boundary data");
        P->hjobs[nj++] = {d_f[i], (double*)(h->ws + h->o_in_f) + (long long)N * b, N};
        P->hjobs[nj++] = {d_g[i], (double*)(h->ws + h->o_in_g) + (long long)N * b, N};
        P->hslots[i] = b;
    }
    CopyJob* djobs = (CopyJob*)(h->ws + h->o_jobs);
    hipError_t e = hipMemcpyAsync(djobs, P->hjobs, sizeof(CopyJob) * nj, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_copy_jobs(nj, djobs, s);
    if (e != hipSuccess) return hip_fail(e, "admission copies");
    int* dslots = (int*)(h->ws + h->o_slots);
    static_assert(sizeof(int) == 4, "int");
    e = hipMemcpyAsync(dslots, P->hslots, sizeof(int) * n, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "slot list upload");
    SetupArgs a;
    setup_args(h, a);
    for (int l = h->l0; l < h->nlev; ++l) a.coords[l] = (const double*)(h->ws + h->o_in_coords[l]);
    a.slots = dslots;
    a.nslots = n;
    pmg_info* info = (pmg_info*)(h->ws + h->o_info);
    e = launch_setup(dim, h->d.p_fine, h->nlev, B, a, info, s);
    for (int l = h->K > 1 ? h->l0 + 1 : 0; l < h->nlev && e == hipSuccess; ++l)   // lower first
        if (h->o_Cc[l])
            e = launch_collapse(dim, 2 << l, h->f32, h->K > 1, n, hier_of(h, h->f32),
                                (double*)(h->ws + h->o_Cc[l]), dslots, s);
    if (e == hipSuccess)
        e = launch_rhs(dim, h->d.p_fine, B, hier64_dev(h), (const double*)(h->ws + h->o_in_f),
                       (const double*)(h->ws + h->o_in_g), (double*)(h->ws + h->o_b),
                       (double*)(h->ws + h->o_V), h->nv * (long long)N, s, dslots, n);
    if (e == hipSuccess)
        e = launch_pool_start(dslots, n, (const int*)(h->ws + h->o_sstatus),
                              (SolveState*)(h->ws + h->o_state), info, s);
    // the staging and the device slot list are reused by the next admission
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? PMG_OK : hip_fail(e, "admission kernels");
}

// Capture the step (one launch of the resumable solve) into a graph on
// stream s; on failure the pool launches directly.
static void pool_capture(pmg_pool* P, hipStream_t s)
{
    pmg_handle* h = P->h;
    SolveArgs a = pool_solve_args(P);
    const void* H = hier_of(h, h->f32);
    hipError_t e;
    {
        // capture the step once; replays reuse it
        e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t el = launch_solve(h->d.dim, h->d.p_fine, h->f32, h->d.batch, H, a, s);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(s, &g);
            if (el == hipSuccess && e == hipSuccess && g) {
                e = hipGraphInstantiate(&P->exec, g, nullptr, nullptr, 0);
                if (e == hipSuccess) {
                    P->graph = g;
                    P->graph_stream = s;
                } else {
                    hipGraphDestroy(g);
                    P->exec = nullptr;
                }
            } else if (g) {
                hipGraphDestroy(g);
            }
        }
        (void)hipGetLastError();
    }
}

int pmg_pool_step(pmg_pool* P, pmg_stream_t stream)
{
    if (!P) return fail(PMG_EINVAL, "pool is NULL");
    pmg_handle* h = P->h;
    hipStream_t s = (hipStream_t)stream;
    SolveArgs a = pool_solve_args(P);
    const void* H = hier_of(h, h->f32);
    hipError_t e;
    if (s && !P->exec) pool_capture(P, s);
    if (P->exec)
        e = hipGraphLaunch(P->exec, s);
    else
        e = launch_solve(h->d.dim, h->d.p_fine, h->f32, h->d.batch, H, a, s);
    return e == hipSuccess ? PMG_OK : hip_fail(e, "pool step");
}

int pmg_pool_poll(pmg_pool* P, int* slot_status, pmg_info* info, pmg_stream_t stream)
{
    if (!P || !slot_status) return fail(PMG_EINVAL, "NULL argument");
    pmg_handle* h = P->h;
    const int B = h->d.batch;
    hipStream_t s = (hipStream_t)stream;
    std::vector<SolveState> st(B);
    hipError_t e = hipMemcpyAsync(st.data(), h->ws + h->o_state, sizeof(SolveState) * B,
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && info)
        e = hipMemcpyAsync(info, h->ws + h->o_info, sizeof(pmg_info) * B, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "pool poll");
    for (int b = 0; b < B; ++b) slot_status[b] = st[b].status;
    return PMG_OK;
}

int pmg_pool_take(pmg_pool* P, int slot, double* d_u, pmg_stream_t stream)
{
    if (!P || !d_u) return fail(PMG_EINVAL, "NULL argument");
    pmg_handle* h = P->h;
    if (slot < 0 || slot >= h->d.batch) return fail(PMG_EINVAL, "slot out of range");
    hipError_t e = launch_pool_take(h->d.dim, h->d.p_fine, slot, (const double*)(h->ws + h->o_x),
                                    (const double*)(h->ws + h->o_in_g), d_u,
                                    (SolveState*)(h->ws + h->o_state), (hipStream_t)stream);
    return e == hipSuccess ? PMG_OK : hip_fail(e, "pool take");
}

// Lift n finished slots at once: h_slots / h_outs are pinned host arrays
// that stay unchanged until the stream has copied them.
static int pool_take_many(pmg_pool* P, int n, const int* h_slots, double* const* h_outs,
                          hipStream_t s)
{
    pmg_handle* h = P->h;
    if (n <= 0) return PMG_OK;
    int* ds = (int*)(h->ws + h->o_take_slots);
    double** dout = (double**)(h->ws + h->o_take_outs);
    hipError_t e = hipMemcpyAsync(ds, h_slots, sizeof(int) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dout, h_outs, sizeof(double*) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = launch_pool_take_many(h->d.dim, h->d.p_fine, n, ds, dout,
                                  (const double*)(h->ws + h->o_x),
                                  (const double*)(h->ws + h->o_in_g),
                                  (SolveState*)(h->ws + h->o_state), s);
    return e == hipSuccess ? PMG_OK : hip_fail(e, "pool take");
}

int pmg_pool_destroy(pmg_pool* P)
{
    if (!P) return PMG_OK;
    if (P->exec) hipGraphExecDestroy(P->exec);
    if (P->graph) hipGraphDestroy(P->graph);
    if (P->hjobs) (void)hipHostFree(P->hjobs);
    if (P->hslots) (void)hipHostFree(P->hslots);
    delete P->h;
    delete P;
    return PMG_OK;
}

// ------------------------------------------------------------------ server

struct pmg_server {
    pmg_server_desc d;
    struct Req {
        long long ticket;
        int cls;
        std::vector<const double*> coords;
        const double* f;
        const double* g;
        double* u;
        int slot = -1;
        bool done = false;
        pmg_info info;
    };
    struct Class {
        pmg_pool* pool = nullptr;
        hipStream_t stream = nullptr;
        size_t footprint = 0;        // bytes per slot
        int resident = 0;            // solve workgroups the device holds at once
        std::vector<long long> slot_req;   // ticket per slot, -1 free
        int running = 0;
        int nlev = 0;
        // a step in flight: its slot states and infos arrive in pinned host
        // buffers, `done` is recorded after the copies
        bool inflight = false;
        hipEvent_t done = nullptr;
        SolveState* hst = nullptr;
        pmg_info* hinfo = nullptr;
        int* htake = nullptr;          // pinned slot / destination lists of a lift
        double** hout = nullptr;
    };
    Class cls[PMG_SERVER_MAX_CLASSES];
    std::vector<Req> reqs;           // indexed by ticket
    std::vector<long long> queue;    // arrival order
    std::vector<long long> retired;  // tickets retired and not yet drained
    std::vector<int> order;          // classes by per-slot footprint, largest first
    size_t in_use = 0;
    long long steps = 0;
    int finished = 0;
};

static int check_server_desc(const pmg_server_desc* d)
{
    if (!d) return fail(PMG_EINVAL, "desc is NULL");
    if (d->n_classes < 1 || d->n_classes > PMG_SERVER_MAX_CLASSES)
        return fail(PMG_EINVAL, "n_classes must be in [1, %d]", PMG_SERVER_MAX_CLASSES);
    if (d->iters_per_step < 1) return fail(PMG_EINVAL, "iters_per_step must be >= 1");
    for (int c = 0; c < d->n_classes; ++c) {
        int rc = check_desc(&d->classes[c]);
        if (rc) return rc;
    }
    return PMG_OK;
}

int pmg_server_workspace_bytes(const pmg_server_desc* d, size_t* bytes)
{
    int rc = check_server_desc(d);
    if (rc) return rc;
    if (!bytes) return fail(PMG_EINVAL, "bytes is NULL");
    size_t tot = 0;
    for (int c = 0; c < d->n_classes; ++c) {
        size_t b = 0;
        if ((rc = pmg_pool_workspace_bytes(&d->classes[c], &b))) return rc;
        tot += (b + 4095) & ~size_t(4095);
    }
    *bytes = tot;
    return PMG_OK;
}

int pmg_server_create(const pmg_server_desc* d, void* d_ws, size_t ws_bytes,
                      const pmg_stream_t* streams, pmg_server** out)
{
    int rc = check_server_desc(d);
    if (rc) return rc;
    if (!d_ws || !out || !streams) return fail(PMG_EINVAL, "NULL argument");
    size_t need = 0;
    pmg_server_workspace_bytes(d, &need);
    if (ws_bytes < need) return fail(PMG_ENOMEM, "server workspace too small: %zu < %zu", ws_bytes, need);
    pmg_server* S = new pmg_server();
    S->d = *d;
    char* base = (char*)d_ws;
    for (int c = 0; c < d->n_classes; ++c) {
        size_t b = 0;
        pmg_pool_workspace_bytes(&d->classes[c], &b);
        pmg_server::Class& C = S->cls[c];
        C.stream = (hipStream_t)streams[c];   // the caller's stream for this class
        hipError_t e;
        if ((rc = pmg_pool_create(&d->classes[c], d->iters_per_step, base, b, (pmg_stream_t)C.stream,
                                  &C.pool))) {
            pmg_server_destroy(S);
            return rc;
        }
        base += (b + 4095) & ~size_t(4095);
        const int B = d->classes[c].batch;
        if ((e = hipEventCreateWithFlags(&C.done, hipEventDisableTiming)) != hipSuccess ||
            (e = hipHostMalloc((void**)&C.hst, sizeof(SolveState) * B, hipHostMallocDefault)) !=
                hipSuccess ||
            (e = hipHostMalloc((void**)&C.hinfo, sizeof(pmg_info) * B, hipHostMallocDefault)) !=
                hipSuccess ||
            (e = hipHostMalloc((void**)&C.htake, sizeof(int) * B, hipHostMallocDefault)) !=
                hipSuccess ||
            (e = hipHostMalloc((void**)&C.hout, sizeof(double*) * B, hipHostMallocDefault)) !=
                hipSuccess) {
            pmg_server_destroy(S);
            return hip_fail(e, "server host buffers");
        }
        C.footprint = b / d->classes[c].batch;
        C.slot_req.assign(d->classes[c].batch, -1);
        C.nlev = ilog2(d->classes[c].p_fine);
    }
    // resident solve workgroups per class: CUs x workgroups per CU
    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 0;
        for (int c = 0; c < d->n_classes; ++c) {
            const pmg_desc& cd = d->classes[c];
            const int per = cd.inner_prec == PMG_F32 ? solve_blocks_per_cu_f32(cd.dim, cd.p_fine)
                                                     : solve_blocks_per_cu_f64(cd.dim, cd.p_fine);
            S->cls[c].resident = cus > 0 && per > 0 ? cus * per : INT_MAX;
        }
        (void)hipGetLastError();
    }
    // the heaviest problems are the longest single solves: their admissions
    // and steps are issued first so that they start first on the device
    for (int c = 0; c < d->n_classes; ++c) S->order.push_back(c);
    std::stable_sort(S->order.begin(), S->order.end(),
                     [S](int a, int b) { return S->cls[a].footprint > S->cls[b].footprint; });
    *out = S;
    return PMG_OK;
}

int pmg_server_submit(pmg_server* S, int c, const double* const* d_coords, const double* d_f,
                      const double* d_g, double* d_u, long long* ticket)
{
    if (!S || !d_coords || !d_f || !d_g || !d_u || !ticket) return fail(PMG_EINVAL, "NULL argument");
    if (c < 0 || c >= S->d.n_classes) return fail(PMG_EINVAL, "class %d out of range", c);
    pmg_server::Req r;
    r.ticket = (long long)S->reqs.size();
    r.cls = c;
    r.coords.assign(d_coords, d_coords + S->cls[c].nlev);
    r.f = d_f;
    r.g = d_g;
    r.u = d_u;
    memset(&r.info, 0, sizeof(r.info));
    S->reqs.push_back(r);
    S->queue.push_back(r.ticket);
    *ticket = r.ticket;
    return PMG_OK;
}

// Retire the finished slots of a class whose step has completed (its slot
// states are in C.hst): lift their solutions into the callers' buffers and
// free slots and budget.
static int server_retire(pmg_server* S, pmg_server::Class& C, int* done)
{
    int rc;
    const int B = (int)C.slot_req.size();
    std::vector<int> taken;
    for (int b = 0; b < B; ++b) {
        if (C.slot_req[b] < 0) continue;
        const int st = C.hst[b].status;
        if (st == ST_RUNNING || st == ST_IDLE) continue;
        pmg_server::Req& r = S->reqs[C.slot_req[b]];
        C.htake[taken.size()] = b;
        C.hout[taken.size()] = r.u;
        r.info = C.hinfo[b];
        r.info.status = st;
        taken.push_back(b);
    }
    if (taken.empty()) return PMG_OK;
    // one launch lifts every finished slot of the class
    if ((rc = pool_take_many(C.pool, (int)taken.size(), C.htake, C.hout, C.stream))) return rc;
    hipError_t e = hipStreamSynchronize(C.stream);   // only the lifts are queued
    if (e != hipSuccess) return hip_fail(e, "server retire");
    for (int b : taken) {
        S->reqs[C.slot_req[b]].done = true;
        S->retired.push_back(C.slot_req[b]);
        C.slot_req[b] = -1;
        C.running--;
        S->in_use -= C.footprint;
        S->finished++;
        ++*done;
    }
    return PMG_OK;
}

int pmg_server_step(pmg_server* S, int* n_done)
{
    if (!S) return fail(PMG_EINVAL, "server is NULL");
    int rc;
    const int nc = S->d.n_classes;
    int done = 0;
    // 1. collect the classes whose step has completed; if none has and some
    //    are in flight, wait a little for one (bounded, so that the caller
    //    can keep submitting arrivals)
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        bool any_inflight = false, any_ready = false;
        for (int c = 0; c < nc; ++c) {
            pmg_server::Class& C = S->cls[c];
            if (!C.inflight) continue;
            hipError_t q = hipEventQuery(C.done);
            if (q == hipErrorNotReady) {
                any_inflight = true;
                continue;
            }
            if (q != hipSuccess) return hip_fail(q, "server step");
            C.inflight = false;
            any_ready = true;
            if ((rc = server_retire(S, C, &done))) return rc;
        }
        if (any_ready || !any_inflight) break;
        if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(2)) break;
        std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    // 2. admissions in arrival order into idle classes, within slots and the
    //    byte budget (a request of a class whose step is in flight waits).
    //    A class is admitted into only while the classes of larger
    //    footprint run fewer requests than the device holds solve
    //    workgroups at once: the heaviest work fills the device by itself
    //    (no other class's working set in the caches beside it), lighter
    //    classes fill what it leaves free.
    std::vector<std::vector<int>> slots(nc);
    std::vector<std::vector<const double*>> coords(nc), fs(nc), gs(nc);
    std::vector<long long> keep;
    for (long long t : S->queue) {
        pmg_server::Req& r = S->reqs[t];
        pmg_server::Class& C = S->cls[r.cls];
        int free_slot = -1;
        int heavier = 0;
        for (int k : S->order) {
            if (k == r.cls) break;
            heavier += S->cls[k].running;
        }
        if (!C.inflight && S->in_use + C.footprint <= S->d.budget_bytes && heavier < C.resident) {
            for (int b = 0; b < (int)C.slot_req.size(); ++b)
                if (C.slot_req[b] < 0) { free_slot = b; break; }
        }
        if (free_slot < 0) { keep.push_back(t); continue; }
        C.slot_req[free_slot] = t;
        r.slot = free_slot;
        S->in_use += C.footprint;
        C.running++;
        slots[r.cls].push_back(free_slot);
        coords[r.cls].insert(coords[r.cls].end(), r.coords.begin(), r.coords.end());
        fs[r.cls].push_back(r.f);
        gs[r.cls].push_back(r.g);
    }
    S->queue.swap(keep);
    for (int c : S->order)
        if (!slots[c].empty() &&
            (rc = pmg_pool_admit(S->cls[c].pool, (int)slots[c].size(), slots[c].data(),
                                 coords[c].data(), fs[c].data(), gs[c].data(),
                                 (pmg_stream_t)S->cls[c].stream)))
            return rc;
    // 3. launch a step of every idle class with running slots; each class runs
    //    on its own stream, so fast classes are not held by slow ones
    for (int c : S->order) {
        pmg_server::Class& C = S->cls[c];
        if (C.inflight || C.running == 0) continue;
        if ((rc = pmg_pool_step(C.pool, (pmg_stream_t)C.stream))) return rc;
        pmg_handle* h = C.pool->h;
        const int B = h->d.batch;
        hipError_t e = hipMemcpyAsync(C.hst, h->ws + h->o_state, sizeof(SolveState) * B,
                                      hipMemcpyDeviceToHost, C.stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(C.hinfo, h->ws + h->o_info, sizeof(pmg_info) * B,
                               hipMemcpyDeviceToHost, C.stream);
        if (e == hipSuccess) e = hipEventRecord(C.done, C.stream);
        if (e != hipSuccess) return hip_fail(e, "server launch");
        C.inflight = true;
    }
    S->steps++;
    if (n_done) *n_done = done;
    return PMG_OK;
}

int pmg_server_poll(pmg_server* S, long long ticket, pmg_info* info)
{
    if (!S || ticket < 0 || ticket >= (long long)S->reqs.size()) return fail(PMG_EINVAL, "bad ticket");
    const pmg_server::Req& r = S->reqs[ticket];
    if (!r.done) return 0;
    if (info) *info = r.info;
    return 1;
}

int pmg_server_drain(pmg_server* S, long long* tickets, int max, int* n)
{
    if (!S || !n || max < 0 || (max > 0 && !tickets)) return fail(PMG_EINVAL, "bad argument");
    const int k = (int)std::min<size_t>((size_t)max, S->retired.size());
    std::copy(S->retired.begin(), S->retired.begin() + k, tickets);
    S->retired.erase(S->retired.begin(), S->retired.begin() + k);
    *n = k;
    return PMG_OK;
}

int pmg_server_stats_get(pmg_server* S, pmg_server_stats* st)
{
    if (!S || !st) return fail(PMG_EINVAL, "NULL argument");
    st->queued = (int)S->queue.size();
    int running = 0;
    for (int c = 0; c < S->d.n_classes; ++c) running += S->cls[c].running;
    st->running = running;
    st->finished = S->finished;
    st->bytes_in_use = S->in_use;
    st->steps = S->steps;
    return PMG_OK;
}

int pmg_server_destroy(pmg_server* S)
{
    if (!S) return PMG_OK;
    for (int c = 0; c < PMG_SERVER_MAX_CLASSES; ++c) {
        pmg_server::Class& C = S->cls[c];
        if (C.stream) hipStreamSynchronize(C.stream);
        if (C.pool) pmg_pool_destroy(C.pool);
        if (C.done) hipEventDestroy(C.done);
        if (C.hst) hipHostFree(C.hst);
        if (C.hinfo) hipHostFree(C.hinfo);
        if (C.htake) hipHostFree(C.htake);
        if (C.hout) hipHostFree(C.hout);
        // the class streams belong to the caller
    }
    delete S;
    return PMG_OK;
}

}  // extern "C"

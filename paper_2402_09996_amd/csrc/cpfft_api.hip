// Host side of the solver and the C-ABI declared in include/cpfft.h.
//
// One load step runs the Green-operator fixed point on the device: each
// iteration is x pass (law + x transforms) -> y pass -> z pass with Gamma0
// -> inverse y pass -> boundary update.  Iterations are queued in chunks
// and every kernel returns at once when the device flag says the step has
// ended, so the host only polls the step status between chunks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/cpfft.h"
#include "cpfft_kernels.hpp"

using namespace cpf;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(call)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(CPF_E_HIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),  \
                        __FILE__, __LINE__);                                               \
    } while (0)

extern "C" int cpf_version(void) { return CPF_VERSION; }

extern "C" const char *cpf_error_string(int code)
{
    switch (code) {
    case CPF_OK: return "ok";
    case CPF_E_INVALID_ARG: return "invalid argument";
    case CPF_E_WORKSPACE: return "workspace missing or too small";
    case CPF_E_HIP: return "HIP runtime error";
    case CPF_E_NOT_CONVERGED: return "fixed point did not converge";
    case CPF_E_NAN: return "non-finite values";
    case CPF_E_UNSUPPORTED_SIZE: return "unsupported grid size";
    case CPF_E_BAD_STATE: return "solver not bound or in a bad state";
    default: return "unknown error";
    }
}

extern "C" const char *cpf_last_error_message(void) { return g_err.c_str(); }

extern "C" void cpf_options_default(cpf_options *o)
{
    if (!o) return;
    o->precision = CPF_PREC_FP64;
    o->tol = 1e-8;
    o->max_iter = 1000;
    o->h_max = 0.05;
    o->rk4_M = 0;
    o->lam0 = 0.0;
    o->mu0 = 0.0;
    o->stag_tol = 0.0;
    o->check_every = 0;
}

// ---------------------------------------------------------------------------
// problem
// ---------------------------------------------------------------------------
struct cpf_problem {
    int nx, ny, nz, nlab, nsys;
    std::vector<int32_t> labels;
    std::vector<double> Q;      // [nlab][9], v_lab = Q v_crystal
    double Cv[36];
    std::vector<double> m;      // [nsys][6] crystal Schmid tensors (tensor comps)
    std::vector<double> tau0;
    std::vector<int> fam;
    cpf_law law[2];
    int twin_mode;
    double Kc, fm, gT, eta;
    int n_slip, n_twin;
};

static bool radix_plan(int n, FftPlan &P)
{
    P.n = n;
    P.npass = 0;
    int r = n;
    while (r % 8 == 0) { P.radix[P.npass++] = 8; r /= 8; }
    if (r % 4 == 0) { P.radix[P.npass++] = 4; r /= 4; }
    if (r % 2 == 0) { P.radix[P.npass++] = 2; r /= 2; }
    while (r % 3 == 0 && P.npass < MAXPASS) { P.radix[P.npass++] = 3; r /= 3; }
    return r == 1 && n >= 2;
}

static bool finite_all(const double *a, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

extern "C" int cpf_problem_create(const cpf_problem_desc *d, cpf_problem **out)
{
    if (!d || !out) return fail(CPF_E_INVALID_ARG, "null argument");
    *out = nullptr;
    FftPlan tmp;
    const int dims[3] = {d->nx, d->ny, d->nz};
    for (int i = 0; i < 3; ++i)
        if (dims[i] < 2 || dims[i] > 256 || !radix_plan(dims[i], tmp))
            return fail(CPF_E_UNSUPPORTED_SIZE, "grid dimension %d: need 2^a 3^b in [2, 256]", dims[i]);
    if (!d->labels || !d->euler || !d->n_miller || !d->l_miller || !d->family || !d->tau0)
        return fail(CPF_E_INVALID_ARG, "null array in problem description");
    if (d->n_labels < 1) return fail(CPF_E_INVALID_ARG, "n_labels must be >= 1");
    if (d->n_sys < 1 || d->n_sys > CPF_MAX_SYSTEMS)
        return fail(CPF_E_INVALID_ARG, "n_sys must be in [1, %d]", CPF_MAX_SYSTEMS);
    if (d->twin_mode != CPF_TWIN_NORTON && d->twin_mode != CPF_TWIN_PAPER)
        return fail(CPF_E_INVALID_ARG, "unknown twin_mode %d", d->twin_mode);
    if (!(d->eta >= 0.0) || !finite_all(d->C_crystal, 36) || !(d->gamma_T > 0.0))
        return fail(CPF_E_INVALID_ARG, "eta must be >= 0, gamma_T > 0 and C finite");
    for (int f = 0; f < 2; ++f) {
        const cpf_law &L = d->law[f];
        const double v[8] = {L.Q, L.b, L.c, L.d, L.K, L.n, L.q_self, L.q_latent};
        if (!finite_all(v, 8) || !(L.n > 0.0) || !(L.K > 0.0))
            return fail(CPF_E_INVALID_ARG, "law of family %d: need finite values, K > 0, n > 0", f);
    }
    cpf_problem *p = new (std::nothrow) cpf_problem();
    if (!p) return fail(CPF_E_INVALID_ARG, "out of host memory");
    p->nx = d->nx; p->ny = d->ny; p->nz = d->nz;
    p->nlab = d->n_labels;
    p->nsys = d->n_sys;
    const size_t nvox = (size_t)d->nx * d->ny * d->nz;
    p->labels.assign(d->labels, d->labels + nvox);
    for (size_t i = 0; i < nvox; ++i)
        if (p->labels[i] < 0 || p->labels[i] >= d->n_labels) {
            delete p;
            return fail(CPF_E_INVALID_ARG, "label %d at voxel %zu outside [0, %d)", d->labels[i], i,
                        d->n_labels);
        }
    p->Q.resize((size_t)p->nlab * 9);
    for (int l = 0; l < p->nlab; ++l) {
        const double a = d->euler[3 * l], b = d->euler[3 * l + 1], c = d->euler[3 * l + 2];
        const double c1 = cos(a), s1 = sin(a), cP = cos(b), sP = sin(b), c2 = cos(c), s2 = sin(c);
        double *Q = &p->Q[9 * l];
        // Q = Rz(phi1) Rx(Phi) Rz(phi2)
        Q[0] = c1 * c2 - s1 * cP * s2; Q[1] = -c1 * s2 - s1 * cP * c2; Q[2] = s1 * sP;
        Q[3] = s1 * c2 + c1 * cP * s2; Q[4] = -s1 * s2 + c1 * cP * c2; Q[5] = -c1 * sP;
        Q[6] = sP * s2;                Q[7] = sP * c2;                 Q[8] = cP;
    }
    memcpy(p->Cv, d->C_crystal, sizeof p->Cv);
    p->m.resize((size_t)p->nsys * 6);
    p->tau0.assign(d->tau0, d->tau0 + p->nsys);
    p->fam.assign(d->family, d->family + p->nsys);
    p->n_slip = p->n_twin = 0;
    for (int s = 0; s < p->nsys; ++s) {
        double n[3], l[3];
        double nn = 0, ll = 0, nl = 0;
        for (int i = 0; i < 3; ++i) {
            n[i] = d->n_miller[3 * s + i];
            l[i] = d->l_miller[3 * s + i];
            nn += n[i] * n[i]; ll += l[i] * l[i]; nl += n[i] * l[i];
        }
        if (!(nn > 0) || !(ll > 0) || fabs(nl) > 1e-9 * sqrt(nn * ll) || (p->fam[s] != 0 && p->fam[s] != 1)) {
            delete p;
            return fail(CPF_E_INVALID_ARG, "system %d: need nonzero orthogonal n, l and family 0/1", s);
        }
        for (int i = 0; i < 3; ++i) { n[i] /= sqrt(nn); l[i] /= sqrt(ll); }
        double *m = &p->m[6 * s];
        m[0] = n[0] * l[0]; m[1] = n[1] * l[1]; m[2] = n[2] * l[2];
        m[3] = 0.5 * (n[1] * l[2] + n[2] * l[1]);
        m[4] = 0.5 * (n[0] * l[2] + n[2] * l[0]);
        m[5] = 0.5 * (n[0] * l[1] + n[1] * l[0]);
        (p->fam[s] ? p->n_twin : p->n_slip)++;
    }
    p->law[0] = d->law[0];
    p->law[1] = d->law[1];
    p->twin_mode = d->twin_mode;
    p->Kc = d->K_c; p->fm = d->f_m; p->gT = d->gamma_T; p->eta = d->eta;
    *out = p;
    return CPF_OK;
}

extern "C" void cpf_problem_destroy(cpf_problem *p) { delete p; }

// Symmetric eigenvalues by cyclic Jacobi (small matrices).
static void jacobi_eigs(int n, double *A, double *w)
{
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) off += A[i * n + j] * A[i * n + j];
        if (off < 1e-30) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[p * n + q];
                if (fabs(apq) < 1e-300) continue;
                const double th = (A[q * n + q] - A[p * n + p]) / (2 * apq);
                const double t = (th >= 0 ? 1 : -1) / (fabs(th) + sqrt(th * th + 1));
                const double c = 1 / sqrt(t * t + 1), s = t * c;
                for (int k = 0; k < n; ++k) {
                    const double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    const double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
            }
    }
    for (int i = 0; i < n; ++i) w[i] = A[i * n + i];
}

extern "C" int cpf_problem_reference_medium(const cpf_problem *p, double *lam0, double *mu0)
{
    if (!p || !lam0 || !mu0) return fail(CPF_E_INVALID_ARG, "null argument");
    // Mandel form of the crystal stiffness
    const double w[6] = {1, 1, 1, M_SQRT2, M_SQRT2, M_SQRT2};
    double CM[36];
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) CM[i * 6 + j] = w[i] * w[j] * p->Cv[i * 6 + j];
    double k0 = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) k0 += CM[i * 6 + j];
    k0 /= 9.0;
    // orthonormal deviatoric basis
    double B[5][6] = {{0}};
    B[0][0] = 1 / M_SQRT2; B[0][1] = -1 / M_SQRT2;
    B[1][0] = B[1][1] = 1 / sqrt(6.0); B[1][2] = -2 / sqrt(6.0);
    B[2][3] = B[3][4] = B[4][5] = 1.0;
    double M5[25];
    for (int a = 0; a < 5; ++a)
        for (int b = 0; b < 5; ++b) {
            double s = 0;
            for (int i = 0; i < 6; ++i)
                for (int j = 0; j < 6; ++j) s += B[a][i] * CM[i * 6 + j] * B[b][j];
            M5[a * 5 + b] = s;
        }
    double ev[5];
    jacobi_eigs(5, M5, ev);
    const double lo = *std::min_element(ev, ev + 5), hi = *std::max_element(ev, ev + 5);
    *mu0 = 0.25 * (lo + hi);
    *lam0 = k0 - 2.0 * (*mu0) / 3.0;
    return CPF_OK;
}

// ---------------------------------------------------------------------------
// solver
// ---------------------------------------------------------------------------
struct cpf_solver {
    cpf_problem pb;
    cpf_options opt;
    int prec;
    int nx, ny, nz, nhx;
    long nvox;
    int D;
    FftPlan px, py, pz;
    int L, tpbx, nbx, ty, nty, tz, ntz, nbz;
    size_t lds_x, lds_y, lds_z;
    double lam0, mu0, K0[36];
    int ns_inst;
    int law_spec;     // LAW_GENERAL or LAW_TABLE1
    // workspace
    unsigned char *ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    bool bound = false;
    size_t off_labels, off_Q, off_eps[2], off_st[2], off_spec, off_tw[3], off_px, off_pz, off_sc, total;
    int eps_cur = 0, st_cur = 0;
    double Sigma_n[6], E_n[6];
    int prev_iters = 8;
    Scalars *hsc = nullptr;   // pinned host mirror
    // kernel timing
    bool timing = false;
    double t_ms[CPF_NKERNELS] = {0};
    long long t_n[CPF_NKERNELS] = {0};
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
};

static int timed_begin(cpf_solver *s, hipEvent_t *a, hipEvent_t *b)
{
    if (!s->timing) return CPF_OK;
    for (hipEvent_t *e : {a, b}) {
        if (s->ev_pool.empty()) {
            HIPCHK(hipEventCreate(e));
        } else {
            *e = s->ev_pool.back();
            s->ev_pool.pop_back();
        }
    }
    HIPCHK(hipEventRecord(*a, s->stream));
    return CPF_OK;
}

static int timed_end(cpf_solver *s, int k, hipEvent_t a, hipEvent_t b)
{
    if (!s->timing) return CPF_OK;
    HIPCHK(hipEventRecord(b, s->stream));
    s->ev_pending.push_back({k, {a, b}});
    return CPF_OK;
}

// After a stream synchronization: fold the pending event pairs into the counters.
static int timed_collect(cpf_solver *s)
{
    for (auto &p : s->ev_pending) {
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, p.second.first, p.second.second));
        s->t_ms[p.first] += ms;
        s->t_n[p.first] += 1;
        s->ev_pool.push_back(p.second.first);
        s->ev_pool.push_back(p.second.second);
    }
    s->ev_pending.clear();
    return CPF_OK;
}

#define TIMED(s, k, launch)                                   \
    do {                                                      \
        hipEvent_t ea_ = nullptr, eb_ = nullptr;              \
        int rc_ = timed_begin(s, &ea_, &eb_);                 \
        if (rc_) return rc_;                                  \
        launch;                                               \
        rc_ = timed_end(s, k, ea_, eb_);                      \
        if (rc_) return rc_;                                  \
    } while (0)

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

template <typename R>
static void layout(cpf_solver *s)
{
    const size_t cb = sizeof(C2<R>);
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
    s->off_labels = take(sizeof(int32_t) * s->nvox);
    s->off_Q = take(sizeof(R) * 9 * s->pb.nlab);
    s->off_eps[0] = take(sizeof(R) * 6 * s->nvox);
    s->off_eps[1] = take(sizeof(R) * 6 * s->nvox);
    s->off_st[0] = take(sizeof(R) * s->D * s->nvox);
    s->off_st[1] = take(sizeof(R) * s->D * s->nvox);
    s->off_spec = take(cb * 6 * (size_t)s->nz * s->ny * s->nhx);
    s->off_tw[0] = take(cb * s->nx);
    s->off_tw[1] = take(cb * s->ny);
    s->off_tw[2] = take(cb * s->nz);
    s->off_px = take(sizeof(double) * NPX * s->nbx);
    s->off_pz = take(sizeof(double) * s->nbz);
    s->off_sc = take(sizeof(Scalars));
    s->total = o;
}

template <typename R>
static void tiling(cpf_solver *s)
{
    const size_t cb = sizeof(C2<R>);
    const bool f32 = sizeof(R) == 4;
    s->L = std::max(1, 256 / s->nx);
    s->tpbx = s->L * s->nx;
    s->nbx = (s->ny * s->nz + s->L - 1) / s->L;
    s->lds_x = 3 * (size_t)s->tpbx * cb;
    const int ty_max = f32 ? 16 : 8;
    s->ty = std::min(std::min(ty_max, std::max(1, 16 * 256 / s->ny)), s->nhx);
    s->nty = (s->nhx + s->ty - 1) / s->ty;
    s->lds_y = (size_t)s->ty * (s->ny + 1) * cb;
    const int ept_z = f32 ? 24 : 12;
    s->tz = std::min(std::min(16, std::max(1, ept_z * 256 / (6 * s->nz))), s->nhx);
    s->ntz = (s->nhx + s->tz - 1) / s->tz;
    s->nbz = s->ntz * s->ny;
    s->lds_z = 6 * (size_t)s->tz * (s->nz + 1) * cb;
}

// The specialized law kernel applies when the systems are those of Table 1
// in order (12 slip, or 12 slip + 4 twin) and the crystal stiffness has the
// orthotropic zero pattern (no normal-shear or shear-shear coupling).
static bool table1_specializable(const cpf_problem &p)
{
    if (p.nsys != 12 && p.nsys != 16) return false;
    for (int s = 0; s < p.nsys; ++s) {
        if (p.fam[s] != (s < 12 ? 0 : 1)) return false;
        for (int i = 0; i < 6; ++i)
            if (fabs(p.m[6 * s + i] - T1_M[s][i]) > 1e-12) return false;
    }
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            const bool nz = (i < 3 && j < 3) || i == j;
            if (!nz && p.Cv[i * 6 + j] != 0.0) return false;
        }
    return true;
}

extern "C" int cpf_solver_create(const cpf_problem *p, const cpf_options *opt, cpf_solver **out)
{
    if (!p || !out) return fail(CPF_E_INVALID_ARG, "null argument");
    *out = nullptr;
    cpf_options o;
    cpf_options_default(&o);
    if (opt) o = *opt;
    if (o.precision != CPF_PREC_FP64 && o.precision != CPF_PREC_FP32)
        return fail(CPF_E_INVALID_ARG, "unknown precision %d", o.precision);
    if (!(o.tol > 0) || o.max_iter < 1 || (o.rk4_M <= 0 && !(o.h_max > 0)) || o.rk4_M > 100000)
        return fail(CPF_E_INVALID_ARG, "need tol > 0, max_iter >= 1 and rk4_M > 0 or h_max > 0");
    cpf_solver *s = new (std::nothrow) cpf_solver();
    if (!s) return fail(CPF_E_INVALID_ARG, "out of host memory");
    s->pb = *p;
    s->opt = o;
    s->prec = o.precision;
    s->nx = p->nx; s->ny = p->ny; s->nz = p->nz;
    s->nhx = p->nx / 2 + 1;
    s->nvox = (long)p->nx * p->ny * p->nz;
    s->D = 6 + 2 * p->nsys;
    radix_plan(s->nx, s->px);
    radix_plan(s->ny, s->py);
    radix_plan(s->nz, s->pz);
    s->ns_inst = p->nsys <= 4 ? 4 : p->nsys <= 12 ? 12 : p->nsys <= 16 ? 16 : 32;
    s->law_spec = table1_specializable(*p) ? LAW_TABLE1 : LAW_GENERAL;
    if (s->prec == CPF_PREC_FP64) { tiling<double>(s); layout<double>(s); }
    else { tiling<float>(s); layout<float>(s); }
    if (o.mu0 > 0) {
        s->lam0 = o.lam0;
        s->mu0 = o.mu0;
    } else {
        cpf_problem_reference_medium(p, &s->lam0, &s->mu0);
    }
    if (!(s->mu0 > 0) || !(s->lam0 + 2 * s->mu0 / 3 > 0)) {
        delete s;
        return fail(CPF_E_INVALID_ARG, "reference medium not positive definite");
    }
    for (int i = 0; i < 36; ++i) s->K0[i] = 0;
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) s->K0[i * 6 + j] = s->lam0;
        s->K0[i * 6 + i] = s->lam0 + 2 * s->mu0;
        s->K0[(i + 3) * 6 + i + 3] = 2 * s->mu0;
    }
    *out = s;
    return CPF_OK;
}

extern "C" int cpf_solver_workspace_size(const cpf_solver *s, size_t *bytes)
{
    if (!s || !bytes) return fail(CPF_E_INVALID_ARG, "null argument");
    *bytes = s->total;
    return CPF_OK;
}

extern "C" void cpf_solver_destroy(cpf_solver *s)
{
    if (!s) return;
    if (s->hsc) (void)hipHostFree(s->hsc);
    for (auto &p : s->ev_pending) {
        (void)hipEventDestroy(p.second.first);
        (void)hipEventDestroy(p.second.second);
    }
    for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
    delete s;
}

extern "C" int cpf_solver_set_timing(cpf_solver *s, int enable)
{
    if (!s) return fail(CPF_E_INVALID_ARG, "null solver");
    if (s->bound) HIPCHK(hipStreamSynchronize(s->stream));
    int rc = timed_collect(s);
    if (rc) return rc;
    s->timing = enable != 0;
    for (int k = 0; k < CPF_NKERNELS; ++k) {
        s->t_ms[k] = 0.0;
        s->t_n[k] = 0;
    }
    return CPF_OK;
}

extern "C" int cpf_solver_get_timing(const cpf_solver *s, double *ms, long long *n)
{
    if (!s || !ms || !n) return fail(CPF_E_INVALID_ARG, "null argument");
    for (int k = 0; k < CPF_NKERNELS; ++k) {
        ms[k] = s->t_ms[k];
        n[k] = s->t_n[k];
    }
    return CPF_OK;
}

template <typename R>
static R *dptr(cpf_solver *s, size_t off) { return reinterpret_cast<R *>(s->ws + off); }

template <typename R>
static LawP<R> make_law(const cpf_solver *s)
{
    const cpf_problem &p = s->pb;
    LawP<R> P;
    memset(&P, 0, sizeof P);
    P.nsys = p.nsys;
    P.twin_mode = p.twin_mode;
    P.twin_mask = 0;
    for (int I = 0; I < 6; ++I)
        for (int J = 0; J < 6; ++J) P.C[I * 6 + J] = R(p.Cv[I * 6 + J] * (J < 3 ? 1.0 : 2.0));
    for (int sy = 0; sy < NSMAX; ++sy) {
        if (sy < p.nsys) {
            for (int i = 0; i < 6; ++i) P.m[sy][i] = R(p.m[6 * sy + i]);
            P.tau0[sy] = R(p.tau0[sy]);
            if (p.fam[sy]) P.twin_mask |= 1u << sy;
        } else {
            for (int i = 0; i < 6; ++i) P.m[sy][i] = R(0);
            P.tau0[sy] = R(1e30);   // padding systems never activate
        }
    }
    for (int f = 0; f < 2; ++f) {
        const cpf_law &L = p.law[f];
        FamP<R> F;
        F.QL = R(L.Q * L.q_latent);
        F.QD = R(L.Q * (L.q_self - L.q_latent));
        F.bl2e = R(L.b * 1.442695040888963407359924681001892137);
        F.c = R(L.c); F.d = R(L.d);
        F.K = R(L.K); F.invK = R(1.0 / L.K);
        F.n = R(L.n); F.inv_n = R(1.0 / L.n); F.nm1 = R(L.n - 1.0);
        F.nm1_int = (L.n == floor(L.n) && L.n >= 1.0 && L.n <= 64.0) ? (int)L.n - 1 : -1;
        (f ? P.ft : P.fs) = F;
    }
    P.Kc_gT = R(p.Kc * p.gT); P.fm = R(p.fm); P.inv_gT = R(1.0 / p.gT);
    P.eta = R(p.eta); P.inv_eta = R(p.eta > 0 ? 1.0 / p.eta : 0.0);
    P.newton_rtol = sizeof(R) == 4 ? R(1e-5) : R(1e-13);
    return P;
}

template <typename R>
static int zero_state(cpf_solver *s)
{
    const long n6 = 6 * s->nvox, nD = (long)s->D * s->nvox;
    hipLaunchKernelGGL(k_fill<R>, dim3(1024), dim3(256), 0, s->stream, dptr<R>(s, s->off_eps[0]), n6, R(0));
    hipLaunchKernelGGL(k_fill<R>, dim3(1024), dim3(256), 0, s->stream, dptr<R>(s, s->off_eps[1]), n6, R(0));
    hipLaunchKernelGGL(k_fill<R>, dim3(1024), dim3(256), 0, s->stream, dptr<R>(s, s->off_st[0]), nD, R(0));
    hipLaunchKernelGGL(k_fill<R>, dim3(1024), dim3(256), 0, s->stream, dptr<R>(s, s->off_st[1]), nD, R(0));
    HIPCHK(hipGetLastError());
    s->eps_cur = s->st_cur = 0;
    for (int i = 0; i < 6; ++i) s->Sigma_n[i] = s->E_n[i] = 0.0;
    s->prev_iters = 8;
    return CPF_OK;
}

template <typename R>
static int bind_impl(cpf_solver *s)
{
    const cpf_problem &p = s->pb;
    std::vector<R> Qr(p.Q.size());
    for (size_t i = 0; i < Qr.size(); ++i) Qr[i] = R(p.Q[i]);
    HIPCHK(hipMemcpyAsync(s->ws + s->off_labels, p.labels.data(), sizeof(int32_t) * s->nvox,
                          hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(s->ws + s->off_Q, Qr.data(), sizeof(R) * Qr.size(), hipMemcpyHostToDevice,
                          s->stream));
    const int ns[3] = {s->nx, s->ny, s->nz};
    std::vector<C2<R>> tw[3];
    for (int a = 0; a < 3; ++a) {
        tw[a].resize(ns[a]);
        for (int k = 0; k < ns[a]; ++k) {
            const long double ang = -2.0L * 3.141592653589793238462643383279502884L * k / ns[a];
            tw[a][k] = C2<R>{R(cosl(ang)), R(sinl(ang))};
        }
        HIPCHK(hipMemcpyAsync(s->ws + s->off_tw[a], tw[a].data(), sizeof(C2<R>) * ns[a],
                              hipMemcpyHostToDevice, s->stream));
    }
    int rc = zero_state<R>(s);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(s->stream));
    return CPF_OK;
}

extern "C" int cpf_solver_bind(cpf_solver *s, void *ws, size_t bytes, void *stream)
{
    if (!s) return fail(CPF_E_INVALID_ARG, "null solver");
    if (!ws || bytes < s->total)
        return fail(CPF_E_WORKSPACE, "workspace of %zu bytes given, %zu needed", bytes, s->total);
    if (((uintptr_t)ws) & 255) return fail(CPF_E_WORKSPACE, "workspace must be 256-byte aligned");
    s->ws = (unsigned char *)ws;
    s->ws_bytes = bytes;
    s->stream = (hipStream_t)stream;
    if (!s->hsc) HIPCHK(hipHostMalloc((void **)&s->hsc, sizeof(Scalars), hipHostMallocDefault));
    int rc = s->prec == CPF_PREC_FP64 ? bind_impl<double>(s) : bind_impl<float>(s);
    s->bound = rc == CPF_OK;
    return rc;
}

extern "C" int cpf_solver_reset(cpf_solver *s)
{
    if (!s || !s->bound) return fail(CPF_E_BAD_STATE, "solver not bound");
    int rc = s->prec == CPF_PREC_FP64 ? zero_state<double>(s) : zero_state<float>(s);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(s->stream));
    return CPF_OK;
}

static int substeps(double dt, double hmax) { return std::max(1, (int)ceil(dt / hmax * (1.0 - 1e-12))); }

// Gauss-Jordan inverse of the S x S block of K0, embedded in 6 x 6.
static void stress_block_inverse(const double K0[36], const int sidx[6], double out[36])
{
    int S[6], n = 0;
    for (int i = 0; i < 6; ++i)
        if (sidx[i]) S[n++] = i;
    double A[6][12] = {{0}};
    for (int a = 0; a < n; ++a) {
        for (int b = 0; b < n; ++b) A[a][b] = K0[S[a] * 6 + S[b]];
        A[a][n + a] = 1.0;
    }
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
        for (int k = 0; k < 2 * n; ++k) std::swap(A[c][k], A[piv][k]);
        const double d = A[c][c];
        for (int k = 0; k < 2 * n; ++k) A[c][k] /= d;
        for (int r = 0; r < n; ++r)
            if (r != c) {
                const double f = A[r][c];
                for (int k = 0; k < 2 * n; ++k) A[r][k] -= f * A[c][k];
            }
    }
    for (int i = 0; i < 36; ++i) out[i] = 0.0;
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) out[S[a] * 6 + S[b]] = A[a][n + b];
}

template <typename R, int NS, int SPEC>
static void launch_xiter(cpf_solver *s, const XArgs<R> &a, const LawP<R> &P, int first)
{
    hipLaunchKernelGGL((k_xpass_iter<R, NS, SPEC>), dim3(s->nbx), dim3(s->tpbx), s->lds_x, s->stream, a, P,
                       s->px, first);
}

template <typename R>
static void launch_xiter_any(cpf_solver *s, const XArgs<R> &a, const LawP<R> &P, int first)
{
    if (s->law_spec == LAW_TABLE1) {
        if (s->ns_inst == 12) launch_xiter<R, 12, LAW_TABLE1>(s, a, P, first);
        else launch_xiter<R, 16, LAW_TABLE1>(s, a, P, first);
        return;
    }
    switch (s->ns_inst) {
    case 4: launch_xiter<R, 4, LAW_GENERAL>(s, a, P, first); break;
    case 12: launch_xiter<R, 12, LAW_GENERAL>(s, a, P, first); break;
    case 16: launch_xiter<R, 16, LAW_GENERAL>(s, a, P, first); break;
    default: launch_xiter<R, 32, LAW_GENERAL>(s, a, P, first); break;
    }
}

template <typename R>
static GreenArgs<R> green_args(const cpf_solver *s)
{
    GreenArgs<R> g;
    g.nx = s->nx; g.ny = s->ny; g.nz = s->nz; g.nhx = s->nhx; g.tz = s->tz;
    g.inv_mu0 = R(1.0 / s->mu0);
    g.coef = R((s->lam0 + s->mu0) / (s->mu0 * (s->lam0 + 2.0 * s->mu0)));
    return g;
}

template <typename R>
static void launch_y(cpf_solver *s, C2<R> *spec, bool inv, const Scalars *sc)
{
    const C2<R> *tw = dptr<C2<R>>(s, s->off_tw[1]);
    dim3 grid(s->nty, s->nz, 6);
    if (inv)
        hipLaunchKernelGGL((k_ypass<R, true, 16>), grid, dim3(256), s->lds_y, s->stream, spec, tw, s->py,
                           s->ny, s->nz, s->nhx, s->ty, sc);
    else
        hipLaunchKernelGGL((k_ypass<R, false, 16>), grid, dim3(256), s->lds_y, s->stream, spec, tw, s->py,
                           s->ny, s->nz, s->nhx, s->ty, sc);
}

template <typename R>
static void launch_z(cpf_solver *s, C2<R> *spec, int mode, const Scalars *sc)
{
    const C2<R> *tw = dptr<C2<R>>(s, s->off_tw[2]);
    dim3 grid(s->ntz, s->ny);
    constexpr int EPT = sizeof(R) == 4 ? 24 : 12;
    hipLaunchKernelGGL((k_zpass_green<R, EPT>), grid, dim3(256), s->lds_z, s->stream, spec, tw, s->pz,
                       green_args<R>(s), dptr<double>(s, s->off_pz), sc, mode);
}

static void launch_bc(cpf_solver *s, const double *px, Scalars *sc, const BcArgs &b)
{
    hipLaunchKernelGGL(k_bc_update, dim3(1), dim3(256), 0, s->stream, px, dptr<double>(s, s->off_pz), sc, b);
}

template <typename R>
static int step_impl(cpf_solver *s, const cpf_path *path, int n, cpf_step_out *out)
{
    const double dt = path->t[n + 1] - path->t[n];
    const int M = s->opt.rk4_M > 0 ? s->opt.rk4_M : substeps(dt, s->opt.h_max);
    StepInit si;
    double dE0[6] = {0, 0, 0, 0, 0, 0};
    for (int i = 0; i < 6; ++i) {
        si.sidx[i] = path->strain_ctrl[6 * n + i] ? 0 : 1;
        si.target[i] = path->target[6 * n + i];
        if (!si.sidx[i]) dE0[i] = si.target[i] - s->E_n[i];
    }
    stress_block_inverse(s->K0, si.sidx, si.K0inv);
    // homogeneous reference-medium prediction of the stress-controlled part
    double rhs[6];
    for (int i = 0; i < 6; ++i) {
        double k = 0;
        for (int j = 0; j < 6; ++j) k += s->K0[i * 6 + j] * dE0[j];
        rhs[i] = si.sidx[i] ? (si.target[i] - s->Sigma_n[i]) - k : 0.0;
    }
    for (int i = 0; i < 6; ++i) {
        double d = 0;
        for (int j = 0; j < 6; ++j) d += si.K0inv[i * 6 + j] * rhs[j];
        if (si.sidx[i]) dE0[i] = d;
        si.dE0[i] = dE0[i];
        si.E0[i] = s->E_n[i] + dE0[i];
    }
    Scalars *sc = dptr<Scalars>(s, s->off_sc);
    hipLaunchKernelGGL(k_begin_step, dim3(1), dim3(64), 0, s->stream, sc, si);

    XArgs<R> a;
    a.labels = dptr<int32_t>(s, s->off_labels);
    a.Qtab = dptr<R>(s, s->off_Q);
    a.eps_n = dptr<R>(s, s->off_eps[s->eps_cur]);
    a.eps_k = dptr<R>(s, s->off_eps[1 - s->eps_cur]);
    a.st_in = dptr<R>(s, s->off_st[s->st_cur]);
    a.st_out = dptr<R>(s, s->off_st[1 - s->st_cur]);
    a.spec = dptr<C2<R>>(s, s->off_spec);
    a.tw = dptr<C2<R>>(s, s->off_tw[0]);
    a.part = dptr<double>(s, s->off_px);
    a.sc = sc;
    a.nx = s->nx; a.ny = s->ny; a.nz = s->nz; a.nhx = s->nhx; a.L = s->L;
    a.nlines = s->ny * s->nz;
    a.nvox = s->nvox;
    a.inv_nvox = R(1.0 / (double)s->nvox);
    a.dt = R(dt);
    a.M = M;
    const LawP<R> P = make_law<R>(s);
    BcArgs b;
    b.nbx = s->nbx; b.nbz = s->nbz;
    b.nvox = (double)s->nvox;
    b.n_slip = s->pb.n_slip; b.n_twin = s->pb.n_twin;
    b.tol = s->opt.tol;
    b.stag_tol = s->opt.stag_tol;
    b.max_iter = s->opt.max_iter;

    int queued = 0;
    int chunk = s->opt.check_every > 0 ? s->opt.check_every : std::max(2, s->prev_iters);
    for (;;) {
        for (int c = 0; c < chunk; ++c, ++queued) {
            TIMED(s, 0, (launch_xiter_any<R>(s, a, P, queued == 0 ? 1 : 0)));
            TIMED(s, 1, (launch_y<R>(s, a.spec, false, sc)));
            TIMED(s, 2, (launch_z<R>(s, a.spec, ZMODE_FWD | ZMODE_GREEN, sc)));
            TIMED(s, 3, (launch_y<R>(s, a.spec, true, sc)));
            TIMED(s, 4, launch_bc(s, a.part, sc, b));
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(s->hsc, sc, sizeof(Scalars), hipMemcpyDeviceToHost, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
        {
            int rc = timed_collect(s);
            if (rc) return rc;
        }
        if (s->hsc->done) break;
        if (queued > s->opt.max_iter + 8)
            return fail(CPF_E_BAD_STATE, "device did not end the step after %d iterations", queued);
        chunk = s->opt.check_every > 0 ? s->opt.check_every : 4;
    }
    const Scalars &h = *s->hsc;
    if (out) {
        for (int i = 0; i < 6; ++i) { out->Sigma[i] = h.Sigma[i]; out->E[i] = h.E[i]; }
        const double p3 = (h.Sigma[0] + h.Sigma[1] + h.Sigma[2]) / 3.0;
        const double a0 = h.Sigma[0] - p3, a1 = h.Sigma[1] - p3, a2 = h.Sigma[2] - p3;
        out->sig_eq_of_mean = sqrt(1.5 * (a0 * a0 + a1 * a1 + a2 * a2 +
                                          2.0 * (h.Sigma[3] * h.Sigma[3] + h.Sigma[4] * h.Sigma[4] +
                                                 h.Sigma[5] * h.Sigma[5])));
        out->mean_sig_eq = h.mean_sig_eq;
        out->mean_v = h.mean_v;
        out->mean_f = h.mean_f;
        out->err_eq = h.err_eq;
        out->err_bc = h.err_bc;
        out->n_active = h.work_active;
        out->n_newton = h.work_newton;
        out->iters = h.iter;
        out->status = h.status;
    }
    if (h.status == -5) return fail(CPF_E_NAN, "non-finite stress or residual in load step %d", n);
    if (h.status == -4)
        return fail(CPF_E_NOT_CONVERGED, "load step %d: no convergence in %d iterations (err %.3g)", n,
                    h.iter, std::max(h.err_eq, h.err_bc));
    // commit: the iterate and the trial state become the committed ones
    s->eps_cur = 1 - s->eps_cur;
    s->st_cur = 1 - s->st_cur;
    for (int i = 0; i < 6; ++i) { s->Sigma_n[i] = h.Sigma[i]; s->E_n[i] = h.E[i]; }
    s->prev_iters = h.iter;
    return CPF_OK;
}

static int check_path(const cpf_path *p)
{
    if (!p || !p->t || !p->strain_ctrl || !p->target || p->n_steps < 1)
        return fail(CPF_E_INVALID_ARG, "path needs n_steps >= 1 and t, strain_ctrl, target");
    for (int n = 0; n < p->n_steps; ++n)
        if (!(p->t[n + 1] > p->t[n])) return fail(CPF_E_INVALID_ARG, "path times must increase");
    return CPF_OK;
}

extern "C" int cpf_solver_step(cpf_solver *s, const cpf_path *path, int n, cpf_step_out *out)
{
    if (!s || !s->bound) return fail(CPF_E_BAD_STATE, "solver not bound");
    int rc = check_path(path);
    if (rc) return rc;
    if (n < 0 || n >= path->n_steps) return fail(CPF_E_INVALID_ARG, "step %d outside the path", n);
    return s->prec == CPF_PREC_FP64 ? step_impl<double>(s, path, n, out) : step_impl<float>(s, path, n, out);
}

extern "C" int cpf_solver_run(cpf_solver *s, const cpf_path *path, cpf_step_out *out)
{
    if (!s || !s->bound) return fail(CPF_E_BAD_STATE, "solver not bound");
    int rc = check_path(path);
    if (rc) return rc;
    for (int n = 0; n < path->n_steps; ++n) {
        rc = cpf_solver_step(s, path, n, out ? out + n : nullptr);
        if (rc) return rc;
    }
    return CPF_OK;
}

template <typename R>
static int field_impl(cpf_solver *s, int field, void *dev_out)
{
    const long nv = s->nvox;
    R *o = (R *)dev_out;
    const R *eps = dptr<R>(s, s->off_eps[s->eps_cur]);
    const R *st = dptr<R>(s, s->off_st[s->st_cur]);
    switch (field) {
    case CPF_FIELD_STRESS:
        hipLaunchKernelGGL(k_stress_field<R>, dim3((nv + 255) / 256), dim3(256), 0, s->stream,
                           dptr<int32_t>(s, s->off_labels), dptr<R>(s, s->off_Q), eps, st, o,
                           make_law<R>(s), nv);
        HIPCHK(hipGetLastError());
        break;
    case CPF_FIELD_STRAIN:
        HIPCHK(hipMemcpyAsync(o, eps, sizeof(R) * 6 * nv, hipMemcpyDeviceToDevice, s->stream));
        break;
    case CPF_FIELD_PLASTIC_STRAIN:
        HIPCHK(hipMemcpyAsync(o, st, sizeof(R) * 6 * nv, hipMemcpyDeviceToDevice, s->stream));
        break;
    case CPF_FIELD_ACC_SLIP:
        HIPCHK(hipMemcpyAsync(o, st + 6 * nv, sizeof(R) * s->pb.nsys * nv, hipMemcpyDeviceToDevice,
                              s->stream));
        break;
    case CPF_FIELD_BACK_STRAIN:
        HIPCHK(hipMemcpyAsync(o, st + (6 + s->pb.nsys) * nv, sizeof(R) * s->pb.nsys * nv,
                              hipMemcpyDeviceToDevice, s->stream));
        break;
    default:
        return fail(CPF_E_INVALID_ARG, "unknown field %d", field);
    }
    HIPCHK(hipStreamSynchronize(s->stream));
    return CPF_OK;
}

extern "C" int cpf_solver_field(cpf_solver *s, int field, void *dev_out)
{
    if (!s || !s->bound) return fail(CPF_E_BAD_STATE, "solver not bound");
    if (!dev_out) return fail(CPF_E_INVALID_ARG, "null output");
    return s->prec == CPF_PREC_FP64 ? field_impl<double>(s, field, dev_out)
                                    : field_impl<float>(s, field, dev_out);
}

// ---------------------------------------------------------------------------
// component operators
// ---------------------------------------------------------------------------
template <typename R>
static int op_fft_impl(cpf_solver *s, const void *field, void *spec)
{
    C2<R> *sp = (C2<R> *)spec;
    hipLaunchKernelGGL(k_xpass_fwd<R>, dim3(s->nbx), dim3(s->tpbx), s->lds_x, s->stream, (const R *)field,
                       sp, dptr<C2<R>>(s, s->off_tw[0]), s->px, s->nx, s->ny, s->nz, s->nhx, s->L,
                       s->ny * s->nz, s->nvox);
    launch_y<R>(s, sp, false, nullptr);
    launch_z<R>(s, sp, ZMODE_FWD, nullptr);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s->stream));
    return CPF_OK;
}

extern "C" int cpf_op_forward_fft(cpf_solver *s, const void *dev_field, void *dev_spec)
{
    if (!s || !s->bound) return fail(CPF_E_BAD_STATE, "solver not bound");
    if (!dev_field || !dev_spec) return fail(CPF_E_INVALID_ARG, "null device pointer");
    return s->prec == CPF_PREC_FP64 ? op_fft_impl<double>(s, dev_field, dev_spec)
                                    : op_fft_impl<float>(s, dev_field, dev_spec);
}

template <typename R>
static int op_green_impl(cpf_solver *s, void *spec, void *outp, double *err2)
{
    C2<R> *sp = (C2<R> *)spec;
    launch_z<R>(s, sp, ZMODE_GREEN, nullptr);
    launch_y<R>(s, sp, true, nullptr);
    hipLaunchKernelGGL(k_xpass_inv<R>, dim3(s->nbx), dim3(s->tpbx), s->lds_x, s->stream, sp, (R *)outp,
                       dptr<C2<R>>(s, s->off_tw[0]), s->px, s->nx, s->ny, s->nz, s->nhx, s->L,
                       s->ny * s->nz, s->nvox, R(1.0 / (double)s->nvox));
    HIPCHK(hipGetLastError());
    if (err2) {
        std::vector<double> pz(s->nbz);
        HIPCHK(hipMemcpyAsync(pz.data(), s->ws + s->off_pz, sizeof(double) * s->nbz, hipMemcpyDeviceToHost,
                              s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
        double t = 0;
        for (double v : pz) t += v;
        *err2 = t;
    }
    HIPCHK(hipStreamSynchronize(s->stream));
    return CPF_OK;
}

extern "C" int cpf_op_green(cpf_solver *s, void *dev_spec, void *dev_out, double *err2)
{
    if (!s || !s->bound) return fail(CPF_E_BAD_STATE, "solver not bound");
    if (!dev_spec || !dev_out) return fail(CPF_E_INVALID_ARG, "null device pointer");
    return s->prec == CPF_PREC_FP64 ? op_green_impl<double>(s, dev_spec, dev_out, err2)
                                    : op_green_impl<float>(s, dev_spec, dev_out, err2);
}

template <typename R, int NS, int SPEC = LAW_GENERAL>
static void launch_cp(cpf_solver *s, const void *e0, const void *e1, const void *s0, void *s1, void *sig,
                      double dt, int M)
{
    hipLaunchKernelGGL((k_constitutive<R, NS, SPEC>), dim3((s->nvox + 255) / 256), dim3(256), 0, s->stream,
                       dptr<int32_t>(s, s->off_labels), dptr<R>(s, s->off_Q), (const R *)e0, (const R *)e1,
                       (const R *)s0, (R *)s1, (R *)sig, make_law<R>(s), s->nvox, R(dt), M);
}

template <typename R>
static int op_cp_impl(cpf_solver *s, const void *e0, const void *e1, const void *s0, void *s1, void *sig,
                      double dt, int M)
{
    if (s->law_spec == LAW_TABLE1) {
        if (s->ns_inst == 12) launch_cp<R, 12, LAW_TABLE1>(s, e0, e1, s0, s1, sig, dt, M);
        else launch_cp<R, 16, LAW_TABLE1>(s, e0, e1, s0, s1, sig, dt, M);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(s->stream));
        return CPF_OK;
    }
    switch (s->ns_inst) {
    case 4: launch_cp<R, 4>(s, e0, e1, s0, s1, sig, dt, M); break;
    case 12: launch_cp<R, 12>(s, e0, e1, s0, s1, sig, dt, M); break;
    case 16: launch_cp<R, 16>(s, e0, e1, s0, s1, sig, dt, M); break;
    default: launch_cp<R, 32>(s, e0, e1, s0, s1, sig, dt, M); break;
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s->stream));
    return CPF_OK;
}

extern "C" int cpf_op_constitutive(cpf_solver *s, const void *e0, const void *e1, const void *s0, void *s1,
                                   void *sig, double dt, int M)
{
    if (!s || !s->bound) return fail(CPF_E_BAD_STATE, "solver not bound");
    if (!e0 || !e1 || !s0 || !s1 || !sig) return fail(CPF_E_INVALID_ARG, "null device pointer");
    if (!(dt > 0) || M < 1) return fail(CPF_E_INVALID_ARG, "need dt > 0 and M >= 1");
    return s->prec == CPF_PREC_FP64 ? op_cp_impl<double>(s, e0, e1, s0, s1, sig, dt, M)
                                    : op_cp_impl<float>(s, e0, e1, s0, s1, sig, dt, M);
}

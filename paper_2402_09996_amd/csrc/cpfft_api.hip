// Host side of the solver and the C-ABI declared in include/cpfft.h.
//
// One load step runs the Green-operator fixed point on the device: each
// iteration is x pass (law + x transforms) -> y pass -> z pass with Gamma0
// -> inverse y pass -> boundary update.  Iterations are queued in chunks
// and every kernel returns at once when the device flag says the step has
// ended, so the host only polls the step status between chunks.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cstddef>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <new>
#include <string>
#include <vector>

#include "../../include/cpfft.h"
#include "cpfft_adjoint.hpp"

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

// roctx range over a scope (host side: the enqueue of a load step, an
// iteration chunk or a pass; a profiler run with marker tracing shows them
// beside the kernels)
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

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

// for the microstructure entry points (another translation unit)
int cpf_internal_fail(int code, const char *msg)
{
    g_err = msg;
    return code;
}

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
    o->green = CPF_GREEN_CONTINUOUS;
    o->rk_tol = 0.0;
    o->aa_depth = 0;
    o->nyquist_mode = CPF_NYQUIST_ZERO;
    o->cutback = 0;
    o->reg_mode = CPF_REG_IMPLICIT;
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
    int ns = 1;
    for (int p = 0; p < P.npass; ++p) {
        P.mag_m[p] = fdiv_magic((unsigned)(n / P.radix[p]));
        P.mag_ns[p] = fdiv_magic((unsigned)ns);
        ns *= P.radix[p];
    }
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
// solver: a batch of RVEs sharing one law (a single solve is a batch of one)
// ---------------------------------------------------------------------------
struct RveHost {
    cpf_problem pb;
    int nx, ny, nz, nhx;
    int nkx, nhp;               // kx columns of the stored spectrum, row pitch
    long nvox;
    FftPlan px, py, pz;
    int L, tpbx, nbx, ty, nty, tz, ntz, nbz;
    bool tiles_fixed = false;   // set explicitly or by the autotuner
    size_t off_labels, off_Q, off_eps[2], off_st[2], off_spec, off_tw[3], off_px, off_pz, off_sc, off_mv;
    size_t off_pb;
    size_t off_lag = 0;         // lagged regularization: raises [S][N]
    size_t off_aa = 0, off_aax = 0, off_aaf = 0, off_aadx = 0, off_aadf = 0, off_aap = 0, off_aac = 0;
    int cur = 0;
    double Sigma_n[6], E_n[6];
    int prev_iters = 8;
};

struct cpf_solver {
    std::vector<RveHost> rv;
    cpf_options opt;
    int prec;
    int D;                      // state components 6 + 2S (shared law)
    int ns_inst, law_spec;
    double lam0, mu0, K0[36];
    int n_slip, n_twin;
    // last adjoint call: forward iterations (with recomputation), adjoint
    // equilibrium iterations, recomputed steps
    long long adj_fwd_iters = 0, adj_eq_iters = 0;
    int adj_recomputed = 0;
    // pass grids over all RVEs
    int nbx_tot = 0, nby_tot = 0, nbz_tot = 0;
    int y_elems = 0, z_elems = 0;   // largest 6 ny ty and 6 nz tz over the RVEs
    int y_kinds = 0, z_kinds = 0;   // y / z kernels needed: bit 0 fixed-length, bit 1 generic
    size_t lds_x = 0, lds_y = 0, lds_z = 0;
    // workspace
    unsigned char *ws = nullptr;
    size_t ws_bytes = 0, total = 0;
    size_t off_dev, off_si, off_opdev, off_hist;
    hipStream_t stream = nullptr;
    bool bound = false;
    Scalars *hsc = nullptr;     // pinned host mirror of the per-RVE scalars
    StepInit *hsi = nullptr;    // pinned per-RVE step records
    // graph launches: G > 0 iterations per replay, CPF_GRAPH_ADAPTIVE
    // lengths from the previous step, 0 direct launches; captured graphs
    // by length
    int graph_iters = 0;
    std::map<int, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
    // kernel timing (timing_xpass: the x pass only)
    bool timing = false;
    bool timing_xpass = false;
    double t_ms[CPF_NKERNELS] = {0};
    long long t_n[CPF_NKERNELS] = {0};
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
};

static bool timed_on(const cpf_solver *s, int k) { return s->timing && (!s->timing_xpass || k == 0); }

static int timed_begin(cpf_solver *s, int k, hipEvent_t *a, hipEvent_t *b)
{
    if (!timed_on(s, k)) return CPF_OK;
    for (hipEvent_t *e : {a, b}) {
        if (s->ev_pool.empty()) {
            // timing markers only (the polls copy the scalars back and
            // synchronize the stream): no system-scope release, which would
            // write the L2 back between every two kernels of an iteration
            HIPCHK(hipEventCreateWithFlags(e, hipEventDisableSystemFence));
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
    if (!timed_on(s, k)) return CPF_OK;
    HIPCHK(hipEventRecord(b, s->stream));
    s->ev_pending.push_back({k, {a, b}});
    return CPF_OK;
}

// Fold the first `count` pending event pairs (all by default) into the
// counters; they must have completed (recorded before a stream
// synchronization).
static int timed_collect(cpf_solver *s, size_t count = (size_t)-1)
{
    const size_t n = std::min(count, s->ev_pending.size());
    for (size_t i = 0; i < n; ++i) {
        auto &p = s->ev_pending[i];
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, p.second.first, p.second.second));
        s->t_ms[p.first] += ms;
        s->t_n[p.first] += 1;
        s->ev_pool.push_back(p.second.first);
        s->ev_pool.push_back(p.second.second);
    }
    s->ev_pending.erase(s->ev_pending.begin(), s->ev_pending.begin() + n);
    return CPF_OK;
}

#define TIMED(s, k, launch)                                   \
    do {                                                      \
        hipEvent_t ea_ = nullptr, eb_ = nullptr;              \
        int rc_ = timed_begin(s, k, &ea_, &eb_);              \
        if (rc_) return rc_;                                  \
        launch;                                               \
        rc_ = timed_end(s, k, ea_, eb_);                      \
        if (rc_) return rc_;                                  \
    } while (0)

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Elements per thread the y and z pass kernels are compiled for (blocks of
// 256 threads; each kernel also has instantiations for a half and a
// quarter of that).
constexpr int EPT_Y = 24;
constexpr int EPT_Z = 24;
constexpr size_t LDS_LIMIT = 64 * 1024;

// Whether the fixed-length kernels do an RVE's y (z) pass: a common length
// and a tile no wider than theirs.
template <typename R>
static bool yfix_of(const RveHost &h, int ty)
{
    return fixed_len(h.ny) && ty <= fixed_tile_of<R>(h.ny);
}
template <typename R>
static bool zfix_of(const RveHost &h, int tz)
{
    return fixed_len(h.nz) && tz <= fixed_tile_of<R>(h.nz);
}

// LDS of the y and z pass blocks: the tile (6 components; the fixed-length
// kernels' own tile width) and the twiddles of the transform length.
template <typename R>
static size_t lds_y_bytes(const RveHost &h, int ty)
{
    const int w = yfix_of<R>(h, ty) ? fixed_tile_of<R>(h.ny) : ty;
    return (6 * (size_t)w * h.ny + h.ny) * sizeof(C2<R>);
}
template <typename R>
static size_t lds_z_bytes(const RveHost &h, int tz)
{
    const int w = zfix_of<R>(h, tz) ? fixed_tile_of<R>(h.nz) : tz;
    return (6 * (size_t)w * h.nz + h.nz) * sizeof(C2<R>);
}
// which kernels a pass needs: bit 0 the fixed-length one, bit 1 the generic one
template <typename R>
static int y_kinds(const RveHost &h, int ty)
{
    return yfix_of<R>(h, ty) ? 1 : 2;
}
template <typename R>
static int z_kinds(const RveHost &h, int tz)
{
    return zfix_of<R>(h, tz) ? 1 : 2;
}

template <typename R>
static bool tiles_valid(const RveHost &h, int ty, int tz)
{
    return ty >= 1 && tz >= 1 && ty <= h.nkx && tz <= h.nkx && 6 * ty * h.ny <= EPT_Y * 256 &&
           6 * tz * h.nz <= EPT_Z * Z_THREADS && lds_y_bytes<R>(h, ty) <= LDS_LIMIT &&
           lds_z_bytes<R>(h, tz) <= LDS_LIMIT;
}

template <typename R>
static void set_tiles(RveHost &h, int ty, int tz)
{
    h.ty = ty;
    h.nty = (h.nkx + ty - 1) / ty;
    h.tz = tz;
    h.ntz = (h.nkx + tz - 1) / tz;
    h.nbz = h.ntz * h.ny;
}

template <typename R>
static void default_tiles(RveHost &h)
{
    const bool f32 = sizeof(R) == 4;
    // rows of 4 columns (6 components each: 192 bytes in FP32) where the
    // registers and the LDS allow it
    (void)f32;
    int ty = std::min(std::min(4, std::max(1, EPT_Y * 256 / (6 * h.ny))), h.nkx);
    int tz = std::min(std::min(4, std::max(1, EPT_Z * Z_THREADS / (6 * h.nz))), h.nkx);
    if (fixed_len(h.ny)) ty = std::min(fixed_tile_of<R>(h.ny), h.nkx);
    if (fixed_len(h.nz)) tz = std::min(fixed_tile_of<R>(h.nz), h.nkx);
    while (!tiles_valid<R>(h, ty, tz) && tz > 1) tz = (tz + 1) / 2;
    while (!tiles_valid<R>(h, ty, tz) && ty > 1) ty = (ty + 1) / 2;
    set_tiles<R>(h, ty, tz);
}

// Grid offsets of every RVE in each pass and the LDS sizes of the launches.
template <typename R>
static void pass_grids(cpf_solver *s)
{
    s->nbx_tot = s->nby_tot = s->nbz_tot = 0;
    // x pass: FFT buffer, then the law's per-thread work area
    s->lds_x = xfft_lds_bytes<R>() + law_lds_bytes_ns<R>(s->ns_inst);
    s->lds_y = s->lds_z = 0;
    s->y_elems = s->z_elems = 0;
    s->y_kinds = s->z_kinds = 0;
    for (auto &h : s->rv) {
        s->y_kinds |= y_kinds<R>(h, h.ty);
        s->z_kinds |= z_kinds<R>(h, h.tz);
        s->nbx_tot += h.nbx;
        s->nby_tot += h.nty * h.nz;
        s->nbz_tot += h.nbz;
        s->lds_y = std::max(s->lds_y, lds_y_bytes<R>(h, h.ty));
        s->y_elems = std::max(s->y_elems, 6 * h.ny * h.ty);
        s->z_elems = std::max(s->z_elems, 6 * h.nz * h.tz);
        s->lds_z = std::max(s->lds_z, lds_z_bytes<R>(h, h.tz));
    }
}

template <typename R>
static void layout(cpf_solver *s)
{
    const size_t cb = sizeof(C2<R>);
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
    for (auto &h : s->rv) {
        h.off_labels = take(sizeof(int32_t) * h.nvox);
        h.off_Q = take(sizeof(R) * 9 * h.pb.nlab);
        h.off_eps[0] = take(sizeof(R) * 6 * h.nvox);
        h.off_eps[1] = take(sizeof(R) * 6 * h.nvox);
        h.off_st[0] = take(sizeof(R) * s->D * h.nvox);
        h.off_st[1] = take(sizeof(R) * s->D * h.nvox);
        h.off_spec = take(cb * 6 * (size_t)h.nz * h.ny * h.nhp);
        h.off_tw[0] = take(cb * h.nx);
        h.off_tw[1] = take(cb * h.ny);
        h.off_tw[2] = take(cb * h.nz);
        h.off_px = take(sizeof(double) * NPX * h.nbx);
        h.off_pz = take(sizeof(double) * h.nhx * h.ny);   // room for the smallest z tile
        h.off_sc = take(sizeof(Scalars));
        h.off_mv = take(sizeof(int32_t) * h.nvox);
        h.off_pb = take(sizeof(double) * (NPX + 1) * BC_CHUNKS);
        if (s->opt.reg_mode == CPF_REG_LAGGED) h.off_lag = take(sizeof(R) * (size_t)(s->D - 6) / 2 * h.nvox);
        if (s->opt.aa_depth > 0) {
            const size_t f6 = sizeof(R) * 6 * h.nvox;
            h.off_aa = take(sizeof(AaState));
            h.off_aax = take(f6);
            h.off_aaf = take(f6);
            h.off_aadx = take(f6 * s->opt.aa_depth);
            h.off_aadf = take(f6 * s->opt.aa_depth);
            h.off_aap = take(sizeof(double) * 2 * AA_MAX * h.nbx);
            h.off_aac = take(sizeof(double) * 2 * AA_MAX * 32);
        }
    }
    const size_t n = s->rv.size();
    s->off_dev = take(sizeof(RveDev<R>) * n);
    s->off_si = take(sizeof(StepInit) * n);
    s->off_opdev = take(sizeof(RveDev<R>));
    s->off_hist = take(sizeof(unsigned long long) * (CPF_MAX_HIST_BINS + 2) + sizeof(double) * (CPF_MAX_HIST_BINS + 1));
    s->total = o;
}

template <typename R>
static R *dptr(cpf_solver *s, size_t off) { return reinterpret_cast<R *>(s->ws + off); }

template <typename R>
static RveDev<R> make_dev(cpf_solver *s, const RveHost &h, int bx0, int by0, int bz0)
{
    RveDev<R> d;
    memset(&d, 0, sizeof d);
    d.nx = h.nx; d.ny = h.ny; d.nz = h.nz; d.nhx = h.nhx;
    d.nkx = h.nkx; d.nhp = h.nhp;
    d.L = h.L; d.tpbx = h.tpbx; d.nlines = h.ny * h.nz;
    d.ty = h.ty; d.nty = h.nty; d.tz = h.tz; d.ntz = h.ntz;
    d.yfix = yfix_of<R>(h, h.ty) ? 1 : 0;
    d.zfix = zfix_of<R>(h, h.tz) ? 1 : 0;
    d.bx0 = bx0; d.by0 = by0; d.bz0 = bz0;
    d.nvox = h.nvox;
    d.inv_nvox = R(1.0 / (double)h.nvox);
    d.px = h.px; d.py = h.py; d.pz = h.pz;
    d.labels = dptr<int32_t>(s, h.off_labels);
    d.Qtab = dptr<R>(s, h.off_Q);
    d.eps[0] = dptr<R>(s, h.off_eps[0]);
    d.eps[1] = dptr<R>(s, h.off_eps[1]);
    d.st[0] = dptr<R>(s, h.off_st[0]);
    d.st[1] = dptr<R>(s, h.off_st[1]);
    d.mv = dptr<int32_t>(s, h.off_mv);
    d.spec = dptr<C2<R>>(s, h.off_spec);
    for (int a = 0; a < 3; ++a) d.tw[a] = dptr<C2<R>>(s, h.off_tw[a]);
    d.part_x = dptr<double>(s, h.off_px);
    d.part_z = dptr<double>(s, h.off_pz);
    d.part_b = dptr<double>(s, h.off_pb);
    d.aa_depth = s->opt.aa_depth;
    d.aa = s->opt.aa_depth > 0 ? dptr<AaState>(s, h.off_aa) : nullptr;
    d.aa_x = s->opt.aa_depth > 0 ? dptr<R>(s, h.off_aax) : nullptr;
    d.aa_f = s->opt.aa_depth > 0 ? dptr<R>(s, h.off_aaf) : nullptr;
    d.aa_dX = s->opt.aa_depth > 0 ? dptr<R>(s, h.off_aadx) : nullptr;
    d.aa_dF = s->opt.aa_depth > 0 ? dptr<R>(s, h.off_aadf) : nullptr;
    d.aa_part = s->opt.aa_depth > 0 ? dptr<double>(s, h.off_aap) : nullptr;
    d.aa_chunk = s->opt.aa_depth > 0 ? dptr<double>(s, h.off_aac) : nullptr;
    d.sc = dptr<Scalars>(s, h.off_sc);
    d.lag = s->opt.reg_mode == CPF_REG_LAGGED ? dptr<R>(s, h.off_lag) : nullptr;
    return d;
}

// Upload the descriptor table of all RVEs (after binding or a tile change).
template <typename R>
static int upload_devs(cpf_solver *s)
{
    pass_grids<R>(s);
    std::vector<RveDev<R>> t;
    int bx = 0, by = 0, bz = 0;
    for (auto &h : s->rv) {
        t.push_back(make_dev<R>(s, h, bx, by, bz));
        bx += h.nbx;
        by += h.nty * h.nz;
        bz += h.nbz;
    }
    HIPCHK(hipMemcpyAsync(s->ws + s->off_dev, t.data(), sizeof(RveDev<R>) * t.size(), hipMemcpyHostToDevice,
                          s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return CPF_OK;
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
        // one initial resistance per kind (the first system of each kind)
        for (int q = 0; q < s; ++q)
            if (T1_KIND[q] == T1_KIND[s] && p.tau0[q] != p.tau0[s]) return false;
    }
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            const bool nz = (i < 3 && j < 3) || i == j;
            if (!nz && p.Cv[i * 6 + j] != 0.0) return false;
        }
    return true;
}

// Members of a batch share the crystal stiffness, the systems and the law.
static bool same_material(const cpf_problem &a, const cpf_problem &b)
{
    if (a.nsys != b.nsys || a.twin_mode != b.twin_mode || a.Kc != b.Kc || a.fm != b.fm || a.gT != b.gT ||
        a.eta != b.eta)
        return false;
    if (memcmp(a.Cv, b.Cv, sizeof a.Cv) != 0 || memcmp(a.law, b.law, sizeof a.law) != 0) return false;
    return a.m == b.m && a.tau0 == b.tau0 && a.fam == b.fam;
}

template <typename R>
static void init_rve(RveHost &h, const cpf_problem &p, int green, int nyquist)
{
    h.pb = p;
    h.nx = p.nx; h.ny = p.ny; h.nz = p.nz;
    h.nhx = p.nx / 2 + 1;
    // With the continuous operator the solve keeps the columns below the
    // Nyquist one (kx < nx/2 for even nx, all nx/2 + 1 for odd nx): Gamma0
    // is zero on the Nyquist column and the residual leaves it out, so the
    // column is neither stored nor transformed along y and z.  The rotated
    // operator, and the continuous one applied at Nyquist frequencies too,
    // act on it, so it is kept.  The spectrum is stored
    // [z][y][kx][c]; rows of nhp columns (a multiple of 8: whole 128-byte
    // lines of 6 components).
    h.nkx = (green == CPF_GREEN_ROTATED || nyquist == CPF_NYQUIST_FORMULA || (p.nx & 1)) ? p.nx / 2 + 1
                                                                                          : p.nx / 2;
    h.nhp = (h.nkx + 7) / 8 * 8;
    h.nvox = (long)p.nx * p.ny * p.nz;
    radix_plan(h.nx, h.px);
    radix_plan(h.ny, h.py);
    radix_plan(h.nz, h.pz);
    h.L = std::max(1, 256 / h.nx);
    h.tpbx = h.L * h.nx;
    h.nbx = (h.ny * h.nz + h.L - 1) / h.L;
    default_tiles<R>(h);
}

extern "C" int cpf_batch_create(int n, const cpf_problem *const *probs, const cpf_options *opt,
                                cpf_solver **out)
{
    if (!probs || !out || n < 1) return fail(CPF_E_INVALID_ARG, "need n >= 1 problems and an output");
    *out = nullptr;
    for (int i = 0; i < n; ++i) {
        if (!probs[i]) return fail(CPF_E_INVALID_ARG, "problem %d is null", i);
        if (!same_material(*probs[0], *probs[i]))
            return fail(CPF_E_INVALID_ARG, "problem %d: batch members must share stiffness, systems and law", i);
    }
    cpf_options o;
    cpf_options_default(&o);
    if (opt) o = *opt;
    if (o.precision != CPF_PREC_FP64 && o.precision != CPF_PREC_FP32)
        return fail(CPF_E_INVALID_ARG, "unknown precision %d", o.precision);
    if (!(o.tol > 0) || o.max_iter < 1 || (o.rk4_M <= 0 && !(o.h_max > 0)) || o.rk4_M > 100000)
        return fail(CPF_E_INVALID_ARG, "need tol > 0, max_iter >= 1 and rk4_M > 0 or h_max > 0");
    if (o.green != CPF_GREEN_CONTINUOUS && o.green != CPF_GREEN_ROTATED)
        return fail(CPF_E_INVALID_ARG, "unknown Green operator %d", o.green);
    if (o.nyquist_mode != CPF_NYQUIST_ZERO && o.nyquist_mode != CPF_NYQUIST_FORMULA)
        return fail(CPF_E_INVALID_ARG, "unknown nyquist_mode %d", o.nyquist_mode);
    if (o.nyquist_mode == CPF_NYQUIST_FORMULA && o.green != CPF_GREEN_CONTINUOUS)
        return fail(CPF_E_INVALID_ARG, "nyquist_mode applies to the continuous Green operator only");
    if (o.cutback < 0 || o.cutback > 20)
        return fail(CPF_E_INVALID_ARG, "cutback must be in [0, 20]");
    if (!(o.rk_tol >= 0.0) || !std::isfinite(o.rk_tol))
        return fail(CPF_E_INVALID_ARG, "rk_tol must be finite and >= 0");
    if (o.aa_depth < 0 || o.aa_depth > AA_MAX)
        return fail(CPF_E_INVALID_ARG, "aa_depth must be in [0, %d]", AA_MAX);
    if (o.aa_depth > 0 && o.rk_tol > 0.0)
        return fail(CPF_E_INVALID_ARG, "Anderson acceleration and error-controlled substeps are exclusive");
    if (o.reg_mode != CPF_REG_IMPLICIT && o.reg_mode != CPF_REG_LAGGED)
        return fail(CPF_E_INVALID_ARG, "unknown reg_mode %d", o.reg_mode);
    if (o.reg_mode == CPF_REG_LAGGED && (o.rk_tol > 0.0 || o.aa_depth > 0))
        return fail(CPF_E_INVALID_ARG, "the lagged regularization runs the basic fixed point with fixed substeps");
    cpf_solver *s = new (std::nothrow) cpf_solver();
    if (!s) return fail(CPF_E_INVALID_ARG, "out of host memory");
    const cpf_problem &p0 = *probs[0];
    s->opt = o;
    s->prec = o.precision;
    s->D = 6 + 2 * p0.nsys;
    s->ns_inst = p0.nsys <= 4 ? 4 : p0.nsys <= 12 ? 12 : p0.nsys <= 16 ? 16 : 32;
    s->law_spec = table1_specializable(p0) ? LAW_TABLE1 : LAW_GENERAL;
    s->n_slip = p0.n_slip;
    s->n_twin = p0.n_twin;
    s->rv.resize(n);
    for (int i = 0; i < n; ++i) {
        if (s->prec == CPF_PREC_FP64) init_rve<double>(s->rv[i], *probs[i], o.green, o.nyquist_mode);
        else init_rve<float>(s->rv[i], *probs[i], o.green, o.nyquist_mode);
    }
    if (s->prec == CPF_PREC_FP64) { layout<double>(s); pass_grids<double>(s); }
    else { layout<float>(s); pass_grids<float>(s); }
    if (o.mu0 > 0) {
        s->lam0 = o.lam0;
        s->mu0 = o.mu0;
    } else {
        cpf_problem_reference_medium(&p0, &s->lam0, &s->mu0);
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

extern "C" int cpf_solver_create(const cpf_problem *p, const cpf_options *opt, cpf_solver **out)
{
    if (!p || !out) return fail(CPF_E_INVALID_ARG, "null argument");
    return cpf_batch_create(1, &p, opt, out);
}

extern "C" int cpf_batch_size(const cpf_solver *s, int *n)
{
    if (!s || !n) return fail(CPF_E_INVALID_ARG, "null argument");
    *n = (int)s->rv.size();
    return CPF_OK;
}

extern "C" int cpf_solver_workspace_size(const cpf_solver *s, size_t *bytes)
{
    if (!s || !bytes) return fail(CPF_E_INVALID_ARG, "null argument");
    *bytes = s->total;
    return CPF_OK;
}

static void drop_graph(cpf_solver *s)
{
    for (auto &g : s->graphs) {
        if (g.second.second) (void)hipGraphExecDestroy(g.second.second);
        if (g.second.first) (void)hipGraphDestroy(g.second.first);
    }
    s->graphs.clear();
}

extern "C" void cpf_solver_destroy(cpf_solver *s)
{
    if (!s) return;
    drop_graph(s);
    if (s->hsc) (void)hipHostFree(s->hsc);
    if (s->hsi) (void)hipHostFree(s->hsi);
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
    if (enable != CPF_TIMING_OFF && enable != CPF_TIMING_ALL && enable != CPF_TIMING_XPASS)
        return fail(CPF_E_INVALID_ARG, "timing mode must be CPF_TIMING_OFF, CPF_TIMING_ALL or CPF_TIMING_XPASS");
    if (s->bound) HIPCHK(hipStreamSynchronize(s->stream));
    int rc = timed_collect(s);
    if (rc) return rc;
    s->timing = enable != CPF_TIMING_OFF;
    s->timing_xpass = enable == CPF_TIMING_XPASS;
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

extern "C" int cpf_solver_set_graph(cpf_solver *s, int iters_per_launch)
{
    if (!s) return fail(CPF_E_INVALID_ARG, "null solver");
    if ((iters_per_launch < 0 && iters_per_launch != CPF_GRAPH_ADAPTIVE) || iters_per_launch > 1024)
        return fail(CPF_E_INVALID_ARG, "iterations per graph launch must be in [0, 1024] or CPF_GRAPH_ADAPTIVE");
    if (s->bound) HIPCHK(hipStreamSynchronize(s->stream));
    drop_graph(s);
    s->graph_iters = iters_per_launch;
    return CPF_OK;
}

// Newton stops when the last step is below rtol times the root.  From
// above the root the iteration converges quadratically, and the relative
// error left after that step is about (n - 1)/2 times the square of the
// step (4.5 rtol^2 at n = 10): 1e-6 in FP32, the fixed point's own
// tolerance in that precision, and 1e-12 in FP64, two orders below the
// 1e-10 to which FP64 runs are held.
constexpr double NEWTON_RTOL_F32 = 4.7e-4;
constexpr double NEWTON_RTOL_F64 = 4.7e-7;

template <typename R>
static LawP<R> make_law(const cpf_solver *s)
{
    const cpf_problem &p = s->rv[0].pb;
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
        F.Q = R(L.Q); F.b = R(L.b); F.qs = R(L.q_self); F.ql = R(L.q_latent);
        (f ? P.ft : P.fs) = F;
    }
    P.Kc_gT = R(p.Kc * p.gT); P.fm = R(p.fm); P.inv_gT = R(1.0 / p.gT);
    P.eta = R(p.eta); P.inv_eta = R(p.eta > 0 ? 1.0 / p.eta : 0.0);
    // per-kind resistances of the Table 1 specialization (kinds absent from
    // the problem never activate)
    for (int k = 0; k < 3; ++k) P.tau0k[k] = R(1e30);
    if (s->law_spec == LAW_TABLE1)
        for (int sy = p.nsys - 1; sy >= 0; --sy) P.tau0k[T1_KIND[sy]] = R(p.tau0[sy]);
    P.newton_rtol = sizeof(R) == 4 ? R(NEWTON_RTOL_F32) : R(NEWTON_RTOL_F64);
    // one integer exponent n - 1 for every family that has systems (the
    // Newton passes mix the families of different lanes)
    bool has[2] = {false, false};
    for (int sy = 0; sy < p.nsys; ++sy) has[p.fam[sy] ? 1 : 0] = true;
    P.nm1_uni = -1;
    for (int f = 0; f < 2; ++f) {
        if (!has[f]) continue;
        const int e = (f ? P.ft : P.fs).nm1_int;
        if (e < 0 || (P.nm1_uni >= 0 && e != P.nm1_uni)) { P.nm1_uni = -1; break; }
        P.nm1_uni = e;
    }
    return P;
}

template <typename R>
static int zero_state(cpf_solver *s)
{
    for (auto &h : s->rv) {
        const long n6 = 6 * h.nvox, nD = (long)s->D * h.nvox;
        for (int b = 0; b < 2; ++b) {
            hipLaunchKernelGGL(k_fill<R>, dim3(512), dim3(256), 0, s->stream, dptr<R>(s, h.off_eps[b]), n6, R(0));
            hipLaunchKernelGGL(k_fill<R>, dim3(512), dim3(256), 0, s->stream, dptr<R>(s, h.off_st[b]), nD, R(0));
        }
        if (s->opt.reg_mode == CPF_REG_LAGGED)
            hipLaunchKernelGGL(k_fill<R>, dim3(512), dim3(256), 0, s->stream, dptr<R>(s, h.off_lag),
                               (long)(s->D - 6) / 2 * h.nvox, R(0));
        h.cur = 0;
        for (int i = 0; i < 6; ++i) h.Sigma_n[i] = h.E_n[i] = 0.0;
        h.prev_iters = 8;
    }
    HIPCHK(hipGetLastError());
    return CPF_OK;
}

template <typename R>
static int bind_impl(cpf_solver *s)
{
    for (auto &h : s->rv) {
        const cpf_problem &p = h.pb;
        std::vector<R> Qr(p.Q.size());
        for (size_t i = 0; i < Qr.size(); ++i) Qr[i] = R(p.Q[i]);
        HIPCHK(hipMemcpyAsync(s->ws + h.off_labels, p.labels.data(), sizeof(int32_t) * h.nvox,
                              hipMemcpyHostToDevice, s->stream));
        HIPCHK(hipMemcpyAsync(s->ws + h.off_Q, Qr.data(), sizeof(R) * Qr.size(), hipMemcpyHostToDevice,
                              s->stream));
        const int ns[3] = {h.nx, h.ny, h.nz};
        for (int a = 0; a < 3; ++a) {
            std::vector<C2<R>> tw(ns[a]);
            for (int k = 0; k < ns[a]; ++k) {
                const long double ang = -2.0L * 3.141592653589793238462643383279502884L * k / ns[a];
                tw[k] = C2<R>{R(cosl(ang)), R(sinl(ang))};
            }
            HIPCHK(hipMemcpyAsync(s->ws + h.off_tw[a], tw.data(), sizeof(C2<R>) * ns[a], hipMemcpyHostToDevice,
                                  s->stream));
        }
        // the host vectors above are pageable: make each copy complete before they go
        HIPCHK(hipStreamSynchronize(s->stream));
        // scalars start as an ended step so that nothing runs before a step begins
        Scalars z;
        memset(&z, 0, sizeof z);
        z.done = 1;
        HIPCHK(hipMemcpyAsync(s->ws + h.off_sc, &z, sizeof z, hipMemcpyHostToDevice, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
    }
    int rc = zero_state<R>(s);
    if (rc) return rc;
    rc = upload_devs<R>(s);
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
    drop_graph(s);
    s->ws = (unsigned char *)ws;
    s->ws_bytes = bytes;
    s->stream = (hipStream_t)stream;
    const size_t n = s->rv.size();
    if (!s->hsc) HIPCHK(hipHostMalloc((void **)&s->hsc, sizeof(Scalars) * n, hipHostMallocDefault));
    if (!s->hsi) HIPCHK(hipHostMalloc((void **)&s->hsi, sizeof(StepInit) * n, hipHostMallocDefault));
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

// ---------------------------------------------------------------------------
// launches (all RVEs per grid)
// ---------------------------------------------------------------------------
template <typename R, int NS, int SPEC>
static void launch_xiter(cpf_solver *s, const LawP<R> &P)
{
    if (s->opt.rk_tol > 0.0) {
        // frozen error-controlled substeps: Richardson's bound (15 tol)^2 on
        // the squared state difference, at most CPF_RK_MAX_DOUBLINGS doublings
        const double lim2 = (15.0 * s->opt.rk_tol) * (15.0 * s->opt.rk_tol);
        hipLaunchKernelGGL((k_xpass_iter<R, NS, SPEC, true>), dim3(s->nbx_tot), dim3(256), s->lds_x, s->stream,
                           dptr<RveDev<R>>(s, s->off_dev), (int)s->rv.size(), P, lim2, CPF_RK_MAX_DOUBLINGS);
    } else if (s->opt.aa_depth > 0) {
        hipLaunchKernelGGL((k_xpass_iter<R, NS, SPEC, false, true>), dim3(s->nbx_tot), dim3(256), s->lds_x,
                           s->stream, dptr<RveDev<R>>(s, s->off_dev), (int)s->rv.size(), P, 0.0, 0);
    } else if (s->opt.reg_mode == CPF_REG_LAGGED) {
        hipLaunchKernelGGL((k_xpass_iter<R, NS, SPEC, false, false, true>), dim3(s->nbx_tot), dim3(256),
                           s->lds_x, s->stream, dptr<RveDev<R>>(s, s->off_dev), (int)s->rv.size(), P, 0.0, 0);
    } else {
        hipLaunchKernelGGL((k_xpass_iter<R, NS, SPEC, false>), dim3(s->nbx_tot), dim3(256), s->lds_x, s->stream,
                           dptr<RveDev<R>>(s, s->off_dev), (int)s->rv.size(), P, 0.0, 0);
    }
}

template <typename R>
static void launch_xiter_any(cpf_solver *s, const LawP<R> &P)
{
    if (s->law_spec == LAW_TABLE1) {
        if (s->ns_inst == 12) launch_xiter<R, 12, LAW_TABLE1>(s, P);
        else launch_xiter<R, 16, LAW_TABLE1>(s, P);
        return;
    }
    switch (s->ns_inst) {
    case 4: launch_xiter<R, 4, LAW_GENERAL>(s, P); break;
    case 12: launch_xiter<R, 12, LAW_GENERAL>(s, P); break;
    case 16: launch_xiter<R, 16, LAW_GENERAL>(s, P); break;
    default: launch_xiter<R, 32, LAW_GENERAL>(s, P); break;
    }
}

// table/nrve/grid default to the whole batch; the component operators and
// the autotuner pass a one-RVE table and an explicit spectrum.  nbc > 0:
// the fixed-length kernel's launch also runs the first stage of the scalar
// reduction in nbc leading blocks (the caller then skips k_bc_partials).
template <typename R>
static void launch_y(cpf_solver *s, bool inv, const RveDev<R> *table = nullptr, int nrve = 0, int grid = 0,
                     size_t lds = 0, C2<R> *spec = nullptr, int elems = 0, int kinds = 0, int nbc = 0)
{
    if (!table) {
        table = dptr<RveDev<R>>(s, s->off_dev);
        nrve = (int)s->rv.size();
        grid = s->nby_tot;
        lds = s->lds_y;
        elems = s->y_elems;
        kinds = s->y_kinds;
    }
    if (kinds & 1) {
        if (inv)
            hipLaunchKernelGGL((k_ypass_fx<R, true>), dim3(grid + nbc), dim3(FX_THREADS), lds, s->stream, table, nrve,
                               spec, nbc);
        else
            hipLaunchKernelGGL((k_ypass_fx<R, false>), dim3(grid + nbc), dim3(FX_THREADS), lds, s->stream, table, nrve,
                               spec, nbc);
    }
    if (!(kinds & 2)) return;
    // registers for fewer elements per thread when the tiles allow it
    constexpr int EQ = EPT_Y / 4, EH = EPT_Y / 2;
    if (elems <= EQ * 256) {
        if (inv)
            hipLaunchKernelGGL((k_ypass<R, true, EQ>), dim3(grid), dim3(256), lds, s->stream, table, nrve, spec);
        else
            hipLaunchKernelGGL((k_ypass<R, false, EQ>), dim3(grid), dim3(256), lds, s->stream, table, nrve, spec);
    } else if (elems <= EH * 256) {
        if (inv)
            hipLaunchKernelGGL((k_ypass<R, true, EH>), dim3(grid), dim3(256), lds, s->stream, table, nrve, spec);
        else
            hipLaunchKernelGGL((k_ypass<R, false, EH>), dim3(grid), dim3(256), lds, s->stream, table, nrve, spec);
    } else {
        if (inv)
            hipLaunchKernelGGL((k_ypass<R, true, EPT_Y>), dim3(grid), dim3(256), lds, s->stream, table, nrve, spec);
        else
            hipLaunchKernelGGL((k_ypass<R, false, EPT_Y>), dim3(grid), dim3(256), lds, s->stream, table, nrve, spec);
    }
}

template <typename R>
static void launch_z(cpf_solver *s, int mode, const RveDev<R> *table = nullptr, int nrve = 0, int grid = 0,
                     size_t lds = 0, C2<R> *spec = nullptr, int elems = 0, int kinds = 0)
{
    if (!table) {
        table = dptr<RveDev<R>>(s, s->off_dev);
        nrve = (int)s->rv.size();
        grid = s->nbz_tot;
        lds = s->lds_z;
        elems = s->z_elems;
        kinds = s->z_kinds;
    }
    const R inv_mu0 = R(1.0 / s->mu0);
    const R coef = R((s->lam0 + s->mu0) / (s->mu0 * (s->lam0 + 2.0 * s->mu0)));
    if ((mode & ZMODE_GREEN) && s->opt.green == CPF_GREEN_ROTATED) mode |= ZMODE_ROTATED;
    if ((mode & ZMODE_GREEN) && s->opt.nyquist_mode == CPF_NYQUIST_FORMULA) mode |= ZMODE_NYQUIST;
    if (kinds & 1)
        hipLaunchKernelGGL(k_zpass_fx<R>, dim3(grid), dim3(FX_THREADS), lds, s->stream, table, nrve, inv_mu0, coef,
                           mode, spec);
    if (!(kinds & 2)) return;
    constexpr int EQ = EPT_Z / 4, EH = EPT_Z / 2;
    if (elems <= EQ * Z_THREADS)
        hipLaunchKernelGGL((k_zpass_green<R, EQ>), dim3(grid), dim3(Z_THREADS), lds, s->stream, table, nrve, inv_mu0,
                           coef, mode, spec);
    else if (elems <= EH * Z_THREADS)
        hipLaunchKernelGGL((k_zpass_green<R, EH>), dim3(grid), dim3(Z_THREADS), lds, s->stream, table, nrve, inv_mu0,
                           coef, mode, spec);
    else
        hipLaunchKernelGGL((k_zpass_green<R, EPT_Z>), dim3(grid), dim3(Z_THREADS), lds, s->stream, table, nrve,
                           inv_mu0, coef, mode, spec);
}

template <typename R>
static void launch_bc(cpf_solver *s, bool partials_done = false)
{
    BcArgs b;
    b.n_slip = s->n_slip;
    b.n_twin = s->n_twin;
    b.tol = s->opt.tol;
    b.stag_tol = s->opt.stag_tol;
    b.max_iter = s->opt.max_iter;
    // two stages: BC_CHUNKS blocks per RVE sum fixed chunks of the block
    // partials (a 128^3 x pass leaves 8192 x 11 doubles), one wave per RVE
    // sums the chunks and updates the scalars
    if (!partials_done)
        hipLaunchKernelGGL(k_bc_partials<R>, dim3(s->rv.size() * BC_CHUNKS), dim3(256), 0, s->stream,
                           dptr<RveDev<R>>(s, s->off_dev));
    hipLaunchKernelGGL(k_bc_update<R>, dim3(s->rv.size()), dim3(64), 0, s->stream,
                       dptr<RveDev<R>>(s, s->off_dev), b);
}

template <typename R>
static int launch_iteration(cpf_solver *s, const LawP<R> &P)
{
    if (s->opt.aa_depth > 0) {
        // Anderson: step of the last iterate, its dot products, the small solve
        const RveDev<R> *tab = dptr<RveDev<R>>(s, s->off_dev);
        const int nrve = (int)s->rv.size();
        hipLaunchKernelGGL(k_aa_resid<R>, dim3(s->nbx_tot), dim3(256), xfft_lds_bytes<R>(), s->stream, tab, nrve);
        hipLaunchKernelGGL(k_aa_partials<R>, dim3(nrve * 32), dim3(256), 0, s->stream, tab);
        hipLaunchKernelGGL(k_aa_solve<R>, dim3(nrve), dim3(64), 0, s->stream, tab);
        hipLaunchKernelGGL(k_aa_update<R>, dim3(s->nbx_tot), dim3(256), 0, s->stream, tab, nrve);
    }
    { TraceRange t("cpf x pass (law, x transforms)"); TIMED(s, 0, launch_xiter_any<R>(s, P)); }
    { TraceRange t("cpf y pass"); TIMED(s, 1, launch_y<R>(s, false)); }
    { TraceRange t("cpf z pass (Green operator)"); TIMED(s, 2, launch_z<R>(s, ZMODE_FWD | ZMODE_GREEN)); }
    // the first stage of the scalar reduction rides in the inverse y pass's
    // launch when the fixed-length kernel runs it (one launch less per
    // iteration)
    const int nbc = (s->y_kinds & 1) ? (int)s->rv.size() * BC_CHUNKS : 0;
    { TraceRange t("cpf y pass (inverse)"); TIMED(s, 3, launch_y<R>(s, true, nullptr, 0, 0, 0, nullptr, 0, 0, nbc)); }
    { TraceRange t("cpf boundary update"); TIMED(s, 4, launch_bc<R>(s, nbc > 0)); }
    return CPF_OK;
}

// The executable graph of `len` iterations of the batch (captured on first
// use, kept until the graphs are dropped).  Every kernel reads the step's
// flags and buffer indices from device memory, so one graph serves every
// load step.
template <typename R>
static int graph_of(cpf_solver *s, const LawP<R> &P, int len, hipGraphExec_t *out)
{
    auto it = s->graphs.find(len);
    if (it != s->graphs.end()) {
        *out = it->second.second;
        return CPF_OK;
    }
    if (!s->stream)
        return fail(CPF_E_INVALID_ARG, "graph launches need a solver bound to a non-default stream");
    const bool was_timing = s->timing;
    s->timing = false;   // events are not recorded inside the graph
    HIPCHK(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
    int rc = CPF_OK;
    for (int i = 0; i < len && rc == CPF_OK; ++i) rc = launch_iteration<R>(s, P);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s->stream, &g);
    s->timing = was_timing;
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(CPF_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(CPF_E_HIP, "graph instantiation failed: %s", hipGetErrorString(e));
    }
    s->graphs[len] = {g, x};
    *out = x;
    return CPF_OK;
}

// Adaptive graph length: the least power of two (8 .. 1024) covering what
// the step is expected to need from here: 1.25 times the previous step's
// largest iteration count plus 2, less what is already queued; once that
// guess is used up, as many as are queued (the total doubles per replay).
static int adaptive_len(int prev, int queued, int max_iter)
{
    int want = prev > 0 ? (prev * 5 + 3) / 4 + 2 - queued : 16 - queued;
    want = std::max(want, std::max(8, queued));
    want = std::min(want, max_iter + 1 - queued);
    int len = 8;
    while (len < want && len < 1024) len *= 2;
    return len;
}

static int check_path(const cpf_path *p)
{
    if (!p || !p->t || !p->strain_ctrl || !p->target || p->n_steps < 1)
        return fail(CPF_E_INVALID_ARG, "path needs n_steps >= 1 and t, strain_ctrl, target");
    for (int n = 0; n < p->n_steps; ++n)
        if (!(p->t[n + 1] > p->t[n])) return fail(CPF_E_INVALID_ARG, "path times must increase");
    for (int i = 0; i < 6 * p->n_steps; ++i)
        if (!std::isfinite(p->target[i])) return fail(CPF_E_INVALID_ARG, "path targets must be finite");
    return CPF_OK;
}

template <typename R>
static int step_impl(cpf_solver *s, const cpf_path *path, int n, cpf_step_out *outs)
{
    TraceRange trace("cpf load step");
    const double dt = path->t[n + 1] - path->t[n];
    const int M = s->opt.rk4_M > 0 ? s->opt.rk4_M : substeps(dt, s->opt.h_max);
    const size_t nr = s->rv.size();
    for (size_t r = 0; r < nr; ++r) {
        RveHost &h = s->rv[r];
        StepInit &si = s->hsi[r];
        double dE0[6] = {0, 0, 0, 0, 0, 0};
        for (int i = 0; i < 6; ++i) {
            si.sidx[i] = path->strain_ctrl[6 * n + i] ? 0 : 1;
            si.target[i] = path->target[6 * n + i];
            if (!si.sidx[i]) dE0[i] = si.target[i] - h.E_n[i];
        }
        stress_block_inverse(s->K0, si.sidx, si.K0inv);
        // homogeneous reference-medium prediction of the stress-controlled part
        double rhs[6];
        for (int i = 0; i < 6; ++i) {
            double k = 0;
            for (int j = 0; j < 6; ++j) k += s->K0[i * 6 + j] * dE0[j];
            rhs[i] = si.sidx[i] ? (si.target[i] - h.Sigma_n[i]) - k : 0.0;
        }
        for (int i = 0; i < 6; ++i) {
            double d = 0;
            for (int j = 0; j < 6; ++j) d += si.K0inv[i * 6 + j] * rhs[j];
            if (si.sidx[i]) dE0[i] = d;
            si.dE0[i] = dE0[i];
            si.E0[i] = h.E_n[i] + dE0[i];
        }
        si.cur = h.cur;
        si.M = M;
        si.dt = dt;
    }
    HIPCHK(hipMemcpyAsync(s->ws + s->off_si, s->hsi, sizeof(StepInit) * nr, hipMemcpyHostToDevice, s->stream));
    hipLaunchKernelGGL(k_begin_step<R>, dim3(nr), dim3(64), 0, s->stream, dptr<RveDev<R>>(s, s->off_dev),
                       dptr<StepInit>(s, s->off_si));

    const LawP<R> P = make_law<R>(s);
    int queued = 0, prev = 0, syncs = 0;
    for (const auto &h : s->rv) prev = std::max(prev, h.prev_iters);
    int chunk = s->opt.check_every > 0 ? s->opt.check_every : std::max(2, prev);
    // timing events known to have completed (recorded before the last poll's
    // synchronization): read after the next launches are queued, while the
    // device works, not between the poll and those launches
    size_t ev_done = 0;
    for (;;) {
        TraceRange chunk_trace("cpf iterations until the next poll");
        if (s->graph_iters != 0) {
            const int len = s->graph_iters > 0 ? s->graph_iters : adaptive_len(prev, queued, s->opt.max_iter);
            hipGraphExec_t x = nullptr;
            int rc = graph_of<R>(s, P, len, &x);
            if (rc) return rc;
            HIPCHK(hipGraphLaunch(x, s->stream));
            queued += len;
        } else {
            for (int c = 0; c < chunk; ++c, ++queued) {
                int rc = launch_iteration<R>(s, P);
                if (rc) return rc;
            }
        }
        HIPCHK(hipGetLastError());
        for (size_t r = 0; r < nr; ++r)
            HIPCHK(hipMemcpyAsync(s->hsc + r, s->ws + s->rv[r].off_sc, sizeof(Scalars), hipMemcpyDeviceToHost,
                                  s->stream));
        {
            int rc = timed_collect(s, ev_done);
            if (rc) return rc;
        }
        HIPCHK(hipStreamSynchronize(s->stream));
        ++syncs;
        ev_done = s->ev_pending.size();
        bool all = true;
        for (size_t r = 0; r < nr; ++r) all = all && s->hsc[r].done;
        if (all) break;
        if (queued > s->opt.max_iter + 8)
            return fail(CPF_E_BAD_STATE, "device did not end the step after %d iterations", queued);
        chunk = s->opt.check_every > 0 ? s->opt.check_every : 4;
    }
    bool all_ok = true;
    for (size_t r = 0; r < nr; ++r) all_ok = all_ok && s->hsc[r].status == 0;
    if (all_ok) {
        // local-stress test of the converged step (k_symptom)
        const double E0 = s->mu0 * (3.0 * s->lam0 + 2.0 * s->mu0) / (s->lam0 + s->mu0);
        for (size_t r = 0; r < nr; ++r) {
            const RveHost &h = s->rv[r];
            double d2 = 0.0;
            for (int i = 0; i < 6; ++i) {
                const double d = s->hsc[r].E[i] - h.E_n[i];
                d2 += (i < 3 ? 1.0 : 2.0) * d * d;
            }
            const int a = h.cur, b = 1 - h.cur;
            unsigned long long *cnt =
                (unsigned long long *)(s->ws + h.off_sc + offsetof(Scalars, n_symptom));
            int *bad = (int *)(s->ws + h.off_sc + offsetof(Scalars, bad_state));
            hipLaunchKernelGGL(k_symptom<R>, dim3((h.nvox + 255) / 256), dim3(256), 0, s->stream,
                               dptr<int32_t>(s, h.off_labels), dptr<R>(s, h.off_Q), dptr<R>(s, h.off_eps[b]),
                               dptr<R>(s, h.off_st[b]), dptr<R>(s, h.off_eps[a]), dptr<R>(s, h.off_st[a]), P,
                               h.nvox, E0 * E0 * d2, s->D, cnt, bad);
            HIPCHK(hipGetLastError());
            static_assert(offsetof(Scalars, bad_state) == offsetof(Scalars, n_symptom) + sizeof(unsigned long long),
                          "the count and the flag are copied back together");
            HIPCHK(hipMemcpyAsync(&s->hsc[r].n_symptom, cnt, sizeof(unsigned long long) + sizeof(int),
                                  hipMemcpyDeviceToHost, s->stream));
        }
        {
            int rc = timed_collect(s);   // no timed launch since the last poll
            if (rc) return rc;
        }
        HIPCHK(hipStreamSynchronize(s->stream));
        for (size_t r = 0; r < nr; ++r)
            if (s->hsc[r].bad_state) {
                s->hsc[r].status = CPF_E_NAN;
                all_ok = false;
            }
    }
    {
        int rc = timed_collect(s);   // the last chunk's events when the check did not run
        if (rc) return rc;
    }
    int worst = CPF_OK, worst_r = -1;
    for (size_t r = 0; r < nr; ++r) {
        const Scalars &h = s->hsc[r];
        if (outs) {
            cpf_step_out *out = outs + r;
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
            out->stagnated = h.stagnated;
            out->host_syncs = syncs;
            out->n_symptom = all_ok ? (long long)h.n_symptom : 0;
            out->cutbacks = 0;
        }
        if (h.status != 0 && worst == CPF_OK) {
            worst = h.status;
            worst_r = (int)r;
        }
    }
    if (worst == CPF_E_NAN)
        return fail(CPF_E_NAN, "non-finite stress, residual or state in load step %d (RVE %d)", n, worst_r);
    if (worst == CPF_E_NOT_CONVERGED)
        return fail(CPF_E_NOT_CONVERGED, "load step %d (RVE %d): no convergence in %d iterations (err %.3g)", n,
                    worst_r, s->hsc[worst_r].iter,
                    std::max(s->hsc[worst_r].err_eq, s->hsc[worst_r].err_bc));
    // commit: the iterate and the trial state become the committed ones
    // (the lagged regularization first takes the raises of the next step
    // from the slip of this one)
    for (size_t r = 0; r < nr; ++r) {
        RveHost &h = s->rv[r];
        if (s->opt.reg_mode == CPF_REG_LAGGED) {
            const int S = (s->D - 6) / 2;
            const long n = (long)S * h.nvox;
            const int nb = (int)std::min<long>(4096, std::max<long>(1, (n + 255) / 256));
            hipLaunchKernelGGL(k_lag_update<R>, dim3(nb), dim3(256), 0, s->stream, dptr<R>(s, h.off_lag),
                               dptr<R>(s, h.off_st[1 - h.cur]), dptr<R>(s, h.off_st[h.cur]), h.nvox, S,
                               R(s->rv[r].pb.eta / dt));
            HIPCHK(hipGetLastError());
        }
        h.cur = 1 - h.cur;
        for (int i = 0; i < 6; ++i) { h.Sigma_n[i] = s->hsc[r].Sigma[i]; h.E_n[i] = s->hsc[r].E[i]; }
        h.prev_iters = s->hsc[r].iter;
    }
    return CPF_OK;
}

// A load step, retried as two half steps when it ends NOT_CONVERGED or NAN
// and halvings are left.  Nothing is committed by a failed attempt, so the
// retry starts from the same committed state.  The half step's targets are
// the midpoints between the committed mean strain (strain-controlled
// components) or mean stress (stress-controlled ones) of the first RVE and
// the step's targets.  Outputs: the last sub-step's, with the iterations
// and local-stress counts of all completed sub-steps summed and the failed
// attempts counted.
static int step_cut(cpf_solver *s, const cpf_path *path, int n, cpf_step_out *outs, int depth)
{
    int rc = s->prec == CPF_PREC_FP64 ? step_impl<double>(s, path, n, outs) : step_impl<float>(s, path, n, outs);
    if ((rc != CPF_E_NOT_CONVERGED && rc != CPF_E_NAN) || depth <= 0) return rc;
    const size_t nr = s->rv.size();
    const RveHost &h0 = s->rv[0];
    double t[3] = {path->t[n], 0.5 * (path->t[n] + path->t[n + 1]), path->t[n + 1]};
    uint8_t ctrl[12];
    double tg[12];
    for (int i = 0; i < 6; ++i) {
        ctrl[i] = ctrl[6 + i] = path->strain_ctrl[6 * n + i];
        const double from = ctrl[i] ? h0.E_n[i] : h0.Sigma_n[i];
        tg[i] = 0.5 * (from + path->target[6 * n + i]);
        tg[6 + i] = path->target[6 * n + i];
    }
    const cpf_path half = {2, t, ctrl, tg};
    std::vector<cpf_step_out> first(nr);
    rc = step_cut(s, &half, 0, outs ? first.data() : nullptr, depth - 1);
    if (rc) return rc;
    rc = step_cut(s, &half, 1, outs, depth - 1);
    if (rc) return rc;
    if (outs)
        for (size_t r = 0; r < nr; ++r) {
            outs[r].iters += first[r].iters;
            outs[r].n_symptom += first[r].n_symptom;
            outs[r].n_active += first[r].n_active;
            outs[r].n_newton += first[r].n_newton;
            outs[r].host_syncs += first[r].host_syncs;
            outs[r].cutbacks += first[r].cutbacks + 1;
        }
    return CPF_OK;
}

extern "C" int cpf_batch_step(cpf_solver *s, const cpf_path *path, int n, cpf_step_out *outs)
{
    if (!s || !s->bound) return fail(CPF_E_BAD_STATE, "solver not bound");
    int rc = check_path(path);
    if (rc) return rc;
    if (n < 0 || n >= path->n_steps) return fail(CPF_E_INVALID_ARG, "step %d outside the path", n);
    return step_cut(s, path, n, outs, s->opt.cutback);
}

extern "C" int cpf_solver_step(cpf_solver *s, const cpf_path *path, int n, cpf_step_out *out)
{
    if (s && s->rv.size() != 1) return fail(CPF_E_INVALID_ARG, "batch solver: use cpf_batch_step");
    return cpf_batch_step(s, path, n, out);
}

extern "C" int cpf_solver_run(cpf_solver *s, const cpf_path *path, cpf_step_out *out)
{
    if (!s || !s->bound) return fail(CPF_E_BAD_STATE, "solver not bound");
    int rc = check_path(path);
    if (rc) return rc;
    const int nr = (int)s->rv.size();
    for (int n = 0; n < path->n_steps; ++n) {
        rc = cpf_batch_step(s, path, n, out ? out + (size_t)n * nr : nullptr);
        if (rc) return rc;
    }
    return CPF_OK;
}

template <typename R>
static int field_impl(cpf_solver *s, int r, int field, void *dev_out)
{
    const RveHost &h = s->rv[r];
    const long nv = h.nvox;
    R *o = (R *)dev_out;
    const R *eps = dptr<R>(s, h.off_eps[h.cur]);
    const R *st = dptr<R>(s, h.off_st[h.cur]);
    const int nsys = h.pb.nsys;
    switch (field) {
    case CPF_FIELD_STRESS:
        hipLaunchKernelGGL(k_stress_field<R>, dim3((nv + 255) / 256), dim3(256), 0, s->stream,
                           dptr<int32_t>(s, h.off_labels), dptr<R>(s, h.off_Q), eps, st, o, make_law<R>(s), nv);
        HIPCHK(hipGetLastError());
        break;
    case CPF_FIELD_STRAIN:
        HIPCHK(hipMemcpyAsync(o, eps, sizeof(R) * 6 * nv, hipMemcpyDeviceToDevice, s->stream));
        break;
    case CPF_FIELD_PLASTIC_STRAIN:
        HIPCHK(hipMemcpyAsync(o, st, sizeof(R) * 6 * nv, hipMemcpyDeviceToDevice, s->stream));
        break;
    case CPF_FIELD_ACC_SLIP:
        HIPCHK(hipMemcpyAsync(o, st + 6 * nv, sizeof(R) * nsys * nv, hipMemcpyDeviceToDevice, s->stream));
        break;
    case CPF_FIELD_BACK_STRAIN:
        HIPCHK(hipMemcpyAsync(o, st + (6 + nsys) * nv, sizeof(R) * nsys * nv, hipMemcpyDeviceToDevice,
                              s->stream));
        break;
    case CPF_FIELD_SUBSTEPS:
        hipLaunchKernelGGL(k_substeps_field<R>, dim3((nv + 255) / 256), dim3(256), 0, s->stream,
                           dptr<int32_t>(s, h.off_mv), dptr<Scalars>(s, h.off_sc), o, nv, s->opt.rk_tol > 0.0 ? 1 : 0);
        HIPCHK(hipGetLastError());
        break;
    default:
        return fail(CPF_E_INVALID_ARG, "unknown field %d", field);
    }
    HIPCHK(hipStreamSynchronize(s->stream));
    return CPF_OK;
}

extern "C" int cpf_batch_field(cpf_solver *s, int rve, int field, void *dev_out)
{
    if (!s || !s->bound) return fail(CPF_E_BAD_STATE, "solver not bound");
    if (!dev_out) return fail(CPF_E_INVALID_ARG, "null output");
    if (rve < 0 || rve >= (int)s->rv.size()) return fail(CPF_E_INVALID_ARG, "RVE %d outside the batch", rve);
    return s->prec == CPF_PREC_FP64 ? field_impl<double>(s, rve, field, dev_out)
                                    : field_impl<float>(s, rve, field, dev_out);
}

extern "C" int cpf_solver_field(cpf_solver *s, int field, void *dev_out)
{
    return cpf_batch_field(s, 0, field, dev_out);
}

// ---------------------------------------------------------------------------
// tile autotuner
// ---------------------------------------------------------------------------
struct TuneKey {
    int nx, ny, nz, prec;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(nx, ny, nz, prec) < std::tie(o.nx, o.ny, o.nz, o.prec);
    }
};
static std::map<TuneKey, std::pair<int, int>> g_tune_cache;
static std::mutex g_tune_mu;

// Time `reps` launches of one pass of RVE r with a one-RVE table.
template <typename R>
static int time_pass(cpf_solver *s, int r, int ty, int tz, bool zpass, int reps, float *ms_out)
{
    RveHost h = s->rv[r];
    set_tiles<R>(h, ty, tz);
    RveDev<R> d = make_dev<R>(s, h, 0, 0, 0);
    RveDev<R> *tab = dptr<RveDev<R>>(s, s->off_opdev);
    HIPCHK(hipMemcpyAsync(tab, &d, sizeof d, hipMemcpyHostToDevice, s->stream));
    hipEvent_t a, b;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    for (int it = 0; it < reps + 1; ++it) {
        if (it == 1) HIPCHK(hipEventRecord(a, s->stream));
        if (zpass)
            launch_z<R>(s, ZMODE_FWD | ZMODE_GREEN, tab, 1, h.ntz * h.ny, lds_z_bytes<R>(h, tz), d.spec,
                        6 * h.nz * tz, z_kinds<R>(h, tz));
        else
            launch_y<R>(s, false, tab, 1, h.nty * h.nz, lds_y_bytes<R>(h, ty), d.spec, 6 * h.ny * ty,
                        y_kinds<R>(h, ty));
    }
    HIPCHK(hipEventRecord(b, s->stream));
    HIPCHK(hipEventSynchronize(b));
    HIPCHK(hipGetLastError());
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *ms_out = ms / reps;
    return CPF_OK;
}

template <typename R>
static int autotune_impl(cpf_solver *s, int *n_timed)
{
    *n_timed = 0;
    for (size_t r = 0; r < s->rv.size(); ++r) {
        RveHost &h = s->rv[r];
        const TuneKey key{h.nx, h.ny, h.nz, (int)sizeof(R)};
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tune_cache.find(key);
            if (it != g_tune_cache.end()) {
                set_tiles<R>(h, it->second.first, it->second.second);
                continue;
            }
        }
        const int cand[] = {1, 2, 4, 6, 8, 12, 16, 24, 32};
        int best_ty = h.ty, best_tz = h.tz;
        float best = 1e30f;
        for (int ty : cand) {
            if (!tiles_valid<R>(h, ty, h.tz)) continue;
            float ms;
            int rc = time_pass<R>(s, (int)r, ty, h.tz, false, 3, &ms);
            if (rc) return rc;
            ++*n_timed;
            if (ms < best) { best = ms; best_ty = ty; }
        }
        best = 1e30f;
        for (int tz : cand) {
            if (!tiles_valid<R>(h, best_ty, tz)) continue;
            float ms;
            int rc = time_pass<R>(s, (int)r, best_ty, tz, true, 3, &ms);
            if (rc) return rc;
            ++*n_timed;
            if (ms < best) { best = ms; best_tz = tz; }
        }
        set_tiles<R>(h, best_ty, best_tz);
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = {best_ty, best_tz};
    }
    // the tuning passes ran on the spectra: restore a clean start
    int rc = zero_state<R>(s);
    if (rc) return rc;
    return upload_devs<R>(s);
}

extern "C" int cpf_solver_autotune(cpf_solver *s, int *n_timed)
{
    if (!s || !s->bound) return fail(CPF_E_BAD_STATE, "solver not bound");
    int dummy = 0;
    drop_graph(s);
    int rc = s->prec == CPF_PREC_FP64 ? autotune_impl<double>(s, n_timed ? n_timed : &dummy)
                                      : autotune_impl<float>(s, n_timed ? n_timed : &dummy);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(s->stream));
    return CPF_OK;
}

template <typename R>
static int set_tiles_impl(cpf_solver *s, int rve, int ty, int tz)
{
    RveHost &h = s->rv[rve];
    if (!tiles_valid<R>(h, ty, tz))
        return fail(CPF_E_INVALID_ARG, "tiles (%d, %d) not valid for a %dx%dx%d grid", ty, tz, h.nx, h.ny, h.nz);
    set_tiles<R>(h, ty, tz);
    pass_grids<R>(s);
    return upload_devs<R>(s);
}

extern "C" int cpf_solver_set_tiles(cpf_solver *s, int rve, int ty, int tz)
{
    if (!s || !s->bound) return fail(CPF_E_BAD_STATE, "solver not bound");
    if (rve < 0 || rve >= (int)s->rv.size()) return fail(CPF_E_INVALID_ARG, "RVE %d outside the batch", rve);
    HIPCHK(hipStreamSynchronize(s->stream));
    drop_graph(s);
    int rc = s->prec == CPF_PREC_FP64 ? set_tiles_impl<double>(s, rve, ty, tz) : set_tiles_impl<float>(s, rve, ty, tz);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(s->stream));
    return CPF_OK;
}

extern "C" int cpf_solver_tiles(const cpf_solver *s, int rve, int *ty, int *tz)
{
    if (!s || !ty || !tz) return fail(CPF_E_INVALID_ARG, "null argument");
    if (rve < 0 || rve >= (int)s->rv.size()) return fail(CPF_E_INVALID_ARG, "RVE %d outside the batch", rve);
    *ty = s->rv[rve].ty;
    *tz = s->rv[rve].tz;
    return CPF_OK;
}

// ---------------------------------------------------------------------------
// component operators (RVE 0)
// ---------------------------------------------------------------------------
// The component operators work on caller spectra [nz][ny][nx/2+1][6]: all
// columns, unpadded rows.
template <typename R>
static RveHost op_host(const RveHost &solve)
{
    RveHost h = solve;
    h.nkx = h.nhp = h.nhx;
    set_tiles<R>(h, std::min(h.ty, h.nkx), std::min(h.tz, h.nkx));
    return h;
}

template <typename R>
static int op_fft_impl(cpf_solver *s, const void *field, void *spec)
{
    const RveHost h = op_host<R>(s->rv[0]);
    C2<R> *sp = (C2<R> *)spec;
    const RveDev<R> d = make_dev<R>(s, h, 0, 0, 0);
    RveDev<R> *tab = dptr<RveDev<R>>(s, s->off_opdev);
    HIPCHK(hipMemcpyAsync(tab, &d, sizeof d, hipMemcpyHostToDevice, s->stream));
    hipLaunchKernelGGL(k_xpass_fwd<R>, dim3(h.nbx), dim3(256), s->lds_x, s->stream, (const R *)field, sp, d);
    launch_y<R>(s, false, tab, 1, h.nty * h.nz, lds_y_bytes<R>(h, h.ty), sp, 6 * h.ny * h.ty, y_kinds<R>(h, h.ty));
    launch_z<R>(s, ZMODE_FWD, tab, 1, h.nbz, lds_z_bytes<R>(h, h.tz), sp, 6 * h.nz * h.tz, z_kinds<R>(h, h.tz));
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
    const RveHost h = op_host<R>(s->rv[0]);
    C2<R> *sp = (C2<R> *)spec;
    const RveDev<R> d = make_dev<R>(s, h, 0, 0, 0);
    RveDev<R> *tab = dptr<RveDev<R>>(s, s->off_opdev);
    HIPCHK(hipMemcpyAsync(tab, &d, sizeof d, hipMemcpyHostToDevice, s->stream));
    launch_z<R>(s, ZMODE_GREEN, tab, 1, h.nbz, lds_z_bytes<R>(h, h.tz), sp, 6 * h.nz * h.tz, z_kinds<R>(h, h.tz));
    launch_y<R>(s, true, tab, 1, h.nty * h.nz, lds_y_bytes<R>(h, h.ty), sp, 6 * h.ny * h.ty, y_kinds<R>(h, h.ty));
    hipLaunchKernelGGL(k_xpass_inv<R>, dim3(h.nbx), dim3(256), s->lds_x, s->stream, sp, (R *)outp, d);
    HIPCHK(hipGetLastError());
    if (err2) {
        std::vector<double> pz(h.nbz);
        HIPCHK(hipMemcpyAsync(pz.data(), s->ws + h.off_pz, sizeof(double) * h.nbz, hipMemcpyDeviceToHost,
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
    const RveHost &h = s->rv[0];
    const size_t lds = law_lds_bytes<R, NS>() + law_items_bytes<R>();
    hipLaunchKernelGGL((k_constitutive<R, NS, SPEC>), dim3((h.nvox + 255) / 256), dim3(256), lds, s->stream,
                       dptr<int32_t>(s, h.off_labels), dptr<R>(s, h.off_Q), (const R *)e0, (const R *)e1,
                       (const R *)s0, (R *)s1, (R *)sig, make_law<R>(s), h.nvox, R(dt), M);
}

template <typename R>
static int op_cp_impl(cpf_solver *s, const void *e0, const void *e1, const void *s0, void *s1, void *sig,
                      double dt, int M)
{
    if (s->law_spec == LAW_TABLE1) {
        if (s->ns_inst == 12) launch_cp<R, 12, LAW_TABLE1>(s, e0, e1, s0, s1, sig, dt, M);
        else launch_cp<R, 16, LAW_TABLE1>(s, e0, e1, s0, s1, sig, dt, M);
    } else {
        switch (s->ns_inst) {
        case 4: launch_cp<R, 4>(s, e0, e1, s0, s1, sig, dt, M); break;
        case 12: launch_cp<R, 12>(s, e0, e1, s0, s1, sig, dt, M); break;
        case 16: launch_cp<R, 16>(s, e0, e1, s0, s1, sig, dt, M); break;
        default: launch_cp<R, 32>(s, e0, e1, s0, s1, sig, dt, M); break;
        }
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
    if (s->opt.reg_mode != CPF_REG_IMPLICIT)
        return fail(CPF_E_INVALID_ARG, "the component operator evaluates the implicit regularization only");
    return s->prec == CPF_PREC_FP64 ? op_cp_impl<double>(s, e0, e1, s0, s1, sig, dt, M)
                                    : op_cp_impl<float>(s, e0, e1, s0, s1, sig, dt, M);
}

// ---------------------------------------------------------------------------
// discrete adjoint of the load-stepped solve (single RVE)
// ---------------------------------------------------------------------------
struct AdjLayout {
    size_t mu, g, A, Sb, eb, scratch, seg, ckpt, th, total;
    int M_max, n_ckpt, C, nblk;
};

template <typename R>
static AdjLayout adj_layout(const cpf_solver *s, const cpf_path *path, int C)
{
    const RveHost &h = s->rv[0];
    const size_t N = h.nvox, D = s->D;
    AdjLayout a;
    a.C = C;
    a.n_ckpt = (path->n_steps + C - 1) / C;
    a.M_max = 1;
    for (int n = 0; n < path->n_steps; ++n) {
        const double dt = path->t[n + 1] - path->t[n];
        a.M_max = std::max(a.M_max, s->opt.rk4_M > 0 ? s->opt.rk4_M : substeps(dt, s->opt.h_max));
    }
    a.nblk = (int)((N + 255) / 256);
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
    a.mu = take(sizeof(R) * 6 * N);
    a.g = take(sizeof(R) * 6 * N);
    a.A = take(sizeof(R) * 36 * N);
    a.Sb = take(sizeof(R) * D * N);
    a.eb = take(sizeof(R) * 6 * N);
    a.scratch = take(sizeof(R) * (size_t)a.M_max * 4 * (D + s->n_slip + s->n_twin) * N);
    // checkpoints at steps 0, C, 2C, ... and the end state; a segment's
    // other start states are recomputed into C - 1 slots
    a.seg = take(sizeof(R) * (size_t)(C - 1) * (6 + D) * N);
    a.ckpt = take(sizeof(R) * (size_t)(a.n_ckpt + 1) * (6 + D) * N);
    a.th = take(sizeof(double) * NTH * a.nblk);
    a.total = o;
    return a;
}

extern "C" int cpf_adjoint_workspace_size(const cpf_solver *s, const cpf_path *path, int checkpoint_every,
                                          size_t *bytes)
{
    if (!s || !bytes) return fail(CPF_E_INVALID_ARG, "null argument");
    if (s->rv.size() != 1) return fail(CPF_E_INVALID_ARG, "the adjoint needs a single-RVE solver");
    if (s->opt.rk_tol > 0.0)
        return fail(CPF_E_INVALID_ARG, "the adjoint replays fixed substep counts: rk_tol must be 0");
    if (s->opt.aa_depth > 0)
        return fail(CPF_E_INVALID_ARG, "the adjoint runs the basic fixed point: aa_depth must be 0");
    if (s->opt.reg_mode != CPF_REG_IMPLICIT)
        return fail(CPF_E_INVALID_ARG, "the adjoint differentiates the implicit regularization only");
    int rc = check_path(path);
    if (rc) return rc;
    if (checkpoint_every < 1) return fail(CPF_E_INVALID_ARG, "checkpoint_every must be >= 1");
    *bytes = s->prec == CPF_PREC_FP64 ? adj_layout<double>(s, path, checkpoint_every).total
                                      : adj_layout<float>(s, path, checkpoint_every).total;
    return CPF_OK;
}

template <typename R, int NS, int SPEC>
static void launch_law_adj(cpf_solver *s, const AdjArgs<R> &a, int what)
{
    const RveHost &h = s->rv[0];
    const dim3 grid((h.nvox + 255) / 256), block(256);
    const LawP<R> P = make_law<R>(s);
    const size_t lds = law_lds_bytes<R, NS>() + law_items_bytes<R>();
    if (what == 0) hipLaunchKernelGGL((k_law_record<R, NS, SPEC>), grid, block, lds, s->stream, a, P);
    else if (what == 1) hipLaunchKernelGGL((k_law_vjp<R, NS, SPEC, VJP_GA>), grid, block, 0, s->stream, a, P);
    else hipLaunchKernelGGL((k_law_vjp<R, NS, SPEC, VJP_F>), grid, block, 0, s->stream, a, P);
}

// what: 0 record the forward stages, 1 g and A sweeps, 2 final sweep
template <typename R>
static int launch_law_adj_any(cpf_solver *s, const AdjArgs<R> &a, int what)
{
    if (s->law_spec == LAW_TABLE1) {
        if (s->ns_inst == 12) launch_law_adj<R, 12, LAW_TABLE1>(s, a, what);
        else launch_law_adj<R, 16, LAW_TABLE1>(s, a, what);
    } else {
        switch (s->ns_inst) {
        case 4: launch_law_adj<R, 4, LAW_GENERAL>(s, a, what); break;
        case 12: launch_law_adj<R, 12, LAW_GENERAL>(s, a, what); break;
        case 16: launch_law_adj<R, 16, LAW_GENERAL>(s, a, what); break;
        default: launch_law_adj<R, 32, LAW_GENERAL>(s, a, what); break;
        }
    }
    HIPCHK(hipGetLastError());
    return CPF_OK;
}

template <typename R>
static int copy_fields(cpf_solver *s, void *dst, const void *src, size_t bytes)
{
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s->stream));
    return CPF_OK;
}

// Solve the transposed-tangent equilibrium of step n for mu (on the device).
template <typename R>
static int adjoint_equilibrium(cpf_solver *s, const cpf_path *path, int n, const AdjArgs<R> &a, double tol,
                               int *iters)
{
    const RveHost &h = s->rv[0];
    StepInit &si = s->hsi[0];
    memset(&si, 0, sizeof si);
    for (int i = 0; i < 6; ++i) si.sidx[i] = path->strain_ctrl[6 * n + i] ? 0 : 1;
    stress_block_inverse(s->K0, si.sidx, si.K0inv);
    si.cur = h.cur;
    si.M = 1;
    si.dt = 1.0;
    HIPCHK(hipMemcpyAsync(s->ws + s->off_si, s->hsi, sizeof(StepInit), hipMemcpyHostToDevice, s->stream));
    hipLaunchKernelGGL(k_begin_step<R>, dim3(1), dim3(64), 0, s->stream, dptr<RveDev<R>>(s, s->off_dev),
                       dptr<StepInit>(s, s->off_si));
    int queued = 0, chunk = 8;
    for (;;) {
        for (int c = 0; c < chunk; ++c, ++queued) {
            hipLaunchKernelGGL(k_adj_xpass<R>, dim3(h.nbx), dim3(256), s->lds_x, s->stream, a);
            launch_y<R>(s, false);
            launch_z<R>(s, ZMODE_FWD | ZMODE_GREEN);
            launch_y<R>(s, true);
            hipLaunchKernelGGL(k_adj_bc<R>, dim3(1), dim3(256), 0, s->stream, dptr<RveDev<R>>(s, s->off_dev), tol,
                               s->opt.max_iter);
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(s->hsc, s->ws + h.off_sc, sizeof(Scalars), hipMemcpyDeviceToHost, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
        if (s->hsc->done) break;
        if (queued > s->opt.max_iter + 16)
            return fail(CPF_E_BAD_STATE, "adjoint equilibrium of step %d did not end", n);
        chunk = 8;
    }
    if (s->hsc->status == CPF_E_NAN) return fail(CPF_E_NAN, "adjoint equilibrium of step %d: non-finite", n);
    if (s->hsc->status == CPF_E_NOT_CONVERGED)
        return fail(CPF_E_NOT_CONVERGED, "adjoint equilibrium of step %d: no convergence in %d iterations", n,
                    s->hsc->iter);
    *iters = s->hsc->iter;
    return CPF_OK;
}

template <typename R>
// target != nullptr: cotangent 2 (Sigma_11 - target_n) e_11 of the stress
// curve loss (returned in *loss); else the caller's sbar[n][6].
static int adjoint_impl(cpf_solver *s, const cpf_path *path, const double *target, const double *sbar, int C,
                        double adj_tol, unsigned char *aws, double *loss, double *grad, double *sig_out)
{
    TraceRange trace("cpf adjoint (forward with checkpoints, then reverse)");
    const AdjLayout L = adj_layout<R>(s, path, C);
    RveHost &h = s->rv[0];
    const long N = h.nvox;
    const int D = s->D, ns = path->n_steps;
    const size_t fe = sizeof(R) * 6 * N, fs = sizeof(R) * D * N, slot = fe + fs;
    auto P = [&](size_t off) { return aws + off; };
    std::vector<double> Sig((size_t)ns * 6), Sbar((size_t)ns * 6, 0.0);
    struct Ck { double Sigma[6], E[6]; int prev; };
    std::vector<Ck> ck(L.n_ckpt);
    cpf_step_out out;

    s->adj_fwd_iters = s->adj_eq_iters = 0;
    s->adj_recomputed = 0;
    // forward with checkpoints
    int rc = zero_state<R>(s);
    if (rc) return rc;
    for (int n = 0; n < ns; ++n) {
        if (n % C == 0) {
            unsigned char *c = P(L.ckpt) + (size_t)(n / C) * slot;
            rc = copy_fields<R>(s, c, s->ws + h.off_eps[h.cur], fe);
            if (!rc) rc = copy_fields<R>(s, c + fe, s->ws + h.off_st[h.cur], fs);
            if (rc) return rc;
            Ck &k = ck[n / C];
            memcpy(k.Sigma, h.Sigma_n, sizeof k.Sigma);
            memcpy(k.E, h.E_n, sizeof k.E);
            k.prev = h.prev_iters;
        }
        rc = step_impl<R>(s, path, n, &out);
        if (rc) return rc;
        for (int c = 0; c < 6; ++c) Sig[(size_t)n * 6 + c] = out.Sigma[c];
        s->adj_fwd_iters += out.iters;
    }
    {
        unsigned char *c = P(L.ckpt) + (size_t)L.n_ckpt * slot;
        rc = copy_fields<R>(s, c, s->ws + h.off_eps[h.cur], fe);
        if (!rc) rc = copy_fields<R>(s, c + fe, s->ws + h.off_st[h.cur], fs);
        if (rc) return rc;
    }
    double Lsum = 0;
    for (int n = 0; n < ns; ++n) {
        if (target) {
            const double r = Sig[(size_t)n * 6] - target[n];
            Lsum += r * r;
            Sbar[(size_t)n * 6] = 2.0 * r;
        } else {
            for (int c = 0; c < 6; ++c) Sbar[(size_t)n * 6 + c] = sbar[(size_t)n * 6 + c];
        }
    }

    // reverse
    AdjArgs<R> a;
    a.rv = dptr<RveDev<R>>(s, s->off_dev);
    a.scratch = (R *)P(L.scratch);
    a.g = (R *)P(L.g);
    a.A = (R *)P(L.A);
    a.mu = (R *)P(L.mu);
    a.Sb = (R *)P(L.Sb);
    a.eb = (R *)P(L.eb);
    a.th_part = (double *)P(L.th);
    hipLaunchKernelGGL(k_fill<R>, dim3(512), dim3(256), 0, s->stream, a.Sb, (long)D * N, R(0));
    hipLaunchKernelGGL(k_fill<R>, dim3(512), dim3(256), 0, s->stream, a.eb, 6L * N, R(0));
    double G[NTH] = {0};
    std::vector<double> thp((size_t)NTH * L.nblk);
    for (int sg = L.n_ckpt - 1; sg >= 0; --sg) {
        const int n0 = sg * C, n1 = std::min(ns, n0 + C);
        // start states of the segment: the checkpoint, then recomputed steps
        const unsigned char *c = P(L.ckpt) + (size_t)sg * slot;
        if (n1 - n0 > 1) {
            rc = copy_fields<R>(s, s->ws + h.off_eps[h.cur], c, fe);
            if (!rc) rc = copy_fields<R>(s, s->ws + h.off_st[h.cur], c + fe, fs);
            if (rc) return rc;
            memcpy(h.Sigma_n, ck[sg].Sigma, sizeof h.Sigma_n);
            memcpy(h.E_n, ck[sg].E, sizeof h.E_n);
            h.prev_iters = ck[sg].prev;
            for (int n = n0; n < n1 - 1; ++n) {
                rc = step_impl<R>(s, path, n, &out);
                if (rc) return rc;
                s->adj_fwd_iters += out.iters;
                s->adj_recomputed += 1;
                unsigned char *sl = P(L.seg) + (size_t)(n - n0) * slot;
                rc = copy_fields<R>(s, sl, s->ws + h.off_eps[h.cur], fe);
                if (!rc) rc = copy_fields<R>(s, sl + fe, s->ws + h.off_st[h.cur], fs);
                if (rc) return rc;
            }
        }
        auto start_of = [&](int n) -> const unsigned char * {
            return n == n0 ? c : n == n1 ? P(L.ckpt) + (size_t)(sg + 1) * slot
                                         : P(L.seg) + (size_t)(n - n0 - 1) * slot;
        };
        for (int n = n1 - 1; n >= n0; --n) {
            TraceRange step_trace("cpf adjoint load step");
            const unsigned char *sl = start_of(n);
            a.e0 = (const R *)sl;
            a.st0 = (const R *)(sl + fe);
            a.e1 = (const R *)start_of(n + 1);
            for (int c = 0; c < 6; ++c) a.sigL[c] = R(Sbar[(size_t)n * 6 + c] / (double)N);
            a.dt = R(path->t[n + 1] - path->t[n]);
            a.M = s->opt.rk4_M > 0 ? s->opt.rk4_M : substeps(path->t[n + 1] - path->t[n], s->opt.h_max);
            rc = launch_law_adj_any<R>(s, a, 0);
            if (!rc) rc = launch_law_adj_any<R>(s, a, 1);
            if (rc) return rc;
            int its = 0;
            rc = adjoint_equilibrium<R>(s, path, n, a, adj_tol, &its);
            if (rc) return rc;
            s->adj_eq_iters += its;
            rc = launch_law_adj_any<R>(s, a, 2);
            if (rc) return rc;
            HIPCHK(hipMemcpyAsync(thp.data(), a.th_part, sizeof(double) * thp.size(), hipMemcpyDeviceToHost,
                                  s->stream));
            HIPCHK(hipStreamSynchronize(s->stream));
            for (int b = 0; b < L.nblk; ++b)
                for (int k = 0; k < NTH; ++k) G[k] += thp[(size_t)b * NTH + k];
        }
    }
    // leave the solver at the undeformed state
    rc = zero_state<R>(s);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(s->stream));
    if (loss) *loss = Lsum;
    for (int k = 0; k < NTH; ++k) grad[k] = G[k];
    if (sig_out)
        for (size_t i = 0; i < Sig.size(); ++i) sig_out[i] = Sig[i];
    return CPF_OK;
}

static int adjoint_entry(cpf_solver *s, const cpf_path *path, const double *target, const double *sbar,
                         int checkpoint_every, double adj_tol, void *dev_ws, size_t bytes, double *loss,
                         double *grad, double *sig_out)
{
    if (!s || !s->bound) return fail(CPF_E_BAD_STATE, "solver not bound");
    if (s->rv.size() != 1) return fail(CPF_E_INVALID_ARG, "the adjoint needs a single-RVE solver");
    if ((!target && !sbar) || !grad) return fail(CPF_E_INVALID_ARG, "null argument");
    if (!(adj_tol > 0)) return fail(CPF_E_INVALID_ARG, "adj_tol must be > 0");
    size_t need = 0;
    int rc = cpf_adjoint_workspace_size(s, path, checkpoint_every, &need);
    if (rc) return rc;
    if (sbar)
        for (int i = 0; i < 6 * path->n_steps; ++i)
            if (!std::isfinite(sbar[i])) return fail(CPF_E_INVALID_ARG, "sigma_bar[%d] is not finite", i);
    if (!dev_ws || bytes < need)
        return fail(CPF_E_WORKSPACE, "adjoint workspace of %zu bytes given, %zu needed", bytes, need);
    if (((uintptr_t)dev_ws) & 255) return fail(CPF_E_WORKSPACE, "adjoint workspace must be 256-byte aligned");
    drop_graph(s);
    const int g = s->graph_iters;
    s->graph_iters = 0;
    rc = s->prec == CPF_PREC_FP64
             ? adjoint_impl<double>(s, path, target, sbar, checkpoint_every, adj_tol, (unsigned char *)dev_ws,
                                    loss, grad, sig_out)
             : adjoint_impl<float>(s, path, target, sbar, checkpoint_every, adj_tol, (unsigned char *)dev_ws,
                                   loss, grad, sig_out);
    s->graph_iters = g;
    if (rc) {
        // back to the undeformed state; the first error stays reported
        if (s->prec == CPF_PREC_FP64) zero_state<double>(s);
        else zero_state<float>(s);
        (void)hipStreamSynchronize(s->stream);
    }
    return rc;
}

extern "C" int cpf_adjoint_gradient(cpf_solver *s, const cpf_path *path, const double *target_xx,
                                    int checkpoint_every, double adj_tol, void *dev_ws, size_t bytes, double *loss,
                                    double *grad, double *sigma_xx)
{
    if (!target_xx || !loss || !grad) return fail(CPF_E_INVALID_ARG, "null argument");
    std::vector<double> sig;
    if (sigma_xx && path && path->n_steps > 0) sig.resize((size_t)path->n_steps * 6);
    const int rc = adjoint_entry(s, path, target_xx, nullptr, checkpoint_every, adj_tol, dev_ws, bytes, loss, grad,
                                 sig.empty() ? nullptr : sig.data());
    if (!rc && !sig.empty())
        for (int n = 0; n < path->n_steps; ++n) sigma_xx[n] = sig[(size_t)n * 6];
    return rc;
}

extern "C" int cpf_adjoint_vjp(cpf_solver *s, const cpf_path *path, const double *sigma_bar, int checkpoint_every,
                               double adj_tol, void *dev_ws, size_t bytes, double *grad, double *sigma)
{
    if (!sigma_bar || !grad) return fail(CPF_E_INVALID_ARG, "null argument");
    return adjoint_entry(s, path, nullptr, sigma_bar, checkpoint_every, adj_tol, dev_ws, bytes, nullptr, grad,
                         sigma);
}

// ---------------------------------------------------------------------------
// von Mises stress histogram of the committed state
// ---------------------------------------------------------------------------
template <typename R>
static int seq_hist_impl(cpf_solver *s, int rve, int nbins, double lo, double hi, unsigned long long *counts)
{
    unsigned long long *dc = dptr<unsigned long long>(s, s->off_hist);
    double *dq = reinterpret_cast<double *>(dc + CPF_MAX_HIST_BINS + 2);
    hipLaunchKernelGGL(k_fill<unsigned long long>, dim3(16), dim3(256), 0, s->stream, dc, (long)nbins + 2, 0ull);
    // squared bin edges: e_k = lo + k w, w = (hi - lo) / nbins; -1 where e_k <= 0
    std::vector<double> q(nbins + 1);
    const double w = (hi - lo) / nbins;
    for (int k = 0; k <= nbins; ++k) {
        const double e = lo + k * w;
        q[k] = e > 0.0 ? e * e : -1.0;
    }
    HIPCHK(hipMemcpyAsync(dq, q.data(), sizeof(double) * q.size(), hipMemcpyHostToDevice, s->stream));
    const LawP<R> P = make_law<R>(s);
    for (int r = 0; r < (int)s->rv.size(); ++r) {
        if (rve >= 0 && r != rve) continue;
        const RveHost &h = s->rv[r];
        // the stress field exactly as cpf_batch_field exports it, staged in
        // the RVE's spectrum area (scratch between load steps: 6 nz ny nhp
        // complex values hold 6 nvox reals)
        R *sig = dptr<R>(s, h.off_spec);
        hipLaunchKernelGGL(k_stress_field<R>, dim3((h.nvox + 255) / 256), dim3(256), 0, s->stream,
                           dptr<int32_t>(s, h.off_labels), dptr<R>(s, h.off_Q), dptr<R>(s, h.off_eps[h.cur]),
                           dptr<R>(s, h.off_st[h.cur]), sig, P, h.nvox);
        const long blocks = std::min<long>((h.nvox + 255) / 256, 2048);
        const size_t lds = sizeof(double) * (nbins + 1) + sizeof(unsigned int) * (nbins + 2);
        hipLaunchKernelGGL(k_seq_hist<R>, dim3(blocks), dim3(256), lds, s->stream, (const R *)sig, h.nvox, nbins,
                           (const double *)dq, dc);
        HIPCHK(hipGetLastError());
    }
    HIPCHK(hipMemcpyAsync(counts, dc, sizeof(unsigned long long) * (nbins + 2), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return CPF_OK;
}

extern "C" int cpf_seq_histogram(cpf_solver *s, int rve, int nbins, double lo, double hi,
                                 unsigned long long *counts)
{
    if (!s || !s->bound) return fail(CPF_E_BAD_STATE, "solver not bound");
    if (!counts) return fail(CPF_E_INVALID_ARG, "null argument");
    if (rve < -1 || rve >= (int)s->rv.size()) return fail(CPF_E_INVALID_ARG, "rve %d out of range", rve);
    if (nbins < 1 || nbins > CPF_MAX_HIST_BINS)
        return fail(CPF_E_INVALID_ARG, "nbins %d: need 1..%d", nbins, CPF_MAX_HIST_BINS);
    if (!std::isfinite(lo) || !std::isfinite(hi) || !(hi > lo))
        return fail(CPF_E_INVALID_ARG, "need finite lo < hi");
    return s->prec == CPF_PREC_FP64 ? seq_hist_impl<double>(s, rve, nbins, lo, hi, counts)
                                    : seq_hist_impl<float>(s, rve, nbins, lo, hi, counts);
}

// ---------------------------------------------------------------------------
// The same histogram of a caller's stress field, with no workspace: the
// device counts and squared edges live in one fixed array per GPU.
// ---------------------------------------------------------------------------
static constexpr size_t HIST_COUNTS_BYTES = sizeof(unsigned long long) * (CPF_MAX_HIST_BINS + 2);
static constexpr size_t HIST_EDGES_OFF = (HIST_COUNTS_BYTES + 255) / 256 * 256;
static_assert(HIST_EDGES_OFF + sizeof(double) * (CPF_MAX_HIST_BINS + 1) <= CPF_HIST_SCRATCH_BYTES,
              "histogram scratch too small");

// Device array of the allocation-free histogram.  In host code this name
// is only a stand-in: the address on each device comes from
// hipGetSymbolAddress (scratch_ptr below) and is what kernels receive.
static __device__ __align__(256) unsigned char scratch[CPF_HIST_SCRATCH_BYTES];

static constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static unsigned char *g_scratch_dev[SCRATCH_MAX_DEVICES];   // per device, set on first use

// Address of `scratch` on the current device (looked up once per device,
// with that device current).
static int scratch_ptr(unsigned char **out)
{
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return fail(CPF_E_INVALID_ARG, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(CPF_E_HIP, "hipGetSymbolAddress returned no address");
        g_scratch_dev[dev] = static_cast<unsigned char *>(p);
    }
    *out = g_scratch_dev[dev];
    return CPF_OK;
}

// Squared bin edges e_k = lo + k w (-1 where e_k <= 0), each operation
// rounded on its own as in the host loop of seq_hist_impl.
__global__ void k_hist_edges(double lo, double w, int nbins, double *q)
{
#pragma clang fp contract(off)
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k <= nbins; k += gridDim.x * blockDim.x) {
        const double e = lo + (double)k * w;
        q[k] = e > 0.0 ? e * e : -1.0;
    }
}

extern "C" int cpf_seq_histogram_field(const void *dev_sig, int precision, long long nvox, int nbins, double lo,
                                       double hi, unsigned long long *counts, void *hip_stream)
{
    if (!counts || (nvox > 0 && !dev_sig)) return fail(CPF_E_INVALID_ARG, "null argument");
    if (precision != CPF_PREC_FP64 && precision != CPF_PREC_FP32)
        return fail(CPF_E_INVALID_ARG, "precision %d", precision);
    if (nvox < 0) return fail(CPF_E_INVALID_ARG, "nvox %lld < 0", nvox);
    if (nbins < 1 || nbins > CPF_MAX_HIST_BINS)
        return fail(CPF_E_INVALID_ARG, "nbins %d: need 1..%d (the fixed device array holds at most %d bins)",
                    nbins, CPF_MAX_HIST_BINS, CPF_MAX_HIST_BINS);
    if (!std::isfinite(lo) || !std::isfinite(hi) || !(hi > lo))
        return fail(CPF_E_INVALID_ARG, "need finite lo < hi");
    unsigned char *base = nullptr;
    if (int rc = scratch_ptr(&base)) return rc;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    unsigned long long *dc = reinterpret_cast<unsigned long long *>(base);
    double *dq = reinterpret_cast<double *>(base + HIST_EDGES_OFF);
    // the array keeps the previous call's counts: clear them (a kernel, no memset node)
    hipLaunchKernelGGL(k_fill<unsigned long long>, dim3(16), dim3(256), 0, st, dc, (long)nbins + 2, 0ull);
    hipLaunchKernelGGL(k_hist_edges, dim3((nbins + 256) / 256), dim3(256), 0, st, lo, (hi - lo) / nbins, nbins, dq);
    if (nvox > 0) {
        const long blocks = std::min<long>((nvox + 255) / 256, 2048);
        const size_t lds = sizeof(double) * (nbins + 1) + sizeof(unsigned int) * (nbins + 2);
        if (precision == CPF_PREC_FP64)
            hipLaunchKernelGGL(k_seq_hist<double>, dim3(blocks), dim3(256), lds, st, (const double *)dev_sig,
                               (long)nvox, nbins, (const double *)dq, dc);
        else
            hipLaunchKernelGGL(k_seq_hist<float>, dim3(blocks), dim3(256), lds, st, (const float *)dev_sig,
                               (long)nvox, nbins, (const double *)dq, dc);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(counts, dc, sizeof(unsigned long long) * (nbins + 2), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return CPF_OK;
}

// ---------------------------------------------------------------------------
// committed state save / restore
// ---------------------------------------------------------------------------
struct SavedHead {
    double Sigma[6], E[6];
    int prev_iters;
    int reg_mode;   // the saving solver's regularization reading (the layout
                    // of the sections that follow depends on it)
};

// Buffer layout: one SavedHead per RVE, then per RVE the committed strain
// [6][N], state [D][N] and, with the lagged regularization, the raises
// [S][N] of the next step, in the solver's precision, 256-byte sections.
static size_t lag_words(const cpf_solver *s, const RveHost &h)
{
    return s->opt.reg_mode == CPF_REG_LAGGED ? (size_t)(s->D - 6) / 2 * h.nvox : 0;
}

static size_t state_layout(const cpf_solver *s, std::vector<size_t> *off)
{
    const size_t rb = s->prec == CPF_PREC_FP64 ? 8 : 4;
    size_t o = align256(sizeof(SavedHead) * s->rv.size());
    for (const auto &h : s->rv) {
        if (off) off->push_back(o);
        o = align256(o + rb * 6 * (size_t)h.nvox);
        if (off) off->push_back(o);
        o = align256(o + rb * (size_t)s->D * h.nvox);
        if (off) off->push_back(o);
        o = align256(o + rb * lag_words(s, h));
    }
    return o;
}

extern "C" int cpf_state_size(const cpf_solver *s, size_t *bytes)
{
    if (!s || !bytes) return fail(CPF_E_INVALID_ARG, "null argument");
    *bytes = state_layout(s, nullptr);
    return CPF_OK;
}

static int state_check(const cpf_solver *s, const void *buf)
{
    if (!s || !s->bound) return fail(CPF_E_BAD_STATE, "solver not bound");
    if (!buf) return fail(CPF_E_INVALID_ARG, "null device buffer");
    if (((uintptr_t)buf) & 255) return fail(CPF_E_WORKSPACE, "state buffer must be 256-byte aligned");
    return CPF_OK;
}

extern "C" int cpf_state_save(cpf_solver *s, void *dev_buf)
{
    int rc = state_check(s, dev_buf);
    if (rc) return rc;
    std::vector<size_t> off;
    state_layout(s, &off);
    const size_t rb = s->prec == CPF_PREC_FP64 ? 8 : 4;
    std::vector<SavedHead> head(s->rv.size());
    unsigned char *b = (unsigned char *)dev_buf;
    for (size_t r = 0; r < s->rv.size(); ++r) {
        const RveHost &h = s->rv[r];
        memcpy(head[r].Sigma, h.Sigma_n, sizeof h.Sigma_n);
        memcpy(head[r].E, h.E_n, sizeof h.E_n);
        head[r].prev_iters = h.prev_iters;
        head[r].reg_mode = s->opt.reg_mode;
        HIPCHK(hipMemcpyAsync(b + off[3 * r], s->ws + h.off_eps[h.cur], rb * 6 * h.nvox, hipMemcpyDeviceToDevice,
                              s->stream));
        HIPCHK(hipMemcpyAsync(b + off[3 * r + 1], s->ws + h.off_st[h.cur], rb * s->D * h.nvox,
                              hipMemcpyDeviceToDevice, s->stream));
        if (lag_words(s, h))
            HIPCHK(hipMemcpyAsync(b + off[3 * r + 2], s->ws + h.off_lag, rb * lag_words(s, h),
                                  hipMemcpyDeviceToDevice, s->stream));
    }
    HIPCHK(hipMemcpyAsync(b, head.data(), sizeof(SavedHead) * head.size(), hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return CPF_OK;
}

extern "C" int cpf_state_restore(cpf_solver *s, const void *dev_buf)
{
    int rc = state_check(s, dev_buf);
    if (rc) return rc;
    std::vector<size_t> off;
    state_layout(s, &off);
    const size_t rb = s->prec == CPF_PREC_FP64 ? 8 : 4;
    std::vector<SavedHead> head(s->rv.size());
    const unsigned char *b = (const unsigned char *)dev_buf;
    HIPCHK(hipMemcpyAsync(head.data(), b, sizeof(SavedHead) * head.size(), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    for (size_t r = 0; r < s->rv.size(); ++r)
        for (int i = 0; i < 6; ++i)
            if (!std::isfinite(head[r].Sigma[i]) || !std::isfinite(head[r].E[i]) ||
                head[r].reg_mode != s->opt.reg_mode)
                return fail(CPF_E_INVALID_ARG, "state buffer does not hold a saved state of this solver "
                                               "(or holds one of the other regularization reading)");
    for (size_t r = 0; r < s->rv.size(); ++r) {
        RveHost &h = s->rv[r];
        memcpy(h.Sigma_n, head[r].Sigma, sizeof h.Sigma_n);
        memcpy(h.E_n, head[r].E, sizeof h.E_n);
        h.prev_iters = std::max(1, head[r].prev_iters);
        HIPCHK(hipMemcpyAsync(s->ws + h.off_eps[h.cur], b + off[3 * r], rb * 6 * h.nvox, hipMemcpyDeviceToDevice,
                              s->stream));
        HIPCHK(hipMemcpyAsync(s->ws + h.off_st[h.cur], b + off[3 * r + 1], rb * s->D * h.nvox,
                              hipMemcpyDeviceToDevice, s->stream));
        if (lag_words(s, h))
            HIPCHK(hipMemcpyAsync(s->ws + h.off_lag, b + off[3 * r + 2], rb * lag_words(s, h),
                                  hipMemcpyDeviceToDevice, s->stream));
    }
    HIPCHK(hipStreamSynchronize(s->stream));
    return CPF_OK;
}

extern "C" int cpf_adjoint_last_stats(const cpf_solver *s, long long *fwd_iters, long long *adj_iters,
                                      int *recomputed_steps)
{
    if (!s || !fwd_iters || !adj_iters || !recomputed_steps) return fail(CPF_E_INVALID_ARG, "null argument");
    *fwd_iters = s->adj_fwd_iters;
    *adj_iters = s->adj_eq_iters;
    *recomputed_steps = s->adj_recomputed;
    return CPF_OK;
}

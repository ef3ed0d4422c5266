/*
 * CPU ORACLE -- test infrastructure only.  Plain FP64 reference for the
 * Meric-Cailletaud crystal-plasticity law of the paper (Section 3) with the
 * viscous-hardening regularization (Section 4, equation "regu"), integrated
 * per material point with classical RK4.  Only tests, the smoke check and
 * the CPU-baseline leg of the benchmark may load this; the GPU product path
 * shares no code with it.
 *
 * Conventions: symmetric second-order tensors are Mandel 6-vectors
 * (11, 22, 33, sqrt2*23, sqrt2*13, sqrt2*12), so double contractions are
 * dot products.  Stiffness and Schmid tensors arrive already rotated to
 * the lab frame, one set per voxel label.  Units: MPa, s.
 *
 * State per point: y = (eps_p[6], v[S], alpha[S]):
 *   eps_p  plastic strain (Section 3, strain split and equation 1)
 *   v      accumulated slip, dv/dt = |gamma_dot| (Section 3, below eq. 4)
 *   alpha  back-strain of Armstrong-Frederick kinematic hardening,
 *          x = c*alpha, dalpha/dt = gamma_dot - d*|gamma_dot|*alpha; the
 *          paper's law is the special case c = 0 (kinematic hardening is
 *          an addition of the synthetic workloads).
 */
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXS 64
#define ORC_FAM_SLIP 0
#define ORC_FAM_TWIN 1
#define ORC_TWIN_NORTON 0
#define ORC_TWIN_PAPER 1

typedef struct {
    int n_sys;
    int n_labels;
    const double *C_lab;   /* [n_labels][6][6] Mandel stiffness, lab frame  */
    const double *m_lab;   /* [n_labels][n_sys][6] Mandel Schmid tensors    */
    const int *family;     /* [n_sys] 0 slip, 1 twin                        */
    const double *tau0;    /* [n_sys] initial resistance                    */
    double Q[2], b[2], c[2], d[2], K[2], n[2], q_self[2], q_lat[2];
    int twin_mode;         /* ORC_TWIN_NORTON or ORC_TWIN_PAPER             */
    double K_c, f_m, gamma_T;
    double eta;            /* viscous-hardening regularization, MPa*s       */
} orc_material;

/*
 * Regularized Norton rate (equations 5 and 6 with equation "regu").
 * With the yield stress raised to r + eta*|g|, the rate magnitude g solves
 *     g = A * < (o - eta*g) / K >^n ,   o = overstress before regularization.
 * Writing y = (o - eta*g)/K >= 0, g = A*y^n and y is the root of
 *     phi(y) = K*y + eta*A*y^n - o .
 * phi is increasing and convex on y > 0; both o/K and (o/(eta*A))^(1/n) are
 * upper bounds of the root, so Newton from their minimum decreases
 * monotonically onto it.  Stop when the step is within 4 ulps of y.
 */
double orc_reg_rate(double o, double A, double K, double n, double eta)
{
    if (!(o > 0.0) || !(A > 0.0))
        return 0.0;
    if (eta == 0.0)
        return A * pow(o / K, n);
    double y = pow(o / (eta * A), 1.0 / n);
    if (K > 0.0 && o / K < y)
        y = o / K;
    for (int it = 0; it < 50; ++it) {
        double yn1 = pow(y, n - 1.0);
        double phi = K * y + eta * A * yn1 * y - o;
        double dphi = K + eta * A * n * yn1;
        double step = phi / dphi;
        y -= step;
        if (fabs(step) <= 4.0 * DBL_EPSILON * y)
            break;
    }
    return A * pow(y, n);
}

/* Rate of the internal variables, dy/dt = F(eps, y), at total strain eps.
 * dr: NULL for the implicit regularization (the rate solves equation
 * "regu" with the rate itself); otherwise the lagged reading: dr[s] =
 * eta |gdot_s| of the previous load step raises the resistance of system s
 * and the rate is the plain Norton law (eta = 0 in it). */
static void rate_dr(const orc_material *mt, int lab, const double eps[6],
                    const double *y, const double *dr, double *dy)
{
    const int S = mt->n_sys;
    const double *C = mt->C_lab + 36 * (long)lab;
    const double *m = mt->m_lab + 6 * (long)S * lab;
    const double *ep = y, *v = y + 6, *al = y + 6 + S;
    double sig[6], gd[ORC_MAXS];

    /* Hooke's law on the elastic strain eps - eps_p */
    for (int i = 0; i < 6; ++i) {
        double s = 0.0;
        for (int j = 0; j < 6; ++j)
            s += C[6 * i + j] * (eps[j] - ep[j]);
        sig[i] = s;
    }

    /* twin volume fractions: gamma_beta = gamma_T * f_beta, so f = v/gamma_T */
    double sum_f = 0.0;
    for (int s = 0; s < S; ++s)
        if (mt->family[s] == ORC_FAM_TWIN)
            sum_f += v[s] / mt->gamma_T;

    /* isotropic hardening, equation 4: the saturating terms 1 - exp(-b v)
     * of every system, summed within the family of the hardened system */
    double hs[ORC_MAXS];
    for (int t = 0; t < S; ++t)
        hs[t] = 1.0 - exp(-mt->b[mt->family[t]] * v[t]);

    for (int s = 0; s < S; ++s) {
        const int f = mt->family[s];
        double r = mt->tau0[s];
        for (int t = 0; t < S; ++t) {
            if (mt->family[t] != f)
                continue;
            double q = (t == s) ? mt->q_self[f] : mt->q_lat[f];
            r += mt->Q[f] * q * hs[t];
        }
        /* resolved shear stress, equation 3 */
        double tau = 0.0;
        for (int i = 0; i < 6; ++i)
            tau += sig[i] * m[6 * s + i];
        double x = mt->c[f] * al[s];
        const double eta = dr ? 0.0 : mt->eta;
        if (dr)
            r += dr[s];
        if (f == ORC_FAM_SLIP) {
            /* equation 5, two-sided */
            double o = fabs(tau - x) - r;
            double g = orc_reg_rate(o, 1.0, mt->K[f], mt->n[f], eta);
            gd[s] = (tau - x >= 0.0) ? g : -g;
        } else {
            /* equation 6, one-sided (twinning is unidirectional) */
            double A = 1.0;
            if (mt->twin_mode == ORC_TWIN_PAPER)
                A = mt->gamma_T * mt->K_c * (mt->f_m - sum_f);
            double o = (tau - x) - r;
            gd[s] = orc_reg_rate(o, A, mt->K[f], mt->n[f], eta);
        }
    }

    /* equation 1: slip contributions weighted by the untwinned fraction */
    double dep[6] = {0, 0, 0, 0, 0, 0};
    for (int s = 0; s < S; ++s) {
        double w = (mt->family[s] == ORC_FAM_SLIP) ? (1.0 - sum_f) * gd[s] : gd[s];
        for (int i = 0; i < 6; ++i)
            dep[i] += w * m[6 * s + i];
    }
    for (int i = 0; i < 6; ++i)
        dy[i] = dep[i];
    for (int s = 0; s < S; ++s) {
        const int f = mt->family[s];
        dy[6 + s] = fabs(gd[s]);
        dy[6 + S + s] = gd[s] - mt->d[f] * fabs(gd[s]) * al[s];
    }
}

void orc_rate(const orc_material *mt, int lab, const double eps[6],
              const double *y, double *dy)
{
    rate_dr(mt, lab, eps, y, NULL, dy);
}

/*
 * One load increment at one point: total strain moves linearly in time
 * from eps0 (start of the increment) to eps1 (end); the internal variables
 * are integrated with classical RK4 over M equal substeps of dt/M.
 * Returns the end state y1 and the end stress sig1 = C:(eps1 - eps_p).
 */
static void integrate_dr(const orc_material *mt, int lab, const double eps0[6],
                         const double eps1[6], const double *y0, const double *dr, double *y1,
                         double sig1[6], double dt, int M);

void orc_integrate_point(const orc_material *mt, int lab, const double eps0[6],
                         const double eps1[6], const double *y0, double *y1,
                         double sig1[6], double dt, int M)
{
    integrate_dr(mt, lab, eps0, eps1, y0, NULL, y1, sig1, dt, M);
}

static void integrate_dr(const orc_material *mt, int lab, const double eps0[6],
                         const double eps1[6], const double *y0, const double *dr, double *y1,
                         double sig1[6], double dt, int M)
{
    const int S = mt->n_sys, D = 6 + 2 * S;
    double y[6 + 2 * ORC_MAXS], k1[6 + 2 * ORC_MAXS], k2[6 + 2 * ORC_MAXS];
    double k3[6 + 2 * ORC_MAXS], k4[6 + 2 * ORC_MAXS], tmp[6 + 2 * ORC_MAXS];
    double e[6];
    const double h = dt / M;
    memcpy(y, y0, sizeof(double) * D);

    for (int j = 0; j < M; ++j) {
        const double s0 = (double)j / M, sh = (j + 0.5) / M, s1 = (double)(j + 1) / M;
        for (int i = 0; i < 6; ++i) e[i] = eps0[i] + s0 * (eps1[i] - eps0[i]);
        rate_dr(mt, lab, e, y, dr, k1);
        for (int i = 0; i < 6; ++i) e[i] = eps0[i] + sh * (eps1[i] - eps0[i]);
        for (int q = 0; q < D; ++q) tmp[q] = y[q] + 0.5 * h * k1[q];
        rate_dr(mt, lab, e, tmp, dr, k2);
        for (int q = 0; q < D; ++q) tmp[q] = y[q] + 0.5 * h * k2[q];
        rate_dr(mt, lab, e, tmp, dr, k3);
        for (int i = 0; i < 6; ++i) e[i] = eps0[i] + s1 * (eps1[i] - eps0[i]);
        for (int q = 0; q < D; ++q) tmp[q] = y[q] + h * k3[q];
        rate_dr(mt, lab, e, tmp, dr, k4);
        for (int q = 0; q < D; ++q)
            y[q] += h / 6.0 * (k1[q] + 2.0 * k2[q] + 2.0 * k3[q] + k4[q]);
    }
    memcpy(y1, y, sizeof(double) * D);
    const double *C = mt->C_lab + 36 * (long)lab;
    for (int i = 0; i < 6; ++i) {
        double s = 0.0;
        for (int q = 0; q < 6; ++q)
            s += C[6 * i + q] * (eps1[q] - y[q]);
        sig1[i] = s;
    }
}

/*
 * Frozen error-controlled substeps (an option: the paper uses a fixed
 * count).  At the first fixed-point iteration of a load step, each point
 * takes the least count M_v = M 2^j, j = 0..maxd, whose RK4 result y(M_v)
 * agrees with y(2 M_v) within Richardson's bound: e(M_v) <= (15 tol)^2,
 * where e is the largest of the squared Frobenius norm of the plastic
 * strain difference and the squared differences of each v and alpha
 * (quantities that do not depend on the frame); j = maxd when none does.
 * The point's result at that iteration is y(M_v), and the count stays for
 * the rest of the load step, so the stress remains a smooth function of the
 * strain iterate.
 */
static double subst_err2(int S, const double *a, const double *b)
{
    double f = 0.0, m = 0.0;
    for (int i = 0; i < 6; ++i) f += (a[i] - b[i]) * (a[i] - b[i]);
    for (int q = 6; q < 6 + 2 * S; ++q) {
        const double d2 = (a[q] - b[q]) * (a[q] - b[q]);
        if (d2 > m) m = d2;
    }
    return f > m ? f : m;
}

int orc_cp_probe(const orc_material *mt, long n_pts, const int *labels, const double *eps0,
                 const double *eps1, const double *y0, double *y1, double *sig1, double dt, int M,
                 double tol, int maxd, int *jsel)
{
    if (mt->n_sys < 0 || mt->n_sys > ORC_MAXS || M < 1 || !(tol > 0.0) || maxd < 0 || maxd > 10)
        return -1;
    const int S = mt->n_sys, D = 6 + 2 * S;
    for (long p = 0; p < n_pts; ++p)
        if (labels[p] < 0 || labels[p] >= mt->n_labels)
            return -1;
    const double lim = (15.0 * tol) * (15.0 * tol);
#pragma omp parallel for schedule(dynamic, 16)
    for (long p = 0; p < n_pts; ++p) {
        double ya[6 + 2 * ORC_MAXS], yb[6 + 2 * ORC_MAXS], sa[6], sb[6];
        orc_integrate_point(mt, labels[p], eps0 + 6 * p, eps1 + 6 * p, y0 + D * p, ya, sa, dt, M);
        int j = 0;
        for (; j < maxd; ++j) {
            orc_integrate_point(mt, labels[p], eps0 + 6 * p, eps1 + 6 * p, y0 + D * p, yb, sb, dt,
                                M << (j + 1));
            const double e = subst_err2(S, ya, yb);
            if (e <= lim) break;
            memcpy(ya, yb, sizeof(double) * D);
            memcpy(sa, sb, sizeof sa);
        }
        jsel[p] = j;
        memcpy(y1 + D * p, ya, sizeof(double) * D);
        memcpy(sig1 + 6 * p, sa, sizeof sa);
    }
    return 0;
}

/* All points with their own substep counts M 2^jsel[p]. */
int orc_cp_update_j(const orc_material *mt, long n_pts, const int *labels, const double *eps0,
                    const double *eps1, const double *y0, double *y1, double *sig1, double dt, int M,
                    const int *jsel)
{
    if (mt->n_sys < 0 || mt->n_sys > ORC_MAXS || M < 1)
        return -1;
    const int D = 6 + 2 * mt->n_sys;
    for (long p = 0; p < n_pts; ++p)
        if (labels[p] < 0 || labels[p] >= mt->n_labels || jsel[p] < 0 || jsel[p] > 10)
            return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (long p = 0; p < n_pts; ++p)
        orc_integrate_point(mt, labels[p], eps0 + 6 * p, eps1 + 6 * p, y0 + D * p, y1 + D * p,
                            sig1 + 6 * p, dt, M << jsel[p]);
    return 0;
}

/* All points of a grid (OpenMP over points).  Arrays are point-major:
 * eps [n][6], state [n][6+2S], sig [n][6].  Returns 0, or -1 on bad input. */
int orc_cp_update(const orc_material *mt, long n_pts, const int *labels,
                  const double *eps0, const double *eps1, const double *y0,
                  double *y1, double *sig1, double dt, int M)
{
    if (mt->n_sys < 0 || mt->n_sys > ORC_MAXS || M < 1)
        return -1;
    const int D = 6 + 2 * mt->n_sys;
    for (long p = 0; p < n_pts; ++p)
        if (labels[p] < 0 || labels[p] >= mt->n_labels)
            return -1;
#pragma omp parallel for schedule(dynamic, 64)
    for (long p = 0; p < n_pts; ++p)
        orc_integrate_point(mt, labels[p], eps0 + 6 * p, eps1 + 6 * p,
                            y0 + D * p, y1 + D * p, sig1 + 6 * p, dt, M);
    return 0;
}

/* orc_cp_update with the lagged regularization: dr [n][S] per point. */
int orc_cp_update_lagged(const orc_material *mt, long n_pts, const int *labels,
                         const double *eps0, const double *eps1, const double *y0,
                         const double *dr, double *y1, double *sig1, double dt, int M)
{
    if (mt->n_sys < 0 || mt->n_sys > ORC_MAXS || M < 1 || !dr)
        return -1;
    const int S = mt->n_sys, D = 6 + 2 * S;
    for (long p = 0; p < n_pts; ++p)
        if (labels[p] < 0 || labels[p] >= mt->n_labels)
            return -1;
#pragma omp parallel for schedule(dynamic, 64)
    for (long p = 0; p < n_pts; ++p)
        integrate_dr(mt, labels[p], eps0 + 6 * p, eps1 + 6 * p, y0 + D * p, dr + (long)S * p,
                     y1 + D * p, sig1 + 6 * p, dt, M);
    return 0;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of the parallel loops above (timing only: every voxel's
 * result is independent of it). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------
 * Reverse mode (adjoint) of the local law, for gradients with respect to
 * the per-family parameters theta[f] = (r0, Q, b, c, d, K, n), f = slip,
 * twin.  Everything is the plain chain rule of the forward definitions
 * above; the regularized rate g(o, A) enters through the implicit-function
 * derivatives of its defining equation K y + eta A y^n = o, g = A y^n:
 *   D = K + eta A n y^(n-1)
 *   dg/do = A n y^(n-1) / D        dg/dA = y^n K / D
 *   dg/dK = -A n y^n / D           dg/dn = A y^n ln(y) K / D
 * ------------------------------------------------------------------------ */
enum { TH_R0 = 0, TH_Q, TH_B, TH_C, TH_D, TH_K, TH_N, TH_NUM };

/* root y of the regularized rate (0 when inactive) */
static double reg_root(double o, double A, double K, double n, double eta)
{
    if (!(o > 0.0) || !(A > 0.0))
        return 0.0;
    if (eta == 0.0)
        return o / K;
    double y = pow(o / (eta * A), 1.0 / n);
    if (K > 0.0 && o / K < y)
        y = o / K;
    for (int it = 0; it < 50; ++it) {
        double yn1 = pow(y, n - 1.0);
        double step = (K * y + eta * A * yn1 * y - o) / (K + eta * A * n * yn1);
        y -= step;
        if (fabs(step) <= 4.0 * DBL_EPSILON * y)
            break;
    }
    return y;
}

static double sgn(double x) { return (x > 0.0) - (x < 0.0); }

/* kb: cotangent of dy/dt = F(eps, y).  Accumulates yb (+=), eb (+=), th (+=). */
void orc_rate_vjp(const orc_material *mt, int lab, const double eps[6], const double *y,
                  const double *kb, double *yb, double *eb, double th[2][TH_NUM])
{
    const int S = mt->n_sys;
    const double *C = mt->C_lab + 36 * (long)lab;
    const double *m = mt->m_lab + 6 * (long)S * lab;
    const double *ep = y, *v = y + 6, *al = y + 6 + S;
    const double *kep = kb, *kv = kb + 6, *kal = kb + 6 + S;
    double sig[6], hs[ORC_MAXS], ex[ORC_MAXS], r[ORC_MAXS], tx[ORC_MAXS], o[ORC_MAXS];
    double A[ORC_MAXS], yr[ORC_MAXS], gd[ORC_MAXS];

    /* forward recomputation */
    for (int i = 0; i < 6; ++i) {
        double s = 0.0;
        for (int j = 0; j < 6; ++j)
            s += C[6 * i + j] * (eps[j] - ep[j]);
        sig[i] = s;
    }
    double sum_f = 0.0;
    for (int s = 0; s < S; ++s)
        if (mt->family[s] == ORC_FAM_TWIN)
            sum_f += v[s] / mt->gamma_T;
    for (int t = 0; t < S; ++t) {
        ex[t] = exp(-mt->b[mt->family[t]] * v[t]);
        hs[t] = 1.0 - ex[t];
    }
    for (int s = 0; s < S; ++s) {
        const int f = mt->family[s];
        double rr = mt->tau0[s];
        for (int t = 0; t < S; ++t)
            if (mt->family[t] == f)
                rr += mt->Q[f] * ((t == s) ? mt->q_self[f] : mt->q_lat[f]) * hs[t];
        r[s] = rr;
        double tau = 0.0;
        for (int i = 0; i < 6; ++i)
            tau += sig[i] * m[6 * s + i];
        tx[s] = tau - mt->c[f] * al[s];
        if (f == ORC_FAM_SLIP) {
            A[s] = 1.0;
            o[s] = fabs(tx[s]) - r[s];
        } else {
            A[s] = (mt->twin_mode == ORC_TWIN_PAPER) ? mt->gamma_T * mt->K_c * (mt->f_m - sum_f) : 1.0;
            o[s] = tx[s] - r[s];
        }
        yr[s] = reg_root(o[s], A[s], mt->K[f], mt->n[f], mt->eta);
        double g = (yr[s] > 0.0) ? A[s] * pow(yr[s], mt->n[f]) : 0.0;
        gd[s] = (f == ORC_FAM_SLIP && tx[s] < 0.0) ? -g : g;
    }

    /* reverse */
    double gdb[ORC_MAXS], sigb[6] = {0, 0, 0, 0, 0, 0}, hb[ORC_MAXS], sumfb = 0.0;
    for (int s = 0; s < S; ++s) {
        const int f = mt->family[s];
        double mk = 0.0;
        for (int i = 0; i < 6; ++i)
            mk += m[6 * s + i] * kep[i];
        if (f == ORC_FAM_SLIP) {
            gdb[s] = (1.0 - sum_f) * mk;
            sumfb -= gd[s] * mk;
        } else {
            gdb[s] = mk;
        }
        gdb[s] += sgn(gd[s]) * kv[s];
        gdb[s] += kal[s] * (1.0 - mt->d[f] * sgn(gd[s]) * al[s]);
        yb[6 + S + s] -= mt->d[f] * fabs(gd[s]) * kal[s];
        th[f][TH_D] -= fabs(gd[s]) * al[s] * kal[s];
        hb[s] = 0.0;
    }
    for (int s = 0; s < S; ++s) {
        const int f = mt->family[s];
        double txb = 0.0, rb = 0.0;
        if (yr[s] > 0.0) {
            const double n = mt->n[f], K = mt->K[f], eta = mt->eta, y1 = yr[s];
            const double yn1 = pow(y1, n - 1.0), yn = yn1 * y1;
            const double D = K + eta * A[s] * n * yn1;
            const double Go = A[s] * n * yn1 / D;
            const double GA = yn * K / D;
            const double GK = -A[s] * n * yn / D;
            const double Gn = A[s] * yn * log(y1) * K / D;
            double gb;
            if (f == ORC_FAM_SLIP) {
                gb = sgn(tx[s]) * gdb[s];            /* g = |gd| */
                const double ob = Go * gb;
                txb = sgn(tx[s]) * ob;
                rb = -ob;
            } else {
                gb = gdb[s];
                const double ob = Go * gb;
                txb = ob;
                rb = -ob;
                if (mt->twin_mode == ORC_TWIN_PAPER)
                    sumfb -= mt->gamma_T * mt->K_c * GA * gb;
            }
            th[f][TH_K] += GK * gb;
            th[f][TH_N] += Gn * gb;
        }
        /* tx = tau - c alpha */
        yb[6 + S + s] -= mt->c[f] * txb;
        th[f][TH_C] -= al[s] * txb;
        for (int i = 0; i < 6; ++i)
            sigb[i] += txb * m[6 * s + i];
        /* r = tau0 + Q sum_t q_st h_t */
        th[f][TH_R0] += rb;
        double qh = 0.0;
        for (int t = 0; t < S; ++t) {
            if (mt->family[t] != f)
                continue;
            const double q = (t == s) ? mt->q_self[f] : mt->q_lat[f];
            qh += q * hs[t];
            hb[t] += mt->Q[f] * q * rb;
        }
        th[f][TH_Q] += qh * rb;
    }
    for (int t = 0; t < S; ++t) {
        const int f = mt->family[t];
        yb[6 + t] += hb[t] * mt->b[f] * ex[t];
        th[f][TH_B] += hb[t] * v[t] * ex[t];
        if (f == ORC_FAM_TWIN)
            yb[6 + t] += sumfb / mt->gamma_T;
    }
    /* sigma = C (eps - eps_p) */
    for (int j = 0; j < 6; ++j) {
        double cs = 0.0;
        for (int i = 0; i < 6; ++i)
            cs += C[6 * i + j] * sigb[i];
        eb[j] += cs;
        yb[j] -= cs;
    }
}

/*
 * Reverse of orc_integrate_point: given cotangents of the end stress (sigb)
 * and end state (ybM), accumulate those of eps0, eps1, y0 and theta.
 * The substep states are recomputed forward and kept; the stage states of
 * each substep are recomputed during its reverse.
 */
void orc_point_vjp(const orc_material *mt, int lab, const double eps0[6], const double eps1[6],
                   const double *y0, double dt, int M, const double sigb[6], const double *ybM,
                   double *e0b, double *e1b, double *y0b, double th[2][TH_NUM])
{
    const int S = mt->n_sys, D = 6 + 2 * S;
    const double h = dt / M;
    double *ys = (double *)malloc(sizeof(double) * (size_t)(M + 1) * D);
    double k1[6 + 2 * ORC_MAXS], k2[6 + 2 * ORC_MAXS], k3[6 + 2 * ORC_MAXS], k4[6 + 2 * ORC_MAXS];
    double z2[6 + 2 * ORC_MAXS], z3[6 + 2 * ORC_MAXS], z4[6 + 2 * ORC_MAXS];
    double yb[6 + 2 * ORC_MAXS], yjb[6 + 2 * ORC_MAXS], kb1[6 + 2 * ORC_MAXS], kb2[6 + 2 * ORC_MAXS];
    double kb3[6 + 2 * ORC_MAXS], kb4[6 + 2 * ORC_MAXS], zb[6 + 2 * ORC_MAXS];
    double e[6], eb[6];
    memcpy(ys, y0, sizeof(double) * D);
    for (int j = 0; j < M; ++j) {
        double *yj = ys + (size_t)j * D, *yn = ys + (size_t)(j + 1) * D;
        const double s0 = (double)j / M, sh = (j + 0.5) / M, s1 = (double)(j + 1) / M;
        for (int i = 0; i < 6; ++i) e[i] = eps0[i] + s0 * (eps1[i] - eps0[i]);
        orc_rate(mt, lab, e, yj, k1);
        for (int i = 0; i < 6; ++i) e[i] = eps0[i] + sh * (eps1[i] - eps0[i]);
        for (int q = 0; q < D; ++q) z2[q] = yj[q] + 0.5 * h * k1[q];
        orc_rate(mt, lab, e, z2, k2);
        for (int q = 0; q < D; ++q) z3[q] = yj[q] + 0.5 * h * k2[q];
        orc_rate(mt, lab, e, z3, k3);
        for (int i = 0; i < 6; ++i) e[i] = eps0[i] + s1 * (eps1[i] - eps0[i]);
        for (int q = 0; q < D; ++q) z4[q] = yj[q] + h * k3[q];
        orc_rate(mt, lab, e, z4, k4);
        for (int q = 0; q < D; ++q)
            yn[q] = yj[q] + h / 6.0 * (k1[q] + 2.0 * k2[q] + 2.0 * k3[q] + k4[q]);
    }
    /* end stress sig = C (eps1 - eps_p(M)) */
    const double *C = mt->C_lab + 36 * (long)lab;
    memcpy(yb, ybM, sizeof(double) * D);
    for (int j = 0; j < 6; ++j) {
        double cs = 0.0;
        for (int i = 0; i < 6; ++i)
            cs += C[6 * i + j] * sigb[i];
        e1b[j] += cs;
        yb[j] -= cs;
    }
    for (int j = M - 1; j >= 0; --j) {
        const double *yj = ys + (size_t)j * D;
        const double sv[4] = {(double)j / M, (j + 0.5) / M, (j + 0.5) / M, (double)(j + 1) / M};
        /* recompute the stage states */
        for (int i = 0; i < 6; ++i) e[i] = eps0[i] + sv[0] * (eps1[i] - eps0[i]);
        orc_rate(mt, lab, e, yj, k1);
        for (int i = 0; i < 6; ++i) e[i] = eps0[i] + sv[1] * (eps1[i] - eps0[i]);
        for (int q = 0; q < D; ++q) z2[q] = yj[q] + 0.5 * h * k1[q];
        orc_rate(mt, lab, e, z2, k2);
        for (int q = 0; q < D; ++q) z3[q] = yj[q] + 0.5 * h * k2[q];
        orc_rate(mt, lab, e, z3, k3);
        for (int q = 0; q < D; ++q) z4[q] = yj[q] + h * k3[q];
        /* y_{j+1} = y_j + h/6 (k1 + 2 k2 + 2 k3 + k4) */
        for (int q = 0; q < D; ++q) {
            yjb[q] = yb[q];
            kb1[q] = h / 6.0 * yb[q];
            kb2[q] = h / 3.0 * yb[q];
            kb3[q] = h / 3.0 * yb[q];
            kb4[q] = h / 6.0 * yb[q];
        }
        const double *zs[4] = {yj, z2, z3, z4};
        double *kbs[4] = {kb1, kb2, kb3, kb4};
        const double cprev[4] = {0.0, 0.5 * h, 0.5 * h, h};
        for (int st = 3; st >= 0; --st) {
            for (int i = 0; i < 6; ++i) e[i] = eps0[i] + sv[st] * (eps1[i] - eps0[i]);
            for (int q = 0; q < D; ++q) zb[q] = 0.0;
            for (int i = 0; i < 6; ++i) eb[i] = 0.0;
            orc_rate_vjp(mt, lab, e, zs[st], kbs[st], zb, eb, th);
            for (int i = 0; i < 6; ++i) {
                e0b[i] += (1.0 - sv[st]) * eb[i];
                e1b[i] += sv[st] * eb[i];
            }
            /* z_st = y_j + cprev * k_{st-1} */
            for (int q = 0; q < D; ++q) {
                yjb[q] += zb[q];
                if (st > 0) kbs[st - 1][q] += cprev[st] * zb[q];
            }
        }
        memcpy(yb, yjb, sizeof(double) * D);
    }
    for (int q = 0; q < D; ++q) y0b[q] += yb[q];
    free(ys);
}

/* Grid version: per point sigb[n][6], ybM[n][D] -> e0b, e1b [n][6], y0b [n][D]
 * (overwritten) and theta[2][7] (summed, overwritten). */
int orc_vjp_grid(const orc_material *mt, long n_pts, const int *labels, const double *eps0,
                 const double *eps1, const double *y0, double dt, int M, const double *sigb,
                 const double *ybM, double *e0b, double *e1b, double *y0b, double *theta)
{
    if (mt->n_sys < 0 || mt->n_sys > ORC_MAXS || M < 1)
        return -1;
    const int D = 6 + 2 * mt->n_sys;
    double tot[2][TH_NUM];
    memset(tot, 0, sizeof tot);
#pragma omp parallel
    {
        double th[2][TH_NUM];
        memset(th, 0, sizeof th);
#pragma omp for schedule(dynamic, 64)
        for (long p = 0; p < n_pts; ++p) {
            memset(e0b + 6 * p, 0, 6 * sizeof(double));
            memset(e1b + 6 * p, 0, 6 * sizeof(double));
            memset(y0b + D * p, 0, D * sizeof(double));
            orc_point_vjp(mt, labels[p], eps0 + 6 * p, eps1 + 6 * p, y0 + D * p, dt, M, sigb + 6 * p,
                          ybM + D * p, e0b + 6 * p, e1b + 6 * p, y0b + D * p, th);
        }
#pragma omp critical
        for (int f = 0; f < 2; ++f)
            for (int k = 0; k < TH_NUM; ++k) tot[f][k] += th[f][k];
    }
    memcpy(theta, tot, sizeof tot);
    return 0;
}

/* Per-point rate VJP for tests. */
void orc_rate_vjp_point(const orc_material *mt, int lab, const double eps[6], const double *y,
                        const double *kb, double *yb, double *eb, double *theta)
{
    double th[2][TH_NUM];
    memset(th, 0, sizeof th);
    orc_rate_vjp(mt, lab, eps, y, kb, yb, eb, th);
    memcpy(theta, th, sizeof th);
}

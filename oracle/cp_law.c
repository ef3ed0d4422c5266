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

/* Rate of the internal variables, dy/dt = F(eps, y), at total strain eps. */
void orc_rate(const orc_material *mt, int lab, const double eps[6],
              const double *y, double *dy)
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
        if (f == ORC_FAM_SLIP) {
            /* equation 5, two-sided */
            double o = fabs(tau - x) - r;
            double g = orc_reg_rate(o, 1.0, mt->K[f], mt->n[f], mt->eta);
            gd[s] = (tau - x >= 0.0) ? g : -g;
        } else {
            /* equation 6, one-sided (twinning is unidirectional) */
            double A = 1.0;
            if (mt->twin_mode == ORC_TWIN_PAPER)
                A = mt->gamma_T * mt->K_c * (mt->f_m - sum_f);
            double o = (tau - x) - r;
            gd[s] = orc_reg_rate(o, A, mt->K[f], mt->n[f], mt->eta);
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

/*
 * One load increment at one point: total strain moves linearly in time
 * from eps0 (start of the increment) to eps1 (end); the internal variables
 * are integrated with classical RK4 over M equal substeps of dt/M.
 * Returns the end state y1 and the end stress sig1 = C:(eps1 - eps_p).
 */
void orc_integrate_point(const orc_material *mt, int lab, const double eps0[6],
                         const double eps1[6], const double *y0, double *y1,
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
        orc_rate(mt, lab, e, y, k1);
        for (int i = 0; i < 6; ++i) e[i] = eps0[i] + sh * (eps1[i] - eps0[i]);
        for (int q = 0; q < D; ++q) tmp[q] = y[q] + 0.5 * h * k1[q];
        orc_rate(mt, lab, e, tmp, k2);
        for (int q = 0; q < D; ++q) tmp[q] = y[q] + 0.5 * h * k2[q];
        orc_rate(mt, lab, e, tmp, k3);
        for (int i = 0; i < 6; ++i) e[i] = eps0[i] + s1 * (eps1[i] - eps0[i]);
        for (int q = 0; q < D; ++q) tmp[q] = y[q] + h * k3[q];
        orc_rate(mt, lab, e, tmp, k4);
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

int orc_max_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

// Reverse mode of the local law and the kernels of the discrete adjoint.
//
// Cotangents are gradients with respect to the stored numbers: symmetric
// tensors as tensor components (11,22,33,23,13,12), so the chain rule is
// plain transposes.  A frame change x_c = Q^T x_l Q maps cotangents as
// c_l = W (Q c_c' Q^T) with c_c' = W^-1 c_c, W = diag(1,1,1,2,2,2) (the
// transpose of the rotation in these coordinates), and conversely.
//
// Per converged load step n (sums over voxels, L the loss):
//   g    = d/d eps_{n+1} [ sigma_bar_L . sigma + S_bar . S_{n+1} ] + eps_bar
//   A    = d sigma / d eps_{n+1}                 (6x6 per voxel)
//   mu   : admissible strain field with W^-1 (A^T W mu - g) weakly
//          equilibrated (Green-operator fixed point, target mean stress 0)
//   then the reverse sweep with sigma_bar = sigma_bar_L - W mu gives
//   S_bar_n, eps_bar_n and the parameter gradient.
// Parameter order per family (slip, twin): r0, Q, b, c, d, K, n.
#pragma once
#include "cpfft_kernels.hpp"

namespace cpf {

constexpr int NTH = 14;

template <typename R>
__device__ __forceinline__ void cot_to_crystal(const R Q[9], const R cl[6], R cc[6])
{
    R t[6] = {cl[0], cl[1], cl[2], R(0.5) * cl[3], R(0.5) * cl[4], R(0.5) * cl[5]};
    rot_to_crystal(Q, t, cc);
    cc[3] *= R(2); cc[4] *= R(2); cc[5] *= R(2);
}

template <typename R>
__device__ __forceinline__ void cot_to_lab(const R Q[9], const R cc[6], R cl[6])
{
    R t[6] = {cc[0], cc[1], cc[2], R(0.5) * cc[3], R(0.5) * cc[4], R(0.5) * cc[5]};
    rot_to_lab(Q, t, cl);
    cl[3] *= R(2); cl[4] *= R(2); cl[5] *= R(2);
}

__device__ __forceinline__ double sgnd(double x) { return (x > 0.0) - (x < 0.0); }

// Root y of the regularized rate (0 below threshold), cold start.
template <typename R>
__device__ __forceinline__ R reg_root(R o, R A, R eta, const FamP<R> &F, R rtol)
{
    if (!(o > R(0)) || !(A > R(0))) return R(0);
    R yw = R(0);
    int na = 0, nn = 0;
    const R etaA = eta * A;
    const R inv_etaA = etaA > R(0) ? R(1) / etaA : R(0);
    reg_rate<R>(o, A, inv_etaA, etaA, eta > R(0) ? R(1) / eta : R(0), F, rtol, yw, na, nn);
    return yw;
}

// Reverse of one rate evaluation dy/dt = F(e, z) in the crystal frame.
// kb: cotangent of the output; accumulates zb, eb and th (FP64).
template <typename R, int NS>
__device__ void rate_vjp(const LawP<R> &P, const R e[6], const R (&zep)[6], const R (&zv)[NS],
                         const R (&zal)[NS], const R (&kep)[6], const R (&kv)[NS], const R (&kal)[NS],
                         R (&zbep)[6], R (&zbv)[NS], R (&zbal)[NS], R eb[6], double (&th)[NTH])
{
    // forward recomputation
    R ee[6], sig[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) ee[i] = e[i] - zep[i];
    hooke_c<R, LAW_GENERAL>(P.C, ee, sig);
    R h[NS];
    R Hs = R(0), Ht = R(0), sumf = R(0);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const bool tw = (P.twin_mask >> s) & 1u;
        const FamP<R> &F = tw ? P.ft : P.fs;
        h[s] = R(1) - exp(-F.b * zv[s]);
        if (tw) { Ht += h[s]; sumf += zv[s] * P.inv_gT; }
        else Hs += h[s];
    }
    const R Atw = P.twin_mode ? P.Kc_gT * (P.fm - sumf) : R(1);
    // reverse: dep, dv, dalpha -> gd; accumulate sigma_bar, h_bar, sumf_bar
    R sigb[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
    R hb[NS];
    R Hsb = R(0), Htb = R(0), sumfb = R(0);
#pragma unroll
    for (int s = 0; s < NS; ++s) hb[s] = R(0);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const bool tw = (P.twin_mask >> s) & 1u;
        const FamP<R> &F = tw ? P.ft : P.fs;
        const int fo = tw ? 7 : 0;
        const R r = P.tau0[s] + F.QL * (tw ? Ht : Hs) + F.QD * h[s];
        R tau = R(0);
#pragma unroll
        for (int i = 0; i < 6; ++i) tau += (i < 3 ? sig[i] : R(2) * sig[i]) * P.m[s][i];
        const R tx = tau - F.c * zal[s];
        const R A = tw ? Atw : R(1);
        const R o = tw ? tx - r : fabs(tx) - r;
        const R y = reg_root<R>(o, A, P.eta, F, P.newton_rtol);
        R g = R(0), Go = R(0), GA = R(0), GK = R(0), Gn = R(0);
        if (y > R(0)) {
            const R yn1 = pow(y, F.nm1), yn = yn1 * y;
            const R Dn = F.K + P.eta * A * F.n * yn1;
            g = A * yn;
            Go = A * F.n * yn1 / Dn;
            GA = yn * F.K / Dn;
            GK = -A * F.n * yn / Dn;
            Gn = A * yn * log(y) * F.K / Dn;
        }
        const R gd = (!tw && tx < R(0)) ? -g : g;
        const R sg = gd > R(0) ? R(1) : (gd < R(0) ? R(-1) : R(0));
        // dep = sum_s w_s gd_s m_s (w = 1 - sumf for slip), dv = |gd|,
        // dalpha = gd - d |gd| alpha
        R mk = R(0);
#pragma unroll
        for (int i = 0; i < 6; ++i) mk += P.m[s][i] * kep[i];
        R gdb = tw ? mk : (R(1) - sumf) * mk;
        if (!tw) sumfb -= gd * mk;
        gdb += sg * kv[s];
        gdb += kal[s] * (R(1) - F.d * sg * zal[s]);
        zbal[s] -= F.d * fabs(gd) * kal[s];
        th[fo + 4] -= (double)(fabs(gd) * zal[s] * kal[s]);
        // gd through the regularized rate
        R txb = R(0), rb = R(0);
        if (y > R(0)) {
            const R gb = tw ? gdb : (tx < R(0) ? -gdb : gdb);
            const R ob = Go * gb;
            txb = tw ? ob : (tx < R(0) ? -ob : ob);
            rb = -ob;
            if (tw && P.twin_mode) sumfb -= P.Kc_gT * GA * gb;
            th[fo + 5] += (double)(GK * gb);
            th[fo + 6] += (double)(Gn * gb);
        }
        // tx = tau - c alpha, tau = sigma : m
        zbal[s] -= F.c * txb;
        th[fo + 3] -= (double)(zal[s] * txb);
#pragma unroll
        for (int i = 0; i < 6; ++i) sigb[i] += txb * (i < 3 ? P.m[s][i] : R(2) * P.m[s][i]);
        // r = tau0 + Q (q_lat H_f + (q_self - q_lat) h_s)
        th[fo + 0] += (double)rb;
        th[fo + 1] += (double)(rb * (F.ql * (tw ? Ht : Hs) + (F.qs - F.ql) * h[s]));
        hb[s] += F.QD * rb;
        if (tw) Htb += F.QL * rb;
        else Hsb += F.QL * rb;
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const bool tw = (P.twin_mask >> s) & 1u;
        const FamP<R> &F = tw ? P.ft : P.fs;
        const int fo = tw ? 7 : 0;
        const R hbt = hb[s] + (tw ? Htb : Hsb);
        const R ex = R(1) - h[s];   // exp(-b v)
        zbv[s] += hbt * F.b * ex;
        th[fo + 2] += (double)(hbt * zv[s] * ex);
        if (tw) zbv[s] += sumfb * P.inv_gT;
    }
    // sigma = C (e - ep)
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        R cs = R(0);
#pragma unroll
        for (int i = 0; i < 6; ++i) cs += P.C[i * 6 + j] * sigb[i];
        eb[j] += cs;
        zbep[j] -= cs;
    }
}

// ---------------------------------------------------------------------------
// Per-voxel reverse sweep of the RK4 law over one load step
// ---------------------------------------------------------------------------
template <typename R>
struct AdjArgs {
    const RveDev<R> *rv;     // the RVE (one-element table)
    const R *e0;             // eps_n   [6][N] lab
    const R *e1;             // eps_n+1 [6][N] lab
    const R *st0;            // S_n     [D][N] lab plastic strain, v, alpha
    R *scratch;              // [M][4][D][N] crystal-frame stage states
    R *g;                    // [6][N]
    R *A;                    // [36][N], row i = d sigma_i / d eps_n+1
    R *mu;                   // [6][N]
    R *Sb;                   // [D][N] cotangent of S (in: S_n+1, out: S_n)
    R *eb;                   // [6][N] cotangent of eps (in: eps_n+1, out: eps_n)
    double *th_part;         // [blocks][NTH]
    R sigL_xx;               // loss cotangent of sigma_xx at every voxel
    R dt;
    int M;
};

constexpr int VJP_GA = 0;   // forward recompute, g and A
constexpr int VJP_F = 1;    // final sweep with sigma_bar_L - W mu (scratch reused)

template <typename R, int NS>
__device__ void sweep(const LawP<R> &P, const AdjArgs<R> &a, long N, long vox, int nsys, const R e0c[6],
                      const R e1c[6], const R sbc[6], const R (&Sbep)[6], const R (&Sbv)[NS],
                      const R (&Sbal)[NS], R e0bc[6], R e1bc[6], R (&ybep)[6], R (&ybv)[NS],
                      R (&ybal)[NS], double (&th)[NTH])
{
    const int D = 6 + 2 * nsys;
    const R h = a.dt / R(a.M);
    const R invM = R(1) / R(a.M);
    // end stress sigma = C (e1 - ep_M)
#pragma unroll
    for (int i = 0; i < 6; ++i) ybep[i] = Sbep[i];
#pragma unroll
    for (int s = 0; s < NS; ++s) { ybv[s] = Sbv[s]; ybal[s] = Sbal[s]; }
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        R cs = R(0);
#pragma unroll
        for (int i = 0; i < 6; ++i) cs += P.C[i * 6 + j] * sbc[i];
        e1bc[j] += cs;
        ybep[j] -= cs;
    }
    for (int j = a.M - 1; j >= 0; --j) {
        R aep[6], av[NS], aal[NS];        // y_j bar accumulator
#pragma unroll
        for (int i = 0; i < 6; ++i) aep[i] = ybep[i];
#pragma unroll
        for (int s = 0; s < NS; ++s) { av[s] = ybv[s]; aal[s] = ybal[s]; }
        R zbep[6] = {R(0), R(0), R(0), R(0), R(0), R(0)}, zbv[NS], zbal[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) { zbv[s] = R(0); zbal[s] = R(0); }
        for (int st = 3; st >= 0; --st) {
            const R wst = (st == 0 || st == 3) ? h * R(1.0 / 6.0) : h * R(1.0 / 3.0);
            const R cn = (st == 2) ? h : h * R(0.5);   // z_{st+1} = y + cn k_st
            // k_bar_st = w_st y_bar + cn z_bar_{st+1}
            R kep[6], kv[NS], kal[NS];
#pragma unroll
            for (int i = 0; i < 6; ++i) kep[i] = wst * ybep[i] + (st < 3 ? cn * zbep[i] : R(0));
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                kv[s] = wst * ybv[s] + (st < 3 ? cn * zbv[s] : R(0));
                kal[s] = wst * ybal[s] + (st < 3 ? cn * zbal[s] : R(0));
            }
            // stage input z_st from the scratch
            const R *zs = a.scratch + (((long)j * 4 + st) * D) * N + vox;
            R zep[6], zv[NS], zal[NS];
#pragma unroll
            for (int i = 0; i < 6; ++i) zep[i] = zs[i * N];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                zv[s] = s < nsys ? zs[(6 + s) * N] : R(0);
                zal[s] = s < nsys ? zs[(6 + nsys + s) * N] : R(0);
            }
            const R sf = (st == 0) ? R(j) * invM : (st == 3) ? R(j + 1) * invM : (R(j) + R(0.5)) * invM;
            R e[6], ebs[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
#pragma unroll
            for (int i = 0; i < 6; ++i) e[i] = e0c[i] + sf * (e1c[i] - e0c[i]);
#pragma unroll
            for (int i = 0; i < 6; ++i) zbep[i] = R(0);
#pragma unroll
            for (int s = 0; s < NS; ++s) { zbv[s] = R(0); zbal[s] = R(0); }
            rate_vjp<R, NS>(P, e, zep, zv, zal, kep, kv, kal, zbep, zbv, zbal, ebs, th);
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                e0bc[i] += (R(1) - sf) * ebs[i];
                e1bc[i] += sf * ebs[i];
                aep[i] += zbep[i];
            }
#pragma unroll
            for (int s = 0; s < NS; ++s) { av[s] += zbv[s]; aal[s] += zbal[s]; }
        }
#pragma unroll
        for (int i = 0; i < 6; ++i) ybep[i] = aep[i];
#pragma unroll
        for (int s = 0; s < NS; ++s) { ybv[s] = av[s]; ybal[s] = aal[s]; }
    }
}

template <typename R, int NS>
__global__ __launch_bounds__(256) void k_law_vjp(AdjArgs<R> a, LawP<R> P, int mode)
{
    const RveDev<R> &d = a.rv[0];
    const long N = d.nvox;
    const long vox = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double th[NTH];
#pragma unroll
    for (int k = 0; k < NTH; ++k) th[k] = 0.0;
    const int nsys = P.nsys;
    if (vox < N) {
        const int D = 6 + 2 * nsys;
        const int lab = d.labels[vox];
        R Q[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) Q[i] = d.Qtab[lab * 9 + i];
        R e0l[6], e1l[6], e0c[6], e1c[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            e0l[c] = a.e0[c * N + vox];
            e1l[c] = a.e1[c * N + vox];
        }
        rot_to_crystal(Q, e0l, e0c);
        rot_to_crystal(Q, e1l, e1c);
        if (mode == VJP_GA) {
            // forward recompute of the stage inputs into the scratch
            R ep[6], v[NS], al[NS];
            load_state<R, NS>(a.st0, N, vox, nsys, Q, ep, v, al);
            const R h = a.dt / R(a.M), invM = R(1) / R(a.M);
            for (int j = 0; j < a.M; ++j) {
                R tep[6], tv[NS], tal[NS], aep[6], av[NS], aal[NS], yw[NS];
#pragma unroll
                for (int i = 0; i < 6; ++i) tep[i] = aep[i] = ep[i];
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    tv[s] = av[s] = v[s];
                    tal[s] = aal[s] = al[s];
                    yw[s] = R(0);
                }
                for (int st = 0; st < 4; ++st) {
                    R *zs = a.scratch + (((long)j * 4 + st) * D) * N + vox;
#pragma unroll
                    for (int i = 0; i < 6; ++i) zs[i * N] = tep[i];
#pragma unroll
                    for (int s = 0; s < NS; ++s)
                        if (s < nsys) {
                            zs[(6 + s) * N] = tv[s];
                            zs[(6 + nsys + s) * N] = tal[s];
                        }
                    const R sf = (st == 0) ? R(j) * invM : (st == 3) ? R(j + 1) * invM : (R(j) + R(0.5)) * invM;
                    const R wacc = (st == 0 || st == 3) ? h * R(1.0 / 6.0) : h * R(1.0 / 3.0);
                    const R cnext = (st == 2) ? h : h * R(0.5);
                    R e[6];
#pragma unroll
                    for (int i = 0; i < 6; ++i) e[i] = e0c[i] + sf * (e1c[i] - e0c[i]);
                    int na = 0, nn = 0;
                    rk_stage<R, NS, LAW_GENERAL>(P, e, tep, tv, tal, ep, v, al, aep, av, aal, yw, wacc, cnext,
                                                 st < 3, na, nn);
                }
#pragma unroll
                for (int i = 0; i < 6; ++i) ep[i] = aep[i];
#pragma unroll
                for (int s = 0; s < NS; ++s) { v[s] = av[s]; al[s] = aal[s]; }
            }
        }
        R Sbep[6], Sbv[NS], Sbal[NS];
        {
            R tl[6], tc[6];
#pragma unroll
            for (int i = 0; i < 6; ++i) tl[i] = a.Sb[i * N + vox];
            cot_to_crystal(Q, tl, tc);
#pragma unroll
            for (int i = 0; i < 6; ++i) Sbep[i] = tc[i];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                Sbv[s] = s < nsys ? a.Sb[(6 + s) * N + vox] : R(0);
                Sbal[s] = s < nsys ? a.Sb[(6 + nsys + s) * N + vox] : R(0);
            }
        }
        R ybep[6], ybv[NS], ybal[NS];
        if (mode == VJP_GA) {
            // g: cotangents (sigma_bar_L, S_bar) plus the carried eps_bar
            R sbl[6] = {a.sigL_xx, R(0), R(0), R(0), R(0), R(0)}, sbc[6];
            cot_to_crystal(Q, sbl, sbc);
            R e0b[6] = {R(0), R(0), R(0), R(0), R(0), R(0)}, e1b[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
            double thd[NTH];
#pragma unroll
            for (int k = 0; k < NTH; ++k) thd[k] = 0.0;
            sweep<R, NS>(P, a, N, vox, nsys, e0c, e1c, sbc, Sbep, Sbv, Sbal, e0b, e1b, ybep, ybv, ybal, thd);
            R gl[6];
            cot_to_lab(Q, e1b, gl);
#pragma unroll
            for (int c = 0; c < 6; ++c) a.g[c * N + vox] = gl[c] + a.eb[c * N + vox];
            // A: rows d sigma_i / d eps_n+1 (sigma_bar = e_i, S_bar = 0)
            R zep6[6] = {R(0), R(0), R(0), R(0), R(0), R(0)}, zv[NS], zal[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) { zv[s] = R(0); zal[s] = R(0); }
            for (int i = 0; i < 6; ++i) {
                R el[6] = {R(0), R(0), R(0), R(0), R(0), R(0)}, ec[6];
                el[i] = R(1);
                cot_to_crystal(Q, el, ec);
                R a0[6] = {R(0), R(0), R(0), R(0), R(0), R(0)}, a1[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
                sweep<R, NS>(P, a, N, vox, nsys, e0c, e1c, ec, zep6, zv, zal, a0, a1, ybep, ybv, ybal, thd);
                R rl[6];
                cot_to_lab(Q, a1, rl);
#pragma unroll
                for (int c = 0; c < 6; ++c) a.A[(i * 6 + c) * N + vox] = rl[c];
            }
        } else {
            // final sweep: sigma_bar = sigma_bar_L - W mu
            R sbl[6], sbc[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                const R w = c < 3 ? R(1) : R(2);
                sbl[c] = (c == 0 ? a.sigL_xx : R(0)) - w * a.mu[c * N + vox];
            }
            cot_to_crystal(Q, sbl, sbc);
            R e0b[6] = {R(0), R(0), R(0), R(0), R(0), R(0)}, e1b[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
            sweep<R, NS>(P, a, N, vox, nsys, e0c, e1c, sbc, Sbep, Sbv, Sbal, e0b, e1b, ybep, ybv, ybal, th);
            R el[6], epl[6];
            cot_to_lab(Q, e0b, el);
            cot_to_lab(Q, ybep, epl);
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                a.eb[c * N + vox] = el[c];
                a.Sb[c * N + vox] = epl[c];
            }
#pragma unroll
            for (int s = 0; s < NS; ++s)
                if (s < nsys) {
                    a.Sb[(6 + s) * N + vox] = ybv[s];
                    a.Sb[(6 + nsys + s) * N + vox] = ybal[s];
                }
        }
    }
    if (mode == VJP_F) block_sum<NTH>(th, a.th_part + (long)blockIdx.x * NTH);
}

// ---------------------------------------------------------------------------
// Adjoint equilibrium iteration: x pass and boundary update.  The y and z
// passes are those of the forward iteration (same spectrum, same flags).
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_adj_xpass(AdjArgs<R> a)
{
    const RveDev<R> &d = a.rv[0];
    Scalars *sc = d.sc;
    if (sc->done) return;
    extern __shared__ unsigned char smem_raw[];
    C2<R> *buf = reinterpret_cast<C2<R> *>(smem_raw);
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int first = sc->iter == 0;
    const int li = tid / d.nx, x = tid - li * d.nx;
    const int line = blockIdx.x * d.L + li;
    const bool valid = tid < d.tpbx && line < d.nlines;
    const int y = valid ? line % d.ny : 0, z = valid ? line / d.ny : 0;
    const long N = d.nvox;
    const long vox = (long)line * d.nx + x;
    R corr[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
    if (!first) {
        if (tid < d.tpbx) load_halfspec_pairs(d.spec, buf, d.nx, d.ny, d.nz, d.nhx, d.L, li, x, y, z, valid);
        __syncthreads();
        lds_fft<R, true, 8>(buf, 3 * d.L, d.nx, d.px, d.tw[0], tid, nthr);
        if (tid < d.tpbx) {
#pragma unroll
            for (int p = 0; p < 3; ++p) {
                const C2<R> zz = buf[(p * d.L + li) * d.nx + x];
                corr[2 * p] = zz.x * d.inv_nvox;
                corr[2 * p + 1] = zz.y * d.inv_nvox;
            }
        }
        __syncthreads();
    }
    R tau[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
    double part[NPX];
#pragma unroll
    for (int i = 0; i < NPX; ++i) part[i] = 0.0;
    if (valid) {
        R m[6], wm[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            m[c] = (first ? R(0) : a.mu[c * N + vox]) - corr[c] + R(sc->dE[c]);
            a.mu[c * N + vox] = m[c];
            wm[c] = c < 3 ? m[c] : R(2) * m[c];
        }
        double g2 = 0.0;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            R t = R(0);
#pragma unroll
            for (int i = 0; i < 6; ++i) t += wm[i] * a.A[(i * 6 + c) * N + vox];
            const R gc = a.g[c * N + vox];
            t -= gc;
            tau[c] = c < 3 ? t : R(0.5) * t;
            g2 += c < 3 ? (double)gc * gc : 0.5 * (double)gc * gc;
            part[c] = (double)tau[c];
        }
        part[6] = g2;
    }
    block_sum<NPX>(part, d.part_x + (long)blockIdx.x * NPX);
    if (tid < d.tpbx) {
#pragma unroll
        for (int p = 0; p < 3; ++p) buf[(p * d.L + li) * d.nx + x] = C2<R>{tau[2 * p], tau[2 * p + 1]};
    }
    __syncthreads();
    lds_fft<R, false, 8>(buf, 3 * d.L, d.nx, d.px, d.tw[0], tid, nthr);
    if (tid < d.tpbx) store_halfspec_pairs(d.spec, buf, d.nx, d.ny, d.nz, d.nhx, d.L, li, x, y, z, valid);
}

template <typename R>
__global__ __launch_bounds__(256) void k_adj_bc(const RveDev<R> *__restrict__ rv, double tol, int max_iter)
{
    const RveDev<R> &d = rv[0];
    Scalars *sc = d.sc;
    if (sc->done) return;
    const int nbx = (d.nlines + d.L - 1) / d.L, nbz = d.ntz * d.ny;
    const double N = (double)d.nvox;
    double acc[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = 0.0;
    for (int j = threadIdx.x; j < nbx; j += blockDim.x)
#pragma unroll
        for (int i = 0; i < 7; ++i) acc[i] += d.part_x[(long)j * NPX + i];
    for (int j = threadIdx.x; j < nbz; j += blockDim.x) acc[7] += d.part_z[j];
    __shared__ double tot[8];
    block_sum<8>(acc, tot);
    __syncthreads();
    if (threadIdx.x != 0) return;
    const int it = sc->iter + 1;
    sc->iter = it;
    const double gn = sqrt(tot[6]);
    if (!(gn > 0.0)) {            // no load on this step: mu = 0
        sc->done = 1;
        return;
    }
    double T[6], TS[6];
    for (int i = 0; i < 6; ++i) {
        T[i] = tot[i] / N;
        TS[i] = sc->sidx[i] ? T[i] : 0.0;
    }
    const double err_eq = sqrt(tot[7]) / (sqrt(N) * gn);
    const double err_bc = sqrt(frob2(TS)) / (gn / sqrt(N));
    sc->err_eq = err_eq;
    sc->err_bc = err_bc;
    if (!(err_eq == err_eq) || !(err_bc == err_bc)) {
        sc->status = -5;
        sc->done = 1;
        return;
    }
    if (err_eq <= tol && err_bc <= tol) {
        sc->done = 1;
        return;
    }
    if (it >= max_iter) {
        sc->status = -4;
        sc->done = 1;
        return;
    }
    for (int i = 0; i < 6; ++i) {
        double dd = 0.0;
        for (int j = 0; j < 6; ++j) dd -= sc->K0inv[i * 6 + j] * TS[j];
        sc->dE[i] = dd;
    }
}

}  // namespace cpf

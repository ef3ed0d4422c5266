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
//
// The forward integration of the step is replayed once per step by
// k_law_record with the solver's own stage code (same specialization, same
// Newton warm starts), so the recorded stage states and Newton roots are
// those of the converged forward step; the reverse sweeps read them and
// never solve for a root.
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

// th[k] (slip) or th[7 + k] (twin) += x with a constant index k, so the
// accumulators stay in registers whether or not the family is known at
// compile time.
__device__ __forceinline__ void th_add(double (&th)[NTH], bool tw, int k, double x)
{
    th[k] += tw ? 0.0 : x;
    th[7 + k] += tw ? x : 0.0;
}

// Transposed elastic product out += C^T v (tensor components, same zero
// pattern as hooke_c).
template <typename R, int SPEC>
__device__ __forceinline__ void hooke_ct(const R (&C)[36], const R v[6], R out[6])
{
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        R s = R(0);
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            const bool nz = SPEC == LAW_GENERAL || (i < 3 && j < 3) || i == j;
            if (nz) s += C[i * 6 + j] * v[i];
        }
        out[j] = s;
    }
}

// Reverse of one rate evaluation dy/dt = F(e, z) in the crystal frame, at
// the recorded stage state z and Newton roots ys (0 where inactive).
// k*: cotangent of the rate; adds to z_bar (zb*), e_bar (eb) and, if TH,
// the parameter gradient th.
template <typename R, int NS, int SPEC, bool TH>
__device__ __forceinline__ void rate_vjp(const LawP<R> &P, const R e[6], const R (&zep)[6], const R (&zv)[NS],
                                         const R (&zal)[NS], const R (&ys)[NS], const R (&kep)[6],
                                         const R (&kv)[NS], const R (&kal)[NS], R (&zbep)[6], R (&zbv)[NS],
                                         R (&zbal)[NS], R (&eb)[6], double (&th)[NTH])
{
    R ee[6], sig[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) ee[i] = e[i] - zep[i];
    hooke_c<R, SPEC>(P.C, ee, sig);
    R h[NS];
    R Hs = R(0), Ht = R(0), sumf = R(0);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const bool tw = is_twin<SPEC>(P, s);
        const R bl = tw ? P.ft.bl2e : P.fs.bl2e;
        h[s] = R(1) - ex2(-bl * zv[s]);
        if (tw) { Ht += h[s]; sumf += zv[s] * P.inv_gT; }
        else Hs += h[s];
    }
    const R Atw = P.twin_mode ? P.Kc_gT * (P.fm - sumf) : R(1);
    R sigb[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
    R hb[NS];
    R Hsb = R(0), Htb = R(0), sumfb = R(0);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        law_fence();
        const bool tw = is_twin<SPEC>(P, s);
        const FamP<R> &F = tw ? P.ft : P.fs;
        R tau = R(0), mk = R(0);
#pragma unroll
        for (int i = 0; i < 6; ++i)
            if (schmid_nonzero<SPEC>(s, i)) {
                const R m = schmid<R, SPEC>(P.m, s, i);
                tau += (i < 3 ? sig[i] : R(2) * sig[i]) * m;
                mk += m * kep[i];
            }
        const R tx = tau - F.c * zal[s];
        const R A = tw ? Atw : R(1);
        const R y = ys[s];
        // g = A y^n with K y + eta A y^n = o: partials of g in o, A, K, n
        R g = R(0), Go = R(0), GA = R(0), GK = R(0), Gn = R(0);
        if (y > R(0)) {
            const R yn1 = pow_nm1(y, F.nm1, F.nm1_int, -1), yn = yn1 * y;
            const R inv_D = R(1) / (F.K + P.eta * A * F.n * yn1);
            g = A * yn;
            Go = A * F.n * yn1 * inv_D;
            GA = yn * F.K * inv_D;
            if constexpr (TH) {
                GK = -A * F.n * yn * inv_D;
                Gn = A * yn * log(y) * F.K * inv_D;
            }
        }
        const bool neg = !tw && tx < R(0);
        const R gd = neg ? -g : g;
        const R sg = gd > R(0) ? R(1) : (gd < R(0) ? R(-1) : R(0));
        // ep' = sum w_s gd_s m_s (w = 1 - sum f for slip), v' = |gd|,
        // alpha' = gd - d |gd| alpha
        R gdb = tw ? mk : (R(1) - sumf) * mk;
        if (!tw) sumfb -= gd * mk;
        gdb += sg * kv[s];
        gdb += kal[s] * (R(1) - F.d * sg * zal[s]);
        zbal[s] -= F.d * fabs(gd) * kal[s];
        if constexpr (TH) th_add(th, tw, 4, -(double)(fabs(gd) * zal[s] * kal[s]));
        R txb = R(0), rb = R(0);
        if (y > R(0)) {
            const R gb = neg ? -gdb : gdb;
            const R ob = Go * gb;
            txb = neg ? -ob : ob;
            rb = -ob;
            if (tw && P.twin_mode) sumfb -= P.Kc_gT * GA * gb;
            if constexpr (TH) {
                th_add(th, tw, 5, (double)(GK * gb));
                th_add(th, tw, 6, (double)(Gn * gb));
            }
        }
        // tx = tau - c alpha, tau = sigma : m
        zbal[s] -= F.c * txb;
        if constexpr (TH) th_add(th, tw, 3, -(double)(zal[s] * txb));
#pragma unroll
        for (int i = 0; i < 6; ++i)
            if (schmid_nonzero<SPEC>(s, i)) {
                const R m = schmid<R, SPEC>(P.m, s, i);
                sigb[i] += txb * (i < 3 ? m : R(2) * m);
            }
        // r = r0 + Q (q_lat H_family + (q_self - q_lat) h_s)
        if constexpr (TH) {
            th_add(th, tw, 0, (double)rb);
            th_add(th, tw, 1, (double)(rb * (F.ql * (tw ? Ht : Hs) + (F.qs - F.ql) * h[s])));
        }
        hb[s] = F.QD * rb;
        if (tw) Htb += F.QL * rb;
        else Hsb += F.QL * rb;
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const bool tw = is_twin<SPEC>(P, s);
        const FamP<R> &F = tw ? P.ft : P.fs;
        const R hbt = hb[s] + (tw ? Htb : Hsb);
        const R ex = R(1) - h[s];   // exp(-b v)
        zbv[s] += hbt * F.b * ex;
        if constexpr (TH) th_add(th, tw, 2, (double)(hbt * zv[s] * ex));
        if (tw) zbv[s] += sumfb * P.inv_gT;
    }
    // sigma = C (e - ep)
    R cs[6];
    hooke_ct<R, SPEC>(P.C, sigb, cs);
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        eb[j] += cs[j];
        zbep[j] -= cs[j];
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
    R *scratch;              // [M][4][D + S][N] crystal-frame stage states and Newton roots
    R *g;                    // [6][N]
    R *A;                    // [36][N], row i = d sigma_i / d eps_n+1
    R *mu;                   // [6][N]
    R *Sb;                   // [D][N] cotangent of S (in: S_n+1, out: S_n)
    R *eb;                   // [6][N] cotangent of eps (in: eps_n+1, out: eps_n)
    double *th_part;         // [blocks][NTH]
    R sigL[6];               // cotangent of the local stress at every voxel (Sigma_bar / N)
    R dt;
    int M;
};

constexpr int VJP_GA = 0;   // g and A (seven sweeps)
constexpr int VJP_F = 1;    // final sweep with sigma_bar_L - W mu, parameter gradient

// Replay of the forward integration of the step (the solver's integrate()
// with every stage input and Newton root written to the scratch).  Dynamic
// LDS: law_lds_bytes<R, NS>() + law_items_bytes<R>().
template <typename R, int NS, int SPEC>
__global__ __launch_bounds__(256, (xpass_min_blocks<R, SPEC>())) void k_law_record(AdjArgs<R> a, LawP<R> P)
{
    const RveDev<R> &d = a.rv[0];
    const long N = d.nvox;
    const long vox = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (vox >= N) return;
    const int nsys = P.nsys, D = 6 + 2 * nsys, DY = D + nsys;
    extern __shared__ unsigned char smem_raw[];
    const LawLds<R> W = law_lds<R, NS>(smem_raw, 0, law_lds_bytes<R, NS>());
    const int lab = d.labels[vox];
    R Q[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) Q[i] = d.Qtab[lab * 9 + i];
    R e0l[6], e1l[6], e0[6], e1[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        e0l[c] = a.e0[c * N + vox];
        e1l[c] = a.e1[c * N + vox];
    }
    rot_to_crystal(Q, e0l, e0);
    rot_to_crystal(Q, e1l, e1);
    R ep[6], v[NS], al[NS];
    load_state<R, NS>(a.st0, N, vox, nsys, Q, ep, v, al);
    const int M = a.M;
    const R h = a.dt / R(M), invM = R(1) / R(M);
    R de[6];
    uint32_t warm = 0;
    law_fam_store<R, NS>(P, W);
#pragma unroll
    for (int i = 0; i < 6; ++i) de[i] = e1[i] - e0[i];
    int nact = 0, nnewt = 0;
#pragma unroll 1
    for (int j = 0; j < M; ++j) {
        R tep[6], tv[NS], tal[NS], aep[6], av[NS], aal[NS];
#pragma unroll
        for (int i = 0; i < 6; ++i) tep[i] = aep[i] = ep[i];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            tv[s] = av[s] = v[s];
            tal[s] = aal[s] = al[s];
        }
#pragma unroll 1
        for (int st = 0; st < 4; ++st) {
            R *zs = a.scratch + (((long)j * 4 + st) * DY) * N + vox;
#pragma unroll
            for (int i = 0; i < 6; ++i) zs[i * N] = tep[i];
#pragma unroll
            for (int s = 0; s < NS; ++s)
                if (s < nsys) {
                    zs[(6 + s) * N] = tv[s];
                    zs[(6 + nsys + s) * N] = tal[s];
                }
            const R sfrac = (st == 0) ? R(j) * invM : (st == 3) ? R(j + 1) * invM : (R(j) + R(0.5)) * invM;
            const R wacc = (st == 0 || st == 3) ? h * R(1.0 / 6.0) : h * R(1.0 / 3.0);
            const R cnext = (st == 2) ? h : h * R(0.5);
            R e[6];
#pragma unroll
            for (int i = 0; i < 6; ++i) e[i] = e0[i] + sfrac * de[i];
            rk_stage<R, NS, SPEC>(P, e, tep, tv, tal, ep, v, al, aep, av, aal, warm, W, wacc, cnext, nact, nnewt);
#pragma unroll
            for (int s = 0; s < NS; ++s)
                if (s < nsys) zs[(D + s) * N] = ((warm >> s) & 1u) ? W.y[s * W.ls] : R(0);
        }
#pragma unroll
        for (int i = 0; i < 6; ++i) ep[i] = aep[i];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            v[s] = av[s];
            al[s] = aal[s];
        }
    }
}

// Reverse RK4 over the recorded stages.  In: cotangents of the end stress
// (sbc) and of the end state (yb*, overwritten with the cotangent of the
// start state).  Adds the strain cotangents to e0bc / e1bc.
template <typename R, int NS, int SPEC, bool TH>
__device__ __forceinline__ void sweep(const LawP<R> &P, const AdjArgs<R> &a, long N, long vox, int nsys,
                                      const R (&e0c)[6], const R (&e1c)[6], const R (&sbc)[6], R (&e0bc)[6],
                                      R (&e1bc)[6], R (&ybep)[6], R (&ybv)[NS], R (&ybal)[NS],
                                      double (&th)[NTH])
{
    const int D = 6 + 2 * nsys, DY = D + nsys;
    const R h = a.dt / R(a.M);
    const R invM = R(1) / R(a.M);
    // end stress sigma = C (e1 - ep_M)
    {
        R cs[6];
        hooke_ct<R, SPEC>(P.C, sbc, cs);
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            e1bc[j] += cs[j];
            ybep[j] -= cs[j];
        }
    }
#pragma unroll 1
    for (int j = a.M - 1; j >= 0; --j) {
        // y_{j+1} = y_j + sum_st w_st k_st, z_0 = y_j, z_{st+1} = y_j + c_st k_st
        R aep[6], av[NS], aal[NS];
#pragma unroll
        for (int i = 0; i < 6; ++i) aep[i] = ybep[i];
#pragma unroll
        for (int s = 0; s < NS; ++s) { av[s] = ybv[s]; aal[s] = ybal[s]; }
        R zbep[6] = {R(0), R(0), R(0), R(0), R(0), R(0)}, zbv[NS], zbal[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) { zbv[s] = R(0); zbal[s] = R(0); }
#pragma unroll 1
        for (int st = 3; st >= 0; --st) {
            const R wst = (st == 0 || st == 3) ? h * R(1.0 / 6.0) : h * R(1.0 / 3.0);
            const R cn = (st == 2) ? h : h * R(0.5);
            const R cz = st < 3 ? cn : R(0);
            // k_bar_st = w_st y_bar + c_st z_bar_{st+1}
            R kep[6], kv[NS], kal[NS];
#pragma unroll
            for (int i = 0; i < 6; ++i) kep[i] = wst * ybep[i] + cz * zbep[i];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                kv[s] = wst * ybv[s] + cz * zbv[s];
                kal[s] = wst * ybal[s] + cz * zbal[s];
            }
            const R *zs = a.scratch + (((long)j * 4 + st) * DY) * N + vox;
            R zep[6], zv[NS], zal[NS], ys[NS];
#pragma unroll
            for (int i = 0; i < 6; ++i) zep[i] = zs[i * N];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                zv[s] = s < nsys ? zs[(6 + s) * N] : R(0);
                zal[s] = s < nsys ? zs[(6 + nsys + s) * N] : R(0);
                ys[s] = s < nsys ? zs[(D + s) * N] : R(0);
            }
            const R sf = (st == 0) ? R(j) * invM : (st == 3) ? R(j + 1) * invM : (R(j) + R(0.5)) * invM;
            R e[6], ebs[6];
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                e[i] = e0c[i] + sf * (e1c[i] - e0c[i]);
                ebs[i] = R(0);
                zbep[i] = R(0);
            }
#pragma unroll
            for (int s = 0; s < NS; ++s) { zbv[s] = R(0); zbal[s] = R(0); }
            rate_vjp<R, NS, SPEC, TH>(P, e, zep, zv, zal, ys, kep, kv, kal, zbep, zbv, zbal, ebs, th);
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

// MODE VJP_GA: seven sweeps of the recorded step, r = 0 with the loss
// cotangent and the carried S_bar (-> g, plus the carried eps_bar), r = 1..6
// with sigma_bar = unit vector r-1 and S_bar = 0 (-> row r-1 of A).
// MODE VJP_F: one sweep with sigma_bar = sigma_bar_L - W mu and the carried
// S_bar; writes S_bar_n, eps_bar_n and the FP64 block partials of the
// parameter gradient.
template <typename R, int NS, int SPEC, int MODE>
__global__ __launch_bounds__(256) void k_law_vjp(AdjArgs<R> a, LawP<R> P)
{
    const RveDev<R> &d = a.rv[0];
    const long N = d.nvox;
    const long vox = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double th[NTH];
#pragma unroll
    for (int k = 0; k < NTH; ++k) th[k] = 0.0;
    const int nsys = P.nsys;
    if (vox < N) {
        const int lab = d.labels[vox];
        R Q[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) Q[i] = d.Qtab[lab * 9 + i];
        R e0c[6], e1c[6];
        {
            R e0l[6], e1l[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                e0l[c] = a.e0[c * N + vox];
                e1l[c] = a.e1[c * N + vox];
            }
            rot_to_crystal(Q, e0l, e0c);
            rot_to_crystal(Q, e1l, e1c);
        }
        // carried cotangent of S_n+1 (crystal frame)
        R Sep[6], Sv[NS], Sal[NS];
        {
            R tl[6];
#pragma unroll
            for (int i = 0; i < 6; ++i) tl[i] = a.Sb[i * N + vox];
            cot_to_crystal(Q, tl, Sep);
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                Sv[s] = s < nsys ? a.Sb[(6 + s) * N + vox] : R(0);
                Sal[s] = s < nsys ? a.Sb[(6 + nsys + s) * N + vox] : R(0);
            }
        }
        if constexpr (MODE == VJP_GA) {
#pragma unroll 1
            for (int r = 0; r < 7; ++r) {
                R sbl[6], sbc[6];
#pragma unroll
                for (int c = 0; c < 6; ++c)
                    sbl[c] = r == 0 ? a.sigL[c] : (c == r - 1 ? R(1) : R(0));
                cot_to_crystal(Q, sbl, sbc);
                R ybep[6], ybv[NS], ybal[NS], e0b[6], e1b[6];
#pragma unroll
                for (int i = 0; i < 6; ++i) {
                    ybep[i] = r == 0 ? Sep[i] : R(0);
                    e0b[i] = e1b[i] = R(0);
                }
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    ybv[s] = r == 0 ? Sv[s] : R(0);
                    ybal[s] = r == 0 ? Sal[s] : R(0);
                }
                sweep<R, NS, SPEC, false>(P, a, N, vox, nsys, e0c, e1c, sbc, e0b, e1b, ybep, ybv, ybal, th);
                R out[6];
                cot_to_lab(Q, e1b, out);
                if (r == 0) {
#pragma unroll
                    for (int c = 0; c < 6; ++c) a.g[c * N + vox] = out[c] + a.eb[c * N + vox];
                } else {
#pragma unroll
                    for (int c = 0; c < 6; ++c) a.A[((r - 1) * 6 + c) * N + vox] = out[c];
                }
            }
        } else {
            R sbl[6], sbc[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                const R w = c < 3 ? R(1) : R(2);
                sbl[c] = a.sigL[c] - w * a.mu[c * N + vox];
            }
            cot_to_crystal(Q, sbl, sbc);
            R e0b[6] = {R(0), R(0), R(0), R(0), R(0), R(0)}, e1b[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
            sweep<R, NS, SPEC, true>(P, a, N, vox, nsys, e0c, e1c, sbc, e0b, e1b, Sep, Sv, Sal, th);
            R el[6], epl[6];
            cot_to_lab(Q, e0b, el);
            cot_to_lab(Q, Sep, epl);
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                a.eb[c * N + vox] = el[c];
                a.Sb[c * N + vox] = epl[c];
            }
#pragma unroll
            for (int s = 0; s < NS; ++s)
                if (s < nsys) {
                    a.Sb[(6 + s) * N + vox] = Sv[s];
                    a.Sb[(6 + nsys + s) * N + vox] = Sal[s];
                }
        }
    }
    if constexpr (MODE == VJP_F) block_sum<NTH>(th, a.th_part + (long)blockIdx.x * NTH);
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
        if (tid < d.tpbx) load_halfspec_pairs(d.spec, buf, d.nx, d.ny, d.nz, d.nkx, d.nhp, d.L, li, x, y, z, valid);
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
    if (tid < d.tpbx) store_halfspec_pairs(d.spec, buf, d.nx, d.ny, d.nz, d.nkx, d.nhp, d.L, li, x, y, z, valid);
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

// Kernels of one fixed-point iteration of the Green-operator scheme, for a
// voxel grid stored [component][z][y][x] (x fastest):
//
//   xpass_iter : inverse x transform of the correction spectrum, strain
//                update eps^{k+1} = eps^k - corr + dE, local law (RK4) at
//                every voxel, FP64 block sums, forward x transform of sigma
//   ypass      : C2C transform along y of the half spectrum (fwd or inv)
//   zpass_green: forward z transform, Gamma0 apply + equilibrium residual
//                (FP64), inverse z transform
//   bc_update  : one block per RVE: reduce the block sums, residuals,
//                convergence decision and mixed-boundary mean-strain correction
//
// Every pass covers all RVEs of a batch in one grid (a single solve is a
// batch of one); blocks of RVEs whose step has ended return at once.
// Plus single-purpose kernels for the component operators and fields.
#pragma once
#include "cpfft_device.hpp"

namespace cpf {

// Device-resident scalars of the running load step of one RVE (FP64).
struct Scalars {
    double dE[6];       // mean-strain increment applied by the next x pass
    double E[6];        // mean strain of the current iterate
    double target[6];   // step targets (strain or stress per component)
    double K0inv[36];   // (C0_SS)^-1 embedded in 6x6 (zero outside S x S)
    int sidx[6];        // 1: stress-controlled component
    int iter;           // constitutive evaluations done in this step
    int done;           // 1: the step has ended (converged or failed)
    int status;         // 0 ok, negative CPF_E_* code
    int stagnated;
    int cur;            // index of the committed strain/state buffers
    int M;              // RK4 substeps of this load step
    double dt;          // load step duration
    double err_hist[8];
    double Sigma[6];    // mean stress of the last evaluated iterate
    double err_eq, err_bc, mean_sig_eq, mean_v, mean_f;
    double work_active, work_newton;   // law work counters summed over the step
    unsigned long long n_symptom;      // voxels of the load step's local-stress test (k_symptom)
    int bad_state;                     // 1: a non-finite value in the converged strain or state
};

// Anderson acceleration of the fixed point (an option): the last AA_MAX
// differences of iterates and basic-scheme steps of one RVE, and the small
// least-squares system built from them (FP64).
constexpr int AA_MAX = 8;
struct AaState {
    int depth;                   // m (0: off)
    int count;                   // stored differences (<= m)
    int head;                    // ring slot of the oldest difference
    int slot;                    // slot written by the current iteration (-1: none)
    int have_prev;               // an earlier iterate and step are stored
    int nk;                      // differences used by the current update
    double G[AA_MAX][AA_MAX];    // dF_s . dF_t by ring slots
    double gamma[AA_MAX];        // coefficients by ring slot
    double E_prev[6], dE_prev[6];
    double dEX[AA_MAX][6], ddE[AA_MAX][6];   // mean-strain parts of dX and dF
};

// One RVE of a (possibly one-element) batch as the kernels see it.  Every
// pass launches one grid over all RVEs; block b belongs to the RVE whose
// first block of that pass (bx0/by0/bz0) is the largest one <= b.
template <typename R>
struct RveDev {
    int nx, ny, nz, nhx;
    int nkx, nhp;              // kx columns held (the continuous operator's solve leaves
                               // out the Nyquist column, which it zeroes) and row pitch
    int L, tpbx, nlines;       // x pass: lines per block, threads used
    int ty, nty, tz, ntz;      // y / z pass tiles (kx columns) and tile counts
    int yfix, zfix;            // 1: the fixed-length kernels do this RVE's y / z passes
    int bx0, by0, bz0;         // first block in the x, y and z pass grids
    long nvox;
    R inv_nvox;
    FftPlan px, py, pz;
    const int32_t *labels;     // [nvox]
    const R *Qtab;             // [n_labels][9]
    R *eps[2];                 // strain [6][nvox]: committed = eps[cur]
    R *st[2];                  // state [6+2S][nvox]: committed = st[cur]
    int32_t *mv;               // [nvox] substep exponent j (count M 2^j) of the current
                               // load step, with error-controlled substeps
    C2<R> *spec;               // [nz][ny][nhp][6], columns kx < nkx
    const C2<R> *tw[3];        // twiddles exp(-2 pi i k / n) along x, y, z
    double *part_x;            // [x blocks][NPX]
    double *part_z;            // [z blocks]
    double *part_b;            // [BC_CHUNKS][NPX + 1]: the x and z block sums in fixed chunks
    AaState *aa;               // Anderson state (null: off)
    int aa_depth;              // m
    R *aa_x, *aa_f;            // last iterate and its basic step [6][nvox]
    R *aa_dX, *aa_dF;          // difference rings [m][6][nvox]
    double *aa_part;           // [x blocks][2 AA_MAX] block dot products
    double *aa_chunk;          // [BC_CHUNKS][2 AA_MAX]
    Scalars *sc;
    R *lag;                    // lagged regularization: [S][nvox] raise of each system's
                               // resistance in the current load step (null: off)
};

// XCD-aware block order.  Consecutive workgroups of a launch are dealt
// round-robin to the 8 XCDs, each with its own L2.  Mapping workgroup b to
// the logical block start(x) + b/8 on XCD x = b % 8 (start(x) = x q +
// min(x, r), n = 8 q + r) is a bijection of [0, n) under which each XCD
// runs a contiguous range of logical blocks in order, so blocks that share
// cache lines (neighbouring kx tiles of one ky row) share one L2.
__device__ __forceinline__ int xcd_block(int b, int n)
{
    const int q = n >> 3, r = n & 7, x = b & 7;
    return x * q + min(x, r) + (b >> 3);
}

template <typename R>
__device__ __forceinline__ int find_rve(const RveDev<R> *__restrict__ rv, int nrve, int b, int pass)
{
    int r = 0;
    for (int i = 1; i < nrve; ++i) {
        const int f = pass == 0 ? rv[i].bx0 : pass == 1 ? rv[i].by0 : rv[i].bz0;
        if (f <= b) r = i;
    }
    return r;
}

// ---------------------------------------------------------------------------
// x pass helpers (LDS layout: pair p, local line li -> (p*L + li)*nx)
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void load_halfspec_pairs(const C2<R> *__restrict__ spec, C2<R> *buf,
                                                    int nx, int ny, int nz, int nkx, int nhp, int L,
                                                    int li, int x, int y, int z, bool valid)
{
    // Z_k = A_k + i B_k over the full x spectrum from the stored halves,
    // using A_{N-k} = conj(A_k); DC and Nyquist bins keep their real parts;
    // bins not stored (k >= nkx) are zero.  Spectrum layout [z][y][kx][c].
    const long row = ((long)z * ny + y) * nhp;
    const bool mirror = x > nx / 2;
    const int k = mirror ? nx - x : x;
    const bool realbin = (k == 0) || ((nx & 1) == 0 && k == nx / 2);
    const C2<R> *bin = spec + (row + k) * 6;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        C2<R> z2 = {R(0), R(0)};
        if (valid && k < nkx) {
            C2<R> A = bin[2 * p];
            C2<R> B = bin[2 * p + 1];
            if (realbin) { A.y = R(0); B.y = R(0); }
            if (mirror) { A.y = -A.y; B.y = -B.y; }
            z2 = {A.x - B.y, A.y + B.x};
        }
        buf[(p * L + li) * nx + x] = z2;
    }
}

template <typename R>
__device__ __forceinline__ void store_halfspec_pairs(C2<R> *__restrict__ spec, const C2<R> *buf,
                                                     int nx, int ny, int nz, int nkx, int nhp, int L,
                                                     int li, int x, int y, int z, bool valid)
{
    // Split Z = FFT(a + i b) into A = FFT(a), B = FFT(b) on k in [0, nkx).
    if (!valid || x >= nkx) return;
    const long row = ((long)z * ny + y) * nhp;
    C2<R> *bin = spec + (row + x) * 6;
    const int xm = x == 0 ? 0 : nx - x;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const C2<R> Zk = buf[(p * L + li) * nx + x];
        const C2<R> Zm = buf[(p * L + li) * nx + xm];
        const C2<R> A = {R(0.5) * (Zk.x + Zm.x), R(0.5) * (Zk.y - Zm.y)};
        const C2<R> B = {R(0.5) * (Zk.y + Zm.y), R(0.5) * (Zm.x - Zk.x)};
        bin[2 * p] = A;
        bin[2 * p + 1] = B;
    }
}

template <typename R, int NS>
__device__ __forceinline__ void load_state(const R *__restrict__ st, long nvox, long vox, int nsys,
                                           const R Q[9], R (&ep)[6], R (&v)[NS], R (&al)[NS])
{
    R epl[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) epl[i] = st[i * nvox + vox];
    rot_to_crystal(Q, epl, ep);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        v[s] = s < nsys ? st[(6 + s) * nvox + vox] : R(0);
        al[s] = s < nsys ? st[(6 + nsys + s) * nvox + vox] : R(0);
    }
}

template <typename R, int NS>
__device__ __forceinline__ void store_state(R *__restrict__ st, long nvox, long vox, int nsys,
                                            const R Q[9], const R (&ep)[6], const R (&v)[NS],
                                            const R (&al)[NS])
{
    R epl[6];
    rot_to_lab(Q, ep, epl);
#pragma unroll
    for (int i = 0; i < 6; ++i) st[i * nvox + vox] = epl[i];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        if (s < nsys) {
            st[(6 + s) * nvox + vox] = v[s];
            st[(6 + nsys + s) * nvox + vox] = al[s];
        }
    }
}

// Local law at one voxel: lab strains in, lab stress out; the committed
// state is read from st_in and the new state written to *st_out.  The
// rotation and the output address are read again after the integration
// (behind a compiler memory fence) instead of being held in registers
// through it.
template <typename R, int NS, int SPEC, bool LAG = false>
__device__ __forceinline__ void voxel_law(const LawP<R> &P, const R *Qrow, const R e0l[6], const R e1l[6],
                                          const R *st_in, R *const *st_out, long nvox, long vox, R dt, int M,
                                          R sigl[6], R (&v)[NS], int &nact, int &nnewt, const LawLds<R> &W,
                                          LagRef<R> lag = {nullptr, 0})
{
    R e0[6], e1[6], ep[6], al[NS];
    {
        R Q[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) Q[i] = Qrow[i];
        rot_to_crystal(Q, e0l, e0);
        rot_to_crystal(Q, e1l, e1);
        load_state<R, NS>(st_in, nvox, vox, P.nsys, Q, ep, v, al);
    }
    integrate<R, NS, SPEC, LAG>(P, e0, e1, ep, v, al, dt, M, nact, nnewt, W, lag);
    asm volatile("" ::: "memory");
    R Q[9], sc[6];
#pragma unroll
    for (int i = 0; i < 9; ++i) Q[i] = Qrow[i];
    if constexpr (law_park_e<R, NS>()) {
        // the end strain comes back from the LDS work area
#pragma unroll
        for (int i = 0; i < 6; ++i) e1[i] = W.e[(6 + i) * W.ls];
    }
    hooke(P, e1, ep, sc);
    rot_to_lab(Q, sc, sigl);
    store_state<R, NS>(*st_out, nvox, vox, P.nsys, Q, ep, v, al);
}

// Frozen error-controlled substep counts (an option; the paper uses a fixed
// count): at the first iteration of a load step each voxel takes the least
// count M 2^j, j <= maxd, whose result agrees with that of twice the count
// within lim2 -- the larger of the squared Frobenius norm of the plastic
// strain difference and the squared differences of each v and alpha, all
// independent of the frame -- keeps the result of that count and stores j
// for the later iterations of the step.  The counts differ between lanes;
// the law path has no block barrier (only wave votes over active lanes).
template <typename R, int NS, int SPEC>
__device__ __forceinline__ void voxel_law_probe(const LawP<R> &P, const R *Qrow, const R e0l[6], const R e1l[6],
                                                const R *st_in, R *const *st_out, long nvox, long vox, R dt,
                                                int M, double lim2, int maxd, int32_t *jout, R sigl[6],
                                                R (&v)[NS], int &nact, int &nnewt, const LawLds<R> &W)
{
    // The candidate result lives in the trial-state buffer (this voxel's
    // own slots), so only one state is held in registers at a time.
    R *so = *st_out;
    R e0[6], e1[6];
    {
        R Q[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) Q[i] = Qrow[i];
        rot_to_crystal(Q, e0l, e0);
        rot_to_crystal(Q, e1l, e1);
    }
    int j = 0;
#pragma unroll 1
    for (int a = 0; a <= maxd; ++a) {
        R ep[6], al[NS], Q[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) Q[i] = Qrow[i];
        load_state<R, NS>(st_in, nvox, vox, P.nsys, Q, ep, v, al);
        integrate<R, NS, SPEC>(P, e0, e1, ep, v, al, dt, M << a, nact, nnewt, W);
        asm volatile("" ::: "memory");
#pragma unroll
        for (int i = 0; i < 9; ++i) Q[i] = Qrow[i];
        if (a > 0) {
            // compare with the stored result of half the count
            R epl[6];
            rot_to_lab(Q, ep, epl);
            double f = 0.0, m = 0.0;
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                const double d = (double)epl[i] - (double)so[i * nvox + vox];
                f += (i < 3 ? 1.0 : 2.0) * d * d;
            }
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                if (q < P.nsys) {
                    const double dv = (double)v[q] - (double)so[(6 + q) * nvox + vox];
                    const double da = (double)al[q] - (double)so[(6 + P.nsys + q) * nvox + vox];
                    m = fmax(m, fmax(dv * dv, da * da));
                }
            }
            if (fmax(f, m) <= lim2) break;   // keep the stored result, count M 2^(a-1)
            j = a;
        }
        store_state<R, NS>(so, nvox, vox, P.nsys, Q, ep, v, al);
    }
    *jout = j;
    // the kept result: state from the trial buffer, stress from its plastic strain
    R Q[9], ep[6], al[NS], sc[6];
#pragma unroll
    for (int i = 0; i < 9; ++i) Q[i] = Qrow[i];
    load_state<R, NS>(so, nvox, vox, P.nsys, Q, ep, v, al);
    if constexpr (law_park_e<R, NS>()) {
#pragma unroll
        for (int i = 0; i < 6; ++i) e1[i] = W.e[(6 + i) * W.ls];
    }
    hooke(P, e1, ep, sc);
    rot_to_lab(Q, sc, sigl);
}

// ---------------------------------------------------------------------------
// Fused x pass of one iteration.  Block = L x-lines of nx voxels.
// ---------------------------------------------------------------------------
// Minimum resident blocks per CU for the law kernels (register budget):
// three 256-thread blocks = 3 waves per SIMD = 168 registers per lane in
// the FP32 Table 1 law (a few spills, but the latency hiding of the third
// wave is worth 20 %); two for the FP32 general law (runtime Schmid
// tensors and stiffness need more registers); one block in FP64.
template <typename R, int SPEC>
constexpr int xpass_min_blocks()
{
    return sizeof(R) == 4 ? (SPEC == LAW_TABLE1 ? 3 : 2) : 1;
}

// The law's LDS work area of this thread inside a 256-thread block's
// dynamic LDS, after `offset` bytes used by the kernel itself: 2 NS words
// per thread (plus 12 when the strain path is parked), column-major
// (compile-time stride: plain shifts), then the family table.
template <typename R, int NS, int BD = 256>
__device__ __forceinline__ LawLds<R> law_lds(unsigned char *smem, size_t offset, size_t items_offset)
{
    R *base = reinterpret_cast<R *>(smem + offset);
    const int t = threadIdx.x;
    R *fam = base + (2 * NS + law_e_rows<R>(NS)) * BD;
    unsigned char *iw = smem + items_offset + (t >> 6) * law_items_wave_bytes<R>();
    uint16_t *items = reinterpret_cast<uint16_t *>(iw);
    R *aw = reinterpret_cast<R *>(iw + 64 * law_items_q<R>() * 2);
    return LawLds<R>{base + t, base + NS * BD + t, base + 2 * NS * BD + t, fam, BD, items, aw,
                     fam + 2 * LAW_FAM_WORDS};
}

// Bytes of the x pass FFT area in dynamic LDS: 3 complex lines of up to
// 256 points, then the twiddles of the line length.  The lines are free
// while the law runs, and hold its Newton item lists then.
template <typename R>
constexpr size_t xfft_lds_bytes()
{
    return (3 * 256 + 256) * sizeof(C2<R>);
}
static_assert(law_items_bytes<float>() <= 3 * 256 * sizeof(C2<float>), "Newton items exceed the FFT lines");
static_assert(law_items_bytes<double>() <= 3 * 256 * sizeof(C2<double>), "Newton items exceed the FFT lines");

// LAG: the lagged regularization (d.lag holds the raises of the step).
template <typename R, int NS, int SPEC, bool ADAPT = false, bool AAM = false, bool LAG = false>
__global__ __launch_bounds__(256, (xpass_min_blocks<R, SPEC>())) void k_xpass_iter(
    const RveDev<R> *__restrict__ rv, int nrve, LawP<R> Parg, double rk_lim2, int rk_maxd)
{
    const int r = find_rve(rv, nrve, (int)blockIdx.x, 0);
    const RveDev<R> &d = rv[r];
    Scalars *sc = d.sc;
    if (sc->done) return;
    const LawP<R> &P = Parg;
    extern __shared__ unsigned char smem_raw[];
    C2<R> *buf = reinterpret_cast<C2<R> *>(smem_raw);
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int first = sc->iter == 0;
    const int cur = sc->cur;
    const int li = tid / d.nx, x = tid - li * d.nx;
    const int line = (blockIdx.x - d.bx0) * d.L + li;
    const bool valid = tid < d.tpbx && line < d.nlines;
    const int y = valid ? line % d.ny : 0, z = valid ? line / d.ny : 0;
    const long vox = (long)line * d.nx + x;
    const R *eps_n = d.eps[cur];
    R *eps_k = d.eps[1 - cur];

    C2<R> *twl = buf + 3 * 256;     // twiddles of the x transforms
    for (int i = tid; i < d.nx; i += nthr) twl[i] = d.tw[0][i];
    R corr[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
    // Anderson mode (AAM): k_aa_update has written the iterate into eps_k
    // (and k_aa_resid did the inverse x transform)
    const bool aam = AAM && !first;
    if (!first && !aam) {
        if (tid < d.tpbx)
            load_halfspec_pairs(d.spec, buf, d.nx, d.ny, d.nz, d.nkx, d.nhp, d.L, li, x, y, z, valid);
        __syncthreads();
        lds_fft<R, true, 8>(buf, 3 * d.L, d.nx, d.px, twl, tid, nthr);
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

    R sig[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
    double part[NPX];
#pragma unroll
    for (int i = 0; i < NPX; ++i) part[i] = 0.0;
    if (valid) {
        const R *base = first ? eps_n : eps_k;
        R e1[6], e0[6];
        if constexpr (AAM) {
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                e1[c] = aam ? base[c * d.nvox + vox] : base[c * d.nvox + vox] + R(sc->dE[c]);
                e0[c] = eps_n[c * d.nvox + vox];
            }
        } else {
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                e1[c] = base[c * d.nvox + vox] - corr[c] + R(sc->dE[c]);
                e0[c] = eps_n[c * d.nvox + vox];
            }
        }
#pragma unroll
        for (int c = 0; c < 6; ++c) eps_k[c * d.nvox + vox] = e1[c];
        const int lab = d.labels[vox];
        R v[NS];
        int nact = 0, nnewt = 0;
        if constexpr (ADAPT) {
            if (first)
                voxel_law_probe<R, NS, SPEC>(P, d.Qtab + lab * 9, e0, e1, d.st[cur], &d.st[1 - cur], d.nvox, vox,
                                             R(sc->dt), sc->M, rk_lim2, rk_maxd, d.mv + vox, sig, v, nact, nnewt,
                                             law_lds<R, NS>(smem_raw, xfft_lds_bytes<R>(), 0));
            else
                voxel_law<R, NS, SPEC>(P, d.Qtab + lab * 9, e0, e1, d.st[cur], &d.st[1 - cur], d.nvox, vox,
                                       R(sc->dt), sc->M << d.mv[vox], sig, v, nact, nnewt,
                                       law_lds<R, NS>(smem_raw, xfft_lds_bytes<R>(), 0));
        } else if constexpr (LAG) {
            voxel_law<R, NS, SPEC, true>(P, d.Qtab + lab * 9, e0, e1, d.st[cur], &d.st[1 - cur], d.nvox, vox,
                                         R(sc->dt), sc->M, sig, v, nact, nnewt,
                                         law_lds<R, NS>(smem_raw, xfft_lds_bytes<R>(), 0),
                                         LagRef<R>{d.lag + vox, d.nvox});
        } else {
            voxel_law<R, NS, SPEC>(P, d.Qtab + lab * 9, e0, e1, d.st[cur], &d.st[1 - cur], d.nvox, vox,
                                   R(sc->dt), sc->M, sig, v, nact, nnewt,
                                   law_lds<R, NS>(smem_raw, xfft_lds_bytes<R>(), 0));
        }
        part[9] = (double)nact;
        part[10] = (double)nnewt;
#pragma unroll
        for (int c = 0; c < 6; ++c) part[c] = (double)sig[c];
        part[6] = (double)von_mises(sig);
        double vs = 0.0, ft = 0.0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (s < P.nsys) {
                if ((P.twin_mask >> s) & 1u) ft += (double)v[s] * (double)P.inv_gT;
                else vs += (double)v[s];
            }
        }
        part[7] = vs;
        part[8] = ft;
    }
    block_sum<NPX, 4>(part, d.part_x + (long)(blockIdx.x - d.bx0) * NPX);

    if (tid < d.tpbx) {
#pragma unroll
        for (int p = 0; p < 3; ++p) buf[(p * d.L + li) * d.nx + x] = C2<R>{sig[2 * p], sig[2 * p + 1]};
    }
    __syncthreads();
    lds_fft<R, false, 8>(buf, 3 * d.L, d.nx, d.px, twl, tid, nthr);
    if (tid < d.tpbx)
        store_halfspec_pairs(d.spec, buf, d.nx, d.ny, d.nz, d.nkx, d.nhp, d.L, li, x, y, z, valid);
}

// Forward x transform of 6 real fields (component operator, one RVE).
template <typename R>
__global__ __launch_bounds__(256) void k_xpass_fwd(const R *__restrict__ f, C2<R> *spec, RveDev<R> d)
{
    extern __shared__ unsigned char smem_raw[];
    C2<R> *buf = reinterpret_cast<C2<R> *>(smem_raw);
    const int tid = threadIdx.x;
    const int li = tid / d.nx, x = tid - li * d.nx;
    const int line = blockIdx.x * d.L + li;
    const bool valid = tid < d.tpbx && line < d.nlines;
    const int y = valid ? line % d.ny : 0, z = valid ? line / d.ny : 0;
    const long vox = (long)line * d.nx + x;
    if (tid < d.tpbx) {
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            C2<R> v = {R(0), R(0)};
            if (valid) v = {f[(2 * p) * d.nvox + vox], f[(2 * p + 1) * d.nvox + vox]};
            buf[(p * d.L + li) * d.nx + x] = v;
        }
    }
    __syncthreads();
    lds_fft<R, false, 8>(buf, 3 * d.L, d.nx, d.px, d.tw[0], tid, blockDim.x);
    if (tid < d.tpbx) store_halfspec_pairs(spec, buf, d.nx, d.ny, d.nz, d.nkx, d.nhp, d.L, li, x, y, z, valid);
}

// Inverse x transform to 6 real fields, scaled by 1/nvox (component operator).
template <typename R>
__global__ __launch_bounds__(256) void k_xpass_inv(const C2<R> *__restrict__ spec, R *f, RveDev<R> d)
{
    extern __shared__ unsigned char smem_raw[];
    C2<R> *buf = reinterpret_cast<C2<R> *>(smem_raw);
    const int tid = threadIdx.x;
    const int li = tid / d.nx, x = tid - li * d.nx;
    const int line = blockIdx.x * d.L + li;
    const bool valid = tid < d.tpbx && line < d.nlines;
    const int y = valid ? line % d.ny : 0, z = valid ? line / d.ny : 0;
    const long vox = (long)line * d.nx + x;
    if (tid < d.tpbx) load_halfspec_pairs(spec, buf, d.nx, d.ny, d.nz, d.nkx, d.nhp, d.L, li, x, y, z, valid);
    __syncthreads();
    lds_fft<R, true, 8>(buf, 3 * d.L, d.nx, d.px, d.tw[0], tid, blockDim.x);
    if (valid) {
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            const C2<R> zz = buf[(p * d.L + li) * d.nx + x];
            f[(2 * p) * d.nvox + vox] = zz.x * d.inv_nvox;
            f[(2 * p + 1) * d.nvox + vox] = zz.y * d.inv_nvox;
        }
    }
}

// ---------------------------------------------------------------------------
// y pass: C2C along y on the half spectrum, stored [z][y][kx][c] (the six
// components of a frequency adjacent).  Block = one z, a tile of ty
// consecutive kx columns: 6 ty lines (column-major, components adjacent),
// each row of the tile one contiguous run of 6 ty values.  The first radix
// pass reads its inputs straight from the rows and the last writes its
// outputs straight back; the middle passes run in LDS laid out [y][line].
// ---------------------------------------------------------------------------
// spec_override (component operators): transform this array instead of the
// RVE's own spectrum, and ignore the step flag.
template <typename R, bool INV, int EPT>
__global__ __launch_bounds__(256) void k_ypass(const RveDev<R> *__restrict__ rv, int nrve,
                                               C2<R> *spec_override)
{
    const int blk = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int r = find_rve(rv, nrve, blk, 1);
    const RveDev<R> &d = rv[r];
    if ((!spec_override && d.sc->done) || d.yfix) return;
    extern __shared__ unsigned char smem_raw[];
    C2<R> *buf = reinterpret_cast<C2<R> *>(smem_raw);
    const int local = blk - d.by0;
    const int tile = local % d.nty, z = local / d.nty;
    const int ny = d.ny, nhp = d.nhp;
    const int kx0 = tile * d.ty;
    const int nl = 6 * min(d.ty, d.nkx - kx0);
    C2<R> *g = (spec_override ? spec_override : d.spec) + ((long)z * ny * nhp + kx0) * 6;
    const int tid = threadIdx.x, nthr = blockDim.x;
    // twiddles after the tile (the launch adds ny entries of LDS); the
    // first pass needs none and ends with a barrier
    C2<R> *twl = buf + (size_t)6 * d.ty * ny;
    for (int i = tid; i < ny; i += nthr) twl[i] = d.tw[1][i];
    const auto gline = [=](int l) { return g + l; };
    strided_fft<R, INV, EPT, true, true>(buf, nl, nl, d.py, twl, tid, nthr, gline, 6L * nhp);
}

// ---------------------------------------------------------------------------
// z pass fused with the Green operator.  Block = one ky, a tile of tz kx
// columns, all kz, all 6 components.
// ---------------------------------------------------------------------------
template <typename R>
struct GreenArgs {
    int nx, ny, nz;
    R inv_mu0;      // 1 / mu0
    R coef;         // (lam0 + mu0) / (mu0 (lam0 + 2 mu0))
    R inv_nx, inv_ny, inv_nz;
};

// sin and cos of the half angle pi m / N of frequency m (exact 1 and 0 at
// Nyquist, m = N/2)
__device__ __forceinline__ void half_angle(int m, int n, float &sn, float &cs)
{
    if (2 * m == n) { sn = 1.0f; cs = 0.0f; return; }
    sincospif((float)m / (float)n, &sn, &cs);
}
__device__ __forceinline__ void half_angle(int m, int n, double &sn, double &cs)
{
    if (2 * m == n) { sn = 1.0; cs = 0.0; return; }
    sincospi((double)m / (double)n, &sn, &cs);
}

// operator of green_point
constexpr int GREEN_CONT = 0;       // continuous, zero at every frequency with a Nyquist component
constexpr int GREEN_ROT = 1;        // rotated finite-difference scheme
constexpr int GREEN_CONT_NYQ = 2;   // continuous, the formula also at Nyquist frequencies

// Gamma0(x) : s for the unit direction x, into o; returns |s . x|^2 (summed
// in R: in FP32 a frequency's six squares need no FP64, the block sums of
// the residual are FP64 all the same).
template <typename R>
__device__ __forceinline__ double green_dir(const C2<R> (&s)[6], R x1, R x2, R x3, const GreenArgs<R> &g,
                                            C2<R> (&o)[6])
{
    // a = tau . xi, b = xi . a
    C2<R> a1, a2, a3;
    a1.x = s[0].x * x1 + s[5].x * x2 + s[4].x * x3;
    a1.y = s[0].y * x1 + s[5].y * x2 + s[4].y * x3;
    a2.x = s[5].x * x1 + s[1].x * x2 + s[3].x * x3;
    a2.y = s[5].y * x1 + s[1].y * x2 + s[3].y * x3;
    a3.x = s[4].x * x1 + s[3].x * x2 + s[2].x * x3;
    a3.y = s[4].y * x1 + s[3].y * x2 + s[2].y * x3;
    double t;
    if constexpr (sizeof(R) == 4)
        t = (double)(a1.x * a1.x + a1.y * a1.y + a2.x * a2.x + a2.y * a2.y + a3.x * a3.x + a3.y * a3.y);
    else
        t = a1.x * a1.x + a1.y * a1.y + a2.x * a2.x + a2.y * a2.y + a3.x * a3.x + a3.y * a3.y;
    const C2<R> b = {a1.x * x1 + a2.x * x2 + a3.x * x3, a1.y * x1 + a2.y * x2 + a3.y * x3};
    const R hm = R(0.5) * g.inv_mu0;
    const R xs[3] = {x1, x2, x3};
    const C2<R> as[3] = {a1, a2, a3};
    const int I[6] = {0, 1, 2, 1, 0, 0}, J[6] = {0, 1, 2, 2, 2, 1};
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const R xi = xs[I[c]], xj = xs[J[c]];
        const R q = g.coef * xi * xj;
        o[c].x = hm * (xi * as[J[c]].x + xj * as[I[c]].x) - q * b.x;
        o[c].y = hm * (xi * as[J[c]].y + xj * as[I[c]].y) - q * b.y;
    }
    return t;
}

template <typename R>
__device__ __forceinline__ void green_point(C2<R> (&s)[6], int kx, int ky, int kz, const GreenArgs<R> &g,
                                            int op, double &err2)
{
    // frequency m_j in (-N_j/2, N_j/2]
    const int my = ky <= g.ny / 2 ? ky : ky - g.ny;
    const int mz = kz <= g.nz / 2 ? kz : kz - g.nz;
    const int qx = (g.nx & 1) == 0 && 2 * kx == g.nx, qy = (g.ny & 1) == 0 && 2 * ky == g.ny,
              qz = (g.nz & 1) == 0 && 2 * kz == g.nz;
    // continuous operator: zero at any Nyquist component; rotated: zero
    // where two or more components are at Nyquist (s = 0 there); continuous
    // with Nyquist frequencies: zero only at the zero frequency
    const bool zero = op == GREEN_ROT ? qx + qy + qz >= 2 : (op == GREEN_CONT && (qx | qy | qz) != 0);
    if (zero || (kx == 0 && my == 0 && mz == 0)) {
#pragma unroll
        for (int c = 0; c < 6; ++c) s[c] = C2<R>{R(0), R(0)};
        return;
    }
    R x1, x2, x3;
    if (op == GREEN_ROT) {
        // rotated scheme: s_j = sin(q_j/2) prod_{l != j} cos(q_l/2)
        R sx, cx, sy, cy, sz, cz;
        half_angle(kx, g.nx, sx, cx);
        half_angle(my, g.ny, sy, cy);
        half_angle(mz, g.nz, sz, cz);
        x1 = sx * cy * cz; x2 = sy * cx * cz; x3 = sz * cx * cy;
    } else if constexpr (sizeof(R) == 4) {
        // direction of (m_x/N_x, m_y/N_y, m_z/N_z), m_j = +N_j/2 at Nyquist
        // (FP32: by the reciprocal sizes, normalized with the hardware
        // reciprocal square root; the direction is good to a few ulps)
        x1 = R(kx) * g.inv_nx; x2 = R(my) * g.inv_ny; x3 = R(mz) * g.inv_nz;
    } else {
        x1 = R(kx) / R(g.nx); x2 = R(my) / R(g.ny); x3 = R(mz) / R(g.nz);
    }
    R inr;
    if constexpr (sizeof(R) == 4) inr = __builtin_amdgcn_rsqf(x1 * x1 + x2 * x2 + x3 * x3);
    else inr = R(1) / sqrt(x1 * x1 + x2 * x2 + x3 * x3);
    x1 *= inr; x2 *= inr; x3 *= inr;
    // Hermitian partner in the half spectrum (the kx = 0 and Nyquist columns
    // hold their own)
    const bool own = kx == 0 || qx;
    C2<R> o[6];
    const double t = green_dir<R>(s, x1, x2, x3, g, o);
    if (op == GREEN_CONT_NYQ && (qx | qy | qz)) {
        // The partner index -k has the same +N/2 at its Nyquist components,
        // i.e. the direction m' = m with those components negated (Gamma0 is
        // even).  The real part of the inverse transform of the formula
        // applied at every frequency is the transform of the Hermitian part
        // 1/2 (Gamma0(m) + Gamma0(m')) : s, stored here; the residual counts
        // the partner with its own direction.
        C2<R> o2[6];
        const double t2 = green_dir<R>(s, qx ? -x1 : x1, qy ? -x2 : x2, qz ? -x3 : x3, g, o2);
        err2 += own ? t : t + t2;
#pragma unroll
        for (int c = 0; c < 6; ++c) s[c] = C2<R>{R(0.5) * (o[c].x + o2[c].x), R(0.5) * (o[c].y + o2[c].y)};
        return;
    }
    err2 += (own ? 1.0 : 2.0) * t;
#pragma unroll
    for (int c = 0; c < 6; ++c) s[c] = o[c];
}

// mode bits: ZMODE_FWD forward z transform; ZMODE_GREEN Gamma0, residual and
// inverse z transform.  The iteration uses both; the component operators
// use one each (with spec_override).
constexpr int ZMODE_FWD = 1;
constexpr int ZMODE_GREEN = 2;
constexpr int ZMODE_ROTATED = 4;   // with ZMODE_GREEN: the rotated-scheme operator
constexpr int ZMODE_NYQUIST = 8;   // with ZMODE_GREEN: the continuous operator also at Nyquist frequencies

__device__ __forceinline__ int green_op(int mode)
{
    return (mode & ZMODE_ROTATED) ? GREEN_ROT : (mode & ZMODE_NYQUIST) ? GREEN_CONT_NYQ : GREEN_CONT;
}

// Block = one ky, a tile of tz kx columns, all kz, all 6 components: the
// 6 tz lines (column-major, components adjacent) of nz points, each row of
// the tile one contiguous run of 6 tz values, laid out [kz][line] in LDS.
// The forward transform reads its first pass from the spectrum rows, the
// Green operator works in LDS (a frequency's six components adjacent), and
// the inverse writes its last pass back to the rows.
constexpr int Z_THREADS = 256;

template <typename R, int EPT>
__global__ __launch_bounds__(Z_THREADS) void k_zpass_green(const RveDev<R> *__restrict__ rv, int nrve, R inv_mu0,
                                                           R coef, int mode, C2<R> *spec_override)
{
    const int blk = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int r = find_rve(rv, nrve, blk, 2);
    const RveDev<R> &d = rv[r];
    if ((!spec_override && d.sc->done) || d.zfix) return;
    extern __shared__ unsigned char smem_raw[];
    C2<R> *buf = reinterpret_cast<C2<R> *>(smem_raw);
    const int local = blk - d.bz0;
    const int tile = local % d.ntz, ky = local / d.ntz;
    const int kx0 = tile * d.tz;
    const int tw_ = min(d.tz, d.nkx - kx0);
    const int nz = d.nz, nl = 6 * tw_;
    C2<R> *spec = (spec_override ? spec_override : d.spec) + ((long)ky * d.nhp + kx0) * 6;
    const long zstride = 6L * d.ny * d.nhp;
    const int tid = threadIdx.x, nthr = blockDim.x;
    // twiddles after the tile (the launch adds nz entries of LDS)
    C2<R> *twl = buf + (size_t)6 * d.tz * nz;
    for (int i = tid; i < nz; i += nthr) twl[i] = d.tw[2][i];
    const unsigned mt = fdiv_magic((unsigned)tw_);
    const auto gline = [=](int l) { return spec + l; };
    if (!(mode & ZMODE_GREEN)) {
        // forward transform only (component operator)
        strided_fft<R, false, EPT, true, true>(buf, nl, nl, d.pz, twl, tid, nthr, gline, zstride);
        return;
    }
    if (mode & ZMODE_FWD) {
        strided_fft<R, false, EPT, true, false>(buf, nl, nl, d.pz, twl, tid, nthr, gline, zstride);
    } else {
        const unsigned ml = fdiv_magic((unsigned)nl);
        for (int i = tid; i < nl * nz; i += nthr) {
            const int e = (int)fdiv((unsigned)i, ml), l = i - e * nl;
            buf[e * nl + l] = gline(l)[e * zstride];
        }
        __syncthreads();
    }
    const GreenArgs<R> g = {d.nx, d.ny, d.nz, inv_mu0, coef, R(1) / R(d.nx), R(1) / R(d.ny), R(1) / R(d.nz)};
    double err2 = 0.0;
    for (int i = tid; i < tw_ * nz; i += nthr) {
        const int kz = (int)fdiv((unsigned)i, mt), col = i - kz * tw_;
        C2<R> sv[6];
        C2<R> *f = buf + kz * nl + col * 6;
#pragma unroll
        for (int c = 0; c < 6; ++c) sv[c] = f[c];
        green_point<R>(sv, kx0 + col, ky, kz, g, green_op(mode), err2);
#pragma unroll
        for (int c = 0; c < 6; ++c) f[c] = sv[c];
    }
    double e[1] = {err2};
    block_sum<1, Z_THREADS / 64>(e, d.part_z + local);
    __syncthreads();
    strided_fft<R, true, EPT, false, true>(buf, nl, nl, d.pz, twl, tid, nthr, gline, zstride);
}

// ---------------------------------------------------------------------------
// First stage of the scalar reduction: BC_CHUNKS blocks per RVE each sum a
// fixed contiguous chunk of the x-pass block sums (NPX values each) and of
// the z-pass residual sums, in a fixed order; b = RVE * BC_CHUNKS + chunk.
// 256 threads.
// ---------------------------------------------------------------------------
constexpr int BC_CHUNKS = 32;

template <typename R>
__device__ __forceinline__ void bc_partials_block(const RveDev<R> *__restrict__ rv, int b)
{
    const RveDev<R> &d = rv[b / BC_CHUNKS];
    const int c = b % BC_CHUNKS;
    if (d.sc->done) return;
    const int nbx = (d.nlines + d.L - 1) / d.L, nbz = d.ntz * d.ny;
    const int x0 = (int)((long)nbx * c / BC_CHUNKS), x1 = (int)((long)nbx * (c + 1) / BC_CHUNKS);
    const int z0 = (int)((long)nbz * c / BC_CHUNKS), z1 = (int)((long)nbz * (c + 1) / BC_CHUNKS);
    double acc[NPX + 1];
#pragma unroll
    for (int i = 0; i < NPX + 1; ++i) acc[i] = 0.0;
    for (int j = x0 + threadIdx.x; j < x1; j += blockDim.x)
#pragma unroll
        for (int i = 0; i < NPX; ++i) acc[i] += d.part_x[(long)j * NPX + i];
    for (int j = z0 + threadIdx.x; j < z1; j += blockDim.x) acc[NPX] += d.part_z[j];
    block_sum<NPX + 1, 4>(acc, d.part_b + (long)c * (NPX + 1));
}

// ---------------------------------------------------------------------------
// Fixed-length y and z passes: the common lengths (fixed_len) with their
// radix plans and the tile width known at compile time (fixed_tile columns
// of 6 components), 256 threads.  The same transforms as k_ypass and
// k_zpass_green; an RVE is done by one kernel or the other (yfix, zfix).
// ---------------------------------------------------------------------------
constexpr int FX_THREADS = 256;   // threads of the fixed-length y and z blocks

__host__ __device__ constexpr bool fixed_len(int n)
{
    return n == 32 || n == 48 || n == 64 || n == 96 || n == 128 || n == 256;
}
template <typename R, int N>
__host__ __device__ constexpr int fixed_tile()
{
    return (sizeof(R) == 8 && N == 256) ? 2 : 4;
}
template <typename R>
__host__ __device__ constexpr int fixed_tile_of(int n)
{
    return (sizeof(R) == 8 && n == 256) ? 2 : 4;
}

template <typename R, bool INV, int N>
__device__ __forceinline__ void ypass_fixed(const RveDev<R> &d, C2<R> *g, C2<R> *buf, int nlv)
{
    constexpr int NL = 6 * fixed_tile<R, N>();
    C2<R> *twl = buf + NL * N;
    const C2<R> *twg = d.tw[1];
    const auto stage = [=]() {
        for (int i = threadIdx.x; i < N; i += FX_THREADS) twl[i] = twg[i];
    };
    const auto gline = [=](int l) { return g + l; };
    fixed_fft<R, INV, N, NL, FX_THREADS, true, true>(buf, nlv, twl, gline, 6L * d.nhp, stage);
}

// nbc > 0 (a multiple of 8, so that the XCD of each transform block is
// unchanged): the first nbc blocks of the launch are the first stage of the
// scalar reduction (bc_partials_block) instead of a launch of their own;
// the x and z passes that wrote its inputs ran before.
template <typename R, bool INV>
__global__ __launch_bounds__(FX_THREADS) void k_ypass_fx(const RveDev<R> *__restrict__ rv, int nrve, C2<R> *spec_override,
                                                  int nbc)
{
    if ((int)blockIdx.x < nbc) {
        bc_partials_block<R>(rv, (int)blockIdx.x);
        return;
    }
    const int blk = xcd_block((int)blockIdx.x - nbc, (int)gridDim.x - nbc);
    const int r = find_rve(rv, nrve, blk, 1);
    const RveDev<R> &d = rv[r];
    if ((!spec_override && d.sc->done) || !d.yfix) return;
    extern __shared__ unsigned char smem_raw[];
    C2<R> *buf = reinterpret_cast<C2<R> *>(smem_raw);
    const int local = blk - d.by0;
    const int tile = local % d.nty, z = local / d.nty;
    const int kx0 = tile * d.ty;
    const int nlv = 6 * min(d.ty, d.nkx - kx0);
    C2<R> *g = (spec_override ? spec_override : d.spec) + ((long)z * d.ny * d.nhp + kx0) * 6;
    switch (d.ny) {
    case 32: ypass_fixed<R, INV, 32>(d, g, buf, nlv); break;
    case 48: ypass_fixed<R, INV, 48>(d, g, buf, nlv); break;
    case 64: ypass_fixed<R, INV, 64>(d, g, buf, nlv); break;
    case 96: ypass_fixed<R, INV, 96>(d, g, buf, nlv); break;
    case 128: ypass_fixed<R, INV, 128>(d, g, buf, nlv); break;
    default: ypass_fixed<R, INV, 256>(d, g, buf, nlv); break;
    }
}

template <typename R, int N>
__device__ __forceinline__ void zpass_fixed(const RveDev<R> &d, C2<R> *spec, C2<R> *buf, int tw_, int kx0, int ky,
                                            int local, R inv_mu0, R coef, int mode)
{
    constexpr int TILE = fixed_tile<R, N>(), NL = 6 * TILE;
    const int nlv = 6 * tw_;
    const long zs = 6L * d.ny * d.nhp;
    C2<R> *twl = buf + NL * N;
    const C2<R> *twg = d.tw[2];
    const auto stage = [=]() {
        for (int i = threadIdx.x; i < N; i += FX_THREADS) twl[i] = twg[i];
    };
    const auto gline = [=](int l) { return spec + l; };
    if (!(mode & ZMODE_GREEN)) {
        fixed_fft<R, false, N, NL, FX_THREADS, true, true>(buf, nlv, twl, gline, zs, stage);
        return;
    }
    if (mode & ZMODE_FWD) {
        fixed_fft<R, false, N, NL, FX_THREADS, true, false>(buf, nlv, twl, gline, zs, stage);
    } else {
        for (int i = threadIdx.x; i < NL * N; i += FX_THREADS) {
            const int e = i / NL, l = i - e * NL;
            buf[i] = l < nlv ? gload(gline(l) + e * zs) : C2<R>{R(0), R(0)};
        }
        stage();
        __syncthreads();
    }
    const GreenArgs<R> g = {d.nx, d.ny, d.nz, inv_mu0, coef, R(1) / R(d.nx), R(1) / R(d.ny), R(1) / R(d.nz)};
    double err2 = 0.0;
    for (int i = threadIdx.x; i < TILE * N; i += FX_THREADS) {
        const int kz = i / TILE, col = i - kz * TILE;
        if (col < tw_) {
            C2<R> sv[6];
            C2<R> *f = buf + kz * NL + col * 6;
#pragma unroll
            for (int c = 0; c < 6; ++c) sv[c] = f[c];
            green_point<R>(sv, kx0 + col, ky, kz, g, green_op(mode), err2);
#pragma unroll
            for (int c = 0; c < 6; ++c) f[c] = sv[c];
        }
    }
    double e[1] = {err2};
    block_sum<1, FX_THREADS / 64>(e, d.part_z + local);
    __syncthreads();
    fixed_fft<R, true, N, NL, FX_THREADS, false, true>(buf, nlv, twl, gline, zs);
}

template <typename R>
__global__ __launch_bounds__(FX_THREADS) void k_zpass_fx(const RveDev<R> *__restrict__ rv, int nrve, R inv_mu0, R coef,
                                                  int mode, C2<R> *spec_override)
{
    const int blk = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int r = find_rve(rv, nrve, blk, 2);
    const RveDev<R> &d = rv[r];
    if ((!spec_override && d.sc->done) || !d.zfix) return;
    extern __shared__ unsigned char smem_raw[];
    C2<R> *buf = reinterpret_cast<C2<R> *>(smem_raw);
    const int local = blk - d.bz0;
    const int tile = local % d.ntz, ky = local / d.ntz;
    const int kx0 = tile * d.tz;
    const int tw_ = min(d.tz, d.nkx - kx0);
    C2<R> *spec = (spec_override ? spec_override : d.spec) + ((long)ky * d.nhp + kx0) * 6;
    switch (d.nz) {
    case 32: zpass_fixed<R, 32>(d, spec, buf, tw_, kx0, ky, local, inv_mu0, coef, mode); break;
    case 48: zpass_fixed<R, 48>(d, spec, buf, tw_, kx0, ky, local, inv_mu0, coef, mode); break;
    case 64: zpass_fixed<R, 64>(d, spec, buf, tw_, kx0, ky, local, inv_mu0, coef, mode); break;
    case 96: zpass_fixed<R, 96>(d, spec, buf, tw_, kx0, ky, local, inv_mu0, coef, mode); break;
    case 128: zpass_fixed<R, 128>(d, spec, buf, tw_, kx0, ky, local, inv_mu0, coef, mode); break;
    default: zpass_fixed<R, 256>(d, spec, buf, tw_, kx0, ky, local, inv_mu0, coef, mode); break;
    }
}

// ---------------------------------------------------------------------------
// Step bookkeeping
// ---------------------------------------------------------------------------
struct StepInit {
    double dE0[6], E0[6], target[6], K0inv[36];
    int sidx[6];
    int cur, M;
    double dt;
};

// One block per RVE: reset the step scalars from the host-prepared record.
template <typename R>
__global__ void k_begin_step(const RveDev<R> *__restrict__ rv, const StepInit *__restrict__ si)
{
    if (threadIdx.x != 0) return;
    Scalars *sc = rv[blockIdx.x].sc;
    const StepInit &q = si[blockIdx.x];
    for (int i = 0; i < 6; ++i) {
        sc->dE[i] = q.dE0[i];
        sc->E[i] = q.E0[i];
        sc->target[i] = q.target[i];
        sc->sidx[i] = q.sidx[i];
        sc->Sigma[i] = 0.0;
    }
    for (int i = 0; i < 36; ++i) sc->K0inv[i] = q.K0inv[i];
    for (int i = 0; i < 8; ++i) sc->err_hist[i] = 0.0;
    sc->iter = 0;
    sc->done = 0;
    sc->status = 0;
    sc->stagnated = 0;
    sc->cur = q.cur;
    sc->M = q.M;
    sc->dt = q.dt;
    sc->err_eq = sc->err_bc = 0.0;
    sc->mean_sig_eq = sc->mean_v = sc->mean_f = 0.0;
    sc->work_active = sc->work_newton = 0.0;
    sc->n_symptom = 0ull;
    sc->bad_state = 0;
    AaState *aa = rv[blockIdx.x].aa;
    if (aa) {
        aa->count = 0;
        aa->head = 0;
        aa->slot = -1;
        aa->have_prev = 0;
        aa->nk = 0;
    }
}

struct BcArgs {
    double n_slip, n_twin;
    double tol, stag_tol;
    int max_iter;
};

__device__ __forceinline__ double frob2(const double a[6])
{
    return a[0] * a[0] + a[1] * a[1] + a[2] * a[2] + 2.0 * (a[3] * a[3] + a[4] * a[4] + a[5] * a[5]);
}

// ---------------------------------------------------------------------------
// Anderson acceleration (an option; Walker and Ni, 2011): with x_j the
// iterates and f_j = -Gamma0 * sigma(x_j) + dE_j the basic scheme's steps,
// x_{k+1} = x_k + f_k - sum_s gamma_s (dX_s + dF_s) over the last (up to)
// m differences dX = x_{j+1} - x_j, dF = f_{j+1} - f_j, gamma solving
// (G + lam I) gamma = dF^T f_k, G = dF^T dF (Frobenius products of the
// fields), lam = 1e-14 trace(G) / m_k.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void aa_ring_after(const AaState &a, int m, int &slot, int &cnt, int &head)
{
    // ring after inserting one difference (only when an earlier step exists)
    if (a.count < m) {
        slot = (a.head + a.count) % m;
        cnt = a.count + 1;
        head = a.head;
    } else {
        slot = a.head;
        cnt = m;
        head = (a.head + 1) % m;
    }
}

// Per x-line block: the inverse x transform of the spectrum (the step of
// the last iterate), the new differences into the rings, and the block
// sums of dF_s . f (slots 0..m-1) and dF_s . dF_new (AA_MAX + slot).
template <typename R>
__global__ __launch_bounds__(256) void k_aa_resid(const RveDev<R> *__restrict__ rv, int nrve)
{
    const int r = find_rve(rv, nrve, (int)blockIdx.x, 0);
    const RveDev<R> &d = rv[r];
    Scalars *sc = d.sc;
    if (!d.aa || sc->done || sc->iter == 0) return;
    extern __shared__ unsigned char smem_raw[];
    C2<R> *buf = reinterpret_cast<C2<R> *>(smem_raw);
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int li = tid / d.nx, x = tid - li * d.nx;
    const int line = (blockIdx.x - d.bx0) * d.L + li;
    const bool valid = tid < d.tpbx && line < d.nlines;
    const int y = valid ? line % d.ny : 0, z = valid ? line / d.ny : 0;
    const long vox = (long)line * d.nx + x;
    C2<R> *twl = buf + 3 * 256;
    for (int i = tid; i < d.nx; i += nthr) twl[i] = d.tw[0][i];
    if (tid < d.tpbx) load_halfspec_pairs(d.spec, buf, d.nx, d.ny, d.nz, d.nkx, d.nhp, d.L, li, x, y, z, valid);
    __syncthreads();
    lds_fft<R, true, 8>(buf, 3 * d.L, d.nx, d.px, twl, tid, nthr);
    const AaState &a = *d.aa;
    const int m = d.aa_depth;
    const bool have = a.have_prev != 0;
    int slot = -1, cnt = 0, head = 0;
    if (have) aa_ring_after(a, m, slot, cnt, head);
    double part[2 * AA_MAX];
#pragma unroll
    for (int i = 0; i < 2 * AA_MAX; ++i) part[i] = 0.0;
    if (valid) {
        R f[6], dF[6];
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            const C2<R> zz = buf[(p * d.L + li) * d.nx + x];
            f[2 * p] = -zz.x * d.inv_nvox + R(sc->dE[2 * p]);
            f[2 * p + 1] = -zz.y * d.inv_nvox + R(sc->dE[2 * p + 1]);
        }
        const R *eps_k = d.eps[1 - sc->cur];
        if (have) {
            const long o = (long)slot * 6 * d.nvox + vox;
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                const long i = (long)c * d.nvox + vox;
                dF[c] = f[c] - d.aa_f[i];
                d.aa_dF[o + c * d.nvox] = dF[c];
                d.aa_dX[o + c * d.nvox] = eps_k[i] - d.aa_x[i];
            }
        }
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const long i = (long)c * d.nvox + vox;
            d.aa_f[i] = f[c];
            d.aa_x[i] = eps_k[i];
        }
        if (have) {
            for (int t = 0; t < cnt; ++t) {
                const int sl = (head + t) % m;
                const long o = (long)sl * 6 * d.nvox + vox;
                double p1 = 0.0, p2 = 0.0;
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    const double w = c < 3 ? 1.0 : 2.0;   // Frobenius product in tensor components
                    const double g = sl == slot ? (double)dF[c] : (double)d.aa_dF[o + c * d.nvox];
                    p1 += w * g * (double)f[c];
                    p2 += w * g * (double)dF[c];
                }
                // slots < AA_MAX: constant indices keep part[] in registers
#pragma unroll
                for (int q = 0; q < AA_MAX; ++q)
                    if (q == sl) {
                        part[q] += p1;
                        part[AA_MAX + q] += p2;
                    }
            }
        }
    }
    block_sum<2 * AA_MAX, 4>(part, d.aa_part + (long)(blockIdx.x - d.bx0) * 2 * AA_MAX);
}

template <typename R>
__global__ __launch_bounds__(256) void k_aa_partials(const RveDev<R> *__restrict__ rv)
{
    const RveDev<R> &d = rv[blockIdx.x / 32];
    const int c = blockIdx.x % 32;
    if (!d.aa || d.sc->done || d.sc->iter == 0) return;
    const int nbx = (d.nlines + d.L - 1) / d.L;
    const int x0 = (int)((long)nbx * c / 32), x1 = (int)((long)nbx * (c + 1) / 32);
    double acc[2 * AA_MAX];
#pragma unroll
    for (int i = 0; i < 2 * AA_MAX; ++i) acc[i] = 0.0;
    for (int j = x0 + threadIdx.x; j < x1; j += blockDim.x)
#pragma unroll
        for (int i = 0; i < 2 * AA_MAX; ++i) acc[i] += d.aa_part[(long)j * 2 * AA_MAX + i];
    block_sum<2 * AA_MAX, 4>(acc, d.aa_chunk + (long)c * 2 * AA_MAX);
}

// One wave per RVE: the Gram row of the new difference, the regularized
// normal equations by Cholesky (FP64), and the same mixing of the mean
// strain E (sc->E holds the basic step's E_{k-1} + dE_{k-1}).
template <typename R>
__global__ __launch_bounds__(64) void k_aa_solve(const RveDev<R> *__restrict__ rv)
{
    const RveDev<R> &d = rv[blockIdx.x];
    Scalars *sc = d.sc;
    if (!d.aa || sc->done || sc->iter == 0) return;
    double acc[2 * AA_MAX];
#pragma unroll
    for (int i = 0; i < 2 * AA_MAX; ++i) acc[i] = 0.0;
    for (int j = threadIdx.x; j < 32; j += blockDim.x)
#pragma unroll
        for (int i = 0; i < 2 * AA_MAX; ++i) acc[i] += d.aa_chunk[(long)j * 2 * AA_MAX + i];
    __shared__ double tot[2 * AA_MAX];
    block_sum<2 * AA_MAX, 1>(acc, tot);
    __syncthreads();
    if (threadIdx.x != 0) return;
    AaState &a = *d.aa;
    const int m = d.aa_depth;
    double Ek[6], dEk[6];
    for (int i = 0; i < 6; ++i) {
        dEk[i] = sc->dE[i];
        Ek[i] = sc->E[i] - sc->dE[i];   // E of the last iterate
    }
    if (!a.have_prev) {
        for (int i = 0; i < 6; ++i) {
            a.E_prev[i] = Ek[i];
            a.dE_prev[i] = dEk[i];
        }
        a.have_prev = 1;
        a.nk = 0;
        a.slot = -1;
        return;   // basic step: E stays E_{k-1} + dE_{k-1}
    }
    int slot, cnt, head;
    aa_ring_after(a, m, slot, cnt, head);
    for (int t = 0; t < cnt; ++t) {
        const int sl = (head + t) % m;
        a.G[slot][sl] = tot[AA_MAX + sl];
        a.G[sl][slot] = tot[AA_MAX + sl];
    }
    for (int i = 0; i < 6; ++i) {
        a.dEX[slot][i] = Ek[i] - a.E_prev[i];
        a.ddE[slot][i] = dEk[i] - a.dE_prev[i];
        a.E_prev[i] = Ek[i];
        a.dE_prev[i] = dEk[i];
    }
    a.count = cnt;
    a.head = head;
    a.slot = slot;
    // (G + lam I) g = b over the slots in ring order, Cholesky L L^T
    double A[AA_MAX][AA_MAX], b[AA_MAX], tr = 0.0;
    for (int t = 0; t < cnt; ++t) tr += a.G[(head + t) % m][(head + t) % m];
    const double lam = 1e-14 * tr / cnt;
    bool ok = tr > 0.0;
    for (int t = 0; t < cnt; ++t) {
        const int st = (head + t) % m;
        b[t] = tot[st];
        for (int u = 0; u < cnt; ++u) A[t][u] = a.G[st][(head + u) % m] + (t == u ? lam : 0.0);
    }
    for (int t = 0; t < cnt && ok; ++t) {
        for (int u = 0; u <= t; ++u) {
            double sum = A[t][u];
            for (int q = 0; q < u; ++q) sum -= A[t][q] * A[u][q];
            if (t == u) {
                if (!(sum > 0.0)) { ok = false; break; }
                A[t][t] = sqrt(sum);
            } else {
                A[t][u] = sum / A[u][u];
            }
        }
    }
    if (!ok) {
        a.nk = 0;   // degenerate history: the basic step
        return;
    }
    double g[AA_MAX];
    for (int t = 0; t < cnt; ++t) {
        double sum = b[t];
        for (int q = 0; q < t; ++q) sum -= A[t][q] * g[q];
        g[t] = sum / A[t][t];
    }
    for (int t = cnt - 1; t >= 0; --t) {
        double sum = g[t];
        for (int q = t + 1; q < cnt; ++q) sum -= A[q][t] * g[q];
        g[t] = sum / A[t][t];
    }
    for (int t = 0; t < cnt; ++t) {
        const int st = (head + t) % m;
        a.gamma[st] = g[t];
        for (int i = 0; i < 6; ++i) sc->E[i] -= g[t] * (a.dEX[st][i] + a.ddE[st][i]);
    }
    a.nk = cnt;
}

// The Anderson iterate x_k = x_{k-1} + f_{k-1} - sum_s gamma_s (dX_s +
// dF_s), written over the iterate buffer (k_aa_resid has kept x_{k-1}).
template <typename R>
__global__ __launch_bounds__(256) void k_aa_update(const RveDev<R> *__restrict__ rv, int nrve)
{
    const int r = find_rve(rv, nrve, (int)blockIdx.x, 0);
    const RveDev<R> &d = rv[r];
    Scalars *sc = d.sc;
    if (!d.aa || sc->done || sc->iter == 0) return;
    const int tid = threadIdx.x;
    const int li = tid / d.nx, x = tid - li * d.nx;
    const int line = (blockIdx.x - d.bx0) * d.L + li;
    if (tid >= d.tpbx || line >= d.nlines) return;
    const long vox = (long)line * d.nx + x;
    const AaState &a = *d.aa;
    const int nk = a.nk, hd = a.head, m = d.aa_depth;
    R *eps_k = d.eps[1 - sc->cur];
    R e[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) e[c] = d.aa_x[c * d.nvox + vox] + d.aa_f[c * d.nvox + vox];
    for (int t = 0; t < nk; ++t) {
        const int sl = (hd + t) % m;
        const R g = R(a.gamma[sl]);
        const long o = (long)sl * 6 * d.nvox + vox;
#pragma unroll
        for (int c = 0; c < 6; ++c) e[c] -= g * (d.aa_dX[o + c * d.nvox] + d.aa_dF[o + c * d.nvox]);
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) eps_k[c * d.nvox + vox] = e[c];
}

// First stage of the scalar reduction as its own launch (the iteration runs
// it inside the inverse y pass's launch where that pass is the fixed-length
// kernel).
template <typename R>
__global__ __launch_bounds__(256) void k_bc_partials(const RveDev<R> *__restrict__ rv)
{
    bc_partials_block<R>(rv, (int)blockIdx.x);
}

// One block per RVE: sum the chunk sums (fixed order), evaluate the
// residuals, decide convergence and correct the stress-controlled mean
// strain.
template <typename R>
__global__ __launch_bounds__(64) void k_bc_update(const RveDev<R> *__restrict__ rv, BcArgs b)
{
    const RveDev<R> &d = rv[blockIdx.x];
    Scalars *sc = d.sc;
    if (sc->done) return;
    const double nvox = (double)d.nvox;
    double acc[NPX + 1];
#pragma unroll
    for (int i = 0; i < NPX + 1; ++i) acc[i] = 0.0;
    for (int j = threadIdx.x; j < BC_CHUNKS; j += blockDim.x)
#pragma unroll
        for (int i = 0; i < NPX + 1; ++i) acc[i] += d.part_b[(long)j * (NPX + 1) + i];
    __shared__ double tot[NPX + 1];
    block_sum<NPX + 1, 1>(acc, tot);
    __syncthreads();
    if (threadIdx.x != 0) return;

    double S[6];
    for (int i = 0; i < 6; ++i) S[i] = tot[i] / nvox;
    const double nrm = sqrt(frob2(S));
    const double num = sqrt(tot[NPX]);
    double dS[6];
    for (int i = 0; i < 6; ++i) dS[i] = sc->sidx[i] ? S[i] - sc->target[i] : 0.0;
    const double nb = sqrt(frob2(dS));
    const double err_eq = nrm > 0.0 ? num / (nvox * nrm) : (num == 0.0 ? 0.0 : INFINITY);
    const double err_bc = nrm > 0.0 ? nb / nrm : (nb == 0.0 ? 0.0 : INFINITY);
    const int it = sc->iter + 1;
    sc->iter = it;
    for (int i = 0; i < 6; ++i) sc->Sigma[i] = S[i];
    sc->err_eq = err_eq;
    sc->err_bc = err_bc;
    sc->mean_sig_eq = tot[6] / nvox;
    sc->mean_v = b.n_slip > 0 ? tot[7] / (nvox * b.n_slip) : 0.0;
    sc->mean_f = b.n_twin > 0 ? tot[8] / (nvox * b.n_twin) : 0.0;
    sc->work_active += tot[9];
    sc->work_newton += tot[10];

    const double err = fmax(err_eq, err_bc);
    if (!(err == err) || isinf(tot[0]) || !(tot[0] == tot[0])) {
        sc->status = -5;  // CPF_E_NAN
        sc->done = 1;
        return;
    }
    if (err_eq <= b.tol && err_bc <= b.tol) {
        sc->done = 1;
        return;
    }
    // stalled residual below the acceptance level (reduced precision)
    const double old = sc->err_hist[it & 7];
    sc->err_hist[it & 7] = err;   // slot of iteration it; read back 8 iterations later
    if (b.stag_tol > 0.0 && err < b.stag_tol && it > 8 && err > 0.99 * old) {
        sc->stagnated = 1;
        sc->done = 1;
        return;
    }
    if (it >= b.max_iter) {
        sc->status = -4;  // CPF_E_NOT_CONVERGED
        sc->done = 1;
        return;
    }
    // mixed conditions: dE_S = (C0_SS)^-1 (Sigma*_S - Sigma_S)
    double rr[6];
    for (int i = 0; i < 6; ++i) rr[i] = sc->sidx[i] ? sc->target[i] - S[i] : 0.0;
    for (int i = 0; i < 6; ++i) {
        double dd = 0.0;
        for (int j = 0; j < 6; ++j) dd += sc->K0inv[i * 6 + j] * rr[j];
        sc->dE[i] = dd;
        sc->E[i] += dd;
    }
}

// ---------------------------------------------------------------------------
// Component operators and field outputs
// ---------------------------------------------------------------------------
template <typename R, int NS, int SPEC>
__global__ __launch_bounds__(256, (xpass_min_blocks<R, SPEC>())) void k_constitutive(
    const int32_t *labels, const R *Qtab, const R *eps0, const R *eps1, const R *st0, R *st1, R *sig,
    LawP<R> Parg, long nvox, R dt, int M)
{
    const LawP<R> &P = Parg;
    extern __shared__ unsigned char smem_raw[];
    const long vox = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (vox >= nvox) return;
    const int lab = labels[vox];
    R e0[6], e1[6], s[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        e0[c] = eps0[c * nvox + vox];
        e1[c] = eps1[c * nvox + vox];
    }
    R v[NS];
    int nact = 0, nnewt = 0;
    voxel_law<R, NS, SPEC>(P, Qtab + lab * 9, e0, e1, st0, &st1, nvox, vox, dt, M, s, v, nact, nnewt,
                           law_lds<R, NS>(smem_raw, 0, law_lds_bytes<R, NS>()));
#pragma unroll
    for (int c = 0; c < 6; ++c) sig[c * nvox + vox] = s[c];
}

// Lagged regularization, at the commit of a load step: the raise of each
// system's resistance in the next step is eta times the system's mean slip
// rate over this one, (v_{n+1} - v_n) eta / dt, with f = eta / dt.  The
// slip rows of the state are contiguous ([6 + s][nvox]), so element i of
// the raise array [S][nvox] pairs with element 6 nvox + i of the state.
template <typename R>
__global__ void k_lag_update(R *__restrict__ lag, const R *__restrict__ st_new, const R *__restrict__ st_old,
                             long nvox, int nsys, R f)
{
    const long n = (long)nsys * nvox;
    const R *vn = st_new + 6 * nvox, *vo = st_old + 6 * nvox;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        lag[i] = f * (vn[i] - vo[i]);
}

// sigma = C_lab : (eps - eps_p) at one voxel from a committed strain and
// state (lab frame, tensor components).
template <typename R>
__device__ __forceinline__ void voxel_stress(const int32_t *labels, const R *Qtab, const R *eps, const R *st,
                                             const LawP<R> &P, long nvox, long vox, R sl[6])
{
    const int lab = labels[vox];
    R Q[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) Q[i] = Qtab[lab * 9 + i];
    R el[6], epl[6], ec[6], epc[6], sc[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        el[c] = eps[c * nvox + vox];
        epl[c] = st[c * nvox + vox];
    }
    rot_to_crystal(Q, el, ec);
    rot_to_crystal(Q, epl, epc);
    hooke(P, ec, epc, sc);
    rot_to_lab(Q, sc, sl);
}

template <typename R>
__global__ __launch_bounds__(256) void k_stress_field(const int32_t *labels, const R *Qtab, const R *eps,
                                                      const R *st, R *sig, LawP<R> P, long nvox)
{
    const long vox = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (vox >= nvox) return;
    R sl[6];
    voxel_stress<R>(labels, Qtab, eps, st, P, nvox, vox, sl);
#pragma unroll
    for (int c = 0; c < 6; ++c) sig[c * nvox + vox] = sl[c];
}

// Voxels whose stress moved by more than E0 |dE| over the load step, the
// situation in which the paper observes that the basic scheme stops
// enforcing equilibrium locally (Section 4): |sigma_{n+1} - sigma_n|_F >
// E0 |E_{n+1} - E_n|_F, Frobenius norms of tensor components, E0 the
// Young's modulus of the reference medium, thr2 = (E0 |dE|_F)^2.  The
// stress difference is Hooke's law of the difference of the elastic
// strains, taken in the crystal frame (the norm does not depend on the
// frame); the norm is summed in FP64.  Block counts are added with one
// integer atomic per block (the total does not depend on the order).  The
// same pass checks every component of the converged strain and state for
// non-finite values (a state variable of an inactive system never reaches
// the stress, so the residual would not show it) and raises *bad.
template <typename R>
__global__ __launch_bounds__(256) void k_symptom(const int32_t *labels, const R *Qtab, const R *e1, const R *s1,
                                                 const R *e0, const R *s0, LawP<R> P, long nvox, double thr2,
                                                 int D, unsigned long long *count, int *bad)
{
    const long vox = (long)blockIdx.x * blockDim.x + threadIdx.x;
    int hit = 0;
    bool finite = true;
    if (vox < nvox) {
        for (int c = 0; c < D; ++c) finite = finite && isfinite(s1[c * nvox + vox]);
#pragma unroll
        for (int c = 0; c < 6; ++c) finite = finite && isfinite(e1[c * nvox + vox]);
    }
    if (__ballot(!finite) && (threadIdx.x & 63u) == 0u) atomicOr(bad, 1);
    if (vox < nvox) {
        const int lab = labels[vox];
        R Q[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) Q[i] = Qtab[lab * 9 + i];
        R dl[6], dc[6], zero[6], sc[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            dl[c] = (e1[c * nvox + vox] - s1[c * nvox + vox]) - (e0[c * nvox + vox] - s0[c * nvox + vox]);
            zero[c] = R(0);
        }
        rot_to_crystal(Q, dl, dc);
        hooke(P, dc, zero, sc);
        double n2 = 0.0;
#pragma unroll
        for (int c = 0; c < 6; ++c) n2 += (c < 3 ? 1.0 : 2.0) * (double)sc[c] * (double)sc[c];
        hit = n2 > thr2;
    }
    __shared__ unsigned int block_count;
    if (threadIdx.x == 0) block_count = 0u;
    __syncthreads();
    const int wc = __popcll(__ballot(hit));
    if ((threadIdx.x & 63u) == 0u && wc) atomicAdd(&block_count, (unsigned int)wc);
    __syncthreads();
    if (threadIdx.x == 0 && block_count) atomicAdd(count, (unsigned long long)block_count);
}

// Square of the von Mises stress in FP64 by a fixed order of single,
// correctly rounded operations, so that a host computation in the same
// order gives the same number (plain operators in a scope with contraction
// off: the rounding intrinsics of the HIP headers are plain operators
// compiled under the default contraction, which fuses them once inlined):
//   m = ((s11 + s22) + s33) / 3,  d_i = s_ii - m,
//   J = ((d1 d1 + d2 d2) + d3 d3) + 2 ((s23 s23 + s13 s13) + s12 s12),
//   sigma_eq^2 = 1.5 J.
template <typename R>
__device__ __forceinline__ double von_mises_sq_exact(const R s[6])
{
#pragma clang fp contract(off)
    const double a = s[0], b = s[1], c = s[2], d = s[3], e = s[4], f = s[5];
    const double m = ((a + b) + c) / 3.0;
    const double d1 = a - m, d2 = b - m, d3 = c - m;
    const double nrm = (d1 * d1 + d2 * d2) + d3 * d3;
    const double sh = (d * d + e * e) + f * f;
    return 1.5 * (nrm + 2.0 * sh);
}

// Histogram of the von Mises stress of a stress field [6][nvox] against
// squared bin edges q[0..nbins] (non-decreasing; -1 for edges <= 0): with
// j the largest index such that q[j] <= sigma_eq^2, counts[0] if there is
// none, counts[1 + j] for j < nbins, counts[nbins + 1] for j = nbins or a
// non-finite value.  Comparing squares keeps square roots (not correctly
// rounded on the device) out of the decision.  Block-local counts in LDS,
// added to the device counts at the end (integer atomics: the result does
// not depend on the order).
template <typename R>
__global__ __launch_bounds__(256) void k_seq_hist(const R *__restrict__ sig, long nvox, int nbins,
                                                  const double *__restrict__ qedge, unsigned long long *counts)
{
    extern __shared__ double lds_q[];
    unsigned int *hist = reinterpret_cast<unsigned int *>(lds_q + nbins + 1);
    const int nb = nbins + 2;
    for (int i = threadIdx.x; i <= nbins; i += blockDim.x) lds_q[i] = qedge[i];
    for (int i = threadIdx.x; i < nb; i += blockDim.x) hist[i] = 0u;
    __syncthreads();
    for (long vox = (long)blockIdx.x * blockDim.x + threadIdx.x; vox < nvox; vox += (long)gridDim.x * blockDim.x) {
        R sl[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) sl[c] = sig[c * nvox + vox];
        const double x = von_mises_sq_exact<R>(sl);
        int k;
        if (!(x == x) || x == INFINITY) {
            k = nbins + 1;
        } else {
            // largest j with lds_q[j] <= x, -1 if none
            int a = -1, b = nbins;
            while (a < b) {
                const int mid = (a + b + 1) >> 1;
                if (lds_q[mid] <= x) a = mid;
                else b = mid - 1;
            }
            k = a + 1;
        }
        atomicAdd(&hist[k], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nb; i += blockDim.x)
        if (hist[i]) atomicAdd(&counts[i], (unsigned long long)hist[i]);
}

// substep counts of the current load step as field values (M 2^j)
template <typename R>
__global__ __launch_bounds__(256) void k_substeps_field(const int32_t *mv, const Scalars *sc, R *out, long nvox,
                                                        int adaptive)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nvox) out[i] = R(adaptive ? sc->M << mv[i] : sc->M);
}

template <typename R>
__global__ void k_fill(R *p, long n, R v)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        p[i] = v;
}

}  // namespace cpf

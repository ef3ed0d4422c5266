// Device building blocks for the gfx950 solver: complex arithmetic, an
// LDS-resident mixed-radix (2,3,4,8) Stockham FFT, the regularized
// Meric-Cailletaud rate with RK4 substepping, and FP64 block reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cpf {

constexpr int NSMAX = 32;    // systems per crystal
constexpr int MAXPASS = 12;  // radix passes per 1D transform
constexpr int NPX = 11;      // per-block FP64 sums of the x pass

template <typename R>
struct alignas(2 * sizeof(R)) C2 {
    R x, y;
};

template <typename R>
__device__ __forceinline__ C2<R> cadd(C2<R> a, C2<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ C2<R> csub(C2<R> a, C2<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ C2<R> cmul(C2<R> a, C2<R> b)
{
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// multiply by -i (forward sign) or +i (inverse sign)
template <typename R, bool INV>
__device__ __forceinline__ C2<R> rot90(C2<R> a)
{
    return INV ? C2<R>{-a.y, a.x} : C2<R>{a.y, -a.x};
}

// Exact quotients by a multiply-high: for 0 <= n < 2^16 and 2 <= d < 2^16,
// floor(n / d) = (n M) >> 32 with M = ceil(2^32 / d) (the rounding error
// n (M d - 2^32) / (d 2^32) stays below 1/d).  M = 0 stands for d = 1.
__host__ __device__ __forceinline__ unsigned fdiv_magic(unsigned d) { return d <= 1u ? 0u : 0xFFFFFFFFu / d + 1u; }
__device__ __forceinline__ unsigned fdiv(unsigned n, unsigned M) { return M ? __umulhi(n, M) : n; }

struct FftPlan {
    int n;
    int npass;
    int radix[MAXPASS];
    unsigned mag_m[MAXPASS];   // fdiv_magic(n / radix[p])
    unsigned mag_ns[MAXPASS];  // fdiv_magic(product of the radices before pass p)
};

// ---------------------------------------------------------------------------
// Small DFTs.  Forward uses exp(-2 pi i pq / r), inverse exp(+2 pi i pq / r).
// ---------------------------------------------------------------------------
template <typename R, bool INV>
__device__ __forceinline__ void dft2(C2<R> *v)
{
    C2<R> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <typename R, bool INV>
__device__ __forceinline__ void dft3(C2<R> *v)
{
    const R h = R(0.5), s3 = R(0.866025403784438646763723170752936183);
    C2<R> a = v[0], bc = cadd(v[1], v[2]), d = csub(v[1], v[2]);
    C2<R> t = {a.x - h * bc.x, a.y - h * bc.y};
    C2<R> s = {s3 * d.x, s3 * d.y};
    v[0] = cadd(a, bc);
    C2<R> ms = rot90<R, INV>(s);  // -i s (forward) / +i s (inverse)
    v[1] = cadd(t, ms);
    v[2] = csub(t, ms);
}

template <typename R, bool INV>
__device__ __forceinline__ void dft4(C2<R> *v)
{
    C2<R> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    C2<R> t2 = cadd(v[1], v[3]), t3 = rot90<R, INV>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
}

template <typename R, bool INV>
__device__ __forceinline__ void dft8(C2<R> *v)
{
    const R c = R(0.707106781186547524400844362104849039);
    C2<R> e[4] = {v[0], v[2], v[4], v[6]};
    C2<R> o[4] = {v[1], v[3], v[5], v[7]};
    dft4<R, INV>(e);
    dft4<R, INV>(o);
    // o[p] *= w8^p (forward w8 = exp(-i pi/4); inverse: conjugate)
    C2<R> o1 = INV ? C2<R>{c * (o[1].x - o[1].y), c * (o[1].x + o[1].y)}
                   : C2<R>{c * (o[1].x + o[1].y), c * (o[1].y - o[1].x)};
    C2<R> o2 = rot90<R, INV>(o[2]);
    C2<R> o3 = INV ? C2<R>{-c * (o[3].x + o[3].y), c * (o[3].x - o[3].y)}
                   : C2<R>{c * (o[3].y - o[3].x), -c * (o[3].x + o[3].y)};
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
}

// 16 points as 4 x 4: 4-point DFTs over the four stride-4 subsequences,
// twiddles exp(-+2 pi i n2 k1 / 16), 4-point DFTs across them.
template <typename R, bool INV>
__device__ __forceinline__ void dft16(C2<R> *v)
{
    // cos and sin of 2 pi p / 16, p = 0..9
    constexpr double C[10] = {1.0, 0.923879532511286756, 0.707106781186547524, 0.382683432365089772, 0.0,
                              -0.382683432365089772, -0.707106781186547524, -0.923879532511286756, -1.0,
                              -0.923879532511286756};
    constexpr double S[10] = {0.0, 0.382683432365089772, 0.707106781186547524, 0.923879532511286756, 1.0,
                              0.923879532511286756, 0.707106781186547524, 0.382683432365089772, 0.0,
                              -0.382683432365089772};
    C2<R> a[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
        for (int n1 = 0; n1 < 4; ++n1) a[n2][n1] = v[4 * n1 + n2];
        dft4<R, INV>(a[n2]);
    }
#pragma unroll
    for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
        for (int k1 = 1; k1 < 4; ++k1) {
            const int p = n2 * k1;
            const C2<R> w = {R(C[p]), INV ? R(S[p]) : R(-S[p])};
            a[n2][k1] = cmul(a[n2][k1], w);
        }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        C2<R> b[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
        dft4<R, INV>(b);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = b[k2];
    }
}

template <typename R, bool INV, int RAD>
__device__ __forceinline__ void dft(C2<R> *v)
{
    if constexpr (RAD == 2) dft2<R, INV>(v);
    else if constexpr (RAD == 3) dft3<R, INV>(v);
    else if constexpr (RAD == 4) dft4<R, INV>(v);
    else if constexpr (RAD == 8) dft8<R, INV>(v);
    else dft16<R, INV>(v);
}

// ---------------------------------------------------------------------------
// One Stockham pass over `nlines` transforms of length N held in LDS (line
// stride ls).  Every thread first pulls all inputs of its butterflies into
// registers, the block synchronizes, then the results are written back in
// place at their autosorted positions.  MAXB bounds the butterflies per
// thread: nlines*N/RAD <= MAXB*nthr must hold.
// tw[k] = exp(-2 pi i k / N).
// ---------------------------------------------------------------------------
template <typename R, bool INV, int RAD, int MAXB>
__device__ __forceinline__ void fft_pass(C2<R> *buf, int nlines, int ls, int N, int Ns, unsigned mag_m,
                                         unsigned mag_ns, const C2<R> *__restrict__ tw, int tid, int nthr)
{
    const int m = N / RAD;
    const int nb = nlines * m;
    const int tstride = N / (Ns * RAD);
    C2<R> v[MAXB][RAD];
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        const int i = tid + b * nthr;
        if (i < nb) {
            const int line = (int)fdiv((unsigned)i, mag_m), j = i - line * m;
            const C2<R> *src = buf + line * ls + j;
#pragma unroll
            for (int q = 0; q < RAD; ++q) v[b][q] = src[q * m];
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        const int i = tid + b * nthr;
        if (i < nb) {
            const int line = (int)fdiv((unsigned)i, mag_m), j = i - line * m;
            const int k = j - (int)fdiv((unsigned)j, mag_ns) * Ns;
            if (k) {
#pragma unroll
                for (int q = 1; q < RAD; ++q) {
                    C2<R> w = tw[q * k * tstride];
                    if (INV) w.y = -w.y;
                    v[b][q] = cmul(v[b][q], w);
                }
            }
            dft<R, INV, RAD>(v[b]);
            C2<R> *dst = buf + line * ls + (j - k) * RAD + k;
#pragma unroll
            for (int q = 0; q < RAD; ++q) dst[q * Ns] = v[b][q];
        }
    }
    __syncthreads();
}

// Full 1D transforms of nlines sequences in LDS.  EPT bounds the elements
// per thread: nlines*N <= EPT*nthr.  Must be called by every thread of the
// block (it synchronizes).
template <typename R, bool INV, int EPT>
__device__ void lds_fft(C2<R> *buf, int nlines, int ls, const FftPlan &P,
                        const C2<R> *__restrict__ tw, int tid, int nthr)
{
    int Ns = 1;
    for (int p = 0; p < P.npass; ++p) {
        const int r = P.radix[p];
        const unsigned mm = P.mag_m[p], mn = P.mag_ns[p];
        if (r == 8)
            fft_pass<R, INV, 8, (EPT + 7) / 8>(buf, nlines, ls, P.n, Ns, mm, mn, tw, tid, nthr);
        else if (r == 4)
            fft_pass<R, INV, 4, (EPT + 3) / 4>(buf, nlines, ls, P.n, Ns, mm, mn, tw, tid, nthr);
        else if (r == 3)
            fft_pass<R, INV, 3, (EPT + 2) / 3>(buf, nlines, ls, P.n, Ns, mm, mn, tw, tid, nthr);
        else
            fft_pass<R, INV, 2, (EPT + 1) / 2>(buf, nlines, ls, P.n, Ns, mm, mn, tw, tid, nthr);
        Ns *= r;
    }
}

// ---------------------------------------------------------------------------
// Transforms of nl lines of length N whose lines are adjacent and whose
// elements are strided: LDS word buf[e * es + l] holds element e of line l.
// Butterfly b of a pass takes line l = b mod nl and index j = b div nl, so
// the lanes of a wave touch adjacent lines at the same element: adjacent
// LDS words, and in global memory adjacent columns of one row (the y and z
// passes' lines are the kx columns of a tile).  The first pass can read
// its inputs straight from global memory and the last can write its
// outputs there, so a tile is never staged through LDS on the way in or
// out: LDS sees the middle passes only.  In global memory element e of
// line l is gline(l)[e * gs] (gs uniform).
// ---------------------------------------------------------------------------
// Loads and stores of one complex value that the compiler may issue as
// global-memory instructions (the pointers come from device tables, where
// their address space is not known to it).
template <typename R>
__device__ __forceinline__ C2<R> gload(const C2<R> *p)
{
    typedef R v2 __attribute__((ext_vector_type(2)));
    const v2 t = *(const __attribute__((address_space(1))) v2 *)p;
    return {t.x, t.y};
}
template <typename R>
__device__ __forceinline__ void gstore(C2<R> *p, C2<R> v)
{
    typedef R v2 __attribute__((ext_vector_type(2)));
    const v2 t = {v.x, v.y};
    *(__attribute__((address_space(1))) v2 *)p = t;
}

// Twiddle and butterfly of one radix-RAD butterfly with index j.
template <typename R, bool INV, int RAD>
__device__ __forceinline__ void strided_bfly(C2<R> (&v)[RAD], int k, int tstride, const C2<R> *__restrict__ tw)
{
    if (k) {
#pragma unroll
        for (int q = 1; q < RAD; ++q) {
            C2<R> w = tw[q * k * tstride];
            if (INV) w.y = -w.y;
            v[q] = cmul(v[q], w);
        }
    }
    dft<R, INV, RAD>(v);
}

template <typename R, bool INV, int RAD, int MAXB, bool SRC_G, bool DST_G, class GL>
__device__ __forceinline__ void strided_pass(C2<R> *buf, int es, int nl, unsigned mag_nl, int N, int Ns,
                                             unsigned mag_ns, const C2<R> *__restrict__ tw, int tid, int nthr,
                                             const GL &gline, long gs)
{
    const int m = N / RAD;
    const int nb = nl * m;
    const int tstride = N / (Ns * RAD);
    if constexpr (SRC_G || DST_G) {
        // reads and writes go to different memories: one butterfly at a
        // time (its RAD loads in flight together)
        const long gq = (long)m * gs;   // global step between the inputs of a butterfly
        for (int i = tid; i < nb; i += nthr) {
            const int j = (int)fdiv((unsigned)i, mag_nl), l = i - j * nl;
            const int k = j - (int)fdiv((unsigned)j, mag_ns) * Ns;
            C2<R> v[RAD];
            if constexpr (SRC_G) {
                const C2<R> *src = gline(l) + j * gs;
#pragma unroll
                for (int q = 0; q < RAD; ++q) v[q] = gload(src + q * gq);
            } else {
                const C2<R> *src = buf + j * es + l;
#pragma unroll
                for (int q = 0; q < RAD; ++q) v[q] = src[q * m * es];
            }
            strided_bfly<R, INV, RAD>(v, k, tstride, tw);
            const int o = (j - k) * RAD + k;
            if constexpr (DST_G) {
                C2<R> *dst = gline(l) + o * gs;
#pragma unroll
                for (int q = 0; q < RAD; ++q) gstore(dst + (long)q * Ns * gs, v[q]);
            } else {
                C2<R> *dst = buf + o * es + l;
#pragma unroll
                for (int q = 0; q < RAD; ++q) dst[q * Ns * es] = v[q];
            }
        }
        if constexpr (!DST_G) __syncthreads();
    } else {
        // in place in LDS: every read before any write
        C2<R> v[MAXB][RAD];
#pragma unroll
        for (int b = 0; b < MAXB; ++b) {
            const int i = tid + b * nthr;
            if (i < nb) {
                const int j = (int)fdiv((unsigned)i, mag_nl), l = i - j * nl;
                const C2<R> *src = buf + j * es + l;
#pragma unroll
                for (int q = 0; q < RAD; ++q) v[b][q] = src[q * m * es];
            }
        }
        __syncthreads();
#pragma unroll
        for (int b = 0; b < MAXB; ++b) {
            const int i = tid + b * nthr;
            if (i < nb) {
                const int j = (int)fdiv((unsigned)i, mag_nl), l = i - j * nl;
                const int k = j - (int)fdiv((unsigned)j, mag_ns) * Ns;
                strided_bfly<R, INV, RAD>(v[b], k, tstride, tw);
                C2<R> *dst = buf + ((j - k) * RAD + k) * es + l;
#pragma unroll
                for (int q = 0; q < RAD; ++q) dst[q * Ns * es] = v[b][q];
            }
        }
        __syncthreads();
    }
}

template <typename R, bool INV, int RAD, int MAXB, class GL>
__device__ __forceinline__ void strided_pass_any(bool src_g, bool dst_g, C2<R> *buf, int es, int nl,
                                                 unsigned mag_nl, int N, int Ns, unsigned mag_ns,
                                                 const C2<R> *__restrict__ tw, int tid, int nthr, const GL &gline,
                                                 long gs)
{
    if (src_g && dst_g)
        strided_pass<R, INV, RAD, MAXB, true, true>(buf, es, nl, mag_nl, N, Ns, mag_ns, tw, tid, nthr, gline, gs);
    else if (src_g)
        strided_pass<R, INV, RAD, MAXB, true, false>(buf, es, nl, mag_nl, N, Ns, mag_ns, tw, tid, nthr, gline, gs);
    else if (dst_g)
        strided_pass<R, INV, RAD, MAXB, false, true>(buf, es, nl, mag_nl, N, Ns, mag_ns, tw, tid, nthr, gline, gs);
    else
        strided_pass<R, INV, RAD, MAXB, false, false>(buf, es, nl, mag_nl, N, Ns, mag_ns, tw, tid, nthr, gline,
                                                      gs);
}

// Whole transforms of the nl lines.  FROM_G: the input is in global memory
// (else in LDS); TO_G: the output goes to global memory (else stays in
// LDS, with the block synchronized).  EPT bounds the elements per thread:
// nl * N <= EPT * nthr.  Twiddles tw[k] = exp(-2 pi i k / N) must be
// readable by the second pass (the first uses none).  Called by every
// thread of the block.
template <typename R, bool INV, int EPT, bool FROM_G, bool TO_G, class GL>
__device__ void strided_fft(C2<R> *buf, int es, int nl, const FftPlan &P, const C2<R> *__restrict__ tw, int tid,
                            int nthr, const GL &gline, long gs)
{
    const unsigned mag_nl = fdiv_magic((unsigned)nl);
    int Ns = 1;
    for (int p = 0; p < P.npass; ++p) {
        const int r = P.radix[p];
        const unsigned mn = P.mag_ns[p];
        const bool sg = FROM_G && p == 0, dg = TO_G && p == P.npass - 1;
        if (r == 8)
            strided_pass_any<R, INV, 8, (EPT + 7) / 8>(sg, dg, buf, es, nl, mag_nl, P.n, Ns, mn, tw, tid, nthr,
                                                       gline, gs);
        else if (r == 4)
            strided_pass_any<R, INV, 4, (EPT + 3) / 4>(sg, dg, buf, es, nl, mag_nl, P.n, Ns, mn, tw, tid, nthr,
                                                       gline, gs);
        else if (r == 3)
            strided_pass_any<R, INV, 3, (EPT + 2) / 3>(sg, dg, buf, es, nl, mag_nl, P.n, Ns, mn, tw, tid, nthr,
                                                       gline, gs);
        else
            strided_pass_any<R, INV, 2, (EPT + 1) / 2>(sg, dg, buf, es, nl, mag_nl, P.n, Ns, mn, tw, tid, nthr,
                                                       gline, gs);
        Ns *= r;
    }
}

// ---------------------------------------------------------------------------
// The same line transforms for lengths known at compile time (the common
// grid sizes): a fixed radix plan of two or three passes, all index
// arithmetic by constants, NL lines and NT threads fixed.  nlv <= NL lines
// hold data (a narrower last tile); the others are never read from or
// written to global memory.
// ---------------------------------------------------------------------------
template <int N> struct FixedPlan { static constexpr int np = 0, r0 = 1, r1 = 1, r2 = 1; };
template <> struct FixedPlan<32> { static constexpr int np = 2, r0 = 8, r1 = 4, r2 = 1; };
template <> struct FixedPlan<48> { static constexpr int np = 2, r0 = 16, r1 = 3, r2 = 1; };
template <> struct FixedPlan<64> { static constexpr int np = 2, r0 = 8, r1 = 8, r2 = 1; };
template <> struct FixedPlan<96> { static constexpr int np = 3, r0 = 8, r1 = 4, r2 = 3; };
template <> struct FixedPlan<128> { static constexpr int np = 2, r0 = 8, r1 = 16, r2 = 1; };
template <> struct FixedPlan<256> { static constexpr int np = 2, r0 = 16, r1 = 16, r2 = 1; };

struct NoHook {
    __device__ void operator()() const {}
};

// hook: run by every thread after its butterflies and before the closing
// barrier of the pass (the first pass stages the twiddles there, so their
// load overlaps the tile's)
template <typename R, bool INV, int N, int NL, int NT, int RAD, int NS, bool SRC_G, bool DST_G, class GL,
          class HK = NoHook>
__device__ __forceinline__ void fixed_pass(C2<R> *buf, int nlv, const C2<R> *__restrict__ tw, const GL &gline,
                                           long gs, const HK &hook = HK())
{
    constexpr int m = N / RAD, nb = NL * m, TS = N / (NS * RAD);
    constexpr int ITER = (nb + NT - 1) / NT;
    const int tid = threadIdx.x;
    if constexpr (SRC_G || DST_G) {
#pragma unroll
        for (int it = 0; it < ITER; ++it) {
            const int i = tid + it * NT;
            if (nb % NT == 0 || i < nb) {
                const int j = i / NL, l = i - j * NL;
                const int k = NS > 1 ? j % NS : 0;
                C2<R> v[RAD];
                if constexpr (SRC_G) {
                    if (l < nlv) {
                        const C2<R> *src = gline(l) + j * gs;
#pragma unroll
                        for (int q = 0; q < RAD; ++q) v[q] = gload(src + (long)q * m * gs);
                    } else {
#pragma unroll
                        for (int q = 0; q < RAD; ++q) v[q] = C2<R>{R(0), R(0)};
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < RAD; ++q) v[q] = buf[(j + q * m) * NL + l];
                }
                if constexpr (NS > 1) {
                    if (k) {
#pragma unroll
                        for (int q = 1; q < RAD; ++q) {
                            C2<R> w = tw[q * k * TS];
                            if (INV) w.y = -w.y;
                            v[q] = cmul(v[q], w);
                        }
                    }
                }
                dft<R, INV, RAD>(v);
                const int o = (j - k) * RAD + k;
                if constexpr (DST_G) {
                    if (l < nlv) {
                        C2<R> *dst = gline(l) + o * gs;
#pragma unroll
                        for (int q = 0; q < RAD; ++q) gstore(dst + (long)q * NS * gs, v[q]);
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < RAD; ++q) buf[(o + q * NS) * NL + l] = v[q];
                }
            }
        }
        hook();
        if constexpr (!DST_G) __syncthreads();
    } else {
        C2<R> v[ITER][RAD];
#pragma unroll
        for (int it = 0; it < ITER; ++it) {
            const int i = tid + it * NT;
            if (nb % NT == 0 || i < nb) {
                const int j = i / NL, l = i - j * NL;
#pragma unroll
                for (int q = 0; q < RAD; ++q) v[it][q] = buf[(j + q * m) * NL + l];
            }
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < ITER; ++it) {
            const int i = tid + it * NT;
            if (nb % NT == 0 || i < nb) {
                const int j = i / NL, l = i - j * NL;
                const int k = j % NS;
                if (k) {
#pragma unroll
                    for (int q = 1; q < RAD; ++q) {
                        C2<R> w = tw[q * k * TS];
                        if (INV) w.y = -w.y;
                        v[it][q] = cmul(v[it][q], w);
                    }
                }
                dft<R, INV, RAD>(v[it]);
                const int o = (j - k) * RAD + k;
#pragma unroll
                for (int q = 0; q < RAD; ++q) buf[(o + q * NS) * NL + l] = v[it][q];
            }
        }
        __syncthreads();
    }
}

// Whole transforms with the plan of N (FixedPlan<N>::np > 0); FROM_G, TO_G
// and the twiddle table as for strided_fft; the LDS buffer is [N][NL].
// hook: run inside the first pass before its barrier (staging the
// twiddles that the later passes read).
template <typename R, bool INV, int N, int NL, int NT, bool FROM_G, bool TO_G, class GL, class HK = NoHook>
__device__ __forceinline__ void fixed_fft(C2<R> *buf, int nlv, const C2<R> *__restrict__ tw, const GL &gline,
                                          long gs, const HK &hook = HK())
{
    using P = FixedPlan<N>;
    static_assert(P::np >= 2, "no fixed plan for this length");
    fixed_pass<R, INV, N, NL, NT, P::r0, 1, FROM_G, false>(buf, nlv, tw, gline, gs, hook);
    if constexpr (P::np == 2) {
        fixed_pass<R, INV, N, NL, NT, P::r1, P::r0, false, TO_G>(buf, nlv, tw, gline, gs);
    } else {
        fixed_pass<R, INV, N, NL, NT, P::r1, P::r0, false, false>(buf, nlv, tw, gline, gs);
        fixed_pass<R, INV, N, NL, NT, P::r2, P::r0 * P::r1, false, TO_G>(buf, nlv, tw, gline, gs);
    }
}

// ---------------------------------------------------------------------------
// FP64 block reductions (deterministic: fixed shuffle tree, then fixed
// order over waves).  Block size <= 1024, wave64.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// MAXW: most waves per block (16 for 1024 threads).
template <int NV, int MAXW = 16>
__device__ void block_sum(double (&v)[NV], double *out /* NV values, thread 0 */)
{
    __shared__ double red[MAXW][NV];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < NV; ++i) red[wid][i] = v[i];
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += red[w][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// ---------------------------------------------------------------------------
// Symmetric tensors as tensor components (11,22,33,23,13,12).
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void sym_full(const R a[6], R A[3][3])
{
    A[0][0] = a[0]; A[1][1] = a[1]; A[2][2] = a[2];
    A[1][2] = A[2][1] = a[3];
    A[0][2] = A[2][0] = a[4];
    A[0][1] = A[1][0] = a[5];
}

// out = Q^T a Q  (lab -> crystal when v_lab = Q v_crystal)
template <typename R>
__device__ __forceinline__ void rot_to_crystal(const R Q[9], const R a[6], R out[6])
{
    R A[3][3], T[3][3];
    sym_full(a, A);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            T[i][j] = A[i][0] * Q[0 * 3 + j] + A[i][1] * Q[1 * 3 + j] + A[i][2] * Q[2 * 3 + j];
    // out_ij = sum_k Q_ki T_kj
    const int I[6] = {0, 1, 2, 1, 0, 0}, J[6] = {0, 1, 2, 2, 2, 1};
#pragma unroll
    for (int c = 0; c < 6; ++c)
        out[c] = Q[0 * 3 + I[c]] * T[0][J[c]] + Q[1 * 3 + I[c]] * T[1][J[c]] +
                 Q[2 * 3 + I[c]] * T[2][J[c]];
}

// out = Q a Q^T  (crystal -> lab)
template <typename R>
__device__ __forceinline__ void rot_to_lab(const R Q[9], const R a[6], R out[6])
{
    R A[3][3], T[3][3];
    sym_full(a, A);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            T[i][j] = A[i][0] * Q[j * 3 + 0] + A[i][1] * Q[j * 3 + 1] + A[i][2] * Q[j * 3 + 2];
    // out_ij = sum_k Q_ik T_kj
    const int I[6] = {0, 1, 2, 1, 0, 0}, J[6] = {0, 1, 2, 2, 2, 1};
#pragma unroll
    for (int c = 0; c < 6; ++c)
        out[c] = Q[I[c] * 3 + 0] * T[0][J[c]] + Q[I[c] * 3 + 1] * T[1][J[c]] +
                 Q[I[c] * 3 + 2] * T[2][J[c]];
}

template <typename R>
__device__ __forceinline__ R von_mises(const R s[6])
{
    const R p = (s[0] + s[1] + s[2]) * R(1.0 / 3.0);
    const R a = s[0] - p, b = s[1] - p, c = s[2] - p;
    return sqrt(R(1.5) * (a * a + b * b + c * c + R(2) * (s[3] * s[3] + s[4] * s[4] + s[5] * s[5])));
}

// ---------------------------------------------------------------------------
// Law parameters, crystal frame (uniform over the grid: kernel arguments).
// Per-family values are separate scalar fields so that the family of a
// system (a uniform bit) selects them without indexing into the argument
// block.
// ---------------------------------------------------------------------------
template <typename R>
struct FamP {
    R QL;      // Q * q_latent
    R QD;      // Q * (q_self - q_latent)
    R bl2e;    // b * log2(e)
    R c, d;    // kinematic hardening
    R K, invK, n, inv_n, nm1;
    int nm1_int;   // n - 1 when n is an integer in [1, 64], else -1
    R Q, b, qs, ql;   // raw values for the reverse mode
};

template <typename R>
struct LawP {
    int nsys;
    int twin_mode;        // 0 Norton, 1 paper twin-fraction law
    uint32_t twin_mask;   // bit s set: system s is a twin system
    R C[36];              // sigma_I = sum_J C[I][J] eps_J on tensor components
    R m[NSMAX][6];        // Schmid tensors, tensor components
    R tau0[NSMAX];
    FamP<R> fs, ft;       // slip, twin
    R Kc_gT, fm, inv_gT, eta, inv_eta;
    R newton_rtol;
    int nm1_uni;          // n - 1 when every family present has the same integer
                          // n in [1, 64] (a wave-uniform exponent), else -1
    R tau0k[3];           // FP32 LAW_TABLE1: initial resistance per kind of
                          // Table 1 system (ordinary, superdislocation, twin)
};

// Math in the working precision.  FP32 uses the hardware transcendental
// instructions directly (v_exp_f32, v_log_f32, v_rcp_f32: about 1 ulp;
// results below the normal range flush to zero, which the law never needs).
__device__ __forceinline__ float lg2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ double lg2(double x) { return log2(x); }
__device__ __forceinline__ float ex2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ double ex2(double x) { return exp2(x); }
__device__ __forceinline__ float fdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double fdiv(double a, double b) { return a / b; }
// Reciprocal for the Newton step, where the last ulp does not matter: the
// hardware estimate refined by two Newton-Raphson steps in FP64 (error
// below an ulp or two) instead of the correctly rounded division sequence;
// in FP32 the hardware reciprocal as in fdiv.
__device__ __forceinline__ float rcp_nr(float b) { return __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double rcp_nr(double b)
{
    double r = __builtin_amdgcn_rcp(b);
    double e = fma(-b, r, 1.0);
    r = fma(r, e, r);
    e = fma(-b, r, 1.0);
    return fma(r, e, r);
}

// y^p for an integer 0 <= p < 64 that is uniform across the wave: six
// squarings with the multiplications selected by scalar branches.
template <typename R>
__device__ __forceinline__ R powi(R y, int p)
{
    R r = R(1), b = y;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        if (p & (1 << k)) r *= b;
        b *= b;
    }
    return r;
}

// y^p for an integer 0 <= p < 64 held in a scalar register (the same in
// every lane): the squarings stop at the highest set bit, so y^9 is three
// squarings and one product.  The products are those of powi in the same
// order (the same rounding).
template <typename R>
__device__ __forceinline__ R powu(R y, int p)
{
    R r = (p & 1) ? y : R(1);
    R b = y;
#pragma unroll
    for (int k = 1; k < 6; ++k) {
        if ((p >> k) == 0) break;
        b *= b;
        if ((p >> k) & 1) r *= b;
    }
    return r;
}

// y^(n-1) in the working precision.  FP32: the hardware exp2/log2 (a
// measured 5 % faster x pass than products under scalar branches).  FP64:
// with an exponent shared by every family (nm1_uni >= 0, a kernel
// argument) the products of powu under scalar branches, else repeated
// squaring when this family's n is an integer (per-lane branches), else
// the software exp2/log2.
template <typename R>
__device__ __forceinline__ R pow_nm1(R y, R nm1, int nm1_int, int nm1_uni)
{
    if constexpr (sizeof(R) == 4) {
        return ex2(nm1 * lg2(y));
    } else {
        if (nm1_uni >= 0) return powu(y, nm1_uni);
        return nm1_int >= 0 ? powi(y, nm1_int) : ex2(nm1 * lg2(y));
    }
}

// Schmid tensors of the paper's system set (Table 1; system 9 read with
// direction [110]): m = (n (x) l + l (x) n)/2 of the unit plane normal and
// direction, tensor components (11,22,33,23,13,12).  Systems 1-12 are slip
// (entries +-1/sqrt6, +-1/(2 sqrt6)), 13-16 twinning.
constexpr double T1_M[16][6] = {
    {0.0, 0.40824829046386302, -0.40824829046386302, 0.0, 0.20412414523193151, 0.20412414523193151},
    {0.40824829046386302, 0.0, -0.40824829046386302, 0.20412414523193151, 0.0, 0.20412414523193151},
    {0.40824829046386302, -0.40824829046386302, 0.0, 0.20412414523193151, -0.20412414523193151, 0.0},
    {0.0, -0.40824829046386302, 0.40824829046386302, 0.0, -0.20412414523193151, 0.20412414523193151},
    {0.40824829046386302, 0.0, -0.40824829046386302, -0.20412414523193151, 0.0, -0.20412414523193151},
    {0.40824829046386302, -0.40824829046386302, 0.0, -0.20412414523193151, -0.20412414523193151, 0.0},
    {0.0, -0.40824829046386302, 0.40824829046386302, 0.0, 0.20412414523193151, 0.20412414523193151},
    {0.40824829046386302, 0.0, -0.40824829046386302, 0.20412414523193151, 0.0, -0.20412414523193151},
    {0.40824829046386302, -0.40824829046386302, 0.0, 0.20412414523193151, 0.20412414523193151, 0.0},
    {0.0, 0.40824829046386302, -0.40824829046386302, 0.0, -0.20412414523193151, 0.20412414523193151},
    {0.40824829046386302, 0.0, -0.40824829046386302, -0.20412414523193151, 0.0, 0.20412414523193151},
    {0.40824829046386302, -0.40824829046386302, 0.0, -0.20412414523193151, 0.20412414523193151, 0.0},
    {0.23570226039551589, 0.23570226039551589, -0.47140452079103179, 0.11785113019775795,
     0.11785113019775795, 0.23570226039551589},
    {0.23570226039551589, 0.23570226039551589, -0.47140452079103179, -0.11785113019775795,
     0.11785113019775795, -0.23570226039551589},
    {0.23570226039551589, 0.23570226039551589, -0.47140452079103179, 0.11785113019775795,
     -0.11785113019775795, -0.23570226039551589},
    {0.23570226039551589, 0.23570226039551589, -0.47140452079103179, -0.11785113019775795,
     -0.11785113019775795, 0.23570226039551589},
};

// Kind of each Table 1 system: 0 ordinary dislocation, 1 superdislocation,
// 2 twin (the table's last column).  The FP32 Table 1 specialization takes
// one initial resistance per kind (LawP::tau0k): three scalar registers in
// place of sixteen, which otherwise are spilled to vector lanes and read
// back at every RK stage (FP64 reads its resistances from LDS).
constexpr int T1_KIND[16] = {1, 1, 0, 1, 1, 0, 1, 1, 0, 1, 1, 0, 2, 2, 2, 2};

// Kernel specializations of the law:
//   LAW_GENERAL : any systems (Schmid tensors and stiffness from the arguments)
//   LAW_TABLE1  : the Table 1 systems in order (12 slip, optionally + 4 twin)
//                 with one initial resistance per kind of system, and a
//                 crystal stiffness with orthotropic zero pattern (cubic,
//                 tetragonal): compile-time Schmid tensors, 12-term Hooke
constexpr int LAW_GENERAL = 0;
constexpr int LAW_TABLE1 = 1;

template <typename R, int SPEC>
__device__ __forceinline__ R schmid(const R (&m)[NSMAX][6], int s, int i)
{
    if constexpr (SPEC == LAW_TABLE1) return R(T1_M[s][i]);
    else return m[s][i];
}

template <int SPEC>
__device__ __forceinline__ bool schmid_nonzero(int s, int i)
{
    if constexpr (SPEC == LAW_TABLE1) return T1_M[s][i] != 0.0;
    else return true;
}

// Family of system s: known at compile time for the Table 1 set (systems
// 13-16 are the twins), from the mask otherwise.
template <int SPEC, typename R>
__device__ __forceinline__ bool is_twin(const LawP<R> &P, int s)
{
    if constexpr (SPEC == LAW_TABLE1) return s >= 12;
    else return (P.twin_mask >> s) & 1u;
}

// Factored Schmid contractions of the Table 1 set.  Every slip tensor has
// one diagonal entry +-A and one -+A (A = 1/sqrt6) and two shear entries
// +-A/2; every twin tensor has the diagonal (B, B, -2B) (B = 1/sqrt18) and
// the shear entries (+-B/2, +-B/2, +-B).  With sa = A sigma, a resolved
// shear stress is then a signed diagonal difference of sa plus two signed
// shear components (slip), or (B/A) times d02 + d12 plus three signed terms
// (twin); the plastic strain rate collects signed sums of the rates per
// pattern before one multiplication.  Only the rounding order differs
// from the plain contraction.
constexpr double T1_A = 0.40824829046386302;
constexpr double T1_B = 0.23570226039551589;
constexpr double T1_BA = T1_B / T1_A;   // 1/sqrt3

constexpr bool t1_pattern_ok()
{
    for (int s = 0; s < 16; ++s) {
        if (s < 12) {
            int np = 0, nn = 0, nsh = 0;
            for (int i = 0; i < 3; ++i) {
                if (T1_M[s][i] == T1_A) ++np;
                else if (T1_M[s][i] == -T1_A) ++nn;
                else if (T1_M[s][i] != 0.0) return false;
            }
            for (int i = 3; i < 6; ++i) {
                if (T1_M[s][i] == T1_A / 2 || T1_M[s][i] == -T1_A / 2) ++nsh;
                else if (T1_M[s][i] != 0.0) return false;
            }
            if (np != 1 || nn != 1 || nsh != 2) return false;
        } else {
            if (T1_M[s][0] != T1_B || T1_M[s][1] != T1_B || T1_M[s][2] != -2 * T1_B) return false;
            for (int i = 3; i < 6; ++i) {
                const double e = i == 5 ? T1_B : T1_B / 2;
                if (T1_M[s][i] != e && T1_M[s][i] != -e) return false;
            }
        }
    }
    return true;
}
static_assert(t1_pattern_ok(), "Table 1 Schmid tensors do not have the factored pattern");

template <int SPEC>
constexpr bool t1_factor()
{
    return SPEC == LAW_TABLE1;
}

// Diagonal pair of slip system s (p < q: 0 = (0,1), 1 = (0,2), 2 = (1,2))
// and the sign of its entry at p.
__host__ __device__ constexpr int t1_pair(int s)
{
    return T1_M[s][2] == 0.0 ? 0 : T1_M[s][1] == 0.0 ? 1 : 2;
}
__host__ __device__ constexpr bool t1_pair_pos(int s)
{
    return T1_M[s][t1_pair(s) == 2 ? 1 : 0] > 0.0;
}

// sa = A sigma, dd = (sa0 - sa1, sa0 - sa2, sa1 - sa2), tT = dd1 + dd2,
// u5 = 2 sa5.
template <typename R>
struct T1Sig {
    R sa[6], dd[3], tT, u5;
};
template <typename R>
__device__ __forceinline__ T1Sig<R> t1_sig(const R sig[6])
{
    T1Sig<R> t;
#pragma unroll
    for (int i = 0; i < 6; ++i) t.sa[i] = R(T1_A) * sig[i];
    t.dd[0] = t.sa[0] - t.sa[1];
    t.dd[1] = t.sa[0] - t.sa[2];
    t.dd[2] = t.sa[1] - t.sa[2];
    t.tT = t.dd[1] + t.dd[2];
    t.u5 = t.sa[5] + t.sa[5];
    return t;
}
template <typename R>
__device__ __forceinline__ R t1_tau(int s, const T1Sig<R> &t)
{
    if (s < 12) {
        const R d = t.dd[t1_pair(s)];
        R x = t1_pair_pos(s) ? d : -d;
#pragma unroll
        for (int i = 3; i < 6; ++i) {
            if (T1_M[s][i] > 0.0) x += t.sa[i];
            else if (T1_M[s][i] < 0.0) x -= t.sa[i];
        }
        return x;
    }
    R x = t.tT;
    x = T1_M[s][3] > 0.0 ? x + t.sa[3] : x - t.sa[3];
    x = T1_M[s][4] > 0.0 ? x + t.sa[4] : x - t.sa[4];
    x = T1_M[s][5] > 0.0 ? x + t.u5 : x - t.u5;
    return R(T1_BA) * x;
}

// Signed rate sums of the factored plastic strain rate.
template <typename R>
struct T1Acc {
    R G[3], Hs[3], W, Ht[3];
};
template <typename R>
__device__ __forceinline__ void t1_acc_init(T1Acc<R> &a)
{
    // -0 is the additive identity: the first sums fold to moves
#pragma unroll
    for (int i = 0; i < 3; ++i) a.G[i] = a.Hs[i] = a.Ht[i] = R(-0.0);
    a.W = R(-0.0);
}
template <typename R>
__device__ __forceinline__ void t1_acc_add(T1Acc<R> &a, int s, R gd)
{
    if (s < 12) {
        const int k = t1_pair(s);
        a.G[k] = t1_pair_pos(s) ? a.G[k] + gd : a.G[k] - gd;
#pragma unroll
        for (int i = 3; i < 6; ++i) {
            if (T1_M[s][i] > 0.0) a.Hs[i - 3] += gd;
            else if (T1_M[s][i] < 0.0) a.Hs[i - 3] -= gd;
        }
    } else {
        a.W += gd;
#pragma unroll
        for (int i = 3; i < 6; ++i) a.Ht[i - 3] = T1_M[s][i] > 0.0 ? a.Ht[i - 3] + gd : a.Ht[i - 3] - gd;
    }
}
// dep = wslip sum_slip gd m + sum_twin gd m
template <typename R>
__device__ __forceinline__ void t1_acc_dep(const T1Acc<R> &a, R wslip, R dep[6])
{
    const R ws = wslip * R(T1_A);
    const R g01 = ws * a.G[0], g02 = ws * a.G[1], g12 = ws * a.G[2];
    const R bw = R(T1_B) * a.W;
    dep[0] = (g01 + g02) + bw;
    dep[1] = (g12 - g01) + bw;
    dep[2] = R(-2) * bw - (g02 + g12);
    const R wh = wslip * R(T1_A / 2);
    dep[3] = wh * a.Hs[0] + R(T1_B / 2) * a.Ht[0];
    dep[4] = wh * a.Hs[1] + R(T1_B / 2) * a.Ht[1];
    dep[5] = wh * a.Hs[2] + R(T1_B) * a.Ht[2];
}

template <typename R, int SPEC>
__device__ __forceinline__ void hooke_c(const R (&C)[36], const R ee[6], R sig[6])
{
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        R s = R(0);
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const bool nz = SPEC == LAW_GENERAL || (i < 3 && j < 3) || i == j;
            if (nz) s += C[i * 6 + j] * ee[j];
        }
        sig[i] = s;
    }
}

// Compiler fence between systems: keeps the per-system law parameters from
// being hoisted (and held in registers) across the whole system loop.
__device__ __forceinline__ void law_fence() { asm volatile("" ::: "memory"); }

// Per-thread LDS work area of a stage: overstress / rate and Newton root
// per system, column of the thread with stride ls.
template <typename R>
struct LawLds {
    R *o;       // [NS] overstress, then rate
    R *y;       // [NS] Newton roots (warm starts)
    R *e;       // [12] start and end strain of the load step
    R *fam;     // [2][LAW_FAM_WORDS] Norton constants of the slip and twin
                // families, one copy per block
    int ls;
    uint16_t *items;   // this wave's Newton items (law_items_q per lane)
    R *aw;             // this wave's twin rate prefactors, one per lane
    R *tau0;           // [NS] initial resistances, one copy per block (FP64)
};

// The Newton solves of a stage are balanced over the lanes of a wave: the
// active systems of all lanes go to a list of 16-bit items (owner lane,
// system, warm-start bit), and the wave's active lanes take the items in
// turn, so a stage needs ceil(items / lanes) passes instead of the largest
// count of one lane.  Up to law_items_q systems of a lane go to the list
// (the rest, rare, are solved by their own lane afterwards).  Per wave:
// the items, then the twin rate prefactor A of each lane (it depends on
// the lane's twin fractions).
template <typename R>
constexpr int law_items_q()
{
    return sizeof(R) == 4 ? 10 : 16;
}
template <typename R>
constexpr size_t law_items_wave_bytes()
{
    return 64 * law_items_q<R>() * 2 + 64 * sizeof(R);
}
// a 256-thread block's item area
template <typename R>
constexpr size_t law_items_bytes()
{
    return 4 * law_items_wave_bytes<R>();
}

// The Newton passes take the constants of each lane's family from a small
// table in LDS instead of selecting every one of them between two scalar
// registers (two instructions each: a scalar source must be moved to a
// vector register first).  Per family: K, 1/K, n, 1/n, n - 1, the integer
// exponent (as a value of R; FP64 only) and two words of padding (16-byte
// aligned rows).  One table per block (64 bytes in FP32): three FP32 law
// blocks per CU leave no room for a table per wave in the 160 KB of LDS.
constexpr int LAW_FAM_WORDS = 8;

// Register relief through the LDS work area: the hardening terms within a
// stage are parked there in FP64 (FP32 keeps them in registers), and the
// strain path of the step in both precisions, except in FP64 beyond 16
// systems, where the x pass's LDS (FFT lines, 2 NS columns, 12 strain
// rows) would exceed the 160 KB a block may use.
template <typename R>
constexpr bool law_park_h()
{
    return sizeof(R) == 8;
}
template <typename R>
constexpr bool law_park_e_ns(int ns)
{
    return !(sizeof(R) == 8 && ns > 16);
}
template <typename R, int NS>
constexpr bool law_park_e()
{
    return law_park_e_ns<R>(NS);
}
template <typename R>
constexpr int law_e_rows(int ns)
{
    return law_park_e_ns<R>(ns) ? 12 : 0;
}

// Bytes of the law's LDS work area of a 256-thread block (2 NS words and the
// strain rows per thread: 44 KB in FP32 at NS = 16), then the family table.
template <typename R>
constexpr size_t law_lds_bytes_ns(int ns)
{
    return ((2 * (size_t)ns + law_e_rows<R>(ns)) * 256 + 2 * LAW_FAM_WORDS + ns) * sizeof(R);
}
template <typename R, int NS>
constexpr size_t law_lds_bytes()
{
    return law_lds_bytes_ns<R>(NS);
}

// Fill the block's family table and, in FP64, its table of initial
// resistances (read from LDS by every system of every stage: held in scalar
// registers next to the FP64 parameters, which take two each, they crowd
// out the rest, which the compiler then parks in vector lanes and reads
// back each stage; 1.7 % of the FP64 x pass, while the FP32 one is 4 %
// faster with the resistances in scalar registers).  Every lane of every
// wave writes the same values before its own first read, so no barrier is
// needed: a read sees either its own wave's write or an identical one.
template <typename R>
constexpr bool law_tau0_lds()
{
    return sizeof(R) == 8;
}
template <typename R, int NS>
__device__ __forceinline__ void law_fam_store(const LawP<R> &P, const LawLds<R> &W)
{
    if constexpr (law_tau0_lds<R>()) {
#pragma unroll
        for (int s = 0; s < NS; ++s) W.tau0[s] = P.tau0[s];
    }
    const FamP<R> *F[2] = {&P.fs, &P.ft};
#pragma unroll
    for (int f = 0; f < 2; ++f) {
        R *t = W.fam + f * LAW_FAM_WORDS;
        t[0] = F[f]->K;
        t[1] = F[f]->invK;
        t[2] = F[f]->n;
        t[3] = F[f]->inv_n;
        t[4] = F[f]->nm1;
        if constexpr (sizeof(R) == 8) t[5] = R(F[f]->nm1_int);
    }
}

// Regularized Norton rate (equations 5/6 with the yield stress raised by
// eta |g|) of one active system: g = A y^n, where y > 0 is the root of
// phi(y) = K y + eta A y^n - o, o > 0.  phi is increasing and convex, so
// Newton converges from any y > 0 and stays above the root after the first
// step.  The iteration starts from the warm start yw (the root found for
// the same system at the previous RK stage, 0 if none), capped by the upper
// bound o/K, or else from the smaller of the two upper bounds o/K and
// (o/(eta A))^(1/n).  With eta > 0 (uniform), A y^n = (o - K y)/eta at the
// root gives g without another power.  A lane stops at |step| <= rtol y or
// after 40 iterations (the loop is not unrolled: an unrolled loop leaves a
// long chain of exec-mask restores at every exit).  yw receives the root.
template <typename R>
__device__ __forceinline__ R newton_solve(R o, R A, R etaA, R inv_etaA, const R *fam, const LawP<R> &P, R &yw,
                                          int &nnewt)
{
    const R K = fam[0], invK = fam[1], n = fam[2], inv_n = fam[3], nm1 = fam[4];
    const int nm1_int = sizeof(R) == 8 ? (int)fam[5] : -1;
    const R yk = o * invK;
    R y = yw > R(0) ? (yw < yk ? yw : yk) : R(0);
    // the cold start only when some lane of the pass has no warm start (a
    // wave vote: most passes are warm after the first stage of a step; the
    // empty asm keeps the block a branch instead of selects after an
    // unconditional log2 and exp2)
    if (__any(!(yw > R(0)))) {
        asm volatile("");
        R yc;
        if constexpr (sizeof(R) == 8) {
            // The start only has to lie above the root: the bound in FP32
            // (hardware log2/exp2, relative error below 1e-6), raised by
            // 1e-5, instead of the FP64 library sequences.  An FP32 overflow
            // gives +inf (start at o/K), an underflow 0 (the first step goes
            // to o/K); both are upper bounds.
            const float q = (float)(o * inv_etaA);
            yc = (double)ex2(lg2(q) * (float)inv_n) * (1.0 + 1e-5);
        } else {
            yc = ex2(lg2(o * inv_etaA) * inv_n);
        }
        if (!(yw > R(0))) y = yk < yc ? yk : yc;
    }
    const R etaAn = etaA * n;
#pragma unroll 1
    for (int it = 0; it < 40; ++it) {
        const R yn1 = pow_nm1(y, nm1, nm1_int, P.nm1_uni);
        const R phi = K * y + etaA * yn1 * y - o;
        const R dphi = K + etaAn * yn1;
        const R step = phi * rcp_nr(dphi);
        y -= step;
        ++nnewt;
        if (fabs(step) <= P.newton_rtol * y) break;
    }
    yw = y;
    if (P.eta > R(0)) return (o - K * y) * P.inv_eta;
    return A * y * pow_nm1(y, nm1, nm1_int, P.nm1_uni);
}

// One RK4 stage of the internal variables in the crystal frame.  Inputs:
// total strain e at the stage time and the stage state t*, overwritten with
// the next stage state y + cnext*k (at the last stage of a substep that
// value is not used: the next substep starts from the accumulated state);
// the stage slope k is accumulated into a* with weight wacc.
// The Newton solves are compacted: the lanes of a wave rarely share their
// active systems (only a third of the systems that some lane needs are
// active in a given lane), so instead of one divergent solve per system,
// every lane takes its own next active system in each pass of the solve
// loop.  Overstresses go to the thread's LDS column, rates and roots come
// back through it; warm holds the systems whose root from the previous
// stage is a valid warm start.
//
// Lagged regularization (LAG): instead of raising the resistance by eta
// times the rate being solved for, each system's resistance is raised by
// a fixed amount for the whole load step, lag.p[s lag.stride] for s <
// n_sys (eta times the system's mean slip rate over the previous step),
// and the rate is the plain Norton law A (o/K)^n: no Newton solve.
template <typename R>
struct LagRef {
    const R *p;      // this voxel's raise of system 0
    long stride;     // between systems
};

template <typename R, int NS, int SPEC, bool LAG = false>
__device__ __forceinline__ void rk_stage(const LawP<R> &P, const R e[6], R (&tep)[6], R (&tv)[NS], R (&tal)[NS],
                                         const R (&yep)[6], const R (&yv)[NS], const R (&yal)[NS], R (&aep)[6],
                                         R (&av)[NS], R (&aal)[NS], uint32_t &warm, const LawLds<R> &W, R wacc,
                                         R cnext, int &nact, int &nnewt, LagRef<R> lag = {nullptr, 0})
{
    R ee[6], sig[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) ee[i] = e[i] - tep[i];
    hooke_c<R, SPEC>(P.C, ee, sig);
    // saturating hardening terms (parked in the LDS column until the family
    // sums are complete when registers are short)
    R h[NS];
    R Hs = R(0), Ht = R(0), sumf = R(0);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        law_fence();
        const bool tw = is_twin<SPEC>(P, s);
        const R bl = tw ? P.ft.bl2e : P.fs.bl2e;
        const R hs = R(1) - ex2(-bl * tv[s]);
        if constexpr (law_park_h<R>()) W.o[s * W.ls] = hs;
        else h[s] = hs;
        if (tw) {
            Ht += hs;
            sumf += tv[s] * P.inv_gT;
        } else {
            Hs += hs;
        }
    }
    const R wslip = R(1) - sumf;
    const R Atw = P.twin_mode ? P.Kc_gT * (P.fm - sumf) : R(1);
    const R etaAtw = P.eta * Atw;
    const R inv_etaAtw = P.twin_mode ? fdiv(R(1), etaAtw) : P.inv_eta;
    // latent hardening per family (one product per family, not per system)
    // (kept as products: fused into every system's resistance they would
    // cost a move of the scalar resistance and an FMA per system instead of
    // one addition)
    R QLHs, QLHt;
    {
#pragma clang fp contract(off)
        QLHs = P.fs.QL * Hs;
        QLHt = P.ft.QL * Ht;
    }
    // overstress of every system, stored with the sign of the slip rate
    // (zero for inactive systems)
    uint32_t act = 0;
    T1Sig<R> t1;
    if constexpr (t1_factor<SPEC>()) t1 = t1_sig(sig);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        law_fence();
        const bool tw = is_twin<SPEC>(P, s);
        const FamP<R> &F = tw ? P.ft : P.fs;
        const R hs = law_park_h<R>() ? W.o[s * W.ls] : h[s];
        R t0;
        if constexpr (law_tau0_lds<R>()) t0 = W.tau0[s];
        else if constexpr (SPEC == LAW_TABLE1) t0 = P.tau0k[T1_KIND[s]];
        else t0 = P.tau0[s];
        R r = (t0 + (tw ? QLHt : QLHs)) + F.QD * hs;
        if constexpr (LAG) {
            // the raises cover the problem's systems only (NS rounds n_sys up)
            if (s < P.nsys) r += lag.p[s * lag.stride];
        }
        R tau = R(0);
        if constexpr (t1_factor<SPEC>()) {
            tau = t1_tau(s, t1);
        } else {
#pragma unroll
            for (int i = 0; i < 6; ++i)
                if (schmid_nonzero<SPEC>(s, i))
                    tau += (i < 3 ? sig[i] : R(2) * sig[i]) * schmid<R, SPEC>(P.m, s, i);
        }
        const R tx = tau - F.c * tal[s];
        const R o = tw ? tx - r : fabs(tx) - r;
        const R A = tw ? Atw : R(1);
        const bool on = o > R(0) && A > R(0);
        if (on) act |= 1u << s;
        // an active slip system has |tx| > r >= 0, so the sign bit of tx is
        // the sign of the rate
        const R os = tw ? o : copysign(o, tx);
        if constexpr (LAG) {
            R g = R(0);
            if (on) {
                const R yk = o * F.invK;
                g = A * yk * pow_nm1(yk, F.nm1, sizeof(R) == 8 ? F.nm1_int : -1, P.nm1_uni);
            }
            W.o[s * W.ls] = tw ? g : copysign(g, tx);
        } else {
            W.o[s * W.ls] = on ? os : R(0);
        }
    }
    nact += __popc(act);
    if constexpr (!LAG) {
    // Newton solves: the first law_items_q active systems of each lane go to
    // the wave's item list, taken in turn by the wave's active lanes
    constexpr int Q = law_items_q<R>();
    const int lane = (int)(threadIdx.x & 63u);
    uint32_t mine = act, rest = 0u;
    int cnt = __popc(act);
    if (cnt > Q) {
        uint32_t m = act;
        for (int k = 0; k < Q; ++k) m &= m - 1u;
        rest = m;
        mine = act & ~m;
        cnt = Q;
    }
    // exclusive prefix sum of the counts over the active lanes (cnt < 32)
    int excl = 0, total = 0;
#pragma unroll
    for (int b = 0; b < 5; ++b) {
        const uint64_t bal = __ballot((cnt >> b) & 1);
        excl += (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u))
                << b;
        total += __popcll(bal) << b;
    }
    {
        uint32_t m = mine;
        int k = excl;
        while (m) {
            const int sy = __builtin_ctz(m);
            m &= m - 1u;
            W.items[k++] = (uint16_t)((lane << 6) | (sy << 1) | ((warm >> sy) & 1u));
        }
    }
    W.aw[lane] = Atw;
    __builtin_amdgcn_wave_barrier();
    const uint64_t ex = __ballot(1);
    const int nlanes = __popcll(ex);
    const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(ex >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)ex, 0u));
    R *const o_wave = W.o - lane;   // column of lane l: o_wave + l
    R *const y_wave = W.y - lane;
    for (int base = 0; base < total; base += nlanes) {
        const int idx = base + rank;
        if (idx < total) {
            const uint32_t it = W.items[idx];
            const int owner = (int)(it >> 6), sy = (int)((it >> 1) & 31u);
            const bool tw = SPEC == LAW_TABLE1 ? sy >= 12 : ((P.twin_mask >> sy) & 1u) != 0u;
            R *const po = o_wave + owner + sy * W.ls;
            R *const py = y_wave + owner + sy * W.ls;
            const R os = *po;
            const R yprev = *py;
            R yw = (it & 1u) ? yprev : R(0);
            R A = R(1), etaA = P.eta, inv_etaA = P.inv_eta;
            if (tw) {
                A = W.aw[owner];
                etaA = P.eta * A;
                if (P.twin_mode) inv_etaA = fdiv(R(1), etaA);
            }
            const R g = newton_solve<R>(fabs(os), A, etaA, inv_etaA, W.fam + (tw ? LAW_FAM_WORDS : 0), P, yw,
                                        nnewt);
            *py = yw;
            *po = os < R(0) ? -g : g;
        }
    }
    __builtin_amdgcn_wave_barrier();
    // systems beyond the list: solved by their own lane
    uint32_t rem = rest;
    while (__any(rem != 0u)) {
        if (rem) {
            const int sy = __builtin_ctz(rem);
            rem &= rem - 1u;
            const bool tw = SPEC == LAW_TABLE1 ? sy >= 12 : ((P.twin_mask >> sy) & 1u) != 0u;
            const R os = W.o[sy * W.ls];
            const R yprev = W.y[sy * W.ls];
            R yw = ((warm >> sy) & 1u) ? yprev : R(0);
            const R g = newton_solve<R>(fabs(os), tw ? Atw : R(1), tw ? etaAtw : P.eta,
                                        tw ? inv_etaAtw : P.inv_eta, W.fam + (tw ? LAW_FAM_WORDS : 0), P, yw,
                                        nnewt);
            W.y[sy * W.ls] = yw;
            W.o[sy * W.ls] = os < R(0) ? -g : g;
        }
    }
    warm = act;
    }
    // rates of the internal variables (signed rates from the LDS column)
    R dep[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
    T1Acc<R> acc;
    if constexpr (t1_factor<SPEC>()) t1_acc_init(acc);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        law_fence();
        const bool tw = is_twin<SPEC>(P, s);
        const FamP<R> &F = tw ? P.ft : P.fs;
        const R gd = W.o[s * W.ls];
        const R ag = fabs(gd);
        const R dal = gd - F.d * ag * tal[s];
        av[s] += wacc * ag;
        aal[s] += wacc * dal;
        tv[s] = yv[s] + cnext * ag;
        tal[s] = yal[s] + cnext * dal;
        if constexpr (t1_factor<SPEC>()) {
            t1_acc_add(acc, s, gd);
        } else {
            const R wg = tw ? gd : wslip * gd;
#pragma unroll
            for (int i = 0; i < 6; ++i)
                if (schmid_nonzero<SPEC>(s, i)) dep[i] += wg * schmid<R, SPEC>(P.m, s, i);
        }
    }
    if constexpr (t1_factor<SPEC>()) t1_acc_dep(acc, wslip, dep);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        aep[i] += wacc * dep[i];
        tep[i] = yep[i] + cnext * dep[i];
    }
}

// Integrate the internal variables over one load increment (crystal frame):
// total strain linear in time from e0 to e1, M classical RK4 substeps.
// W: LDS work area.
template <typename R, int NS, int SPEC, bool LAG = false>
__device__ void integrate(const LawP<R> &P, const R e0[6], const R e1[6], R (&ep)[6], R (&v)[NS],
                          R (&al)[NS], R dt, int M, int &nact, int &nnewt, const LawLds<R> &W,
                          LagRef<R> lag = {nullptr, 0})
{
    const R h = dt / R(M);
    const R invM = R(1) / R(M);
    R de[6];
    uint32_t warm = 0;
#pragma unroll
    for (int i = 0; i < 6; ++i) de[i] = e1[i] - e0[i];
    law_fam_store<R, NS>(P, W);
    if constexpr (law_park_e<R, NS>()) {
        // the strain path lives in LDS through the integration
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            W.e[i * W.ls] = e0[i];
            W.e[(6 + i) * W.ls] = e1[i];
        }
    }
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
            const R sfrac = (st == 0) ? R(j) * invM : (st == 3) ? R(j + 1) * invM : (R(j) + R(0.5)) * invM;
            const R wacc = (st == 0 || st == 3) ? h * R(1.0 / 6.0) : h * R(1.0 / 3.0);
            const R cnext = (st == 2) ? h : h * R(0.5);
            R e[6];
            if constexpr (law_park_e<R, NS>()) {
#pragma unroll
                for (int i = 0; i < 6; ++i) {
                    const R a = W.e[i * W.ls];
                    e[i] = a + sfrac * (W.e[(6 + i) * W.ls] - a);
                }
            } else {
#pragma unroll
                for (int i = 0; i < 6; ++i) e[i] = e0[i] + sfrac * de[i];
            }
            rk_stage<R, NS, SPEC, LAG>(P, e, tep, tv, tal, ep, v, al, aep, av, aal, warm, W, wacc, cnext, nact,
                                       nnewt, lag);
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

template <typename R>
__device__ __forceinline__ void hooke(const LawP<R> &P, const R e[6], const R ep[6], R sig[6])
{
    R ee[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) ee[i] = e[i] - ep[i];
    hooke_c<R, LAW_GENERAL>(P.C, ee, sig);
}

}  // namespace cpf

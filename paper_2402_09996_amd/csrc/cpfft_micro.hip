// Stochastic 3D microstructure model (Section 2) on the device, and the
// C-ABI of include/cpfft_micro.h.
//
// The voxel work runs in four kernels: Matern thinning of the primary
// points, the periodic Voronoi labels (16^3 groups and 8^3 tiles searching
// candidate lists of generators), the grain graph with grain volumes, and
// the inclusion slabs.  The graph-level steps (drawing twin pairs and
// orientations, one grain at a time from one random stream) run on the
// host between the launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/cpfft.h"
#include "../../include/cpfft_micro.h"

// Arithmetic in the order written, host and device (no fused multiply-add):
// the Poisson inversion and the lattice draws must give the same integers
// wherever they are evaluated, and the slab test the same decision as a
// host evaluation in the same order.
#pragma clang fp contract(off)

// error state shared with the solver's entry points
int cpf_internal_fail(int code, const char *msg);

namespace cpfm {

static int failf(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return cpf_internal_fail(code, buf);
}

#define MCHK(call)                                                                                      \
    do {                                                                                                \
        hipError_t e_ = (call);                                                                         \
        if (e_ != hipSuccess) return failf(CPF_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned int periodic_d2(int ax, int ay, int az, int bx, int by, int bz, int Lx, int Ly,
                                                    int Lz)
{
    int dx = abs(ax - bx), dy = abs(ay - by), dz = abs(az - bz);
    dx = min(dx, Lx - dx);
    dy = min(dy, Ly - dy);
    dz = min(dz, Lz - dz);
    // each term <= 2^30, the sum < 2^32
    return (unsigned int)(dx * dx) + (unsigned int)(dy * dy) + (unsigned int)(dz * dz);
}

// Matern type II with the index as the mark: i survives iff no j < i lies
// within r (squared lattice distance <= r2).  One wave per point: the
// lanes split the earlier points and vote.
__global__ __launch_bounds__(256) void k_thin(const int4 *__restrict__ pts, int n, int Lx, int Ly, int Lz,
                                              double r2, uint8_t *__restrict__ keep)
{
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;   // whole waves leave together
    const int4 p = pts[i];
    bool hit = false;
    for (int j = lane; j < i; j += 64) {
        const int4 o = pts[j];
        hit = hit || (double)periodic_d2(p.x, p.y, p.z, o.x, o.y, o.z, Lx, Ly, Lz) <= r2;
    }
    const bool any = __any(hit);
    if (lane == 0) keep[i] = any ? 0 : 1;
}

constexpr int VT = 8;            // tile edge (voxels)
constexpr int VG = 2 * VT;       // group edge: 2x2x2 tiles per block
constexpr int VCAP = 1024;       // tile candidate list capacity
constexpr int VGCAP = 2048;      // group candidate list capacity
constexpr int VD2 = 4096;        // generators whose group-centre distance is kept in LDS

// Candidate screening: for a box of voxel centres with centre c and half
// diagonal R, and any generator at distance D from c, every voxel's nearest
// generators (ties included) lie within D + 2R of c (|s - c| <= |s - v| +
// R <= |s* - v| + R <= D + 2R).  Each block screens all generators once for
// its 16^3 group (D the least distance found), then, for each 8^3 tile of
// the group, the group's list (D the least distance over that list: an
// upper bound of the true one, which keeps the argument valid); each voxel
// takes the least (squared distance, index) over its tile's list.  A list
// that overflows is replaced by the list it was taken from (the group's,
// or all generators).
__global__ __launch_bounds__(256) void k_voronoi(const int4 *__restrict__ seeds, int n, int nx, int ny, int nz,
                                                 int q, int ngx, int ngy, int32_t *__restrict__ labels,
                                                 int32_t *fallback)
{
    __shared__ unsigned int d2c[VD2];
    __shared__ int gidx[VGCAP];
    __shared__ int cidx[VCAP];
    __shared__ unsigned int dmin;
    __shared__ int ncnt;
    const int tid = threadIdx.x;
    const int b = blockIdx.x;
    const int gx = b % ngx, gy = (b / ngx) % ngy, gz = b / (ngx * ngy);
    const int ox = gx * VG, oy = gy * VG, oz = gz * VG;
    const int Lx = q * nx, Ly = q * ny, Lz = q * nz;
    const int h = q / 2;
    auto radius = [&](int ex, int ey, int ez) {
        return 0.5 * (double)q * sqrt((double)((ex - 1) * (ex - 1) + (ey - 1) * (ey - 1) + (ez - 1) * (ez - 1)));
    };

    // group list
    {
        const int ex = min(VG, nx - ox), ey = min(VG, ny - oy), ez = min(VG, nz - oz);
        const int cx = ox * q + h + (ex - 1) * h, cy = oy * q + h + (ey - 1) * h, cz = oz * q + h + (ez - 1) * h;
        if (tid == 0) {
            dmin = 0xffffffffu;
            ncnt = 0;
        }
        __syncthreads();
        unsigned int my = 0xffffffffu;
        for (int j = tid; j < n; j += blockDim.x) {
            const int4 s = seeds[j];
            const unsigned int d2 = periodic_d2(cx, cy, cz, s.x, s.y, s.z, Lx, Ly, Lz);
            if (j < VD2) d2c[j] = d2;
            my = min(my, d2);
        }
        atomicMin(&dmin, my);
        __syncthreads();
        // a margin of 2 lattice units over the rounding of the roots
        const double bd = sqrt((double)dmin) + 2.0 * radius(ex, ey, ez) + 2.0;
        const double b2 = bd * bd;
        for (int j = tid; j < n; j += blockDim.x) {
            unsigned int d2;
            if (j < VD2) {
                d2 = d2c[j];
            } else {
                const int4 s = seeds[j];
                d2 = periodic_d2(cx, cy, cz, s.x, s.y, s.z, Lx, Ly, Lz);
            }
            if ((double)d2 <= b2) {
                const int slot = atomicAdd(&ncnt, 1);
                if (slot < VGCAP) gidx[slot] = j;
            }
        }
        __syncthreads();
    }
    const int ng = ncnt;
    const bool gfull = ng > VGCAP;
    const int nl = gfull ? n : ng;             // the list the tiles screen
    if (gfull && tid == 0 && fallback) atomicAdd(fallback, 1);

    const int lx = tid & 7, ly = (tid >> 3) & 7, lz0 = tid >> 6;
    for (int t = 0; t < 8; ++t) {
        const int x0 = ox + (t & 1) * VT, y0 = oy + ((t >> 1) & 1) * VT, z0 = oz + (t >> 2) * VT;
        if (x0 >= nx || y0 >= ny || z0 >= nz) continue;   // uniform over the block
        const int ex = min(VT, nx - x0), ey = min(VT, ny - y0), ez = min(VT, nz - z0);
        const int cx = x0 * q + h + (ex - 1) * h, cy = y0 * q + h + (ey - 1) * h, cz = z0 * q + h + (ez - 1) * h;
        __syncthreads();   // the previous tile's list is no longer read
        if (tid == 0) {
            dmin = 0xffffffffu;
            ncnt = 0;
        }
        __syncthreads();
        unsigned int my = 0xffffffffu;
        for (int k = tid; k < nl; k += blockDim.x) {
            const int4 s = seeds[gfull ? k : gidx[k]];
            my = min(my, periodic_d2(cx, cy, cz, s.x, s.y, s.z, Lx, Ly, Lz));
        }
        atomicMin(&dmin, my);
        __syncthreads();
        const double bd = sqrt((double)dmin) + 2.0 * radius(ex, ey, ez) + 2.0;
        const double b2 = bd * bd;
        for (int k = tid; k < nl; k += blockDim.x) {
            const int j = gfull ? k : gidx[k];
            const int4 s = seeds[j];
            if ((double)periodic_d2(cx, cy, cz, s.x, s.y, s.z, Lx, Ly, Lz) <= b2) {
                const int slot = atomicAdd(&ncnt, 1);
                if (slot < VCAP) cidx[slot] = j;
            }
        }
        __syncthreads();
        const int nc = ncnt;
        const bool tfull = nc > VCAP;
        const int nv = tfull ? nl : nc;
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            const int lz = lz0 + 4 * v;
            if (lx >= ex || ly >= ey || lz >= ez) continue;
            const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
            const int px = x * q + h, py = y * q + h, pz = z * q + h;
            unsigned int best = 0xffffffffu;
            int bi = 0x7fffffff;
            for (int k = 0; k < nv; ++k) {
                const int j = tfull ? (gfull ? k : gidx[k]) : cidx[k];
                const int4 s = seeds[j];
                const unsigned int d2 = periodic_d2(px, py, pz, s.x, s.y, s.z, Lx, Ly, Lz);
                if (d2 < best || (d2 == best && j < bi)) {
                    best = d2;
                    bi = j;
                }
            }
            labels[((long)z * ny + y) * nx + x] = bi;
        }
    }
}

template <typename T>
__global__ void k_zero(T *p, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = T(0);
}

__device__ __forceinline__ void set_adj(uint32_t *adj, int W, int a, int b)
{
    uint32_t *w = adj + (long)a * W + (b >> 5);
    const uint32_t bit = 1u << (b & 31);
    if (!(__atomic_load_n(w, __ATOMIC_RELAXED) & bit)) atomicOr(w, bit);
}

// Each block takes a contiguous run of voxels: face neighbours along +x,
// +y, +z (periodic) with another label set both bits of the pair; voxel
// counts go to block-local LDS counters when n fits, added once per block.
__global__ __launch_bounds__(256) void k_graph(const int32_t *__restrict__ lab, int nx, int ny, int nz, int n,
                                               int W, long chunk, uint32_t *adj, unsigned long long *vol,
                                               int lds_counts)
{
    extern __shared__ unsigned int cnt[];
    const int tid = threadIdx.x;
    if (lds_counts) {
        for (int i = tid; i < n; i += blockDim.x) cnt[i] = 0u;
        __syncthreads();
    }
    const long nvox = (long)nx * ny * nz;
    const long v0 = (long)blockIdx.x * chunk, v1 = min(nvox, v0 + chunk);
    // coordinates of the first voxel once, then advanced by the stride
    // with 32-bit carries (no 64-bit division in the loop)
    int x = 0, y = 0, z = 0;
    if (v0 + tid < v1) {
        const long v = v0 + tid;
        x = (int)(v % nx);
        const long r = v / nx;
        y = (int)(r % ny);
        z = (int)(r / ny);
    }
    for (long v = v0 + tid; v < v1; v += blockDim.x) {
        if (v != v0 + tid) {
            x += (int)blockDim.x;
            const unsigned cx = (unsigned)x / (unsigned)nx;
            x -= (int)(cx * nx);
            y += (int)cx;
            const unsigned cy = (unsigned)y / (unsigned)ny;
            y -= (int)(cy * ny);
            z += (int)cy;
        }
        const int g = lab[v];
        const bool ok = (unsigned)g < (unsigned)n;   // labels outside [0, n) are not counted
        // one counter update for a wave whose voxels share a label (the
        // common case inside grains), else one per lane
        const int g0 = __shfl(g, 0);
        const unsigned c = (unsigned)__popcll(__ballot(1));   // active lanes (a prefix of the wave)
        if (__all(g == g0)) {
            if ((threadIdx.x & 63) == 0 && ok) {
                if (lds_counts) atomicAdd(&cnt[g], c);
                else atomicAdd(&vol[g], (unsigned long long)c);
            }
        } else if (ok) {
            if (lds_counts) atomicAdd(&cnt[g], 1u);
            else atomicAdd(&vol[g], 1ull);
        }
        if (!ok) continue;
        const long nbx = v - x + (x + 1 == nx ? 0 : x + 1);
        const long nby = v + (long)((y + 1 == ny ? 0 : y + 1) - y) * nx;
        const long nbz = v + (long)((z + 1 == nz ? 0 : z + 1) - z) * nx * ny;
        const int m[3] = {lab[nbx], lab[nby], lab[nbz]};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (m[k] != g && (unsigned)m[k] < (unsigned)n) {
                set_adj(adj, W, g, m[k]);
                set_adj(adj, W, m[k], g);
            }
        }
    }
    if (lds_counts) {
        __syncthreads();
        for (int i = tid; i < n; i += blockDim.x)
            if (cnt[i]) atomicAdd(&vol[i], (unsigned long long)cnt[i]);
    }
}

// Inclusion slabs: the decision |n . d| <= half in single, correctly
// rounded double operations.
__global__ __launch_bounds__(256) void k_slabs(int32_t *__restrict__ lab, int nx, int ny, int nz, int q, int n,
                                               const int32_t *__restrict__ slab_of,
                                               const double *__restrict__ slabs)
{
    // grid: x covers one z plane, y the planes
    const unsigned plane = (unsigned)nx * (unsigned)ny;
    const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= plane) return;
    const int z = (int)blockIdx.y;
    const long v = (long)z * plane + i;
    const int g = lab[v];
    if (g < 0 || g >= n) return;
    const int s = slab_of[g];
    if (s < 0) return;
    const double *S = slabs + 8 * (long)s;
    const int x = (int)(i % (unsigned)nx), y = (int)(i / (unsigned)nx);
    const double c[3] = {(double)(x * q + q / 2), (double)(y * q + q / 2), (double)(z * q + q / 2)};
    const double L[3] = {(double)q * nx, (double)q * ny, (double)q * nz};
    double d[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double t = c[k] - S[3 + k];
        if (t > 0.5 * L[k]) t = t - L[k];
        else if (t < -0.5 * L[k]) t = t + L[k];
        d[k] = t;
    }
    const double t = (S[0] * d[0] + S[1] * d[1]) + S[2] * d[2];
    if (fabs(t) <= S[6]) lab[v] = (int32_t)S[7];
}

// ---------------------------------------------------------------------------
// host: random stream and the graph-level steps
// ---------------------------------------------------------------------------
struct Stream {
    uint64_t s;
    long long count = 0;
    explicit Stream(uint64_t seed) : s(seed) {}
    uint64_t u64()
    {
        // SplitMix64 (Steele, Lea and Flood, 2014)
        s += 0x9E3779B97F4A7C15ull;
        uint64_t z = s;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        ++count;
        return z ^ (z >> 31);
    }
    double uniform() { return (double)(u64() >> 11) * 0x1.0p-53; }
    int below(uint32_t m) { return (int)(((u64() >> 32) * (uint64_t)m) >> 32); }
};

// Poisson(mu) conditioned on N <= kmax, by inversion of u.
static int poisson_inverse(double u, double mu, int kmax)
{
    if (!(mu > 0.0) || kmax <= 0) return 0;
    const int m = std::min((int)mu, kmax);
    std::vector<double> w(kmax + 1, 0.0);
    w[m] = 1.0;
    for (int k = m + 1; k <= kmax; ++k) w[k] = w[k - 1] * mu / (double)k;
    for (int k = m - 1; k >= 0; --k) w[k] = w[k + 1] * (double)(k + 1) / mu;
    double T = 0.0;
    for (int k = 0; k <= kmax; ++k) T += w[k];
    const double target = u * T;
    double acc = 0.0;
    for (int k = 0; k <= kmax; ++k) {
        acc += w[k];
        if (acc > target) return k;
    }
    return kmax;
}

static int poisson_kmax(double mu) { return (int)(mu + 20.0 * std::sqrt(mu) + 20.0); }

struct M3 {
    double a[9];
};

static M3 mul(const M3 &A, const M3 &B)
{
    M3 C;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            C.a[3 * i + j] = A.a[3 * i] * B.a[j] + A.a[3 * i + 1] * B.a[3 + j] + A.a[3 * i + 2] * B.a[6 + j];
    return C;
}

static void apply(const M3 &A, const double v[3], double out[3])
{
    for (int i = 0; i < 3; ++i) out[i] = A.a[3 * i] * v[0] + A.a[3 * i + 1] * v[1] + A.a[3 * i + 2] * v[2];
}

// right-handed rotation by ang about the unit vector k (Rodrigues)
static M3 axis_rot(const double k[3], double ang)
{
    const double s = std::sin(ang), c1 = 1.0 - std::cos(ang);
    const double K[9] = {0.0, -k[2], k[1], k[2], 0.0, -k[0], -k[1], k[0], 0.0};
    M3 R;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double kk = K[3 * i] * K[j] + K[3 * i + 1] * K[3 + j] + K[3 * i + 2] * K[6 + j];
            R.a[3 * i + j] = (i == j ? 1.0 : 0.0) + s * K[3 * i + j] + c1 * kk;
        }
    return R;
}

// crystal habit normal for the twin axis: [100] -> (011), [010] -> (101);
// a/c = tan(theta/2)
static void habit(int axis, double theta, double h[3])
{
    const double ac = std::tan(0.5 * theta);
    const double v[3] = {axis == 0 ? 0.0 : 1.0, axis == 0 ? 1.0 : 0.0, ac};
    const double nrm = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int i = 0; i < 3; ++i) h[i] = v[i] / nrm;
}

// the twin: theta about [100] (right-handed) or [010] (left-handed), the
// senses that carry the habit plane onto one of the twin's
static M3 twin_of(const M3 &O, int axis, double theta)
{
    const double ex[3] = {1.0, 0.0, 0.0}, ey[3] = {0.0, 1.0, 0.0};
    return mul(O, axis == 0 ? axis_rot(ex, theta) : axis_rot(ey, -theta));
}

// least rotation taking unit h to unit f
static M3 least_rot(const double h[3], const double f[3])
{
    const double v[3] = {h[1] * f[2] - h[2] * f[1], h[2] * f[0] - h[0] * f[2], h[0] * f[1] - h[1] * f[0]};
    const double s = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    const double c = h[0] * f[0] + h[1] * f[1] + h[2] * f[2];
    if (s < 1e-15) {
        if (c > 0) {
            M3 I = {{1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0}};
            return I;
        }
        double p[3] = {1.0, 0.0, 0.0};
        if (std::fabs(h[0]) >= 0.9) { p[0] = 0.0; p[1] = 1.0; }
        const double ph = p[0] * h[0] + p[1] * h[1] + p[2] * h[2];
        for (int i = 0; i < 3; ++i) p[i] -= ph * h[i];
        const double pn = std::sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
        for (int i = 0; i < 3; ++i) p[i] /= pn;
        return axis_rot(p, M_PI);
    }
    const double k[3] = {v[0] / s, v[1] / s, v[2] / s};
    return axis_rot(k, std::atan2(s, c));
}

static M3 haar(double u1, double u2, double u3)
{
    // Shoemake's uniform unit quaternion (w, x, y, z)
    const double a = std::sqrt(1.0 - u1), b = std::sqrt(u1);
    const double w = a * std::sin(2.0 * M_PI * u2), x = a * std::cos(2.0 * M_PI * u2);
    const double y = b * std::sin(2.0 * M_PI * u3), z = b * std::cos(2.0 * M_PI * u3);
    M3 R;
    const double r[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z),     2 * (x * z + w * y),
                         2 * (x * y + w * z),     1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                         2 * (x * z - w * y),     2 * (y * z + w * x),     1 - 2 * (x * x + y * y)};
    memcpy(R.a, r, sizeof r);
    return R;
}

// Bunge angles with Q = Rz(phi1) Rx(Phi) Rz(phi2)
static void to_bunge(const M3 &Q, double e[3])
{
    const double c = std::max(-1.0, std::min(1.0, Q.a[8]));
    const double Phi = std::acos(c);
    if (std::sin(Phi) > 1e-12) {
        e[0] = std::atan2(Q.a[2], -Q.a[5]);
        e[1] = Phi;
        e[2] = std::atan2(Q.a[6], Q.a[7]);
    } else {
        e[0] = std::atan2(Q.a[3], Q.a[0]);
        e[1] = Phi;
        e[2] = 0.0;
    }
}

struct P4 {
    int32_t x, y, z, w;
};

static bool params_ok(const cpf_micro_params *p)
{
    return p && p->nx >= 1 && p->ny >= 1 && p->nz >= 1 && p->q >= 2 && (p->q & 1) == 0 &&
           (long)p->q * std::max(p->nx, std::max(p->ny, p->nz)) <= 65536 &&
           (long)p->nx * p->ny * p->nz <= (1L << 31) && p->lambda >= 0.0 &&
           std::isfinite(p->lambda) && p->r >= 0.0 && std::isfinite(p->r) && p->p_neigh >= 0.0 &&
           p->p_neigh <= 1.0 && p->p_incl >= 0.0 && p->p_incl <= 1.0 && p->delta_lo >= 0.0 &&
           p->delta_lo <= p->delta_hi && p->delta_hi <= 1.0 && p->theta > 0.0 && p->theta < M_PI;
}

struct WsLayout {
    size_t pts, keep, seeds, adj, vol, slab_of, slabs, fb, total;
    int kmax, W;
};

static WsLayout ws_layout(const cpf_micro_params *p)
{
    WsLayout L;
    const double mu = p->lambda * (double)p->nx * (double)p->ny * (double)p->nz;
    L.kmax = poisson_kmax(mu);
    L.W = (L.kmax + 31) / 32;
    size_t o = 0;
    auto take = [&](size_t b) {
        const size_t at = o;
        o += (b + 255) / 256 * 256;
        return at;
    };
    const size_t k = (size_t)std::max(L.kmax, 1);
    L.pts = take(sizeof(P4) * k);
    L.keep = take(k);
    L.seeds = take(sizeof(P4) * k);
    L.adj = take(sizeof(uint32_t) * k * (size_t)L.W);
    L.vol = take(sizeof(unsigned long long) * k);
    L.slab_of = take(sizeof(int32_t) * k);
    L.slabs = take(sizeof(double) * 8 * k);
    L.fb = take(sizeof(int32_t));
    L.total = o;
    return L;
}

// Generators binned on a periodic grid of cells (for the ray search).
struct CellGrid {
    int nc[3];
    double cs[3];
    std::vector<int> start, items;
};

static CellGrid make_cells(const std::vector<P4> &seeds, const double L[3])
{
    CellGrid G;
    for (int i = 0; i < 3; ++i) {
        G.nc[i] = std::max(1, (int)(L[i] / 256.0));   // cells of about 16 voxels at q = 16
        G.cs[i] = L[i] / G.nc[i];
    }
    const int ncell = G.nc[0] * G.nc[1] * G.nc[2];
    auto cell_of = [&](const P4 &s) {
        const int c[3] = {std::min(G.nc[0] - 1, (int)(s.x / G.cs[0])), std::min(G.nc[1] - 1, (int)(s.y / G.cs[1])),
                          std::min(G.nc[2] - 1, (int)(s.z / G.cs[2]))};
        return (c[2] * G.nc[1] + c[1]) * G.nc[0] + c[0];
    };
    G.start.assign(ncell + 1, 0);
    for (const P4 &s : seeds) ++G.start[cell_of(s) + 1];
    for (int c = 0; c < ncell; ++c) G.start[c + 1] += G.start[c];
    G.items.resize(seeds.size());
    std::vector<int> fill(G.start.begin(), G.start.end() - 1);
    for (int m = 0; m < (int)seeds.size(); ++m) G.items[fill[cell_of(seeds[m])]++] = m;
    return G;
}

// Exact exit parameter of the ray sg + t dir from the periodic Voronoi cell
// of generator g: t = min over (m, image) != (g, 0) with D.dir > 0 of
// |D|^2 / (2 D.dir).  Every such t is at least |D|/2, so with t_up the
// value over the grid neighbours (an upper bound) only images with
// |D| <= 2 t_up can matter; the cells covering that box (plus one cell each
// side) are searched, or every generator and image when the box spans half
// the window or more.  The result is the
// same minimum as the search over every generator and image.
static double ray_exit(int g, const double sg[3], const double dir[3], const std::vector<P4> &seeds,
                       const std::vector<int> &nb, const CellGrid &G, const double L[3])
{
    auto t_of = [&](int m, double sx, double sy, double sz, double &t) {
        const double df[3] = {seeds[m].x + sx - sg[0], seeds[m].y + sy - sg[1], seeds[m].z + sz - sg[2]};
        const double den = df[0] * dir[0] + df[1] * dir[1] + df[2] * dir[2];
        if (den > 0.0) {
            const double num = df[0] * df[0] + df[1] * df[1] + df[2] * df[2];
            t = std::min(t, num / (2.0 * den));
        }
    };
    double tup = INFINITY;
    for (int m : nb)
        for (int ix = -1; ix <= 1; ++ix)
            for (int iy = -1; iy <= 1; ++iy)
                for (int iz = -1; iz <= 1; ++iz) t_of(m, ix * L[0], iy * L[1], iz * L[2], tup);
    const double R = 2.0 * tup;
    double t = INFINITY;
    if (!(R < 0.5 * std::min(L[0], std::min(L[1], L[2])))) {
        for (int ix = -1; ix <= 1; ++ix)
            for (int iy = -1; iy <= 1; ++iy)
                for (int iz = -1; iz <= 1; ++iz)
                    for (int m = 0; m < (int)seeds.size(); ++m) {
                        if (m == g && ix == 0 && iy == 0 && iz == 0) continue;
                        t_of(m, ix * L[0], iy * L[1], iz * L[2], t);
                    }
        return t;
    }
    int lo[3], hi[3];
    for (int i = 0; i < 3; ++i) {   // one more cell each side covers the rounding of the binning
        lo[i] = (int)std::floor((sg[i] - R) / G.cs[i]) - 1;
        hi[i] = (int)std::floor((sg[i] + R) / G.cs[i]) + 1;
    }
    for (int cz = lo[2]; cz <= hi[2]; ++cz)
        for (int cy = lo[1]; cy <= hi[1]; ++cy)
            for (int cx = lo[0]; cx <= hi[0]; ++cx) {
                const int c[3] = {cx, cy, cz};
                int w[3], sh[3];
                for (int i = 0; i < 3; ++i) {
                    sh[i] = (int)std::floor((double)c[i] / G.nc[i]);
                    w[i] = c[i] - sh[i] * G.nc[i];
                }
                const int cell = (w[2] * G.nc[1] + w[1]) * G.nc[0] + w[0];
                for (int q = G.start[cell]; q < G.start[cell + 1]; ++q) {
                    const int m = G.items[q];
                    if (m == g && sh[0] == 0 && sh[1] == 0 && sh[2] == 0) continue;
                    t_of(m, sh[0] * L[0], sh[1] * L[1], sh[2] * L[2], t);
                }
            }
    return t;
}

static int launch_label(int nx, int ny, int nz, int q, int n, const int32_t *seeds, int32_t *labels, int32_t *fb,
                        hipStream_t st)
{
    const int ngx = (nx + VG - 1) / VG, ngy = (ny + VG - 1) / VG, ngz = (nz + VG - 1) / VG;
    const long blocks = (long)ngx * ngy * ngz;   // < 2^31: at most 2^31 voxels
    hipLaunchKernelGGL(k_voronoi, dim3((unsigned)blocks), dim3(256), 0, st, (const int4 *)seeds, n, nx, ny, nz, q,
                       ngx, ngy, labels, fb);
    MCHK(hipGetLastError());
    return CPF_OK;
}

static int launch_graph(int nx, int ny, int nz, const int32_t *labels, int n, uint32_t *adj,
                        unsigned long long *vol, hipStream_t st)
{
    const int W = (n + 31) / 32;
    hipLaunchKernelGGL(k_zero<uint32_t>, dim3(256), dim3(256), 0, st, adj, (long)n * W);
    hipLaunchKernelGGL(k_zero<unsigned long long>, dim3(64), dim3(256), 0, st, vol, (long)n);
    const long nvox = (long)nx * ny * nz;
    const long blocks = std::max(1L, std::min(2048L, (nvox + 1023) / 1024));
    const long chunk = (nvox + blocks - 1) / blocks;
    const int lds = n <= 16384 ? 1 : 0;
    hipLaunchKernelGGL(k_graph, dim3((unsigned)blocks), dim3(256), lds ? sizeof(unsigned int) * n : 0, st, labels,
                       nx, ny, nz, n, W, chunk, adj, vol, lds);
    MCHK(hipGetLastError());
    return CPF_OK;
}

}  // namespace cpfm

using namespace cpfm;

extern "C" int cpf_micro_workspace_size(const cpf_micro_params *p, size_t *bytes)
{
    if (!params_ok(p) || !bytes) return failf(CPF_E_INVALID_ARG, "invalid microstructure parameters");
    *bytes = ws_layout(p).total;
    return CPF_OK;
}

extern "C" int cpf_micro_thin(int n, const int32_t *dev_pts, int Lx, int Ly, int Lz, double r_q, uint8_t *dev_keep,
                              void *stream)
{
    if (n < 0 || (n > 0 && (!dev_pts || !dev_keep)) || Lx < 1 || Ly < 1 || Lz < 1 || Lx > 65536 || Ly > 65536 ||
        Lz > 65536 || !(r_q >= 0.0) || !std::isfinite(r_q))
        return failf(CPF_E_INVALID_ARG, "cpf_micro_thin: bad arguments");
    if (n == 0) return CPF_OK;
    hipLaunchKernelGGL(k_thin, dim3((n + 3) / 4), dim3(256), 0, (hipStream_t)stream, (const int4 *)dev_pts, n,
                       Lx, Ly, Lz, r_q * r_q, dev_keep);
    MCHK(hipGetLastError());
    return CPF_OK;
}

extern "C" int cpf_micro_label(int nx, int ny, int nz, int q, int n, const int32_t *dev_seeds, int32_t *dev_labels,
                               int32_t *dev_fallback, void *stream)
{
    if (nx < 1 || ny < 1 || nz < 1 || q < 2 || (q & 1) || (long)q * std::max(nx, std::max(ny, nz)) > 65536 ||
        (long)nx * ny * nz > (1L << 31) || n < 1 || !dev_seeds || !dev_labels)
        return failf(CPF_E_INVALID_ARG, "cpf_micro_label: bad arguments");
    return launch_label(nx, ny, nz, q, n, dev_seeds, dev_labels, dev_fallback, (hipStream_t)stream);
}

extern "C" int cpf_micro_graph(int nx, int ny, int nz, const int32_t *dev_labels, int n, uint32_t *dev_adj,
                               unsigned long long *dev_vol, void *stream)
{
    if (nx < 1 || ny < 1 || nz < 1 || n < 1 || !dev_labels || !dev_adj || !dev_vol)
        return failf(CPF_E_INVALID_ARG, "cpf_micro_graph: bad arguments");
    return launch_graph(nx, ny, nz, dev_labels, n, dev_adj, dev_vol, (hipStream_t)stream);
}

extern "C" int cpf_micro_slabs(int nx, int ny, int nz, int q, int32_t *dev_labels, int n, const int32_t *dev_slab_of,
                               const double *dev_slabs, void *stream)
{
    if (nx < 1 || ny < 1 || nz < 1 || q < 2 || (q & 1) || (long)nx * ny * nz > (1L << 31) || n < 1 ||
        !dev_labels || !dev_slab_of || !dev_slabs)
        return failf(CPF_E_INVALID_ARG, "cpf_micro_slabs: bad arguments");
    const long plane = (long)nx * ny;
    hipLaunchKernelGGL(k_slabs, dim3((unsigned)((plane + 255) / 256), (unsigned)nz), dim3(256), 0,
                       (hipStream_t)stream, dev_labels, nx, ny, nz, q, n, dev_slab_of, dev_slabs);
    MCHK(hipGetLastError());
    return CPF_OK;
}

extern "C" int cpf_micro_generate(const cpf_micro_params *p, void *dev_workspace, size_t ws_bytes, void *stream,
                                  int32_t *dev_labels, int max_labels, double *rot_out, double *euler_out,
                                  int32_t *pairs_out, cpf_micro_info *info)
{
    if (!params_ok(p)) return failf(CPF_E_INVALID_ARG, "invalid microstructure parameters");
    if (!dev_workspace || !dev_labels || !rot_out || !info || max_labels < 1)
        return failf(CPF_E_INVALID_ARG, "cpf_micro_generate: missing buffer");
    const WsLayout L = ws_layout(p);
    if (ws_bytes < L.total || ((uintptr_t)dev_workspace & 255))
        return failf(CPF_E_WORKSPACE, "workspace needs %zu bytes, 256-byte aligned", L.total);
    hipStream_t st = (hipStream_t)stream;
    unsigned char *ws = (unsigned char *)dev_workspace;
    memset(info, 0, sizeof *info);
    const int nx = p->nx, ny = p->ny, nz = p->nz, q = p->q;
    const int Lx = q * nx, Ly = q * ny, Lz = q * nz;

    // primary points
    Stream rs(p->seed);
    const double mu = p->lambda * (double)nx * (double)ny * (double)nz;
    const int np = poisson_inverse(rs.uniform(), mu, L.kmax);
    std::vector<P4> pts(std::max(np, 1));
    for (int i = 0; i < np; ++i) {
        pts[i].x = rs.below((uint32_t)Lx);
        pts[i].y = rs.below((uint32_t)Ly);
        pts[i].z = rs.below((uint32_t)Lz);
        pts[i].w = 0;
    }
    info->n_primary = np;
    if (np < 1) return failf(CPF_E_INVALID_ARG, "the primary process drew no point (lambda too small)");
    MCHK(hipMemcpyAsync(ws + L.pts, pts.data(), sizeof(P4) * np, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_thin, dim3((np + 3) / 4), dim3(256), 0, st, (const int4 *)(ws + L.pts), np, Lx, Ly,
                       Lz, (p->r * q) * (p->r * q), (uint8_t *)(ws + L.keep));
    MCHK(hipGetLastError());
    std::vector<uint8_t> keep(np);
    MCHK(hipMemcpyAsync(keep.data(), ws + L.keep, np, hipMemcpyDeviceToHost, st));
    MCHK(hipStreamSynchronize(st));
    std::vector<P4> seeds;
    for (int i = 0; i < np; ++i)
        if (keep[i]) seeds.push_back(pts[i]);
    const int nw = (int)seeds.size();
    info->n_grains = nw;
    if (nw > max_labels) return failf(CPF_E_WORKSPACE, "max_labels %d < %d grains", max_labels, nw);

    // tessellation and grain graph
    MCHK(hipMemcpyAsync(ws + L.seeds, seeds.data(), sizeof(P4) * nw, hipMemcpyHostToDevice, st));
    int32_t *fb = (int32_t *)(ws + L.fb);
    hipLaunchKernelGGL(k_zero<int32_t>, dim3(1), dim3(64), 0, st, fb, 1L);
    int rc = launch_label(nx, ny, nz, q, nw, (const int32_t *)(ws + L.seeds), dev_labels, fb, st);
    if (rc) return rc;
    uint32_t *adj_d = (uint32_t *)(ws + L.adj);
    unsigned long long *vol_d = (unsigned long long *)(ws + L.vol);
    rc = launch_graph(nx, ny, nz, dev_labels, nw, adj_d, vol_d, st);
    if (rc) return rc;
    const int W = (nw + 31) / 32;
    std::vector<uint32_t> adj((size_t)nw * W);
    std::vector<unsigned long long> vol(nw);
    int32_t nfb = 0;
    MCHK(hipMemcpyAsync(adj.data(), adj_d, sizeof(uint32_t) * adj.size(), hipMemcpyDeviceToHost, st));
    MCHK(hipMemcpyAsync(vol.data(), vol_d, sizeof(unsigned long long) * nw, hipMemcpyDeviceToHost, st));
    MCHK(hipMemcpyAsync(&nfb, fb, sizeof nfb, hipMemcpyDeviceToHost, st));
    MCHK(hipStreamSynchronize(st));
    info->fallback_tiles = nfb;
    // neighbour lists, ascending, and the number of free neighbours
    std::vector<std::vector<int>> nbrs(nw);
    for (int a = 0; a < nw; ++a)
        for (int b = 0; b < nw; ++b)
            if ((adj[(size_t)a * W + (b >> 5)] >> (b & 31)) & 1u) nbrs[a].push_back(b);
    std::vector<int> free_nb(nw);
    for (int a = 0; a < nw; ++a) free_nb[a] = (int)nbrs[a].size();

    // neighbouring twins
    std::vector<M3> rot(nw);
    std::vector<char> assigned(nw, 0);
    int npairs = 0;
    if (p->p_neigh > 0.0 && nw >= 2) {
        const int nn = poisson_inverse(rs.uniform(), p->p_neigh * nw / 2.0, nw / 2);
        info->n_neigh_drawn = nn;
        std::vector<int> cand, nb;
        while (npairs < nn) {
            cand.clear();
            for (int k = 0; k < nw; ++k)
                if (!assigned[k] && free_nb[k] > 0) cand.push_back(k);
            if (cand.empty()) break;
            const int k = cand[rs.below((uint32_t)cand.size())];
            nb.clear();
            for (int m : nbrs[k])
                if (!assigned[m]) nb.push_back(m);
            const int l = nb[rs.below((uint32_t)nb.size())];
            const int a = rs.below(2);
            const double psi = 2.0 * M_PI * rs.uniform();
            // facet normal: minimum-image difference of the generators
            const int Ls[3] = {Lx, Ly, Lz};
            const int sk[3] = {seeds[k].x, seeds[k].y, seeds[k].z}, sl[3] = {seeds[l].x, seeds[l].y, seeds[l].z};
            double f[3];
            for (int i = 0; i < 3; ++i) {
                int d = sl[i] - sk[i];
                if (2 * d > Ls[i]) d -= Ls[i];
                else if (2 * d < -Ls[i]) d += Ls[i];
                f[i] = (double)d;
            }
            const double fn = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
            for (int i = 0; i < 3; ++i) f[i] /= fn;
            double h[3];
            habit(a, p->theta, h);
            const M3 Ok = mul(axis_rot(f, psi), least_rot(h, f));
            rot[k] = Ok;
            rot[l] = twin_of(Ok, a, p->theta);
            assigned[k] = assigned[l] = 1;
            for (int m : nbrs[k]) --free_nb[m];
            for (int m : nbrs[l]) --free_nb[m];
            if (pairs_out && npairs < max_labels / 2) {
                pairs_out[3 * npairs] = k;
                pairs_out[3 * npairs + 1] = l;
                pairs_out[3 * npairs + 2] = a;
            }
            ++npairs;
        }
    }
    info->n_pairs = npairs;
    for (int g = 0; g < nw; ++g)
        if (!assigned[g]) {
            const double u1 = rs.uniform(), u2 = rs.uniform(), u3 = rs.uniform();
            rot[g] = haar(u1, u2, u3);
        }

    // inclusion twins
    std::vector<double> slabs;
    std::vector<int32_t> slab_of(nw, -1);
    int ninc = 0;
    if (p->p_incl > 0.0) {
        const double Ld[3] = {(double)Lx, (double)Ly, (double)Lz};
        const CellGrid grid = make_cells(seeds, Ld);
        for (int g = 0; g < nw; ++g) {
            if (!(rs.uniform() < p->p_incl)) continue;
            const int a = rs.below(2);
            const double zc = 1.0 - 2.0 * rs.uniform();
            const double phi = 2.0 * M_PI * rs.uniform();
            const double rho = std::sqrt(std::max(0.0, 1.0 - zc * zc));
            const double dir[3] = {rho * std::cos(phi), rho * std::sin(phi), zc};
            const double u = rs.uniform();
            // exit point of the ray from the generator through the cell: the
            // least t = |D|^2 / (2 D.dir) over the other generators and their
            // periodic images D ahead of the ray
            const double sg[3] = {(double)seeds[g].x, (double)seeds[g].y, (double)seeds[g].z};
            const double tbest = ray_exit(g, sg, dir, seeds, nbrs[g], grid, Ld);
            double x0[3];
            for (int i = 0; i < 3; ++i) {
                const double xi = sg[i] + tbest * dir[i];
                x0[i] = xi - Ld[i] * std::floor(xi / Ld[i]);
            }
            const double ved = std::pow(6.0 * (double)vol[g] / M_PI, 1.0 / 3.0);
            const double delta = (p->delta_lo + (p->delta_hi - p->delta_lo) * u) * ved;
            const double half = 0.5 * delta * q;
            double h[3], nrm[3];
            habit(a, p->theta, h);
            apply(rot[g], h, nrm);
            const int child = nw + ninc;
            if (child >= max_labels) return failf(CPF_E_WORKSPACE, "max_labels %d too small", max_labels);
            slab_of[g] = ninc;
            const double rec[8] = {nrm[0], nrm[1], nrm[2], x0[0], x0[1], x0[2], half, (double)child};
            slabs.insert(slabs.end(), rec, rec + 8);
            rot.push_back(twin_of(rot[g], a, p->theta));
            ++ninc;
        }
    }
    info->n_inclusions = ninc;
    info->n_labels = nw + ninc;
    info->draws = rs.count;
    if (ninc > 0) {
        MCHK(hipMemcpyAsync(ws + L.slab_of, slab_of.data(), sizeof(int32_t) * nw, hipMemcpyHostToDevice, st));
        MCHK(hipMemcpyAsync(ws + L.slabs, slabs.data(), sizeof(double) * slabs.size(), hipMemcpyHostToDevice, st));
        const long plane = (long)nx * ny;
        hipLaunchKernelGGL(k_slabs, dim3((unsigned)((plane + 255) / 256), (unsigned)nz), dim3(256), 0, st,
                           dev_labels, nx, ny, nz, q, nw, (const int32_t *)(ws + L.slab_of),
                           (const double *)(ws + L.slabs));
        MCHK(hipGetLastError());
    }
    MCHK(hipStreamSynchronize(st));
    for (int g = 0; g < nw + ninc; ++g) {
        memcpy(rot_out + 9 * (size_t)g, rot[g].a, sizeof(double) * 9);
        if (euler_out) to_bunge(rot[g], euler_out + 3 * (size_t)g);
    }
    return CPF_OK;
}

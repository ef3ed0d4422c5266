/* Stochastic 3D microstructure model of Section 2 on the GPU: Matern
 * hard-core generators, the periodic Voronoi tessellation on the voxel
 * centres, the grain graph, neighbouring twins and inclusion twins of the
 * tetragonal lattice (misorientation theta = 2 atan(a/c)).
 *
 * Conventions shared by all calls:
 *   - The window is [0, nx) x [0, ny) x [0, nz) voxels, periodic.  Points
 *     live on a lattice of q points per voxel edge: integer coordinates in
 *     [0, q n_d); voxel (i, j, k) has centre (q i + q/2, q j + q/2,
 *     q k + q/2).  q is even and q * max(n_d) <= 65536, so squared
 *     minimum-image distances are exact 32-bit integers; nx ny nz <= 2^31.
 *   - Labels are int32 [nz][ny][nx], x fastest (the solver's layout).
 *   - Rotations are row-major 3x3, crystal to lab (v_lab = O v_crystal).
 *   - Device pointers must be valid on the current HIP device; `stream` is
 *     a hipStream_t (NULL: the default stream).  The component calls only
 *     queue work; cpf_micro_generate synchronizes the stream.
 *   - Errors: CPF_OK or a negative CPF_E_* code (include/cpfft.h) with a
 *     message in cpf_last_error_message(); CPF_E_INVALID_ARG for bad sizes
 *     or parameters, CPF_E_WORKSPACE for a short workspace or output.
 *   - The library allocates no device memory: the caller passes every
 *     buffer, and keeps ownership. */
#ifndef CPFFT_MICRO_H
#define CPFFT_MICRO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cpf_micro_params {
    int nx, ny, nz;          /* window, voxels (each >= 1)                     */
    int q;                   /* lattice points per voxel edge (even, >= 2)     */
    double lambda;           /* primary Poisson intensity, per voxel^3         */
    double r;                /* hard-core radius, voxels (>= 0)                */
    double p_neigh;          /* neighbouring-twin parameter in [0, 1]          */
    double p_incl;           /* inclusion-twin probability in [0, 1]           */
    double delta_lo, delta_hi; /* relative inclusion thickness, 0<=lo<=hi<=1   */
    double theta;            /* twin misorientation angle, radians (0, pi)     */
    uint64_t seed;           /* SplitMix64 state of the random stream          */
} cpf_micro_params;

typedef struct cpf_micro_info {
    int n_primary;           /* points of the primary Poisson process          */
    int n_grains;            /* generators kept by the thinning (N_W)          */
    int n_neigh_drawn;       /* N_neigh drawn for the neighbouring twins       */
    int n_pairs;             /* twin pairs made                                */
    int n_inclusions;        /* inclusion twins made                           */
    int n_labels;            /* n_grains + n_inclusions                        */
    long long draws;         /* 64-bit words taken from the stream             */
    int fallback_tiles;      /* 16^3 voxel groups whose candidate list overflowed */
} cpf_micro_info;

/* Device workspace for cpf_micro_generate (bytes; depends on the window,
 * lambda and q only). */
int cpf_micro_workspace_size(const cpf_micro_params *p, size_t *bytes);

/* The whole model of Section 2.  Random numbers: one SplitMix64 stream
 * (Steele, Lea and Flood, 2014) from p->seed, each 64-bit output used as a
 * uniform double (top 53 bits times 2^-53) or an integer below m (high 32
 * bits times m, shifted right by 32), taken in this order:
 *   1 uniform: the primary count, Poisson(lambda nx ny nz) by inversion
 *     (weights relative to the mode, ratio recursion, ascending sums);
 *   3 integers per primary point: x, y, z lattice coordinates;
 *   then (device) Matern thinning of type II with the generation order as
 *     the mark (kept iff no earlier point lies within r), the periodic
 *     Voronoi labels (ties to the lowest generator index) and the grain
 *     graph (face-adjacent voxels, periodic) with grain volumes;
 *   [p_neigh > 0, N_W >= 2] 1 uniform: N_neigh ~ Poisson(p_neigh N_W / 2)
 *     conditioned on N_neigh <= N_W / 2 (the rejection of Section 2.2.1);
 *     per pair: the first grain (below the number of free grains with a
 *     free neighbour, ascending), its partner (below its number of free
 *     neighbours, ascending), the twin axis (below 2: [100] with habit
 *     plane (011), or [010] with (101)), the angle psi (2 pi uniform) about
 *     the facet normal f (the minimum-image difference of the generators);
 *     O_first = R_f(psi) A, A the least rotation taking the crystal habit
 *     normal to f; O_second = O_first R, R the rotation by theta about the
 *     axis in the sense that carries the habit plane onto one of the
 *     twin's (right-handed about [100], left-handed about [010]);
 *   3 uniforms per other grain, ascending: Haar orientation (Shoemake);
 *   [p_incl > 0] per grain, ascending: 1 uniform (selected iff < p_incl);
 *     if selected: the axis (below 2), a ray direction from the generator
 *     (z = 1 - 2u, phi = 2 pi u), the relative thickness (1 uniform).  The
 *     ray meets the continuous periodic Voronoi cell boundary at x0; the
 *     grain's voxels with |n . (y - x0)| <= delta/2 (n the lab habit
 *     normal, delta = (lo + (hi - lo) u) ved, ved the volume-equivalent
 *     diameter of the grain's voxels) become grain N_W + j, j the rank of
 *     the inclusion, with the parent's orientation times R.
 * dev_labels: device int32 [nz][ny][nx] (output).  rot_out: host
 * [max_labels][9]; euler_out (may be NULL): host [max_labels][3] Bunge
 * angles of the same rotations (the solver's convention).  pairs_out (may
 * be NULL): host [max_labels / 2][3] (first, second, axis).  info: host.
 * CPF_E_WORKSPACE if ws_bytes or max_labels is too small. */
int cpf_micro_generate(const cpf_micro_params *p, void *dev_workspace, size_t ws_bytes, void *stream,
                       int32_t *dev_labels, int max_labels, double *rot_out, double *euler_out,
                       int32_t *pairs_out, cpf_micro_info *info);

/* Matern type II thinning (Section 2.1): keep[i] = 1 iff no point j < i
 * lies within distance r_q (lattice units, minimum image in the periodic
 * box [0,Lx) x [0,Ly) x [0,Lz)).  dev_pts: int32 [n][4] (x, y, z, unused);
 * dev_keep: uint8 [n]. */
int cpf_micro_thin(int n, const int32_t *dev_pts, int Lx, int Ly, int Lz, double r_q, uint8_t *dev_keep,
                   void *stream);

/* Periodic Voronoi labels of the voxel centres (the tessellation equation
 * of Section 2.1): the generator at the least squared minimum-image
 * distance, the lowest index among equals.  dev_seeds: int32 [n][4],
 * coordinates in [0, q n_d); dev_labels: int32 [nz][ny][nx].
 * dev_fallback (may be NULL): int32 counter, incremented per 16^3 group
 * of voxels whose candidate list overflowed (its tiles then search every
 * generator; the result is the same). */
int cpf_micro_label(int nx, int ny, int nz, int q, int n, const int32_t *dev_seeds, int32_t *dev_labels,
                    int32_t *dev_fallback, void *stream);

/* Grain graph: dev_adj uint32 [n][(n+31)/32] bit matrix, bit m of row g
 * set iff a voxel of g and a voxel of m share a face (periodic); dev_vol
 * uint64 [n] voxel counts.  Both are cleared by the call. */
int cpf_micro_graph(int nx, int ny, int nz, const int32_t *dev_labels, int n, uint32_t *dev_adj,
                    unsigned long long *dev_vol, void *stream);

/* Inclusion slabs (Section 2.2.2): each voxel of a grain g with
 * dev_slab_of[g] = s >= 0 takes label child_s if |n . d| <= half_s, where
 * d = y - x0_s with y the voxel centre and x0_s already wrapped into the
 * window, each component shifted by -L (+L) where it exceeds L/2 (is below
 * -L/2), and the dot product (n0 d0 + n1 d1) + n2 d2 is taken in single,
 * correctly rounded double operations (no contraction).  dev_slabs: double
 * [m][8] = (n0, n1, n2, x0, y0, z0, half, child), lattice units.
 * dev_labels is updated in place; n is the number of labels before. */
int cpf_micro_slabs(int nx, int ny, int nz, int q, int32_t *dev_labels, int n, const int32_t *dev_slab_of,
                    const double *dev_slabs, void *stream);

#ifdef __cplusplus
}
#endif

#endif

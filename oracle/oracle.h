/*
 * oracle.h -- plain FP64 CPU reference for the echo-simulation hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or calls
 * this code; only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no source with the GPU path.
 *
 * Method: Jansen & Steckel, "Hardware-Accelerated Geometrical Simulation of Biological
 * and Engineered In-Air Ultrasonic Systems" (SonoTraceUE), arXiv 2602.19652.
 *   - ray tracing with specular bounces: Section III-C, Algorithm 1
 *   - per-point magnitude and transfer function: Eqs. (2)-(4)
 *   - curvature metric: Section III-B, Eq. (1), Meyer et al. 2003 operator
 *   - Monte Carlo diffraction and its transfer function: Section III-D, Eqs. (7)-(8)
 *   - passive component (direct emitter-receiver path): Section III-E, Eqs. (11)-(13)
 *
 * All arithmetic is IEEE double, compiled with -ffp-contract=off.  Brute force: no
 * acceleration structure anywhere.  Every function returns 0 on success, a negative
 * value on invalid arguments.
 */
#ifndef ECHO_ORACLE_H
#define ECHO_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Algorithm 1 (with the readings listed in the design notes): brute-force FP64
 * closest-hit tracing of N rays, per-hit visibility ray toward x_ref, and the
 * per-segment margin predicate that certifies a ray as free of near-ties.
 * Records are written in (ray, bounce) order; capacity must be >= N*B.  With rec_rxvis
 * (non-NULL; 1 <= M <= 64 receivers at rx_pos) the visibility ray toward x_ref is replaced by
 * one line-of-sight ray to each receiver: bit m of rec_rxvis[n] says receiver m sees the
 * point, rec_vis[n] whether any does. */
int orc_trace(int64_t V, int64_t T, const float* verts, const int32_t* tris, const int32_t* tri_mat,
              const double* emitter_pos, const double* emitter_rot, int64_t N, const float* dirs,
              int32_t max_bounces, double max_distance, const double* x_ref, double t_eps,
              double kappa, double mu_g, int64_t capacity,
              int64_t* n_rec, int32_t* rec_ray, int32_t* rec_bounce, int32_t* rec_tri, int32_t* rec_mat,
              double* rec_p, double* rec_din, double* rec_dout, double* rec_rtot, uint8_t* rec_vis,
              uint8_t* ray_certified, int32_t* ray_nseg, int32_t M, const double* rx_pos, uint64_t* rec_rxvis);

/* Eqs. (2)-(4) and (7)-(8): direct spectral sum over records for the listed bins.
 * kind[n] = 0 specular (uses dout, lobe, refl_k), 1 diffraction (uses diff_coef),
 * 2 passive (the emitter itself as the point, rtot 0, passive_coef [Bk]; it reaches only
 * the receiver whose id equals mat[n]; rx_id[m] gives the ids of the rx_pos rows, NULL
 * for 0..M-1).  Records with vis[n]==0 contribute nothing; with rxvis (per-receiver line of
 * sight, bit r for receiver id r) record n reaches receiver id r only when that bit is set.
 * path_product: a specular record's reflection magnitude is the product of k over its ray's
 * reflections up to it (rec_ray, rec_bounce identify them) instead of its own triangle's k.
 * out is [M][nk][2] (re, im). */
int orc_synth(int64_t n_rec, const double* p, const double* dout, const double* rtot, const int32_t* mat,
              const uint8_t* kind, const uint8_t* vis, int32_t M, const double* rx_pos, const double* rx_rot,
              double f_lo, double f_hi, int32_t F, int32_t nk, const int32_t* k_list,
              double c, double A0, double A1, double p_s, int32_t sigma,
              int32_t Q, int32_t Bk, const float* refl_k, const float* beta, const float* diff_coef,
              int32_t Bd, int32_t El, int32_t Az, const float* directivity, const float* passive_coef,
              const int32_t* rx_id, double* out, const uint64_t* rxvis, const int32_t* rec_ray,
              const int32_t* rec_bounce, int path_product);

/* Analytic gradient of L = sum_{m,k} |H_mk - H*_mk|^2 given g = H - H* ([M][F][2]),
 * with respect to refl_k [Q][Bk] and the receiver positions [M][3], over fixed records.
 * Receiver directivity (rx_rot, Bd, El, Az, directivity as in orc_synth; NULL for none)
 * enters the receiver gradient through the direction of arrival; the path-product reading
 * is not an input of this gradient; rxvis as in orc_synth. */
int orc_grad(int64_t n_rec, const double* p, const double* dout, const double* rtot, const int32_t* mat,
             const uint8_t* kind, const uint8_t* vis, int32_t M, const double* rx_pos,
             double f_lo, double f_hi, int32_t F, double c, double A0, double A1, double p_s, int32_t sigma,
             int32_t Q, int32_t Bk, const float* refl_k, const float* beta, const float* diff_coef,
             const float* passive_coef, const double* g, double* grad_k, double* grad_x, const uint64_t* rxvis,
             const double* rx_rot, int32_t Bd, int32_t El, int32_t Az, const float* directivity);

/* Passive component: line of sight from the emitter to each receiver (vis[M]) and whether
 * that decision is certified against FP32 traversal (certified[M], may be NULL). */
int orc_passive(int64_t V, int64_t T, const float* verts, const int32_t* tris, const double* emitter_pos,
                int32_t M, const double* rx_pos, double t_eps, double kappa, uint8_t* vis, uint8_t* certified);

/* Section III-B, Eq. (1): per-vertex mean-curvature magnitude G_v (Meyer et al.
 * cotangent operator with mixed Voronoi areas) and per-triangle metric
 * C_i = eta * w(A_i) * (max G - min G), eta = 1, w(A) = min(1, A / a_ref). */
int orc_curvature(int64_t V, int64_t T, const float* verts, const int32_t* tris, double a_ref,
                  double* G_v, double* C);

/* SplitMix64 finaliser applied to key + (counter+1)*golden-gamma (Steele, Lea & Flood 2014). */
uint64_t orc_splitmix(uint64_t key, uint64_t counter);

/* Section III-D: curvature-importance Monte Carlo diffraction candidates, dithered
 * integer CDF, line-of-sight and incidence-angle filters.  per_mesh = 0: K samples from one
 * CDF over all eligible triangles.  per_mesh = 1: K samples for each mesh (object) with
 * eligible triangles, in increasing object order, each from its own CDF; at most max_meshes
 * meshes (returns 1 when more are eligible).  *n_samples receives the number written; the
 * sample arrays hold K (or K * max_meshes) entries. */
int orc_diffraction(int64_t V, int64_t T, const float* verts, const int32_t* tris, const int32_t* tri_obj,
                    int32_t n_obj, const double* C, const double* emitter_pos, const double* emitter_rot,
                    double cone_half_angle, double tau, uint64_t seed, int64_t K, double max_incidence,
                    double t_eps, double kappa, int per_mesh, int64_t max_meshes,
                    uint64_t* q_out, int64_t* n_elig, int64_t* n_samples, int32_t* samp_tri, double* samp_o,
                    double* samp_r, uint8_t* samp_keep, uint8_t* samp_certified);

#ifdef __cplusplus
}
#endif
#endif

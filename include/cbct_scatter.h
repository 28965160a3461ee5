/*
 * cbct_scatter.h -- quasi-Monte Carlo scatter simulator of libcbct.so
 * (arXiv 2512.21180, Sec. 2.3: the scatter signal at a detector element as
 * an integral over photon paths, evaluated by sampling paths with a
 * quasi-random sequence, Alg. 2 SamplePath, and integrating each path's
 * interaction points toward every detector element, Alg. 3 Integrate;
 * appendix: the escape probability by the Beer-Lambert law, the
 * travel-distance measure and its inverse-transform sampling, the material
 * and interaction-type choices, the Compton energy
 * e' = e / (1 + e (1 - cos theta) / m_e c^2)).  The full scatter estimate of
 * projection i is I_Sigma / |Src| times Integrate(SamplePath(...)).
 *
 * Readings of the paper (it states the model, not its discretisation):
 *   - The patient is the volume of a geometry handle with water and bone
 *     relative densities rho = [2][nz][ny][nx] (cbct_water_bone's layout),
 *     constant on each voxel cube, zero outside; mu_tot,e(x) =
 *     rho_w(x) mu_w(e) + rho_b(x) mu_b(e).
 *   - Cross sections (cbct_xs): per material (0 water, 1 bone) the
 *     photoelectric, Compton and Rayleigh attenuation at unit density on the
 *     energy grid e0 + k de (k < K), linear in energy, constant beyond the
 *     grid; per material and scatter type (0 Compton, 1 Rayleigh) the
 *     inverse CDF of cos(theta) at u = j / (J - 1) and the density of scatter
 *     directions per steradian at cos(theta) = -1 + 2 i / (I - 1), bilinear.
 *     The caller supplies them (the paper reads them from a cross-section
 *     database).
 *   - Source photons: src = [N][4], a unit direction for the source at angle
 *     0 (S = (sid, 0, 0)) and an energy in keV; at projection `angle` both
 *     are rotated about z with the source.  qmc = [N][5 n + 1] points in
 *     [0, 1): coordinate 0 for the first distance, then per scatter
 *     j = 1..n at k = 1 + 5 (j - 1): material, type, cos(theta), azimuth,
 *     next distance.  The caller draws them (e.g. a Sobol sequence).
 *   - Each leg: tau = optical depth to the volume's exit, p0 = exp(-tau),
 *     w *= 1 - p0, the interaction point at depth -log(1 - (1 - p0) u)
 *     (a ray that misses the volume keeps w = 0 and does not move).  A
 *     scatter: material water when u < mu_w / mu_tot at the point (water
 *     where mu_tot = 0), Compton when u < mu_c / (mu_c + mu_r) of that
 *     material, w *= 1 - mu_p / mu_tot of that material, cos(theta) from the
 *     inverse CDF, azimuth 2 pi u in the frame a = normalise(v x z)
 *     (v x x when |v_z| >= 0.9), b = v x a; Compton lowers the energy.
 *   - Records: rec = [N][n + 1][8], per interaction point its position, the
 *     direction and energy the photon arrived with, and its weight.
 *   - Integrate scores each record toward each pixel centre sigma of the
 *     handle's panel at `angle`:
 *       s w |<n, v_s>| du dv / |sigma - x|^2,
 *       s = s_c p0(x, v_s, e') resp(e') + s_r p0(x, v_s, e) resp(e),
 *     s_T = sum_m (mu_m / mu_tot)(x) (mu_T,m / mu_tot,m)(e) dens_T,m(cos, e),
 *     p0 from the material line integrals from x to sigma, resp piecewise
 *     linear through (20, 5), (60, 20), (120, 10) keV, n the panel normal.
 *     The sum runs over records in order (deterministic).
 * Everything on the device is FP32; every pointer below except xs and the
 * handle is a device pointer owned by the caller.  Calls enqueue on `stream`.
 */
#ifndef CBCT_SCATTER_H
#define CBCT_SCATTER_H

#include "cbct.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int K;              /* energy grid points (>= 2) */
    double e0, de;      /* grid start and step, keV (de > 0) */
    const float *mu;    /* device [2][3][K]: photoelectric, Compton, Rayleigh (mm^-1) */
    int J;              /* inverse-CDF points (>= 2) */
    const float *icdf;  /* device [2][2][K][J] */
    int I;              /* density points (>= 2) */
    const float *dens;  /* device [2][2][K][I] */
} cbct_xs;

/* SamplePath at projection `angle` of handle g for n_photons source photons
 * and n_scatter scatters each (0..16); writes rec [N][n_scatter + 1][8].
 * CBCT_E_SHAPE for an angle, count or order out of range; CBCT_E_ARG for a
 * host-only handle or incomplete tables. */
cbct_status cbct_scatter_paths(const cbct_geom *g, const float *rho, const cbct_xs *xs,
                               int angle, int64_t n_photons, const float *src, const float *qmc,
                               int n_scatter, float *rec, void *stream);

/* Integrate n_rec records toward every pixel of g's panel at `angle`:
 * out [nv][nu] (overwritten), before the I_Sigma / |Src| scale. */
cbct_status cbct_scatter_integrate(const cbct_geom *g, const float *rho, const cbct_xs *xs,
                                   int angle, int64_t n_rec, const float *rec, float *out,
                                   void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CBCT_SCATTER_H */

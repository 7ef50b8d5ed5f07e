/*
 * hfd_mm.h -- micromagnetic energy of one magnetic layer on the lateral grid
 * of the demagnetization library (include/hfd.h), for the hysteresis
 * simulation of Sec. 4 of the paper (CoFe free layer of an MRAM cell, two
 * pinned SAFM layers, field along z, energy minimization by L-BFGS per field
 * step).  The paper names the terms (exchange, uniaxial anisotropy along +z,
 * external field, demagnetization) and the material constants; the
 * discretization used here is the usual finite-difference one:
 *
 *   e(m) = E / (mu0 Ms^2 V_cell)
 *        = sum over magnetic cells c of
 *            - 1/2 m_c . (h_ex + h_an + h_d)(c) - m_c . (h_ext + h_bias)(c)
 *
 *   h_ex(c) = cex_x sum_{x-neighbours n} (m_n - m_c) + cex_y sum_{y-neighbours n} (m_n - m_c)
 *             (neighbours inside the mask only: free surfaces), cex = 2A / (mu0 Ms^2 d^2)
 *   h_an(c) = hk m_z(c) z,  hk = 2 K_u / (mu0 Ms^2)
 *   h_d     = - N * m       of the layer itself (hfd_demag_field on a one-layer plan)
 *   h_ext   = applied field / Ms (uniform), h_bias = field of fixed sources / Ms
 *             (the stray field of the pinned layers), both given by the caller
 *
 * All fields in units of Ms.  m = u / |u| on the cells of the mask and 0
 * elsewhere, for an unnormalized vector field u (the minimizer's variables);
 * the gradient returned is d e / d u = -(h_eff - (m . h_eff) m) / |u|, the
 * tangential part of -h_eff.
 *
 * Layout: u, grad, h_eff, h_bias are DEVICE arrays [3][ny][nx] of doubles
 * (x fastest), owned by the caller.  The mask is a HOST array [ny][nx] of
 * bytes (non-zero = magnetic), copied at creation.  Errors as in hfd.h.
 */
#ifndef HFD_MM_H
#define HFD_MM_H

#include "hfd.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hfd_mm_s *hfd_mm;

/* Energy object on the grid of `demag_plan`, which must be an FP64 plan of one
 * layer (nz = 1, n_geom = 1) and stays owned by the caller (it must outlive the
 * object).  cex_x, cex_y >= 0 and hk finite as defined above.  Allocates its
 * device workspace; `stream` is used for the mask upload and synchronized. */
hfd_status hfd_mm_create(hfd_mm *out, hfd_plan demag_plan, const unsigned char *mask, double cex_x,
                         double cex_y, double hk, void *stream);

/* Copy the field of the fixed sources h_bias (DEVICE [3][ny][nx], units of Ms)
 * into the object (zero until set). */
hfd_status hfd_mm_set_bias(hfd_mm mm, const double *h_bias, void *stream);

/* Reduced energy e(u), its gradient d e / d u (DEVICE grad), optionally the
 * effective field (DEVICE h_eff, may be NULL) and the unit magnetization
 * (DEVICE m, may be NULL) for the applied field h_ext[3] (HOST, units of Ms).
 * Cells with |u| = 0 inside the mask return HFD_EINVAL through a flag checked
 * after the kernels.  Synchronizes `stream` (the energy is returned on the
 * host). */
hfd_status hfd_mm_energy_grad(hfd_mm mm, const double *u, const double *h_ext, double *grad,
                              double *h_eff, double *m, double *energy, void *stream);

hfd_status hfd_mm_destroy(hfd_mm mm);

#ifdef __cplusplus
}
#endif
#endif /* HFD_MM_H */

// plate_system.cpp -- FP64 surface system of the discretised flat plate.
//
// The surface matrix (Sec. III-A, Eq. 8) holds n.K_j(r_ci) for bound vortex
// columns (singular kernel, Eq. 4) and shed-vortex columns (regularised
// kernel, Eq. 5), closed by a Kelvin row of ones (Eq. 7). Both kernels depend
// only on relative positions and rotate with the plate, and the normal turns
// with it, so every entry is the same at every pose: the matrix is built once
// in the plate's own frame and inverted once per geometry, after which each
// step's solve (Eq. 11) is one FP64 matrix-vector product.
#include <cmath>
#include <utility>
#include <vector>

#include "host_common.h"

namespace vpm {

namespace {

// Plate frame: mid-chord at the origin, leading edge at +c/2, the tangent
// pointing from LE to TE along -x and the normal along +z. Positions are
// arclengths from the LE: collocation i at i*lb (i = 0..nb), bound j at
// (j + 1/2) lb, LEV at -delta_s, TEV at c + delta_s.
double along(double s, double c) { return 0.5 * c - s; }

// z-component (the normal) of the kernel from a source at x_s to a target at
// x_t on the chord line, per unit circulation, times 2 pi.
double normal_sing(double xt, double xs) { return 1.0 / (xt - xs); }
double normal_reg(double xt, double xs, double rc) {
  double d = xt - xs;
  return d / std::sqrt(rc * rc * rc * rc + d * d * d * d);
}

}  // namespace

int plate_inverse_T(int nb, double chord, double shed_frac, double r_core,
                    int mode, std::vector<double> &inv_t) {
  const int S = system_size(nb, mode);
  const double lb = chord / nb, ds = shed_frac * chord;
  const double inv2pi = 1.0 / (2.0 * M_PI);
  std::vector<double> a(static_cast<size_t>(S) * S, 0.0);
  const int r0 = first_row(mode);
  for (int r = 0; r < S - 1; ++r) {
    double xt = along((r0 + r) * lb, chord);
    int col = 0;
    for (int j = 0; j < nb; ++j)
      a[r * S + col++] = inv2pi * normal_sing(xt, along((j + 0.5) * lb, chord));
    if (mode == VPM_SHED_BOTH)
      a[r * S + col++] = inv2pi * normal_reg(xt, along(-ds, chord), r_core);
    if (mode != VPM_SHED_NONE)
      a[r * S + col++] =
          inv2pi * normal_reg(xt, along(chord + ds, chord), r_core);
  }
  for (int col = 0; col < S; ++col) a[(S - 1) * S + col] = 1.0;

  // Gauss-Jordan elimination with partial pivoting on [A | I].
  std::vector<double> inv(static_cast<size_t>(S) * S, 0.0);
  for (int i = 0; i < S; ++i) inv[i * S + i] = 1.0;
  for (int k = 0; k < S; ++k) {
    int piv = k;
    for (int i = k + 1; i < S; ++i)
      if (std::fabs(a[i * S + k]) > std::fabs(a[piv * S + k])) piv = i;
    double pv = a[piv * S + k];
    if (!(std::fabs(pv) > 0.0) || !std::isfinite(pv)) return VPM_ESINGULAR;
    if (piv != k)
      for (int j = 0; j < S; ++j) {
        std::swap(a[k * S + j], a[piv * S + j]);
        std::swap(inv[k * S + j], inv[piv * S + j]);
      }
    const double rp = 1.0 / a[k * S + k];
    for (int j = 0; j < S; ++j) {
      a[k * S + j] *= rp;
      inv[k * S + j] *= rp;
    }
    for (int i = 0; i < S; ++i) {
      if (i == k) continue;
      const double f = a[i * S + k];
      if (f == 0.0) continue;
      for (int j = 0; j < S; ++j) {
        a[i * S + j] -= f * a[k * S + j];
        inv[i * S + j] -= f * inv[k * S + j];
      }
    }
  }
  inv_t.assign(static_cast<size_t>(S) * S, 0.0);
  for (int i = 0; i < S; ++i)
    for (int j = 0; j < S; ++j) inv_t[j * S + i] = inv[i * S + j];
  return VPM_OK;
}

}  // namespace vpm

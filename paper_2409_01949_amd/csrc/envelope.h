// Per-axis envelope table entries of one subdomain along one axis, shared by the single-problem
// and batched assembly (Sec. 4.1 eq. window_func; hard constraint Sec. 4.3).
//
// For grid index m of the segment, with x the grid coordinate, w the subdomain's raw window
// factor and S the sum of the raw factors of every subdomain of the level covering m along the
// axis, the normalised factor is g = w / S, and with the ansatz factor a(x) the entries are
// E = a g, E' = a'g + a g', E'' = a''g + 2a'g' + a g''.  On an L-shaped domain the level sum of
// the kept 2D windows does not factor per axis: there the entries hold the raw factor (g = w)
// and the entry kernel divides by the 2D sum.
#pragma once

#include "device.h"
#include "kernels.h"

namespace elmfb {

// Entries for grid indices sg.m0..sg.m1-1, strided over the workgroup's threads; cov gives, per
// (level, axis, grid index), the covering subdomain range [jlo, jhi].
__device__ inline void axis_segment_entries(const Geo& g, const AxisSeg& sg,
                                            const int32_t* __restrict__ cov,
                                            double* __restrict__ tab) {
  const int l = sg.level, a = sg.axis;
  const int J = g.J[l][a];
  const double sigma = g.sigma[l][a];
  const double muj = centre(g, l, a, sg.j);
  for (int m = sg.m0 + threadIdx.x; m < sg.m1; m += blockDim.x) {
    double e = 1.0, e1 = 0.0, e2 = 0.0;
    if (a < g.dim) {
      const double x = grid_coord(g, a, m);
      double gv = 1.0, g1 = 0.0, g2 = 0.0;
      if (J > 1) {
        double w, w1, w2;
        raw_window(x, muj, sigma, w, w1, w2);
        if (g.domain == ELMFB_DOMAIN_L) {
          gv = w;
          g1 = w1;
          g2 = w2;
        } else {
          const int jlo = cov[g.cov_off[l][a] + 2 * m], jhi = cov[g.cov_off[l][a] + 2 * m + 1];
          double S = 0.0, S1 = 0.0, S2 = 0.0;
          for (int jj = jlo; jj <= jhi; ++jj) {
            double v, v1, v2;
            raw_window(x, centre(g, l, a, jj), sigma, v, v1, v2);
            S += v; S1 += v1; S2 += v2;
          }
          gv = w / S;
          g1 = (w1 - gv * S1) / S;
          g2 = (w2 - 2.0 * g1 * S1 - gv * S2) / S;
        }
      }
      double c, c1, c2;
      ansatz_axis(g, a, x, c, c1, c2);
      e = c * gv;
      e1 = c1 * gv + c * g1;
      e2 = c2 * gv + 2.0 * c1 * g1 + c * g2;
    }
    const int64_t o = 3 * (int64_t)(sg.tab_off + (m - sg.m0));
    tab[o] = e;
    tab[o + 1] = e1;
    tab[o + 2] = e2;
  }
}

}  // namespace elmfb

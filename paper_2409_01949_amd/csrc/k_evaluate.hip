// Evaluation of the fitted solution at arbitrary points (Sec. 3 eq. multilevel_solution, times
// the hard-constraint factor of Sec. 4.3):
//   u(x) = C(x) (1/L) sum_l sum_{j : x in supp omega_j} omega_j(x) sum_k a_q tanh(W_q xbar + b_q).
// One wavefront per point: the lanes take the features of each covering subdomain (64 at a time)
// and the point's sum is reduced across the wavefront at the end in a fixed order (a sum over
// ~16 subdomains x K features per point, so one thread per point left most of the device idle on
// check grids of 16,384 points).  Per level the covering subdomains along each axis are found
// from the centre spacing and checked with the support test |x - mu| < sigma; the per-axis
// window sums give the partition-of-unity normalisation.  Bound by the FP64 tanh throughput.
#include "device.h"
#include "kernels.h"

namespace elmfb {

constexpr int kMaxCover = 8;   // covering subdomains per axis and level (width ratio < 7)

__device__ __forceinline__ int cover_axis(const Geo& g, int l, int a, double x, int* js,
                                          double* ws) {
  const int J = g.J[l][a];
  if (J == 1 || a >= g.dim) {
    js[0] = 0;
    ws[0] = 1.0;
    return 1;
  }
  const double h = g.cen_h[l][a], sigma = g.sigma[l][a];
  int j0 = (int)floor((x - g.lo[a] - sigma) / h) - 1;
  int j1 = (int)ceil((x - g.lo[a] + sigma) / h) + 1;
  if (j0 < 0) j0 = 0;
  if (j1 > J - 1) j1 = J - 1;
  int n = 0;
  double S = 0.0;
  for (int j = j0; j <= j1 && n < kMaxCover; ++j) {
    const double mu = centre(g, l, a, j);
    if (fabs(x - mu) < sigma) {
      double w, w1, w2;
      raw_window(x, mu, sigma, w, w1, w2);
      js[n] = j;
      ws[n] = w;
      S += w;
      ++n;
    }
  }
  for (int i = 0; i < n; ++i) ws[i] = ws[i] / S;
  return n;
}

// The same covering subdomains with their raw window factors (not normalised), the sum S of
// those factors and the sum D over the ones whose centre lies above the domain's midpoint (the
// discarded subdomains of an L-shaped domain are the products of such centres on both axes).
__device__ __forceinline__ int cover_axis_raw(const Geo& g, int l, int a, double x, int* js,
                                              double* ws, double& S, double& D) {
  S = 1.0;
  D = 0.0;
  const int J = g.J[l][a];
  if (J == 1 || a >= g.dim) {
    js[0] = 0;
    ws[0] = 1.0;
    return 1;
  }
  const double h = g.cen_h[l][a], sigma = g.sigma[l][a];
  int j0 = (int)floor((x - g.lo[a] - sigma) / h) - 1;
  int j1 = (int)ceil((x - g.lo[a] + sigma) / h) + 1;
  if (j0 < 0) j0 = 0;
  if (j1 > J - 1) j1 = J - 1;
  int n = 0;
  S = 0.0;
  for (int j = j0; j <= j1 && n < kMaxCover; ++j) {
    const double mu = centre(g, l, a, j);
    if (fabs(x - mu) < sigma) {
      double w, w1, w2;
      raw_window(x, mu, sigma, w, w1, w2);
      js[n] = j;
      ws[n] = w;
      S += w;
      if (mu > g.lmid[a]) D += w;
      ++n;
    }
  }
  return n;
}

__global__ void __launch_bounds__(256) k_evaluate(Geo g, const double* __restrict__ W,
                                                  const double* __restrict__ bias,
                                                  const double* __restrict__ coef,
                                                  const double* __restrict__ pts, int64_t n_pts,
                                                  double* __restrict__ u) {
  const int lane = threadIdx.x & 63;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; i < n_pts;
       i += nwaves) {
    const double x = pts[i * g.dim];
    const double y = (g.dim == 2) ? pts[i * g.dim + 1] : 0.0;
    double total = 0.0;
    const bool lshape = g.domain == ELMFB_DOMAIN_L;
    for (int l = 0; l < g.n_levels; ++l) {
      int jxs[kMaxCover], jys[kMaxCover];
      double wxs[kMaxCover], wys[kMaxCover];
      int nxc, nyc;
      double inv_s = 1.0;
      if (lshape) {
        // windows normalised over the kept subdomains: S = Sx Sy - Dx Dy
        double Sx, Dx, Sy, Dy;
        nxc = cover_axis_raw(g, l, 0, x, jxs, wxs, Sx, Dx);
        nyc = cover_axis_raw(g, l, 1, y, jys, wys, Sy, Dy);
        inv_s = 1.0 / (Sx * Sy - Dx * Dy);
      } else {
        nxc = cover_axis(g, l, 0, x, jxs, wxs);
        nyc = cover_axis(g, l, 1, y, jys, wys);
      }
      double lev = 0.0;
      for (int ax = 0; ax < nxc; ++ax) {
        const double xb = feat_in(g, l, 0, jxs[ax], x);
        for (int ay = 0; ay < nyc; ++ay) {
          const double yb = (g.dim == 2) ? feat_in(g, l, 1, jys[ay], y) : 0.0;
          int bi = g.bbase[l] + jxs[ax] * g.J[l][1] + jys[ay];
          if (lshape) {
            bi = g.bmap[g.bmap_off[l] + jxs[ax] * g.J[l][1] + jys[ay]];
            if (bi < 0) continue;   // discarded subdomain
          }
          const int64_t q0 = (int64_t)bi * g.K;
          double acc = 0.0;
          for (int k = lane; k < g.K; k += 64) {
            const int64_t q = q0 + k;
            const double z = W[2 * q] * xb + ((g.dim == 2) ? W[2 * q + 1] * yb : 0.0) + bias[q];
            acc += coef[q] * tanh(z);
          }
          lev += (wxs[ax] * wys[ay]) * acc;
        }
      }
      total += lshape ? lev * inv_s : lev;
    }
    total = wave_sum(total);
    double cx, c1, c2, cy;
    ansatz_axis(g, 0, x, cx, c1, c2);
    ansatz_axis(g, 1, y, cy, c1, c2);
    if (lane == 0) u[i] = total * (cx * cy) * g.inv_levels;
  }
}

__global__ void __launch_bounds__(256) k_rel_l2_partials(const double* __restrict__ u,
                                                         const double* __restrict__ ref,
                                                         int64_t n, double* __restrict__ red) {
  __shared__ double sh[4];
  double a = 0.0, b = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double d = u[i] - ref[i];
    a += d * d;
    b += ref[i] * ref[i];
  }
  const double sa = block_sum256(a, sh);
  const double sb = block_sum256(b, sh);
  if (threadIdx.x == 0) {
    red[2 * blockIdx.x] = sa;
    red[2 * blockIdx.x + 1] = sb;
  }
}

__global__ void __launch_bounds__(256) k_rel_l2_final(const double* __restrict__ red, int n,
                                                      SolveState* st) {
  __shared__ double sh[4];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    a += red[2 * i];
    b += red[2 * i + 1];
  }
  const double sa = block_sum256(a, sh);
  const double sb = block_sum256(b, sh);
  if (threadIdx.x == 0) {
    const double r = sqrt(sa) / sqrt(sb);
    st->rel_l2 = r;
    if (st->target > 0.0 && r <= st->target) {
      st->target_hit = 1;
      st->istop = 8;
      st->done = 1;
    }
  }
}

hipError_t launch_evaluate(const Geo& g, const double* W, const double* b, const double* coef,
                           const double* pts, int64_t n_pts, double* u, hipStream_t s) {
  if (n_pts == 0) return hipSuccess;
  int64_t nb = (n_pts + 3) / 4;   // 4 points (wavefronts) per workgroup
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_evaluate, dim3((unsigned)nb), dim3(256), 0, s, g, W, b, coef, pts, n_pts, u);
  return hipGetLastError();
}

hipError_t launch_check_rel_l2(const double* u, const double* ref, int64_t n, SolveState* st,
                               double* red, int n_wg, hipStream_t s) {
  hipLaunchKernelGGL(k_rel_l2_partials, dim3(n_wg), dim3(256), 0, s, u, ref, n, red);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rel_l2_final, dim3(1), dim3(256), 0, s, red, n_wg, st);
  return hipGetLastError();
}

}  // namespace elmfb

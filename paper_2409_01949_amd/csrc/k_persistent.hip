// LSQR (Sec. 3: the method's least-squares solver, Paige-Saunders recurrences) for systems that
// fit in one compute unit: one workgroup of 512 threads runs whole iterations, with u, v, w,
// x, the per-block-point partials t_j, the soft-constraint rows and the index tables held in
// LDS; the FP64 matrix is copied into LDS too when the device's per-workgroup limit allows it,
// else read from global memory, where it stays in the CU's caches.  A step here costs its
// arithmetic and a few workgroup barriers instead of the ~9 kernel launches per step of the
// multi-workgroup path, which dominate when the system holds only thousands of entries (the
// damped oscillator of Sec. 4.2, eq. harm_oscillator).
//
// The step is the same one the multi-workgroup path takes, on the same stored (unnormalised)
// u and v with their scales su = 1/beta and sv = 1/alpha:
//   t_j[p] = sum_k M_j[k][p] v[q0_j + k] sv                    (per block point)
//   u_r    = sum over covering blocks of t_j[p_j(r)] - alpha su u_r      (collocation rows)
//   u_b    = sum_q B[b][q] v[q] sv - alpha su u_b              (soft-constraint rows)
//   beta   = ||u||, x_q = sum_p M_j[k][p] u[r(p)] su + sum_b B[b][q] u_b su,
//   v      = x - beta sv v, alpha = ||v||, the plane rotation, x += t1 w, w = v sv + t2 w,
// then the stopping tests.  Built once per launch: the block table, the block and row of every
// block point, and for every row the block points it sums, in the order of the covering loop
// (level, then x, then y subdomain index), as a compressed row list.  Each reduction is a
// fixed-order wavefront butterfly and a fixed-order sum of the 8 wavefront partials that every
// thread reads, so every thread holds the same scalar state and the result is deterministic.
// 512 threads measured faster than 256 or 1024 on the oscillator (5.9 against 6.7 and 7.4 us
// per step).
#include "device.h"
#include "kernels.h"

namespace elmfb {

namespace {

constexpr int kPThreads = 512;
constexpr int kPWaves = kPThreads / 64;

// A double moved across lanes by a DPP control (both halves); lanes without a source get 0.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double read_lane(double v, int lane) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                          __builtin_amdgcn_readlane(__double2loint(v), lane));
}

// Fixed-order sum over a full wavefront, the same value in every lane: a scan by row shifts of
// 1, 2, 4 and 8 leaves each 16-lane row's sum in its last lane, and the four row sums are added
// as (r0 + r1) + (r2 + r3).  DPP moves and lane reads stay in the vector unit, where the LDS
// permutes of a shuffle butterfly cost a round trip each.
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_move<0x111>(v);   // row_shr:1
  v += dpp_move<0x112>(v);   // row_shr:2
  v += dpp_move<0x114>(v);   // row_shr:4
  v += dpp_move<0x118>(v);   // row_shr:8
  return (read_lane(v, 15) + read_lane(v, 31)) + (read_lane(v, 47) + read_lane(v, 63));
}

// Sum over aligned groups of T lanes (T a power of two <= 64), the same value in each lane of
// a group: quad permutes for the first two steps, shuffles beyond.
__device__ __forceinline__ double group_sum(double s, int T) {
  if (T >= 2) s += dpp_move<0xB1>(s);   // quad_perm [1,0,3,2]: lane ^ 1
  if (T >= 4) s += dpp_move<0x4E>(s);   // quad_perm [2,3,0,1]: lane ^ 2
  for (int o = 4; o < T; o <<= 1) s += __shfl_xor(s, o, 64);
  return s;
}

// Fixed-order sum over the workgroup; every thread returns the same value (each wavefront
// sums the kPWaves partials the same way).  slot holds kPWaves doubles and must not be
// rewritten before every thread has passed a later barrier.
__device__ __forceinline__ double wg_sum(double v, double* slot) {
  v = wave_sum_dpp(v);
  const int lane = threadIdx.x & 63;
  if (lane == 0) slot[threadIdx.x >> 6] = v;
  __syncthreads();
  return wave_sum_dpp(lane < kPWaves ? slot[lane] : 0.0);
}

// Doubles ahead of the index tables, rounded up to an even count so the int4 block table
// starts on a 16-byte boundary.
__host__ __device__ __forceinline__ int64_t persistent_doubles(const Geo& g, int64_t n_pts,
                                                               int64_t n_store, bool a_in_lds) {
  int64_t d = g.n_rows + g.n_bc + 3 * g.n_phi + n_pts + 3 * kPWaves + (int64_t)g.n_bc * g.n_phi;
  if (a_in_lds) d += n_store + g.n_phi;   // rows of (n_j | 1) <= ld_j + 1 entries
  return (d + 1) & ~(int64_t)1;
}

// In wavefront 0: exclusive prefix sum of a[0], a[stride], ... (n entries) in place; returns
// the total in lane 0..63 of wavefront 0.
__device__ __forceinline__ int wave0_exclusive_scan(int32_t* a, int64_t n, int stride) {
  const int lane = threadIdx.x & 63;
  int run = 0;
  for (int64_t base = 0; base < n; base += 64) {
    const int64_t i = base + lane;
    const int c = i < n ? a[i * stride] : 0;
    int incl = c;
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(incl, o, 64);
      if (lane >= o) incl += t;
    }
    if (i < n) a[i * stride] = run + incl - c;
    run += __shfl(incl, 63, 64);
  }
  return run;
}

}  // namespace

// LDS bytes of a launch: the vectors, partials, reduction slots, constraint rows and index
// tables, plus the matrix copy when a_in_lds.
size_t persistent_lds_bytes(const Geo& g, int64_t n_pts, int64_t n_store, bool a_in_lds) {
  const int64_t i = 5 * (int64_t)g.n_blocks + 3 * n_pts + g.n_rows + 1;
  return (size_t)(8 * persistent_doubles(g, n_pts, n_store, a_in_lds) + 4 * i);
}

template <bool ALDS>
__global__ void __launch_bounds__(kPThreads) k_lsqr_persistent(
    Geo g, const DevBlock* __restrict__ blocks, const int32_t* __restrict__ cov,
    const double* __restrict__ A_g, const double* __restrict__ bc_g, double* __restrict__ u_g,
    double* __restrict__ v_g, double* __restrict__ w_g, double* __restrict__ x_g,
    SolveState* st, double* __restrict__ hist, int n_iter, int64_t n_pts, int64_t n_store) {
  if (st->done) return;
  extern __shared__ double lds[];
  const int64_t nrt = g.n_rows + g.n_bc;
  const int64_t n_phi = g.n_phi;
  const int nb = g.n_blocks;
  double* u = lds;
  double* v = u + nrt;
  double* w = v + n_phi;
  double* x = w + n_phi;
  double* tp = x + n_phi;
  double* slot = tp + n_pts;                  // 3 x kPWaves reduction slots
  double* bc = slot + 3 * kPWaves;            // [n_bc][n_phi]
  double* As = bc + (int64_t)g.n_bc * n_phi;  // the matrix copy (ALDS)
  int32_t* ib = reinterpret_cast<int32_t*>(lds + persistent_doubles(g, n_pts, n_store, ALDS));
  int4* bt = reinterpret_cast<int4*>(ib);     // per block: a_off, ld, q0, p_off
  int32_t* bn = ib + 4 * nb;                  // per block: points
  int32_t* pblk = bn + nb;                    // per block point: its block
  int32_t* prow = pblk + n_pts;               // per block point: its row
  int32_t* rp = prow + n_pts;                 // per row: first entry of its list (n_rows + 1)
  int32_t* ridx = rp + g.n_rows + 1;          // the lists: block point indices
  const double* A = ALDS ? As : A_g;
  const int tid = threadIdx.x;
  const int K = g.K;

  for (int64_t i = tid; i < nrt; i += kPThreads) u[i] = u_g[i];
  for (int64_t i = tid; i < n_phi; i += kPThreads) {
    v[i] = v_g[i];
    w[i] = w_g[i];
    x[i] = x_g[i];
  }
  for (int64_t i = tid; i < (int64_t)g.n_bc * n_phi; i += kPThreads) bc[i] = bc_g[i];
  // block table: the global offset and row stride, or (ALDS) the LDS copy's, whose rows hold
  // n_j | 1 entries so that the columns a wavefront reads in M^T u fall in different banks
  for (int j = tid; j < nb; j += kPThreads) {
    const DevBlock& B = blocks[j];
    const int ldl = B.n | 1;
    bt[j] = ALDS ? make_int4(K * ldl, ldl, B.q0, (int)B.p_off)
                 : make_int4((int)B.a_off, B.ld, B.q0, (int)B.p_off);
    bn[j] = B.n;
    for (int p = 0; p < B.n; ++p) {
      const int px = p / B.ny, py = p - px * B.ny;
      pblk[B.p_off + p] = j;
      prow[B.p_off + p] = (B.ix0 + px) * g.ny + (B.iy0 + py);
    }
  }
  if (ALDS) {
    __syncthreads();
    if (tid < 64) wave0_exclusive_scan(reinterpret_cast<int32_t*>(bt), nb, 4);
    __syncthreads();
    for (int j = tid >> 6; j < nb; j += kPWaves) {   // one wavefront per block
      const DevBlock& B = blocks[j];
      const int4 L = bt[j];
      for (int e = tid & 63; e < K * B.n; e += 64) {
        const int k = e / B.n, p = e - k * B.n;
        As[L.x + k * L.y + p] = A_g[B.a_off + (int64_t)k * B.ld + p];
      }
    }
  }
  // the row lists: count, exclusive scan (wavefront 0), fill in the covering loop's order
  for (int pass = 0; pass < 2; ++pass) {
    for (int64_t r = tid; r < g.n_rows; r += kPThreads) {
      const int ix = (int)(r / g.ny), iy = (int)(r - (int64_t)ix * g.ny);
      int c = 0, at = pass ? rp[r] : 0;
      for (int l = 0; l < g.n_levels; ++l) {
        const int jx0 = cov[g.cov_off[l][0] + 2 * ix], jx1 = cov[g.cov_off[l][0] + 2 * ix + 1];
        const int jy0 = cov[g.cov_off[l][1] + 2 * iy], jy1 = cov[g.cov_off[l][1] + 2 * iy + 1];
        const int Jy = g.J[l][1];
        for (int jx = jx0; jx <= jx1; ++jx)
          for (int jy = jy0; jy <= jy1; ++jy) {
            if (pass) {
              const DevBlock& B = blocks[g.bbase[l] + jx * Jy + jy];
              // every (row, covering block) pair is one block point: at < n_pts
              if (at < n_pts) ridx[at] = (int)B.p_off + (ix - B.ix0) * B.ny + (iy - B.iy0);
              ++at;
            }
            ++c;
          }
      }
      if (!pass) rp[r] = c;
    }
    __syncthreads();
    if (!pass && tid < 64) {
      const int run = wave0_exclusive_scan(rp, g.n_rows, 1);
      if (tid == 0) rp[g.n_rows] = run;
    }
    __syncthreads();
  }

  // scalar state: the same copy in every thread
  double alpha = st->alpha, beta = st->beta, su = st->su, sv = st->sv;
  double rhobar = st->rhobar, phibar = st->phibar, anorm = st->anorm;
  double xnorm = st->xnorm, rnorm = st->rnorm, arnorm = st->arnorm, t1 = st->t1, t2 = st->t2;
  const double bnorm = st->bnorm, atol = st->atol, btol = st->btol;
  const int iter_lim = st->iter_lim;
  int itn = st->itn, istop = st->istop, done = 0;

  // threads per column of M^T u: the largest power of two with n_phi * T <= kPThreads, at most 64
  int T = 1;
  while (T < 64 && (int64_t)(2 * T) * n_phi <= kPThreads) T *= 2;
  const int sub = tid & (T - 1);
  const int wave = tid >> 6, lane = tid & 63;

  for (int it = 0; it < n_iter && !done; ++it) {
    // t_j[p] = sum_k M_j[k][p] v[q0_j + k] sv
    for (int64_t f = tid; f < n_pts; f += kPThreads) {
      const int4 B = bt[pblk[f]];
      const double* a = A + B.x + (f - B.w);
      const double* vb = v + B.z;
      const int ld = B.y;
      double c[4] = {0.0, 0.0, 0.0, 0.0};
      int k = 0;
      for (; k + 8 <= K; k += 8) {
        double t[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) t[e] = a[(k + e) * ld];
#pragma unroll
        for (int e = 0; e < 8; ++e) c[e & 3] += t[e] * vb[k + e];
      }
      for (; k < K; ++k) c[k & 3] += a[k * ld] * vb[k];
      tp[f] = ((c[0] + c[1]) + (c[2] + c[3])) * sv;
    }
    __syncthreads();

    // u = M v sv - alpha su u over the collocation rows, then the soft-constraint rows
    const double coef_u = alpha * su;
    double acc = 0.0;
    for (int64_t r = tid; r < g.n_rows; r += kPThreads) {
      double y = 0.0;
      const int e1 = rp[r + 1];
      for (int e = rp[r]; e < e1; ++e) y += tp[ridx[e]];
      const double un = y - coef_u * u[r];
      u[r] = un;
      acc += un * un;
    }
    // constraint row cb on the last wavefronts, which hold the fewest collocation rows
    const int cb = kPWaves - 1 - wave;
    if (cb < g.n_bc) {
      double d = 0.0;
      for (int64_t q = lane; q < n_phi; q += 64) d += bc[(int64_t)cb * n_phi + q] * v[q];
      d = wave_sum_dpp(d) * sv;
      if (lane == 0) {
        const double un = d - coef_u * u[g.n_rows + cb];
        u[g.n_rows + cb] = un;
        acc += un * un;
      }
    }
    beta = sqrt(wg_sum(acc, slot));
    if (tid == 0 && hist && itn + 1 < kHistCap) hist[2 * (itn + 1) + 1] = beta;
    if (beta > 0.0) {
      su = 1.0 / beta;
      anorm = sqrt(anorm * anorm + alpha * alpha + beta * beta);
    }

    // v = M^T u su - beta sv v (v and alpha stay when beta == 0)
    const double coef_v = beta * sv;
    const bool keep = !(beta > 0.0);
    acc = 0.0;
    const int64_t qspan = (n_phi + (kPThreads / T) - 1) / (kPThreads / T) * (kPThreads / T);
    for (int64_t q = tid / T; q < qspan; q += kPThreads / T) {
      // all T threads of a column take this branch together, so the butterfly below reads
      // only active lanes
      if (q < n_phi) {
        const int b = (int)(q / K), k = (int)(q - (int64_t)b * K);
        const int4 B = bt[b];
        const int n = bn[b];
        const double* a = A + B.x + k * B.y;
        const int32_t* pr = prow + B.w;
        double s4[4] = {0.0, 0.0, 0.0, 0.0};
        int p = sub;
        for (; p + 3 * T < n; p += 4 * T) {
          double t[4];
          int rr[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            t[e] = a[p + e * T];
            rr[e] = pr[p + e * T];
          }
#pragma unroll
          for (int e = 0; e < 4; ++e) s4[e] += t[e] * u[rr[e]];
        }
        for (int e = 0; p < n; p += T, ++e) s4[e] += a[p] * u[pr[p]];
        double s = (s4[0] + s4[1]) + (s4[2] + s4[3]);
        s = group_sum(s, T);
        double xq = s * su;
        for (int r = 0; r < g.n_bc; ++r) xq += bc[(int64_t)r * n_phi + q] * (u[g.n_rows + r] * su);
        if (sub == 0) {
          double vq = v[q];
          if (!keep) {
            vq = xq - coef_v * vq;
            v[q] = vq;
          }
          acc += vq * vq;
        }
      }
    }
    const double sa = wg_sum(acc, slot + kPWaves);
    if (beta > 0.0) {
      alpha = sqrt(sa);
      if (alpha > 0.0) sv = 1.0 / alpha;
    }
    if (tid == 0 && hist && itn + 1 < kHistCap) hist[2 * (itn + 1)] = alpha;
    const double rho = sqrt(rhobar * rhobar + beta * beta);
    const double c = rhobar / rho, sn = beta / rho;
    const double theta = sn * alpha;
    rhobar = -c * alpha;
    const double phi = c * phibar;
    phibar = sn * phibar;
    t1 = phi / rho;
    t2 = -theta / rho;
    rnorm = phibar;
    arnorm = alpha * fabs(c) * phibar;

    // x += t1 w, w = v sv + t2 w
    acc = 0.0;
    for (int64_t q = tid; q < n_phi; q += kPThreads) {
      const double wq = w[q];
      const double xq = x[q] + t1 * wq;
      x[q] = xq;
      w[q] = v[q] * sv + t2 * wq;
      acc += xq * xq;
    }
    xnorm = sqrt(wg_sum(acc, slot + 2 * kPWaves));
    itn += 1;

    // stopping tests (conlim off)
    const double eps = 2.220446049250313e-16;
    const double test1 = rnorm / bnorm;
    const double test2 = arnorm / (anorm * rnorm + eps);
    const double tt = test1 / (1.0 + anorm * xnorm / bnorm);
    const double rtol = btol + atol * anorm * xnorm / bnorm;
    int is = 0;
    if (1.0 + test2 <= 1.0) is = 5;
    if (1.0 + tt <= 1.0) is = 4;
    if (test2 <= atol) is = 2;
    if (test1 <= rtol) is = 1;
    if (is == 0 && itn >= iter_lim) is = 7;
    if (is != 0) {
      istop = is;
      done = 1;
    }
  }
  __syncthreads();

  for (int64_t i = tid; i < nrt; i += kPThreads) u_g[i] = u[i];
  for (int64_t i = tid; i < n_phi; i += kPThreads) {
    v_g[i] = v[i];
    w_g[i] = w[i];
    x_g[i] = x[i];
  }
  if (tid == 0) {
    st->alpha = alpha;
    st->beta = beta;
    st->su = su;
    st->sv = sv;
    st->rhobar = rhobar;
    st->phibar = phibar;
    st->anorm = anorm;
    st->xnorm = xnorm;
    st->rnorm = rnorm;
    st->arnorm = arnorm;
    st->t1 = t1;
    st->t2 = t2;
    st->itn = itn;
    st->istop = istop;
    st->done = done;
  }
}

hipError_t launch_lsqr_persistent(const Geo& g, const DevBlock* blocks, const int32_t* cov,
                                  const double* A, const double* bc, double* u, double* v,
                                  double* w, double* x, SolveState* st, double* hist, int n_iter,
                                  int64_t n_pts, int64_t n_store, int* lds_mode, hipStream_t s) {
  size_t lds = persistent_lds_bytes(g, n_pts, n_store, false);
  if (lds > kPersistMaxLds || n_iter <= 0) return hipErrorInvalidValue;
  const size_t lds_a = persistent_lds_bytes(g, n_pts, n_store, true);
  // The matrix joins the vectors in LDS when the device allows that much per workgroup.  The
  // decision (device query and kernel attribute) is taken on the first launch for this system
  // and kept by the caller in *lds_mode: 1 matrix in LDS, 0 vectors only, -1 not decided yet.
  if (*lds_mode < 0) {
    int dev = 0, max_lds = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
      e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return e;
    // the attribute is the kernel's, shared by every handle: raise it to the device limit so a
    // later system with a smaller matrix never lowers it under an earlier one's launches
    *lds_mode = lds_a <= (size_t)max_lds &&
                hipFuncSetAttribute(reinterpret_cast<const void*>(&k_lsqr_persistent<true>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    max_lds) == hipSuccess;
    (void)hipGetLastError();
  }
  if (*lds_mode == 1)
    hipLaunchKernelGGL(k_lsqr_persistent<true>, dim3(1), dim3(kPThreads), lds_a, s, g, blocks,
                       cov, A, bc, u, v, w, x, st, hist, n_iter, n_pts, n_store);
  else
    hipLaunchKernelGGL(k_lsqr_persistent<false>, dim3(1), dim3(kPThreads), lds, s, g, blocks,
                       cov, A, bc, u, v, w, x, st, hist, n_iter, n_pts, n_store);
  return hipGetLastError();
}

}  // namespace elmfb

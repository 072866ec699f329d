// Host runtime behind the C ABI: descriptor checks, decomposition planner, device memory,
// assembly, block-sparse products, LSQR/CGLS drivers with hipGraph-captured iteration loops,
// and evaluation.
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "common.h"
#include "kernels.h"

// Geometry decisions (grid coordinates, centres, support membership) must reproduce the same
// doubles on every implementation: no contraction of a*b+c into fused multiply-adds here.
#pragma clang fp contract(off)

using namespace elmfb;

static thread_local std::string g_thread_error;

struct elmfb_problem_s {
  elmfb_problem_desc desc{};
  Geo geo{};
  int prec = ELMFB_FP64;
  std::string err;

  // host tables
  std::vector<DevBlock> blocks;
  std::vector<Tile> tiles, chunks;
  std::vector<int32_t> chunk_start, cov;
  std::vector<AxisSeg> segs;
  int64_t nnz = 0, n_block_points = 0, n_tab = 0;
  int64_t bytes_device = 0;

  // device memory
  std::vector<void*> allocs;
  DevBlock* d_blocks = nullptr;
  Tile* d_tiles = nullptr;
  Tile* d_chunks = nullptr;
  int32_t* d_cstart = nullptr;
  int32_t* d_cov = nullptr;
  AxisSeg* d_segs = nullptr;
  double* d_tab = nullptr;
  double* d_W = nullptr;
  double* d_b = nullptr;
  void* d_A = nullptr;
  double* d_h = nullptr;
  double* d_tpart = nullptr;
  double* d_part = nullptr;
  double* d_red = nullptr;      // 4 * kRedBlocks * 2 partial sums
  double* d_u = nullptr;        // LSQR u / CGLS r
  double* d_t = nullptr;        // CGLS t = A p
  double* d_v = nullptr;        // LSQR v / CGLS s
  double* d_w = nullptr;        // LSQR w / CGLS p
  double* d_x = nullptr;
  double* d_scalar = nullptr;   // scratch scalar
  SolveState* d_state = nullptr;
  int32_t* d_flag = nullptr;
  double* d_eval = nullptr;     // solution-check buffer
  int64_t eval_cap = 0;

  bool assembled = false;
  double anorm_f = -1.0;        // exact Frobenius norm of the stored matrix (lazy)
  hipStream_t stream = nullptr; // internal stream for captured solves
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  std::map<std::pair<int, int>, hipGraphExec_t> graphs;   // (method, iterations) -> exec
};

namespace {

elmfb_status fail(elmfb_problem h, elmfb_status code, const std::string& msg) {
  if (h) h->err = msg;
  g_thread_error = msg;
  return code;
}

#define HIP_OR_FAIL(h, expr)                                                             \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail((h), ELMFB_E_DEVICE,                                                   \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                    \
  } while (0)

double grid_x(double lo, double hi, int n, int m) {
  if (n == 1) return lo;
  if (m == n - 1) return hi;
  const double step = (hi - lo) / (double)(n - 1);
  const double t = (double)m * step;
  return t + lo;
}

double centre_x(double lo, double hi, int J, int j) {
  if (J == 1) return 0.5 * (lo + hi);
  const double h = (hi - lo) / (double)(J - 1);
  const double t = (double)j * h;
  return t + lo;
}

std::string validate(const elmfb_problem_desc* d) {
  if (!d) return "descriptor is NULL";
  if (d->abi_version != ELMFB_ABI_VERSION) return "abi_version mismatch";
  if (d->dim != 1 && d->dim != 2) return "dim must be 1 or 2";
  if (d->op == ELMFB_OP_D1 && d->dim != 1) return "ELMFB_OP_D1 needs dim = 1";
  if (d->op == ELMFB_OP_NEG_LAPLACE && d->dim != 2) return "ELMFB_OP_NEG_LAPLACE needs dim = 2";
  if (d->op != ELMFB_OP_D1 && d->op != ELMFB_OP_NEG_LAPLACE && d->op != ELMFB_OP_IDENTITY)
    return "unknown operator";
  if (d->ansatz != ELMFB_ANSATZ_NONE && d->ansatz != ELMFB_ANSATZ_TANH_ORIGIN &&
      d->ansatz != ELMFB_ANSATZ_TANH_BOX)
    return "unknown ansatz";
  if (d->ansatz == ELMFB_ANSATZ_TANH_ORIGIN && d->dim != 1) return "TANH_ORIGIN needs dim = 1";
  if (!std::isfinite(d->ansatz_omega)) return "ansatz_omega must be finite";
  for (int a = 0; a < d->dim; ++a) {
    if (!(std::isfinite(d->lo[a]) && std::isfinite(d->hi[a]) && d->lo[a] < d->hi[a]))
      return "domain bounds must be finite with lo < hi";
    if (d->n_points[a] < 2) return "n_points must be >= 2 on every axis";
  }
  if (d->n_levels < 1 || d->n_levels > ELMFB_MAX_LEVELS) return "n_levels out of range";
  if (!(std::isfinite(d->delta) && d->delta > 1.0 && d->delta < 7.0))
    return "delta must satisfy 1 < delta < 7";
  if (d->K < 1 || d->K > 256) return "K must be in 1..256";
  for (int l = 0; l < d->n_levels; ++l)
    for (int a = 0; a < d->dim; ++a)
      if (d->J[l][a] < 1 || d->J[l][a] > 4096) return "J out of range";
  if (d->store_prec != ELMFB_FP64 && d->store_prec != ELMFB_FP32 && d->store_prec != ELMFB_BF16)
    return "unknown store precision";
  if (!d->W_host || !d->b_host) return "W_host and b_host are required";
  return "";
}

// Build every host table of the decomposition.
std::string plan(elmfb_problem h) {
  const elmfb_problem_desc& d = h->desc;
  Geo& g = h->geo;
  std::memset(&g, 0, sizeof(g));
  g.dim = d.dim;
  g.nx = d.n_points[0];
  g.ny = d.dim == 2 ? d.n_points[1] : 1;
  g.n_levels = d.n_levels;
  g.K = d.K;
  g.op = d.op;
  g.ansatz = d.ansatz;
  g.ansatz_omega = d.ansatz_omega;
  const int npts[2] = {g.nx, g.ny};
  double lo[2] = {d.lo[0], d.dim == 2 ? d.lo[1] : 0.0};
  double hi[2] = {d.hi[0], d.dim == 2 ? d.hi[1] : 1.0};
  for (int a = 0; a < 2; ++a) {
    g.lo[a] = lo[a];
    g.hi[a] = hi[a];
    g.step[a] = npts[a] > 1 ? (hi[a] - lo[a]) / (double)(npts[a] - 1) : 0.0;
  }
  g.n_rows = (int64_t)g.nx * g.ny;
  const double sqn = std::sqrt((double)g.n_rows);
  g.inv_scale = 1.0 / (sqn * (double)d.n_levels);
  g.inv_sqrt_n = 1.0 / sqn;
  g.inv_levels = 1.0 / (double)d.n_levels;

  std::vector<double> xs[2];
  for (int a = 0; a < 2; ++a) {
    xs[a].resize(npts[a]);
    for (int m = 0; m < npts[a]; ++m) xs[a][m] = grid_x(lo[a], hi[a], npts[a], m);
  }

  // per level, per axis: centres, half-width, per-subdomain ranges, per-point cover ranges
  std::vector<int> m0s[kMaxLevels][2], m1s[kMaxLevels][2];
  h->cov.clear();
  int nb = 0;
  for (int l = 0; l < d.n_levels; ++l) {
    g.bbase[l] = nb;
    for (int a = 0; a < 2; ++a) {
      const int J = (a < d.dim) ? d.J[l][a] : 1;
      g.J[l][a] = J;
      const int n = npts[a];
      m0s[l][a].assign(J, 0);
      m1s[l][a].assign(J, 0);
      if (J == 1) {
        g.mid[l][a] = 0.5 * (lo[a] + hi[a]);
        g.sigma[l][a] = 0.5 * (hi[a] - lo[a]);
        g.cen_h[l][a] = 0.0;
        m0s[l][a][0] = 0;
        m1s[l][a][0] = n;
      } else {
        const double hc = (hi[a] - lo[a]) / (double)(J - 1);
        g.cen_h[l][a] = hc;
        const double prod = d.delta * hc;
        g.sigma[l][a] = prod / 2.0;
        const double sigma = g.sigma[l][a];
        for (int j = 0; j < J; ++j) {
          const double mu = centre_x(lo[a], hi[a], J, j);
          int first = -1, last = -2;
          for (int m = 0; m < n; ++m) {
            if (std::fabs(xs[a][m] - mu) < sigma) {
              if (first < 0) first = m;
              if (last >= 0 && last != m - 1) return "non-contiguous support";
              last = m;
            }
          }
          if (first < 0) { m0s[l][a][j] = 0; m1s[l][a][j] = 0; }
          else { m0s[l][a][j] = first; m1s[l][a][j] = last + 1; }
        }
      }
      // cover ranges per grid index
      g.cov_off[l][a] = (int32_t)h->cov.size();
      for (int m = 0; m < n; ++m) {
        int jlo = -1, jhi = -2;
        for (int j = 0; j < J; ++j) {
          if (m >= m0s[l][a][j] && m < m1s[l][a][j]) {
            if (jlo < 0) jlo = j;
            if (jhi >= 0 && jhi != j - 1) return "non-contiguous cover";
            jhi = j;
          }
        }
        if (jlo < 0) { jlo = 0; jhi = -1; }
        h->cov.push_back(jlo);
        h->cov.push_back(jhi);
      }
    }
    nb += g.J[l][0] * g.J[l][1];
  }
  g.n_blocks = nb;
  g.n_phi = (int64_t)nb * d.K;

  // axis segments and the envelope table layout
  h->segs.clear();
  std::vector<int> segoff[kMaxLevels][2];
  int32_t tab = 0;
  for (int l = 0; l < d.n_levels; ++l)
    for (int a = 0; a < 2; ++a) {
      segoff[l][a].assign(g.J[l][a], 0);
      for (int j = 0; j < g.J[l][a]; ++j) {
        AxisSeg s{l, a, j, m0s[l][a][j], m1s[l][a][j], tab};
        segoff[l][a][j] = tab;
        tab += m1s[l][a][j] - m0s[l][a][j];
        h->segs.push_back(s);
      }
    }
  h->n_tab = tab;

  // blocks, tiles, chunks
  h->blocks.clear();
  h->tiles.clear();
  h->chunks.clear();
  h->chunk_start.clear();
  int64_t a_off = 0, p_off = 0;
  for (int l = 0; l < d.n_levels; ++l)
    for (int jx = 0; jx < g.J[l][0]; ++jx)
      for (int jy = 0; jy < g.J[l][1]; ++jy) {
        DevBlock B{};
        B.a_off = a_off;
        B.p_off = p_off;
        B.q0 = (int32_t)(h->blocks.size() * (size_t)d.K);
        B.ix0 = m0s[l][0][jx];
        B.nx = m1s[l][0][jx] - m0s[l][0][jx];
        B.iy0 = m0s[l][1][jy];
        B.ny = m1s[l][1][jy] - m0s[l][1][jy];
        const int64_t n = (int64_t)B.nx * B.ny;
        if (n > (int64_t)1 << 30) return "block too large";
        B.n = (int32_t)n;
        B.tabx = segoff[l][0][jx];
        B.taby = segoff[l][1][jy];
        B.level = l;
        const int b = (int)h->blocks.size();
        for (int64_t p0 = 0; p0 < n; p0 += kTile) h->tiles.push_back(Tile{b, (int32_t)p0});
        h->chunk_start.push_back((int32_t)h->chunks.size());
        for (int64_t p0 = 0; p0 < n; p0 += kChunkPts) h->chunks.push_back(Tile{b, (int32_t)p0});
        h->blocks.push_back(B);
        a_off += n * d.K;
        p_off += n;
      }
  h->chunk_start.push_back((int32_t)h->chunks.size());
  h->nnz = a_off;
  h->n_block_points = p_off;
  return "";
}

int64_t elem_size(int prec) { return prec == ELMFB_FP64 ? 8 : (prec == ELMFB_FP32 ? 4 : 2); }

int64_t footprint(elmfb_problem h) {
  const Geo& g = h->geo;
  int64_t b = 0;
  auto add = [&](int64_t n) { b += (n + 255) / 256 * 256; };
  add(h->nnz * elem_size(h->prec));                       // A
  add(h->n_block_points * 8);                             // tpart
  add((int64_t)h->chunks.size() * g.K * 8);               // part
  add(4 * 2 * kRedBlocks * 8);                            // reductions
  add(3 * g.n_rows * 8);                                  // h, u, t
  add(4 * g.n_phi * 8);                                   // v, w, x + W-side
  add(g.n_phi * 2 * 8 + g.n_phi * 8);                     // W, b
  add(h->n_tab * 3 * 8);
  add((int64_t)h->blocks.size() * sizeof(DevBlock));
  add((int64_t)(h->tiles.size() + h->chunks.size()) * sizeof(Tile));
  add((int64_t)(h->chunk_start.size() + h->cov.size()) * 4);
  add((int64_t)h->segs.size() * sizeof(AxisSeg));
  add(sizeof(SolveState) + 64);
  return b;
}

template <typename T>
hipError_t dalloc(elmfb_problem h, T** p, int64_t bytes) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, (size_t)(bytes > 0 ? bytes : 16));
  if (e != hipSuccess) return e;
  h->allocs.push_back(q);
  *p = static_cast<T*>(q);
  return hipSuccess;
}

void release(elmfb_problem h) {
  for (auto& kv : h->graphs) hipGraphExecDestroy(kv.second);
  h->graphs.clear();
  for (void* p : h->allocs) hipFree(p);
  h->allocs.clear();
  if (h->ev_in) hipEventDestroy(h->ev_in);
  if (h->ev_out) hipEventDestroy(h->ev_out);
  if (h->stream) hipStreamDestroy(h->stream);
  h->ev_in = h->ev_out = nullptr;
  h->stream = nullptr;
}

const double* state_field(elmfb_problem h, size_t off) {
  return reinterpret_cast<const double*>(reinterpret_cast<const char*>(h->d_state) + off);
}

}  // namespace

extern "C" {

elmfb_status elmfb_define_problem(const elmfb_problem_desc* desc, elmfb_problem* out) {
  if (!out) return fail(nullptr, ELMFB_E_INVALID, "out is NULL");
  *out = nullptr;
  const std::string v = validate(desc);
  if (!v.empty()) return fail(nullptr, ELMFB_E_INVALID, v);
  elmfb_problem h = new (std::nothrow) elmfb_problem_s();
  if (!h) return fail(nullptr, ELMFB_E_NOMEM, "host allocation failed");
  h->desc = *desc;
  h->prec = desc->store_prec;
  const std::string pe = plan(h);
  if (!pe.empty()) {
    delete h;
    return fail(nullptr, ELMFB_E_INVALID, pe);
  }
  h->bytes_device = footprint(h);
  if (const char* cap = std::getenv("ELMFB_MEM_CAP")) {
    const long long c = std::atoll(cap);
    if (c > 0 && h->bytes_device > c) {
      const std::string m = "device footprint " + std::to_string(h->bytes_device) +
                            " B exceeds ELMFB_MEM_CAP";
      delete h;
      return fail(nullptr, ELMFB_E_NOMEM, m);
    }
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    delete h;
    return fail(nullptr, ELMFB_E_DEVICE, "no HIP device available");
  }
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    delete h;
    return fail(nullptr, ELMFB_E_DEVICE, "cannot query the HIP device");
  }
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    const std::string m = std::string("device is ") + prop.gcnArchName + ", need gfx950";
    delete h;
    return fail(nullptr, ELMFB_E_DEVICE, m);
  }
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && (size_t)h->bytes_device > free_b) {
    const std::string m = "device footprint " + std::to_string(h->bytes_device) +
                          " B exceeds free memory " + std::to_string(free_b) + " B";
    delete h;
    return fail(nullptr, ELMFB_E_NOMEM, m);
  }

  const Geo& g = h->geo;
#define ALLOC(p, bytes)                                                     \
  do {                                                                      \
    hipError_t e_ = dalloc(h, &(p), (bytes));                               \
    if (e_ != hipSuccess) {                                                 \
      release(h);                                                           \
      delete h;                                                             \
      return fail(nullptr, ELMFB_E_NOMEM, std::string("hipMalloc: ") +     \
                                              hipGetErrorString(e_));      \
    }                                                                       \
  } while (0)
  ALLOC(h->d_A, h->nnz * elem_size(h->prec));
  ALLOC(h->d_tpart, h->n_block_points * 8);
  ALLOC(h->d_part, (int64_t)h->chunks.size() * g.K * 8);
  ALLOC(h->d_red, 4 * 2 * kRedBlocks * 8);
  ALLOC(h->d_h, g.n_rows * 8);
  ALLOC(h->d_u, g.n_rows * 8);
  ALLOC(h->d_t, g.n_rows * 8);
  ALLOC(h->d_v, g.n_phi * 8);
  ALLOC(h->d_w, g.n_phi * 8);
  ALLOC(h->d_x, g.n_phi * 8);
  ALLOC(h->d_W, g.n_phi * 2 * 8);
  ALLOC(h->d_b, g.n_phi * 8);
  ALLOC(h->d_tab, h->n_tab * 3 * 8);
  ALLOC(h->d_blocks, (int64_t)h->blocks.size() * sizeof(DevBlock));
  ALLOC(h->d_tiles, (int64_t)h->tiles.size() * sizeof(Tile));
  ALLOC(h->d_chunks, (int64_t)h->chunks.size() * sizeof(Tile));
  ALLOC(h->d_cstart, (int64_t)h->chunk_start.size() * 4);
  ALLOC(h->d_cov, (int64_t)h->cov.size() * 4);
  ALLOC(h->d_segs, (int64_t)h->segs.size() * sizeof(AxisSeg));
  ALLOC(h->d_state, sizeof(SolveState));
  ALLOC(h->d_scalar, 64);
  ALLOC(h->d_flag, 64);
#undef ALLOC

  // W padded to two columns
  std::vector<double> W2((size_t)g.n_phi * 2, 0.0);
  for (int64_t q = 0; q < g.n_phi; ++q)
    for (int a = 0; a < desc->dim; ++a) W2[2 * q + a] = desc->W_host[q * desc->dim + a];
  for (int64_t q = 0; q < g.n_phi * desc->dim; ++q)
    if (!std::isfinite(desc->W_host[q])) { elmfb_destroy(h); return fail(nullptr, ELMFB_E_NUMERIC, "W has non-finite values"); }
  for (int64_t q = 0; q < g.n_phi; ++q)
    if (!std::isfinite(desc->b_host[q])) { elmfb_destroy(h); return fail(nullptr, ELMFB_E_NUMERIC, "b has non-finite values"); }

#define H2D(dst, src, bytes)                                                          \
  do {                                                                                \
    hipError_t e_ = hipMemcpy((dst), (src), (size_t)(bytes), hipMemcpyHostToDevice);  \
    if (e_ != hipSuccess) {                                                           \
      elmfb_destroy(h);                                                               \
      return fail(nullptr, ELMFB_E_DEVICE, std::string("hipMemcpy: ") +              \
                                               hipGetErrorString(e_));               \
    }                                                                                 \
  } while (0)
  H2D(h->d_W, W2.data(), W2.size() * 8);
  H2D(h->d_b, desc->b_host, g.n_phi * 8);
  if (!h->blocks.empty()) H2D(h->d_blocks, h->blocks.data(), h->blocks.size() * sizeof(DevBlock));
  if (!h->tiles.empty()) H2D(h->d_tiles, h->tiles.data(), h->tiles.size() * sizeof(Tile));
  if (!h->chunks.empty()) H2D(h->d_chunks, h->chunks.data(), h->chunks.size() * sizeof(Tile));
  H2D(h->d_cstart, h->chunk_start.data(), h->chunk_start.size() * 4);
  if (!h->cov.empty()) H2D(h->d_cov, h->cov.data(), h->cov.size() * 4);
  if (!h->segs.empty()) H2D(h->d_segs, h->segs.data(), h->segs.size() * sizeof(AxisSeg));
#undef H2D
  h->desc.W_host = nullptr;
  h->desc.b_host = nullptr;

  if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_out, hipEventDisableTiming) != hipSuccess) {
    elmfb_destroy(h);
    return fail(nullptr, ELMFB_E_DEVICE, "stream/event creation failed");
  }
  // envelope tables depend only on the geometry: build them once here
  hipError_t e = launch_axis_tables(g, h->d_segs, (int)h->segs.size(), h->d_cov, h->d_tab, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    const std::string m = std::string("axis tables: ") + hipGetErrorString(e);
    elmfb_destroy(h);
    return fail(nullptr, ELMFB_E_DEVICE, m);
  }
  *out = h;
  return ELMFB_OK;
}

elmfb_status elmfb_query(elmfb_problem h, elmfb_sizes* out) {
  if (!h || !out) return fail(h, ELMFB_E_INVALID, "NULL argument");
  out->n_rows = h->geo.n_rows;
  out->n_phi = h->geo.n_phi;
  out->nnz = h->nnz;
  out->n_blocks = h->geo.n_blocks;
  out->n_block_points = h->n_block_points;
  out->bytes_device = h->bytes_device;
  return ELMFB_OK;
}

elmfb_status elmfb_points(elmfb_problem h, double* xy_dev, void* stream) {
  if (!h || !xy_dev) return fail(h, ELMFB_E_INVALID, "NULL argument");
  HIP_OR_FAIL(h, launch_points(h->geo, xy_dev, (hipStream_t)stream));
  return ELMFB_OK;
}

elmfb_status elmfb_assemble(elmfb_problem h, const double* f_dev, void* stream) {
  if (!h || !f_dev) return fail(h, ELMFB_E_INVALID, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  const Geo& g = h->geo;
  HIP_OR_FAIL(h, hipMemsetAsync(h->d_flag, 0, 4, s));
  HIP_OR_FAIL(h, launch_rhs(g, f_dev, h->d_h, h->d_flag, s));
  HIP_OR_FAIL(h, launch_assemble(g, h->prec, h->d_blocks, h->d_tiles, (int64_t)h->tiles.size(),
                                 h->d_tab, h->d_W, h->d_b, h->d_A, s));
  int32_t bad = 0;
  HIP_OR_FAIL(h, hipMemcpyAsync(&bad, h->d_flag, 4, hipMemcpyDeviceToHost, s));
  HIP_OR_FAIL(h, hipStreamSynchronize(s));
  if (bad) {
    h->assembled = false;
    return fail(h, ELMFB_E_NUMERIC, "f holds non-finite values");
  }
  h->assembled = true;
  h->anorm_f = -1.0;
  return ELMFB_OK;
}

elmfb_status elmfb_matvec(elmfb_problem h, const double* v_dev, double* y_dev, void* stream) {
  if (!h || !v_dev || !y_dev) return fail(h, ELMFB_E_INVALID, "NULL argument");
  if (!h->assembled) return fail(h, ELMFB_E_STATE, "matvec before assemble");
  hipStream_t s = (hipStream_t)stream;
  const Geo& g = h->geo;
  HIP_OR_FAIL(h, launch_mv_blocks(g, h->prec, h->d_blocks, h->d_tiles, (int64_t)h->tiles.size(),
                                  h->d_A, v_dev, nullptr, h->d_tpart, nullptr, s));
  HIP_OR_FAIL(h, launch_gather_rows(g, h->d_blocks, h->d_cov, h->d_tpart, ROW_STORE, y_dev,
                                    nullptr, nullptr, h->d_red, rows_wg(g), s));
  return ELMFB_OK;
}

elmfb_status elmfb_rmatvec(elmfb_problem h, const double* u_dev, double* x_dev, void* stream) {
  if (!h || !u_dev || !x_dev) return fail(h, ELMFB_E_INVALID, "NULL argument");
  if (!h->assembled) return fail(h, ELMFB_E_STATE, "rmatvec before assemble");
  hipStream_t s = (hipStream_t)stream;
  const Geo& g = h->geo;
  HIP_OR_FAIL(h, launch_rmv_chunks(g, h->prec, h->d_blocks, h->d_chunks,
                                   (int64_t)h->chunks.size(), h->d_A, u_dev, nullptr, h->d_part,
                                   nullptr, s));
  HIP_OR_FAIL(h, launch_rmv_finish(g, h->d_cstart, h->d_part, COL_STORE, x_dev, nullptr,
                                   h->d_red, cols_wg(g), s));
  return ELMFB_OK;
}

elmfb_status elmfb_copy_rhs(elmfb_problem h, double* h_dev, void* stream) {
  if (!h || !h_dev) return fail(h, ELMFB_E_INVALID, "NULL argument");
  if (!h->assembled) return fail(h, ELMFB_E_STATE, "copy_rhs before assemble");
  HIP_OR_FAIL(h, hipMemcpyAsync(h_dev, h->d_h, (size_t)h->geo.n_rows * 8,
                                hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return ELMFB_OK;
}

elmfb_status elmfb_copy_blocks(elmfb_problem h, void* dst_dev, int64_t* table_host,
                               void* stream) {
  if (!h) return fail(h, ELMFB_E_INVALID, "NULL handle");
  if (table_host) {
    for (size_t b = 0; b < h->blocks.size(); ++b) {
      const DevBlock& B = h->blocks[b];
      int64_t* t = table_host + 8 * b;
      t[0] = B.level;
      t[1] = (b - (size_t)h->geo.bbase[B.level]) / h->geo.J[B.level][1];
      t[2] = (b - (size_t)h->geo.bbase[B.level]) % h->geo.J[B.level][1];
      t[3] = B.ix0; t[4] = B.nx; t[5] = B.iy0; t[6] = B.ny; t[7] = B.a_off;
    }
  }
  if (dst_dev) {
    if (!h->assembled) return fail(h, ELMFB_E_STATE, "copy_blocks before assemble");
    HIP_OR_FAIL(h, hipMemcpyAsync(dst_dev, h->d_A, (size_t)(h->nnz * elem_size(h->prec)),
                                  hipMemcpyDeviceToDevice, (hipStream_t)stream));
  }
  return ELMFB_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------- solve drivers
namespace {

hipError_t lsqr_iteration(elmfb_problem h, hipStream_t s) {
  const Geo& g = h->geo;
  SolveState* st = h->d_state;
  double* red1 = h->d_red;
  double* red2 = h->d_red + 2 * kRedBlocks;
  double* red3 = h->d_red + 4 * kRedBlocks;
  const int rw = rows_wg(g), cw = cols_wg(g);
  hipError_t e;
  if ((e = launch_mv_blocks(g, h->prec, h->d_blocks, h->d_tiles, (int64_t)h->tiles.size(), h->d_A,
                            h->d_v, state_field(h, offsetof(SolveState, sv)), h->d_tpart, st, s)))
    return e;
  if ((e = launch_gather_rows(g, h->d_blocks, h->d_cov, h->d_tpart, ROW_LSQR_U, h->d_u, nullptr,
                              st, red1, rw, s)))
    return e;
  if ((e = launch_lsqr_beta(st, red1, rw, s))) return e;
  if ((e = launch_rmv_chunks(g, h->prec, h->d_blocks, h->d_chunks, (int64_t)h->chunks.size(),
                             h->d_A, h->d_u, state_field(h, offsetof(SolveState, su)), h->d_part,
                             st, s)))
    return e;
  if ((e = launch_rmv_finish(g, h->d_cstart, h->d_part, COL_LSQR_V, h->d_v, st, red2, cw, s)))
    return e;
  if ((e = launch_lsqr_alpha(st, red2, cw, s))) return e;
  if ((e = launch_lsqr_update(g, h->d_x, h->d_w, h->d_v, st, red3, cw, s))) return e;
  return launch_lsqr_stop(st, red3, cw, s);
}

hipError_t cgls_iteration(elmfb_problem h, hipStream_t s) {
  const Geo& g = h->geo;
  SolveState* st = h->d_state;
  double* red1 = h->d_red;
  double* red2 = h->d_red + 2 * kRedBlocks;
  double* red3 = h->d_red + 4 * kRedBlocks;
  const int rw = rows_wg(g), cw = cols_wg(g);
  hipError_t e;
  // t = A p
  if ((e = launch_mv_blocks(g, h->prec, h->d_blocks, h->d_tiles, (int64_t)h->tiles.size(), h->d_A,
                            h->d_w, nullptr, h->d_tpart, st, s)))
    return e;
  if ((e = launch_gather_rows(g, h->d_blocks, h->d_cov, h->d_tpart, ROW_STORE_SQ, h->d_t, nullptr,
                              st, red1, rw, s)))
    return e;
  if ((e = launch_cgls_step_a(st, red1, rw, s))) return e;
  if ((e = launch_cgls_update_x(g, h->d_x, h->d_w, st, s))) return e;
  if ((e = launch_cgls_update_r(g, h->d_u, h->d_t, st, red2, rw, s))) return e;
  // s = A^T r
  if ((e = launch_rmv_chunks(g, h->prec, h->d_blocks, h->d_chunks, (int64_t)h->chunks.size(),
                             h->d_A, h->d_u, nullptr, h->d_part, st, s)))
    return e;
  if ((e = launch_rmv_finish(g, h->d_cstart, h->d_part, COL_STORE_SQ, h->d_v, st, red3, cw, s)))
    return e;
  if ((e = launch_cgls_step_b(st, red2, rw, red3, cw, s))) return e;
  return launch_cgls_update_p(g, h->d_w, h->d_v, st, s);
}

hipError_t solve_init(elmfb_problem h, int method, const double* x0, hipStream_t s) {
  const Geo& g = h->geo;
  double* red1 = h->d_red;
  double* red2 = h->d_red + 2 * kRedBlocks;
  double* red3 = h->d_red + 4 * kRedBlocks;
  double* red4 = h->d_red + 6 * kRedBlocks;
  const int rw = rows_wg(g), cw = cols_wg(g);
  hipError_t e;
  // u (LSQR) or r (CGLS) = h - A x0
  if (x0) {
    if ((e = launch_mv_blocks(g, h->prec, h->d_blocks, h->d_tiles, (int64_t)h->tiles.size(),
                              h->d_A, x0, nullptr, h->d_tpart, nullptr, s)))
      return e;
    if ((e = launch_gather_rows(g, h->d_blocks, h->d_cov, h->d_tpart, ROW_RESID, h->d_u, h->d_h,
                                nullptr, red2, rw, s)))
      return e;
  } else {
    if ((e = launch_copy(h->d_h, h->d_u, g.n_rows, s))) return e;
    if ((e = launch_sumsq(h->d_u, g.n_rows, red2, rw, s))) return e;
  }
  if ((e = launch_sumsq(h->d_h, g.n_rows, red1, rw, s))) return e;
  if (method == ELMFB_LSQR) {
    if ((e = launch_lsqr_init(h->d_state, red1, rw, red2, rw, s))) return e;
    if ((e = launch_rmv_chunks(g, h->prec, h->d_blocks, h->d_chunks, (int64_t)h->chunks.size(),
                               h->d_A, h->d_u, state_field(h, offsetof(SolveState, su)),
                               h->d_part, nullptr, s)))
      return e;
    if ((e = launch_rmv_finish(g, h->d_cstart, h->d_part, COL_STORE_SQ, h->d_v, nullptr, red3, cw,
                               s)))
      return e;
    if ((e = launch_lsqr_init_alpha(h->d_state, red3, cw, s))) return e;
    return launch_init_xw(g, x0, h->d_x, h->d_w, h->d_v, h->d_state, s);
  }
  // CGLS: s = A^T r, p = s, x = x0
  if ((e = launch_rmv_chunks(g, h->prec, h->d_blocks, h->d_chunks, (int64_t)h->chunks.size(),
                             h->d_A, h->d_u, nullptr, h->d_part, nullptr, s)))
    return e;
  if ((e = launch_rmv_finish(g, h->d_cstart, h->d_part, COL_STORE_SQ, h->d_v, nullptr, red3, cw,
                             s)))
    return e;
  (void)red4;
  if ((e = launch_cgls_init(h->d_state, red1, rw, red2, rw, red3, cw, h->anorm_f, s))) return e;
  if ((e = launch_copy(h->d_v, h->d_w, g.n_phi, s))) return e;
  if (x0) return launch_copy(x0, h->d_x, g.n_phi, s);
  return hipMemsetAsync(h->d_x, 0, (size_t)g.n_phi * 8, s);
}

hipError_t enqueue_iterations(elmfb_problem h, int method, int n, hipStream_t s) {
  for (int i = 0; i < n; ++i) {
    hipError_t e = method == ELMFB_LSQR ? lsqr_iteration(h, s) : cgls_iteration(h, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t get_graph(elmfb_problem h, int method, int n, hipGraphExec_t* out) {
  auto key = std::make_pair(method, n);
  auto it = h->graphs.find(key);
  if (it != h->graphs.end()) { *out = it->second; return hipSuccess; }
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  hipError_t e2 = enqueue_iterations(h, method, n, h->stream);
  e = hipStreamEndCapture(h->stream, &graph);
  if (e2 != hipSuccess) { if (graph) hipGraphDestroy(graph); return e2; }
  if (e != hipSuccess) return e;
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (e != hipSuccess) return e;
  h->graphs[key] = exec;
  *out = exec;
  return hipSuccess;
}

}  // namespace

extern "C" {

elmfb_status elmfb_solve(elmfb_problem h, const elmfb_solve_opts* opts, double* coef_dev,
                         elmfb_solve_info* info, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!h || !opts || !coef_dev) return fail(h, ELMFB_E_INVALID, "NULL argument");
  if (!h->assembled) return fail(h, ELMFB_E_STATE, "solve before assemble");
  if (opts->method != ELMFB_LSQR && opts->method != ELMFB_CGLS)
    return fail(h, ELMFB_E_UNSUPPORTED, "unknown solve method");
  if (opts->iter_lim < 0 || opts->check_every < 1 || opts->check_every > 100000)
    return fail(h, ELMFB_E_INVALID, "iter_lim >= 0 and 1 <= check_every <= 100000 required");
  if (!(opts->atol >= 0.0) || !(opts->btol >= 0.0))
    return fail(h, ELMFB_E_INVALID, "atol and btol must be >= 0");
  if (opts->n_check < 0 || (opts->n_check > 0 && (!opts->check_pts_dev || !opts->check_ref_dev)))
    return fail(h, ELMFB_E_INVALID, "check points need check_pts_dev and check_ref_dev");
  const Geo& g = h->geo;
  hipStream_t caller = (hipStream_t)stream;
  hipStream_t s = h->stream;
  HIP_OR_FAIL(h, hipEventRecord(h->ev_in, caller));
  HIP_OR_FAIL(h, hipStreamWaitEvent(s, h->ev_in, 0));

  if (opts->method == ELMFB_CGLS && h->anorm_f < 0.0) {
    const int nw = kRedBlocks;
    HIP_OR_FAIL(h, launch_sumsq_entries(h->prec, h->d_A, h->nnz, h->d_red, nw, s));
    HIP_OR_FAIL(h, launch_reduce_to(h->d_red, nw, h->d_scalar, s));
    double ss = 0.0;
    HIP_OR_FAIL(h, hipMemcpyAsync(&ss, h->d_scalar, 8, hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(h, hipStreamSynchronize(s));
    h->anorm_f = std::sqrt(ss);
  }
  if (opts->n_check > h->eval_cap) {
    if (h->d_eval) {
      for (auto it = h->allocs.begin(); it != h->allocs.end(); ++it)
        if (*it == h->d_eval) { hipFree(*it); h->allocs.erase(it); break; }
      h->d_eval = nullptr;
      h->eval_cap = 0;
    }
    HIP_OR_FAIL(h, dalloc(h, &h->d_eval, opts->n_check * 8));
    h->eval_cap = opts->n_check;
  }

  SolveState init{};
  init.atol = opts->atol;
  init.btol = opts->btol;
  init.iter_lim = opts->iter_lim;
  init.target = opts->n_check > 0 ? opts->target_rel_l2 : 0.0;
  init.rel_l2 = -1.0;
  HIP_OR_FAIL(h, hipMemcpyAsync(h->d_state, &init, sizeof(init), hipMemcpyHostToDevice, s));
  HIP_OR_FAIL(h, solve_init(h, opts->method, opts->x0_dev, s));

  SolveState st{};
  HIP_OR_FAIL(h, hipMemcpyAsync(&st, h->d_state, sizeof(st), hipMemcpyDeviceToHost, s));
  HIP_OR_FAIL(h, hipStreamSynchronize(s));
  const int chunk = opts->check_every;
  while (!st.done) {
    if (opts->use_graph) {
      hipGraphExec_t exec = nullptr;
      HIP_OR_FAIL(h, get_graph(h, opts->method, chunk, &exec));
      HIP_OR_FAIL(h, hipGraphLaunch(exec, s));
    } else {
      HIP_OR_FAIL(h, enqueue_iterations(h, opts->method, chunk, s));
    }
    if (opts->n_check > 0) {
      HIP_OR_FAIL(h, launch_evaluate(g, h->d_W, h->d_b, h->d_x, opts->check_pts_dev,
                                     opts->n_check, h->d_eval, s));
      int nw = (int)((opts->n_check + 255) / 256);
      if (nw > kRedBlocks) nw = kRedBlocks;
      HIP_OR_FAIL(h, launch_check_rel_l2(h->d_eval, opts->check_ref_dev, opts->n_check,
                                         h->d_state, h->d_red + 6 * kRedBlocks, nw, s));
    }
    HIP_OR_FAIL(h, hipMemcpyAsync(&st, h->d_state, sizeof(st), hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(h, hipStreamSynchronize(s));
  }
  HIP_OR_FAIL(h, hipMemcpyAsync(coef_dev, h->d_x, (size_t)g.n_phi * 8, hipMemcpyDeviceToDevice, s));
  HIP_OR_FAIL(h, hipEventRecord(h->ev_out, s));
  HIP_OR_FAIL(h, hipStreamWaitEvent(caller, h->ev_out, 0));
  if (info) {
    info->istop = st.istop;
    info->iters = st.itn;
    info->rnorm = st.rnorm;
    info->arnorm = st.arnorm;
    info->anorm = st.anorm;
    info->xnorm = st.xnorm;
    info->rel_l2 = st.rel_l2;
    info->ms_solve =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return ELMFB_OK;
}

elmfb_status elmfb_evaluate(elmfb_problem h, const double* coef_dev, const double* pts_dev,
                            int64_t n_pts, double* u_dev, void* stream) {
  if (!h || n_pts < 0 || (n_pts > 0 && (!coef_dev || !pts_dev || !u_dev)))
    return fail(h, ELMFB_E_INVALID, "bad argument");
  HIP_OR_FAIL(h, launch_evaluate(h->geo, h->d_W, h->d_b, coef_dev, pts_dev, n_pts, u_dev,
                                 (hipStream_t)stream));
  return ELMFB_OK;
}

elmfb_status elmfb_time_kernels(elmfb_problem h, int32_t reps, double* ms_host, void* stream) {
  if (!h || !ms_host || reps < 1) return fail(h, ELMFB_E_INVALID, "bad argument");
  if (!h->assembled) return fail(h, ELMFB_E_STATE, "time_kernels before assemble");
  hipStream_t s = (hipStream_t)stream;
  const Geo& g = h->geo;
  // v = 1 (in d_x), u = 1 (in d_t)
  std::vector<double> ones((size_t)(g.n_rows > g.n_phi ? g.n_rows : g.n_phi), 1.0);
  HIP_OR_FAIL(h, hipMemcpyAsync(h->d_x, ones.data(), (size_t)g.n_phi * 8, hipMemcpyHostToDevice, s));
  HIP_OR_FAIL(h, hipMemcpyAsync(h->d_t, ones.data(), (size_t)g.n_rows * 8, hipMemcpyHostToDevice, s));
  hipEvent_t e0, e1, e2;
  HIP_OR_FAIL(h, hipEventCreate(&e0));
  HIP_OR_FAIL(h, hipEventCreate(&e1));
  HIP_OR_FAIL(h, hipEventCreate(&e2));
  hipError_t e = hipEventRecord(e0, s);
  for (int i = 0; i < reps && e == hipSuccess; ++i)
    e = launch_mv_blocks(g, h->prec, h->d_blocks, h->d_tiles, (int64_t)h->tiles.size(), h->d_A,
                         h->d_x, nullptr, h->d_tpart, nullptr, s);
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  for (int i = 0; i < reps && e == hipSuccess; ++i)
    e = launch_rmv_chunks(g, h->prec, h->d_blocks, h->d_chunks, (int64_t)h->chunks.size(),
                          h->d_A, h->d_t, nullptr, h->d_part, nullptr, s);
  if (e == hipSuccess) e = hipEventRecord(e2, s);
  if (e == hipSuccess) e = hipEventSynchronize(e2);
  float t01 = 0.f, t12 = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t01, e0, e1);
  if (e == hipSuccess) e = hipEventElapsedTime(&t12, e1, e2);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipEventDestroy(e2);
  HIP_OR_FAIL(h, e);
  ms_host[0] = (double)t01 / reps;
  ms_host[1] = (double)t12 / reps;
  return ELMFB_OK;
}

void elmfb_destroy(elmfb_problem h) {
  if (!h) return;
  if (h->stream) hipStreamSynchronize(h->stream);
  release(h);
  delete h;
}

const char* elmfb_last_error(elmfb_problem h) {
  if (h) return h->err.c_str();
  return g_thread_error.c_str();
}

}  // extern "C"

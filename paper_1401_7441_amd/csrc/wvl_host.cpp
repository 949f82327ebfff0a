// Host side of the C ABI declared in include/wvl.h: argument validation,
// localization-region construction, plans (device copies of the segment
// lists, row tables, workspace layout in chunks) and launch sequencing.
// Built with -ffp-contract=off so that the sphere membership test rounds
// exactly as written.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <new>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <memory>
#include <vector>

#include "wvl_internal.h"

using namespace wvl;

// kernel kinds for tracing
enum KernelKind {
  KK_GATHER, KK_SCATTER, KK_UNPACK, KK_UP_X, KK_UP_Y, KK_POT_COLUMN, KK_KIN_XCOL, KK_KIN_YCOL, KK_KIN_ZCOL,
  KK_BACK_Y, KK_BACK_X, KK_FINALIZE, KK_PATTERN, KK_SPARSE_S, KK_SPARSE_H,
  KK_UPDATE, KK_UP_Z, KK_DENS_TILE, KK_FOE_MM, KK_FOE, KK_GRADIENT, KK_COUNT
};
static const char* kKernelNames[KK_COUNT] = {
    "uncompress", "compress", "unpack", "up_x", "up_y", "pot_column", "kin_xcol", "kin_ycol", "kin_zcol",
    "back_y", "back_x", "finalize", "pattern", "sparse_s", "sparse_h", "update",
    "up_z", "dens_tile", "foe_mm", "foe", "gradient"};

// LDS a block of the fused plane kernels may use (gfx950: 160 KiB per block),
// less what their fixed-order reductions declare statically
static const int64_t kLdsBudget = 160 * 1024 - 1024;

struct wvl_ctx {
  wvl_grid grid;
  hipStream_t stream;
  std::string err;
  bool prof = false;
  struct Rec { int kind; hipEvent_t a, b; };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  int64_t launches[KK_COUNT] = {};
  double ms[KK_COUNT] = {};
};

namespace {

thread_local std::string g_err;

wvl_status fail(wvl_ctx* ctx, wvl_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (ctx)
    ctx->err = buf;
  else
    g_err = buf;
  return st;
}

// WVL_EDEVICE with the failing HIP call (name or expression), its status
// name and its description, after `what` (the operation that needed it)
static wvl_status hip_fail(wvl_ctx* ctx, const char* what, const char* call, hipError_t e) {
  return fail(ctx, WVL_EDEVICE, "%s: %s returned %s (%s)", what, call, hipGetErrorName(e),
              hipGetErrorString(e));
}

#define WVL_HIP(ctx, call)                                                               \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess) return hip_fail(ctx, __func__, #call, e_);                     \
  } while (0)

hipEvent_t take_event(wvl_ctx* ctx) {
  if (!ctx->pool.empty()) {
    hipEvent_t e = ctx->pool.back();
    ctx->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// brackets one launch with events when tracing is on
struct Trace {
  wvl_ctx* ctx;
  int kind;
  hipEvent_t a = nullptr, b = nullptr;
  Trace(wvl_ctx* c, int k) : ctx(c), kind(k) {
    if (ctx->prof) {
      a = take_event(ctx);
      b = take_event(ctx);
      if (a && b) (void)hipEventRecord(a, ctx->stream);
    }
  }
  ~Trace() {
    if (ctx->prof && a && b) {
      (void)hipEventRecord(b, ctx->stream);
      ctx->pending.push_back({kind, a, b});
    } else {
      if (a) ctx->pool.push_back(a);
      if (b) ctx->pool.push_back(b);
    }
  }
};

#define WVL_LAUNCH(ctx, kind, call)                                                      \
  do {                                                                                   \
    int e_;                                                                              \
    {                                                                                    \
      Trace tr_(ctx, kind);                                                              \
      e_ = (call);                                                                       \
    }                                                                                    \
    if (e_ != 0)                                                                         \
      return fail(ctx, WVL_EDEVICE, "launch of %s failed: %s (%s)", kKernelNames[kind],  \
                  hipGetErrorName((hipError_t)e_), hipGetErrorString((hipError_t)e_));   \
  } while (0)

inline int64_t align64(int64_t n) { return (n + 63) & ~int64_t(63); }
inline int64_t align_bytes(int64_t n) { return (n + 255) & ~int64_t(255); }

struct PatternCache {
  bool ready = false;
  int64_t nnz = 0;
  int64_t* d_rowptr = nullptr;
  int32_t* d_col = nullptr;
  int32_t* d_row = nullptr;
  int32_t* d_order = nullptr;   // processing order of the pairs (CSR positions)
  // S pattern, bra = ket: the pairs a <= b in processing order, and for each
  // the position of (b, a) (-1 on the diagonal); empty when not symmetric
  int32_t* d_order_u = nullptr;
  int32_t* d_mirror_u = nullptr;
  int64_t nnz_u = 0;
  // S pattern only (Fermi operator expansion): position of the transposed
  // entry, and of the entry and its transpose in the H pattern
  int64_t* d_tpos = nullptr;
  int64_t* d_hpos = nullptr;
  int64_t* d_htpos = nullptr;
  int64_t* d_dpos = nullptr;    // diagonal entry of every row
  int32_t* d_foe_rows = nullptr;   // rows by decreasing product work
  int maxdeg = 0;               // longest row
};

// 3D Morton code of a non-negative grid point (10 bits per axis)
inline uint32_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  auto spread = [](uint32_t v) {
    v &= 0x3ff;
    v = (v | (v << 16)) & 0x030000ff;
    v = (v | (v << 8)) & 0x0300f00f;
    v = (v | (v << 4)) & 0x030c30c3;
    v = (v | (v << 2)) & 0x09249249;
    return v;
  };
  return spread(x) | (spread(y) << 1) | (spread(z) << 2);
}

}  // namespace

// Workspace layout of a plan: the functions in processing order (sorted by
// box volume, largest first), cut into `nbins` bins of equal count; a bin is
// split further into chunks when a workspace bound is given.  Without a
// bound every chunk has its own workspace region (chunks are independent and
// may run concurrently); with one, chunks reuse the region one after the
// other.
struct Layout {
  std::vector<ChunkDev> chunks;
  std::vector<SfWork> wk;        // per position of the processing order
  bool disjoint = true;
  int nbins = 1;
  bool zmfma = false;            // z part of the kinetic term on the matrix cores
  int64_t elems_span = 0;        // elements of the compute type before the partials
  int64_t parts_span = 0;        // doubles of energy partials
  int64_t bytes(int sz) const { return align_bytes(elems_span * sz) + parts_span * 8; }
};

struct wvl_graph {
  wvl_plan* plan = nullptr;
  int64_t layout_version = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<hipEvent_t> events;   // fork/join events of the capture, kept with the graph
};

// Chebyshev coefficients c_0..c_npl on [-1, 1] of
// f(x) = erfc((x / sigma + tau - mu) / delta) / 2, by the defining integral
// c_i = (2 / pi) int_0^pi f(cos t) cos(i t) dt on m midpoints (exact for the
// cosine series up to degree 2m - 1).  The node table is kept with the plan.
struct FoeCoef {
  int npl, m;
  std::vector<double> x, cs;   // nodes cos t_k; cos(i t_k), [k][i]
  explicit FoeCoef(int npl_) : npl(npl_), m(std::max(8 * npl_, 2048)) {
    const double pi = 3.14159265358979323846;
    x.resize(m);
    cs.resize((size_t)m * (npl + 1));
    for (int k = 0; k < m; ++k) {
      const double t = pi * (k + 0.5) / m;
      x[k] = std::cos(t);
      for (int i = 0; i <= npl; ++i) cs[(size_t)k * (npl + 1) + i] = std::cos(i * t);
    }
  }
  // erfc(z) rounds to 2 for z <= -6 and to 0 for z >= 28 in double, so the
  // call is needed only in between (most nodes lie outside when delta is
  // small against the spectral range)
  double f(int k, double sigma, double tau, double mu, double delta) const {
    const double z = (x[k] / sigma + tau - mu) / delta;
    if (z <= -6.0) return 1.0;
    if (z >= 28.0) return 0.0;
    return 0.5 * std::erfc(z);
  }
  void operator()(double sigma, double tau, double mu, double delta,
                  std::vector<double>* c) const {
    c->assign(npl + 1, 0.0);
    for (int k = 0; k < m; ++k) {
      const double fk = f(k, sigma, tau, mu, delta);
      const double* row = &cs[(size_t)k * (npl + 1)];
      for (int i = 0; i <= npl; ++i) (*c)[i] += fk * row[i];
    }
    for (int i = 0; i <= npl; ++i) (*c)[i] *= 2.0 / m;
  }
  // c_0 / 2 tr_0 + sum_i c_i tr_i = (2 / m) sum_k f(x_k) g_k with
  // g_k = tr_0 / 2 + sum_i cos(i t_k) tr_i: the node weights of the traces
  void weights(const std::vector<double>& tr, std::vector<double>* g) const {
    g->resize(m);
    for (int k = 0; k < m; ++k) {
      const double* row = &cs[(size_t)k * (npl + 1)];
      double v = 0.5 * row[0] * tr[0];
      for (int i = 1; i <= npl; ++i) v += row[i] * tr[i];
      (*g)[k] = v;
    }
  }
  double trace(const std::vector<double>& g, double sigma, double tau, double mu,
               double delta) const {
    double v = 0.0;
    for (int k = 0; k < m; ++k) v += f(k, sigma, tau, mu, delta) * g[k];
    return v * (2.0 / m);
  }
};

struct wvl_plan {
  wvl_ctx* ctx = nullptr;
  int nsf = 0;
  std::vector<SfDev> h_sf;
  std::vector<int32_t> order;         // processing position -> function index
  size_t max_ws = 0;                  // the caller's workspace bound (0: none)
  Layout lay;
  int64_t ws_cap[2] = {0, 0};         // workspace bytes reported (F32, F64)
  std::vector<hipStream_t> streams;   // branch streams of captured graphs
  int64_t layout_version = 0;         // bumped when the autotuner changes the layout
  bool in_sub_out = false;            // input patterns inside output patterns (wvl_update)
  int64_t max_in_segs = 0;            // largest input segment count of a function
  SfDev* d_sf = nullptr;
  wvl_seg* d_seg = nullptr;
  int32_t* d_rt = nullptr;
  RowRun* d_rr = nullptr;
  SfWork* d_wk = nullptr;
  int64_t* d_foff = nullptr;          // fine-box offsets (wvl_synthesize), function order
  int64_t max_fine = 0;               // largest fine box (elements)
  int64_t* d_cptr = nullptr;          // density: functions meeting each k_dens_tile tile
  int32_t* d_csf = nullptr;
  int32_t* d_tord[2] = {nullptr, nullptr};   // tiles, one-chunk ones first (FP32, FP64)
  int64_t dens_one[2] = {0, 0};              // how many of them have one chunk
  wvl_plan_info info{};
  PatternCache pat[2];
  std::unique_ptr<FoeCoef> foe_coef;  // Chebyshev node table of the last wvl_foe degree
};

namespace {

// --------------------------------------------------------------------------
// validation
// --------------------------------------------------------------------------

int64_t seg_len(const wvl_seg& s) { return (int64_t)s.i1e - s.i1s + 1; }

// checks one segment list: sorted, disjoint, inside [blo, bhi] box and the
// grid, offsets = running sums; returns total length or -1
int64_t check_list(wvl_ctx* ctx, wvl_status* st, int k, const char* name, const wvl_seg* segs,
                   int64_t nsegs, int64_t first, int64_t count, const int* blo, const int* bhi,
                   const int32_t* gn) {
  if (first < 0 || count < 0 || first > nsegs || count > nsegs - first) {
    *st = fail(ctx, WVL_EINVAL, "function %d: %s segment range [%lld, +%lld) outside [0, %lld)", k,
               name, (long long)first, (long long)count, (long long)nsegs);
    return -1;
  }
  int64_t total = 0;
  for (int64_t q = 0; q < count; ++q) {
    const wvl_seg& s = segs[first + q];
    if (s.i1s > s.i1e) {
      *st = fail(ctx, WVL_EINVAL, "function %d: %s segment %lld has i1s > i1e", k, name,
                 (long long)(first + q));
      return -1;
    }
    if (s.i1s < blo[0] || s.i1e > bhi[0] || s.i2 < blo[1] || s.i2 > bhi[1] || s.i3 < blo[2] ||
        s.i3 > bhi[2] || s.i1s < 0 || s.i1e >= gn[0] || s.i2 < 0 || s.i2 >= gn[1] || s.i3 < 0 ||
        s.i3 >= gn[2]) {
      *st = fail(ctx, WVL_EINVAL, "function %d: %s segment %lld lies outside its box or the grid",
                 k, name, (long long)(first + q));
      return -1;
    }
    if (q > 0) {
      const wvl_seg& p = segs[first + q - 1];
      const bool later_row = s.i3 > p.i3 || (s.i3 == p.i3 && s.i2 > p.i2);
      const bool same_row_after = s.i3 == p.i3 && s.i2 == p.i2 && s.i1s > p.i1e;
      if (!later_row && !same_row_after) {
        *st = fail(ctx, WVL_EINVAL,
                   "function %d: %s segment %lld not sorted by (i3, i2, i1) or overlaps the one "
                   "before",
                   k, name, (long long)(first + q));
        return -1;
      }
    }
    if (s.off != total) {
      *st = fail(ctx, WVL_EINVAL,
                 "function %d: %s segment %lld has off %lld, expected running sum %lld", k, name,
                 (long long)(first + q), (long long)s.off, (long long)total);
      return -1;
    }
    total += seg_len(s);
  }
  return total;
}

// every fine segment inside a coarse segment of the same row
bool fine_in_coarse(const wvl_seg* segs, int64_t c0, int64_t nc, int64_t f0, int64_t nf,
                    int64_t* bad) {
  int64_t q = 0;
  for (int64_t r = 0; r < nf; ++r) {
    const wvl_seg& f = segs[f0 + r];
    while (q < nc) {
      const wvl_seg& c = segs[c0 + q];
      if (c.i3 < f.i3 || (c.i3 == f.i3 && c.i2 < f.i2) ||
          (c.i3 == f.i3 && c.i2 == f.i2 && c.i1e < f.i1s))
        ++q;
      else
        break;
    }
    if (q >= nc) {
      *bad = f0 + r;
      return false;
    }
    const wvl_seg& c = segs[c0 + q];
    if (!(c.i3 == f.i3 && c.i2 == f.i2 && c.i1s <= f.i1s && f.i1e <= c.i1e)) {
      *bad = f0 + r;
      return false;
    }
  }
  return true;
}

void bbox(const wvl_seg* segs, int64_t first, int64_t count, int32_t* bb) {
  bb[0] = bb[2] = bb[4] = 1 << 30;
  bb[1] = bb[3] = bb[5] = -(1 << 30);
  for (int64_t q = 0; q < count; ++q) {
    const wvl_seg& s = segs[first + q];
    bb[0] = std::min(bb[0], s.i1s);
    bb[1] = std::max(bb[1], s.i1e);
    bb[2] = std::min(bb[2], s.i2);
    bb[3] = std::max(bb[3], s.i2);
    bb[4] = std::min(bb[4], s.i3);
    bb[5] = std::max(bb[5], s.i3);
  }
}

// row table of one pattern: rt[r] .. rt[r+1] are the global segment indices
// of box row r = (i3 - oz) * by + (i2 - oy)
// compact per-row runs of one pattern over its box rows (see RowRun)
void row_runs(const wvl_seg* segs, int64_t first, int64_t count, int oy, int oz, int by, int bz,
              std::vector<RowRun>& rr) {
  const size_t base = rr.size();
  rr.resize(base + (size_t)by * bz, RowRun{0, 0, 0});
  for (int64_t q = 0; q < count; ++q) {
    const wvl_seg& s = segs[first + q];
    RowRun& r = rr[base + (size_t)(s.i3 - oz) * by + (s.i2 - oy)];
    if (r.len == 0) {
      r.x0 = (uint16_t)s.i1s;
      r.len = (uint16_t)(s.i1e - s.i1s + 1);
      r.off = (int32_t)s.off;
    } else {
      r.len = kMultiRun;
    }
  }
}

void row_table(const wvl_seg* segs, int64_t first, int64_t count, int ox, int oy, int oz, int by,
               int bz, std::vector<int32_t>& rt) {
  (void)ox;
  const int64_t nrows = (int64_t)by * bz;
  const size_t base = rt.size();
  rt.resize(base + nrows + 1, 0);
  std::vector<int32_t> cnt(nrows, 0);
  for (int64_t q = 0; q < count; ++q) {
    const wvl_seg& s = segs[first + q];
    cnt[(int64_t)(s.i3 - oz) * by + (s.i2 - oy)]++;
  }
  int32_t run = (int32_t)first;
  for (int64_t r = 0; r < nrows; ++r) {
    rt[base + r] = run;
    run += cnt[r];
  }
  rt[base + nrows] = run;
}

template <typename P>
wvl_status upload(wvl_ctx* ctx, P** dst, const void* src, size_t bytes) {
  *dst = nullptr;
  if (bytes == 0) return WVL_OK;
  hipError_t e = hipMalloc((void**)dst, bytes);
  if (e != hipSuccess) {
    *dst = nullptr;
    return fail(ctx, WVL_ENOMEM, "hipMalloc(%zu) returned %s (%s)", bytes, hipGetErrorName(e),
                hipGetErrorString(e));
  }
  WVL_HIP(ctx, hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, ctx->stream));
  return WVL_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// public entry points
// ---------------------------------------------------------------------------

extern "C" {

const char* wvl_last_error(const wvl_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_err.c_str();
}

wvl_status wvl_build_locregs(const wvl_grid* grid, int32_t nsf, const double* centers,
                             const double* radii, const double* fine_radii, int32_t ext,
                             wvl_locreg* lr, wvl_seg* segs, int64_t* nsegs) {
  if (!grid || !nsegs || nsf < 0 || (nsf > 0 && (!centers || !radii || !fine_radii || !lr)))
    return fail(nullptr, WVL_EINVAL, "wvl_build_locregs: null argument or nsf < 0");
  const double h = grid->h;
  const int32_t* gn = grid->n;
  if (!(h > 0) || gn[0] <= 0 || gn[1] <= 0 || gn[2] <= 0 || ext < 0 || ext > 16)
    return fail(nullptr, WVL_EINVAL, "wvl_build_locregs: bad grid or ext");
  // Three phases: (A, parallel over functions) input box and masks, and the
  // global fine union F as one bit per grid point; (B, parallel) output
  // masks and the four segment lists of each function; (C, sequential)
  // global segment indices and coefficient offsets.  The result does not
  // depend on the number of threads.
  struct Sf {
    int lo[3], hi[3], olo[3];
    int err = 0;                       // 1 negative radius, 2 empty region
    std::vector<uint8_t> m, f;         // coarse / fine masks over the box [z][y][x]
    std::vector<wvl_seg> seg[4];       // in-coarse, in-fine, out-coarse, out-fine
    int64_t tot[4] = {0, 0, 0, 0};
  };
  std::vector<Sf> sfs(nsf);
  const int64_t ngrid = (int64_t)gn[0] * gn[1] * gn[2];
  std::vector<uint64_t> Fbits((size_t)((ngrid + 63) >> 6), 0);
  auto inside = [&](const double* c, double r, int i1, int i2, int i3) {
    const double dx = h * (double)i1 - c[0];
    const double dy = h * (double)i2 - c[1];
    const double dz = h * (double)i3 - c[2];
    const double d2 = (dx * dx + dy * dy) + dz * dz;
    return d2 <= r * r;
  };
#pragma omp parallel for schedule(dynamic, 4)
  for (int k = 0; k < nsf; ++k) {
    Sf& b = sfs[k];
    const double* c = centers + 3 * k;
    const double R = radii[k];
    if (!(R >= 0) || !(fine_radii[k] >= 0)) {
      b.err = 1;
      continue;
    }
    int clo[3], chi[3];
    for (int a = 0; a < 3; ++a) {
      clo[a] = std::max(0, (int)std::floor((c[a] - R) / h) - 1);
      chi[a] = std::min(gn[a] - 1, (int)std::ceil((c[a] + R) / h) + 1);
    }
    int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-1, -1, -1};
    for (int i3 = clo[2]; i3 <= chi[2]; ++i3)
      for (int i2 = clo[1]; i2 <= chi[1]; ++i2)
        for (int i1 = clo[0]; i1 <= chi[0]; ++i1)
          if (inside(c, R, i1, i2, i3)) {
            lo[0] = std::min(lo[0], i1); hi[0] = std::max(hi[0], i1);
            lo[1] = std::min(lo[1], i2); hi[1] = std::max(hi[1], i2);
            lo[2] = std::min(lo[2], i3); hi[2] = std::max(hi[2], i3);
          }
    if (hi[0] < 0) {
      b.err = 2;
      continue;
    }
    std::copy(lo, lo + 3, b.lo);
    std::copy(hi, hi + 3, b.hi);
    const int n0 = hi[0] - lo[0] + 1, n1 = hi[1] - lo[1] + 1, n2 = hi[2] - lo[2] + 1;
    b.m.assign((size_t)n0 * n1 * n2, 0);
    b.f.assign((size_t)n0 * n1 * n2, 0);
    for (int i3 = lo[2]; i3 <= hi[2]; ++i3)
      for (int i2 = lo[1]; i2 <= hi[1]; ++i2)
        for (int i1 = lo[0]; i1 <= hi[0]; ++i1) {
          const size_t p = ((size_t)(i3 - lo[2]) * n1 + (i2 - lo[1])) * n0 + (i1 - lo[0]);
          if (inside(c, R, i1, i2, i3)) {
            b.m[p] = 1;
            if (inside(c, fine_radii[k], i1, i2, i3)) {
              b.f[p] = 1;
              const int64_t key = ((int64_t)i3 * gn[1] + i2) * gn[0] + i1;
              __atomic_fetch_or(&Fbits[(size_t)(key >> 6)], uint64_t(1) << (key & 63),
                                __ATOMIC_RELAXED);
            }
          }
        }
  }
  for (int k = 0; k < nsf; ++k) {
    if (sfs[k].err == 1) return fail(nullptr, WVL_EINVAL, "function %d: negative radius", k);
    if (sfs[k].err == 2)
      return fail(nullptr, WVL_EINVAL, "function %d: empty localization region", k);
  }
  auto inF = [&](int i1, int i2, int i3) {
    const int64_t key = ((int64_t)i3 * gn[1] + i2) * gn[0] + i1;
    return (Fbits[(size_t)(key >> 6)] >> (key & 63)) & 1;
  };
  // maximal runs of a mask over a box at origin olo, rows (z, y) in order
  auto runs = [](const std::vector<uint8_t>& m, const int* olo, int n0, int n1, int n2,
                 std::vector<wvl_seg>* out) {
    int64_t off = 0;
    for (int z = 0; z < n2; ++z)
      for (int y = 0; y < n1; ++y) {
        const uint8_t* row = m.data() + ((size_t)z * n1 + y) * n0;
        int x = 0;
        while (x < n0) {
          if (row[x]) {
            const int x0 = x;
            while (x < n0 && row[x]) ++x;
            out->push_back(wvl_seg{olo[0] + x0, olo[0] + x - 1, olo[1] + y, olo[2] + z, off});
            off += x - x0;
          } else {
            ++x;
          }
        }
      }
    return off;
  };
#pragma omp parallel for schedule(dynamic, 4)
  for (int k = 0; k < nsf; ++k) {
    Sf& b = sfs[k];
    const double* c = centers + 3 * k;
    const int n0 = b.hi[0] - b.lo[0] + 1, n1 = b.hi[1] - b.lo[1] + 1, n2 = b.hi[2] - b.lo[2] + 1;
    b.tot[0] = runs(b.m, b.lo, n0, n1, n2, &b.seg[0]);
    b.tot[1] = runs(b.f, b.lo, n0, n1, n2, &b.seg[1]);
    std::vector<uint8_t>().swap(b.m);
    std::vector<uint8_t>().swap(b.f);
    // output pattern over the grown box, clipped to the grid
    int ohi[3];
    for (int a = 0; a < 3; ++a) {
      b.olo[a] = std::max(0, b.lo[a] - ext);
      ohi[a] = std::min(gn[a] - 1, b.hi[a] + ext);
    }
    const int m0 = ohi[0] - b.olo[0] + 1, m1 = ohi[1] - b.olo[1] + 1, m2 = ohi[2] - b.olo[2] + 1;
    std::vector<uint8_t> om((size_t)m0 * m1 * m2, 0), of((size_t)m0 * m1 * m2, 0);
    const double Rp = radii[k] + ext * h;
    for (int i3 = b.olo[2]; i3 <= ohi[2]; ++i3)
      for (int i2 = b.olo[1]; i2 <= ohi[1]; ++i2)
        for (int i1 = b.olo[0]; i1 <= ohi[0]; ++i1)
          if (inside(c, Rp, i1, i2, i3)) {
            const size_t p = ((size_t)(i3 - b.olo[2]) * m1 + (i2 - b.olo[1])) * m0 + (i1 - b.olo[0]);
            om[p] = 1;
            if (inF(i1, i2, i3)) of[p] = 1;
          }
    b.tot[2] = runs(om, b.olo, m0, m1, m2, &b.seg[2]);
    b.tot[3] = runs(of, b.olo, m0, m1, m2, &b.seg[3]);
  }
  // global indices, coefficient offsets, copy-out
  const int64_t cap = *nsegs;
  int64_t nout = 0, coef = 0, ocoef = 0;
  for (int k = 0; k < nsf; ++k) {
    Sf& b = sfs[k];
    const double* c = centers + 3 * k;
    wvl_locreg& L = lr[k];
    std::memset(&L, 0, sizeof L);
    std::copy(c, c + 3, L.center);
    L.radius = radii[k];
    L.fine_radius = fine_radii[k];
    L.ext = ext;
    std::copy(b.lo, b.lo + 3, L.lo);
    for (int a = 0; a < 3; ++a) L.dims[a] = b.hi[a] - b.lo[a] + 1;
    int64_t* first[4] = {&L.seg_c, &L.seg_f, &L.oseg_c, &L.oseg_f};
    int64_t* count[4] = {&L.nseg_c, &L.nseg_f, &L.noseg_c, &L.noseg_f};
    for (int p = 0; p < 4; ++p) {
      *first[p] = nout;
      *count[p] = (int64_t)b.seg[p].size();
      if (segs && nout + (int64_t)b.seg[p].size() <= cap)
        std::copy(b.seg[p].begin(), b.seg[p].end(), segs + nout);
      nout += (int64_t)b.seg[p].size();
      std::vector<wvl_seg>().swap(b.seg[p]);
    }
    L.n_c = b.tot[0];
    L.n_f = b.tot[1];
    L.on_c = b.tot[2];
    L.on_f = b.tot[3];
    L.coef_off = coef;
    coef += L.n_c + 7 * L.n_f;
    L.ocoef_off = ocoef;
    ocoef += L.on_c + 7 * L.on_f;
  }
  *nsegs = nout;
  if (segs && nout > cap)
    return fail(nullptr, WVL_EINVAL, "wvl_build_locregs: segs holds %lld, %lld needed",
                (long long)cap, (long long)nout);
  return WVL_OK;
}

wvl_status wvl_create(wvl_ctx** ctx, const wvl_grid* grid, void* hip_stream) {
  if (!ctx || !grid) return fail(nullptr, WVL_EINVAL, "wvl_create: null argument");
  *ctx = nullptr;
  if (!(grid->h > 0) || grid->n[0] <= 0 || grid->n[1] <= 0 || grid->n[2] <= 0)
    return fail(nullptr, WVL_EINVAL, "wvl_create: grid needs h > 0 and n > 0");
  wvl_ctx* c = new (std::nothrow) wvl_ctx;
  if (!c) return fail(nullptr, WVL_ENOMEM, "wvl_create: out of host memory");
  c->grid = *grid;
  c->stream = (hipStream_t)hip_stream;
  *ctx = c;
  return WVL_OK;
}

void wvl_destroy(wvl_ctx* ctx) {
  if (!ctx) return;
  for (auto& r : ctx->pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : ctx->pool) (void)hipEventDestroy(e);
  delete ctx;
}

wvl_status wvl_profile_enable(wvl_ctx* ctx, int enable) {
  if (!ctx) return fail(nullptr, WVL_EINVAL, "wvl_profile_enable: null context");
  ctx->prof = enable != 0;
  return WVL_OK;
}

static wvl_status fold_events(wvl_ctx* ctx) {
  if (ctx->pending.empty()) return WVL_OK;
  WVL_HIP(ctx, hipStreamSynchronize(ctx->stream));
  for (auto& r : ctx->pending) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
      ctx->launches[r.kind] += 1;
      ctx->ms[r.kind] += t;
    }
    ctx->pool.push_back(r.a);
    ctx->pool.push_back(r.b);
  }
  ctx->pending.clear();
  return WVL_OK;
}

wvl_status wvl_profile_reset(wvl_ctx* ctx) {
  if (!ctx) return fail(nullptr, WVL_EINVAL, "wvl_profile_reset: null context");
  wvl_status st = fold_events(ctx);
  for (int k = 0; k < KK_COUNT; ++k) {
    ctx->launches[k] = 0;
    ctx->ms[k] = 0.0;
  }
  return st;
}

int32_t wvl_profile_count(void) { return KK_COUNT; }

wvl_status wvl_profile_read(wvl_ctx* ctx, int32_t id, const char** name, int64_t* launches,
                            double* total_ms) {
  if (!ctx || id < 0 || id >= KK_COUNT)
    return fail(ctx, WVL_EINVAL, "wvl_profile_read: null context or id out of range");
  wvl_status st = fold_events(ctx);
  if (st != WVL_OK) return st;
  if (name) *name = kKernelNames[id];
  if (launches) *launches = ctx->launches[id];
  if (total_ms) *total_ms = ctx->ms[id];
  return WVL_OK;
}

static void free_pattern(PatternCache& p) {
  if (p.d_rowptr) (void)hipFree(p.d_rowptr);
  if (p.d_col) (void)hipFree(p.d_col);
  if (p.d_row) (void)hipFree(p.d_row);
  if (p.d_order) (void)hipFree(p.d_order);
  if (p.d_order_u) (void)hipFree(p.d_order_u);
  if (p.d_mirror_u) (void)hipFree(p.d_mirror_u);
  if (p.d_tpos) (void)hipFree(p.d_tpos);
  if (p.d_hpos) (void)hipFree(p.d_hpos);
  if (p.d_htpos) (void)hipFree(p.d_htpos);
  if (p.d_dpos) (void)hipFree(p.d_dpos);
  if (p.d_foe_rows) (void)hipFree(p.d_foe_rows);
  p = PatternCache{};
}

void wvl_plan_destroy(wvl_plan* plan) {
  if (!plan) return;
  if (plan->d_sf) (void)hipFree(plan->d_sf);
  if (plan->d_seg) (void)hipFree(plan->d_seg);
  if (plan->d_foff) (void)hipFree(plan->d_foff);
  if (plan->d_cptr) (void)hipFree(plan->d_cptr);
  if (plan->d_csf) (void)hipFree(plan->d_csf);
  for (int d = 0; d < 2; ++d)
    if (plan->d_tord[d]) (void)hipFree(plan->d_tord[d]);
  if (plan->d_rt) (void)hipFree(plan->d_rt);
  if (plan->d_rr) (void)hipFree(plan->d_rr);
  if (plan->d_wk) (void)hipFree(plan->d_wk);
  free_pattern(plan->pat[0]);
  free_pattern(plan->pat[1]);
  for (hipStream_t st : plan->streams) (void)hipStreamDestroy(st);
  delete plan;
}

// bin counts the autotuner tries (the plan's workspace covers all of them)
static const int kTuneBins[] = {1, 2, 3, 4, 6, 8};

static int64_t sf_elems(const SfDev& S) {
  const int64_t n0 = S.n[0], n1 = S.n[1], n2 = S.n[2], e = S.ext;
  const int64_t r0 = 2 * n0 + 29, r1 = 2 * n1 + 29;
  const int64_t o0 = n0 + 2 * e, o1 = n1 + 2 * e, o2 = n2 + 2 * e;
  return 2 * align64(8 * n0 * n1 * n2) + align64(2 * n2 * r0 * r1) + align64(2 * o2 * r0 * r1) +
         align64(4 * o2 * r0 * qrow_stride((int)o1)) + align64(8 * n2 * o0 * n1) +
         align64(8 * n2 * qrow_stride((int)o1) * n0) +
         align64(8 * o2 * n0 * n1) + align64(4 * n2 * n1 * r0);
}

// Builds the layout for `nbins` bins; false (with a message) when a box
// does not fit the kernels' LDS stages.
static bool make_layout(const wvl_plan* P, int nbins, bool zmfma, Layout* L, std::string* err) {
  const int nsf = P->nsf;
  L->chunks.clear();
  L->wk.assign(nsf, SfWork{});
  L->nbins = nbins;
  L->zmfma = zmfma;
  L->disjoint = P->max_ws == 0;
  L->elems_span = 0;
  L->parts_span = 0;
  nbins = std::max(1, std::min(nbins, nsf));
  int64_t ebase = 0, pbase = 0;   // running offsets (disjoint layouts)
  for (int bin = 0; bin < nbins; ++bin) {
    const int b0 = (int)((int64_t)nsf * bin / nbins), b1 = (int)((int64_t)nsf * (bin + 1) / nbins);
    int k = b0;
    while (k < b1) {
      ChunkDev ch{};
      ch.sf0 = k;
      int64_t elems = 0;
      int j = k;
      for (; j < b1; ++j) {
        const int64_t need = sf_elems(P->h_sf[P->order[j]]);
        // partial slots are at most a few per 256 output points
        const int64_t bytes = align_bytes((elems + need) * 8) + (int64_t)(j - k + 1) * 4096 * 8;
        if (j > k && P->max_ws > 0 && (size_t)bytes > P->max_ws) break;
        if (j - k >= 65535) break;
        elems += need;
      }
      ch.nsf = j - k;
      int64_t off = L->disjoint ? ebase : 0;
      const int64_t off0 = off;
      for (int q = k; q < j; ++q) {
        const int id = P->order[q];
        const SfDev& S = P->h_sf[id];
        const int64_t n0 = S.n[0], n1 = S.n[1], n2 = S.n[2], e = S.ext;
        const int64_t r0 = 2 * n0 + 29, r1 = 2 * n1 + 29;
        const int64_t o0 = n0 + 2 * e, o1 = n1 + 2 * e, o2 = n2 + 2 * e;
        SfWork& W = L->wk[q];
        W.id = id;
        W.c8 = off;  off += align64(8 * n0 * n1 * n2);
        W.c8x = off; off += align64(8 * n0 * n1 * n2);
        W.g1 = off;  off += align64(2 * n2 * r0 * r1);
        W.g2 = off;  off += align64(2 * o2 * r0 * r1);
        W.q = off;   off += align64(4 * o2 * r0 * qrow_stride((int)o1));
        W.ox = off;  off += align64(8 * n2 * o0 * n1);
        W.oy = off;  off += align64(8 * n2 * qrow_stride((int)o1) * n0);
        W.oz = off;  off += align64(8 * o2 * n0 * n1);
        W.gx = off;  off += align64(4 * n2 * n1 * r0);
        ch.maxbox_in = std::max(ch.maxbox_in, 8 * n0 * n1 * n2);
        ch.grid_u[0] = (int32_t)std::max<int64_t>(ch.grid_u[0], n2);   // planes; scaled below
        ch.grid_ux = (int32_t)std::max<int64_t>(ch.grid_ux, (4 * n2 * n1 + 63) / 64);
        ch.grid_uy = (int32_t)std::max<int64_t>(ch.grid_uy, (2 * n2 * r0 + 255) / 256);
        for (int d = 0; d < 2; ++d)
          ch.lds_u[d] = std::max<int64_t>(ch.lds_u[d], n1 * (n0 + 1) * (d ? 8 : 4));   // one plane
        ch.grid_b = (int32_t)std::max<int64_t>(ch.grid_b, (r0 * r1 + 255) / 256);
        ch.grid_kx = std::max(ch.grid_kx, kin_blocks(0, (int)n0, (int)n1, (int)n2));
        ch.grid_ky = std::max(ch.grid_ky, kin_blocks(1, (int)n0, (int)n1, (int)n2));
        ch.grid_kz = std::max(ch.grid_kz, kin_blocks(2, (int)n0, (int)n1, (int)n2, zmfma));
        ch.grid_by = (int32_t)std::max<int64_t>(ch.grid_by, (2 * o2 * r0 + 63) / 64);
        ch.grid_bx = (int32_t)std::max<int64_t>(ch.grid_bx, (o1 * o2 + kBackOutRows - 1) / kBackOutRows);
      }
      // k_unpack: as many components per block as the LDS stage fits
      const int64_t nz = ch.grid_u[0];
      for (int d = 0; d < 2; ++d) {
        if (ch.lds_u[d] > kLdsBudget) {
          *err = "a box's x-y plane (" + std::to_string(ch.lds_u[d]) +
                 " bytes) does not fit the unpack stage's LDS";
          return false;
        }
        int g = 8;   // grouped stages stay within 64 KiB of dynamic LDS
        while (g > 1 && g * ch.lds_u[d] > 64 * 1024) g /= 2;
        ch.group_u[d] = g;
        ch.grid_u[d] = (int32_t)((8 / g) * nz);
        ch.lds_u[d] *= g;
      }
      ch.nblk_pot = ch.grid_b;
      ch.nblk_kin = ch.grid_kx + ch.grid_ky + ch.grid_kz;
      int64_t poff = L->disjoint ? pbase : 0;
      for (int q = k; q < j; ++q) {
        const SfDev& S = P->h_sf[P->order[q]];
        SfWork& W = L->wk[q];
        W.epart = poff;
        poff += ch.nblk_pot;
        W.kpart = poff;
        W.nkpart = kin_blocks(0, S.n[0], S.n[1], S.n[2]) + kin_blocks(1, S.n[0], S.n[1], S.n[2]) +
                   kin_blocks(2, S.n[0], S.n[1], S.n[2], zmfma);
        poff += ch.nblk_kin;
      }
      L->chunks.push_back(ch);
      if (L->disjoint) {
        ebase = off;
        pbase = poff;
        L->elems_span = ebase;
        L->parts_span = pbase;
      } else {
        L->elems_span = std::max(L->elems_span, off - off0);
        L->parts_span = std::max(L->parts_span, poff);
      }
      k = j;
    }
  }
  return true;
}

wvl_status wvl_plan_create(wvl_ctx* ctx, int32_t nsf, const wvl_locreg* lr, const wvl_seg* segs,
                           int64_t nsegs, size_t max_workspace_bytes, wvl_plan** plan_out,
                           size_t* workspace_bytes) {
  if (!ctx) return fail(nullptr, WVL_EINVAL, "wvl_plan_create: null context");
  if (!plan_out) return fail(ctx, WVL_EINVAL, "wvl_plan_create: null plan pointer");
  *plan_out = nullptr;
  if (nsf < 0 || nsegs < 0 || (nsf > 0 && !lr) || (nsegs > 0 && !segs))
    return fail(ctx, WVL_EINVAL, "wvl_plan_create: bad counts or null arrays");
  if (nsegs >= (int64_t)1 << 31)
    return fail(ctx, WVL_EUNSUPPORTED, "wvl_plan_create: more than 2^31 segments");
  const int32_t* gn = ctx->grid.n;
  if (gn[0] > 65535)
    return fail(ctx, WVL_EUNSUPPORTED, "wvl_plan_create: grid wider than 65535 points along x");
  wvl_status st = WVL_OK;
  bool in_sub_out = true;   // every input pattern inside its output pattern
  std::vector<std::pair<int64_t, int64_t>> outs;
  for (int k = 0; k < nsf; ++k) {
    const wvl_locreg& L = lr[k];
    for (int a = 0; a < 3; ++a) {
      if (L.dims[a] < 1 || L.lo[a] < 0 || (int64_t)L.lo[a] + L.dims[a] > gn[a])
        return fail(ctx, WVL_EINVAL, "function %d: input box outside the grid (axis %d)", k, a);
      if (L.dims[a] > 4096)
        return fail(ctx, WVL_EUNSUPPORTED, "function %d: box wider than 4096 points", k);
    }
    if (L.ext < 0 || L.ext > 16) return fail(ctx, WVL_EINVAL, "function %d: ext outside [0, 16]", k);
    int blo[3], bhi[3], olo[3], ohi[3];
    for (int a = 0; a < 3; ++a) {
      blo[a] = L.lo[a];
      bhi[a] = L.lo[a] + L.dims[a] - 1;
      olo[a] = L.lo[a] - L.ext;
      ohi[a] = bhi[a] + L.ext;
    }
    const int64_t nc = check_list(ctx, &st, k, "input coarse", segs, nsegs, L.seg_c, L.nseg_c, blo,
                                  bhi, gn);
    if (nc < 0) return st;
    const int64_t nf = check_list(ctx, &st, k, "input fine", segs, nsegs, L.seg_f, L.nseg_f, blo,
                                  bhi, gn);
    if (nf < 0) return st;
    const int64_t onc = check_list(ctx, &st, k, "output coarse", segs, nsegs, L.oseg_c, L.noseg_c,
                                   olo, ohi, gn);
    if (onc < 0) return st;
    const int64_t onf = check_list(ctx, &st, k, "output fine", segs, nsegs, L.oseg_f, L.noseg_f,
                                   olo, ohi, gn);
    if (onf < 0) return st;
    if (nc != L.n_c || nf != L.n_f || onc != L.on_c || onf != L.on_f)
      return fail(ctx, WVL_EINVAL,
                  "function %d: point counts (n_c %lld, n_f %lld, on_c %lld, on_f %lld) differ "
                  "from the segment lists (%lld, %lld, %lld, %lld)",
                  k, (long long)L.n_c, (long long)L.n_f, (long long)L.on_c, (long long)L.on_f,
                  (long long)nc, (long long)nf, (long long)onc, (long long)onf);
    int64_t bad = -1;
    if (!fine_in_coarse(segs, L.seg_c, L.nseg_c, L.seg_f, L.nseg_f, &bad))
      return fail(ctx, WVL_EINVAL, "function %d: input fine segment %lld not inside a coarse one",
                  k, (long long)bad);
    if (!fine_in_coarse(segs, L.oseg_c, L.noseg_c, L.oseg_f, L.noseg_f, &bad))
      return fail(ctx, WVL_EINVAL, "function %d: output fine segment %lld not inside a coarse one",
                  k, (long long)bad);
    if (L.coef_off < 0 || L.ocoef_off < 0)
      return fail(ctx, WVL_EINVAL, "function %d: negative coefficient offset", k);
    // wvl_update projects H psi (output pattern) onto the input pattern
    int64_t bad2 = -1;
    if (!fine_in_coarse(segs, L.oseg_c, L.noseg_c, L.seg_c, L.nseg_c, &bad2) ||
        !fine_in_coarse(segs, L.oseg_f, L.noseg_f, L.seg_f, L.nseg_f, &bad2))
      in_sub_out = false;
    outs.emplace_back(L.ocoef_off, L.on_c + 7 * L.on_f);
  }
  std::sort(outs.begin(), outs.end());
  for (size_t q = 1; q < outs.size(); ++q)
    if (outs[q].second > 0 && outs[q - 1].first + outs[q - 1].second > outs[q].first)
      return fail(ctx, WVL_EINVAL, "output coefficient ranges of two functions overlap");

  wvl_plan* P = new (std::nothrow) wvl_plan;
  if (!P) return fail(ctx, WVL_ENOMEM, "wvl_plan_create: out of host memory");
  P->ctx = ctx;
  P->nsf = nsf;
  P->h_sf.resize(nsf);
  std::vector<int32_t> rt;
  std::vector<RowRun> rr;
  int64_t box_in = 0, box_out = 0, in_coefs = 0, out_coefs = 0;
  for (int k = 0; k < nsf; ++k) {
    const wvl_locreg& L = lr[k];
    SfDev& S = P->h_sf[k];
    std::memset(&S, 0, sizeof S);
    for (int a = 0; a < 3; ++a) {
      S.lo[a] = L.lo[a];
      S.n[a] = L.dims[a];
    }
    S.ext = L.ext;
    S.cin = L.coef_off;
    S.cout = L.ocoef_off;
    S.n_c = L.n_c;
    S.n_f = L.n_f;
    S.on_c = L.on_c;
    std::copy(L.center, L.center + 3, S.c);
    S.on_f = L.on_f;
    S.box_in = box_in;
    S.box_out = box_out;
    const int e = L.ext;
    box_in += 8ll * L.dims[0] * L.dims[1] * L.dims[2];
    box_out += 8ll * (L.dims[0] + 2 * e) * (L.dims[1] + 2 * e) * (L.dims[2] + 2 * e);
    in_coefs = std::max<int64_t>(in_coefs, L.coef_off + L.n_c + 7 * L.n_f);
    out_coefs = std::max<int64_t>(out_coefs, L.ocoef_off + L.on_c + 7 * L.on_f);
    const int64_t firsts[4] = {L.seg_c, L.seg_f, L.oseg_c, L.oseg_f};
    const int64_t counts[4] = {L.nseg_c, L.nseg_f, L.noseg_c, L.noseg_f};
    for (int p = 0; p < 4; ++p) {
      const int g = p < 2 ? 0 : e;
      S.rt[p] = (int64_t)rt.size();
      row_table(segs, firsts[p], counts[p], L.lo[0] - g, L.lo[1] - g, L.lo[2] - g,
                L.dims[1] + 2 * g, L.dims[2] + 2 * g, rt);
      S.rr[p] = (int64_t)rr.size();
      row_runs(segs, firsts[p], counts[p], L.lo[1] - g, L.lo[2] - g, L.dims[1] + 2 * g,
               L.dims[2] + 2 * g, rr);
    }
    bbox(segs, L.seg_c, L.nseg_c, S.bb_in);
    bbox(segs, L.oseg_c, L.noseg_c, S.bb_out);
  }
  // processing order: largest boxes first, ties by index
  P->order.resize(nsf);
  for (int k = 0; k < nsf; ++k) P->order[k] = k;
  std::stable_sort(P->order.begin(), P->order.end(), [&](int a, int b) {
    const SfDev &A = P->h_sf[a], &B = P->h_sf[b];
    return (int64_t)A.n[0] * A.n[1] * A.n[2] > (int64_t)B.n[0] * B.n[1] * B.n[2];
  });
  P->max_ws = max_workspace_bytes;
  P->in_sub_out = in_sub_out;
  for (int k = 0; k < nsf; ++k)
    P->max_in_segs = std::max<int64_t>(P->max_in_segs, lr[k].nseg_c + lr[k].nseg_f);
  // the workspace reported covers every layout the autotuner may pick
  for (int zm = 0; zm < 2; ++zm)
    for (int nb : kTuneBins) {
      Layout L;
      std::string err;
      if (!make_layout(P, nb, zm != 0, &L, &err)) {
        wvl_plan_destroy(P);
        return fail(ctx, WVL_EUNSUPPORTED, "%s", err.c_str());
      }
      P->ws_cap[0] = std::max(P->ws_cap[0], L.bytes(4));
      P->ws_cap[1] = std::max(P->ws_cap[1], L.bytes(8));
      if (nb == 1 && zm == 0) P->lay = std::move(L);
    }
  const int64_t best_f32 = P->ws_cap[0], best_f64 = P->ws_cap[1];
  P->info.nsf = nsf;
  P->info.in_coefs = in_coefs;
  P->info.out_coefs = out_coefs;
  P->info.in_box = box_in;
  P->info.out_box = box_out;
  P->info.workspace_f32 = best_f32;
  P->info.workspace_f64 = best_f64;
  P->info.chunks = (int64_t)P->lay.chunks.size();
  std::vector<int64_t> foff(nsf + 1, 0);
  for (int k = 0; k < nsf; ++k) {
    const SfDev& S = P->h_sf[k];
    const int64_t v = (int64_t)(2 * S.n[0] + 29) * (2 * S.n[1] + 29) * (2 * S.n[2] + 29);
    foff[k + 1] = foff[k] + v;
    P->max_fine = std::max(P->max_fine, v);
  }
  P->info.fine_box = foff[nsf];
  if ((st = upload(ctx, &P->d_sf, P->h_sf.data(), sizeof(SfDev) * nsf)) != WVL_OK ||
      (st = upload(ctx, &P->d_seg, segs, sizeof(wvl_seg) * nsegs)) != WVL_OK ||
      (st = upload(ctx, &P->d_rt, rt.data(), sizeof(int32_t) * rt.size())) != WVL_OK ||
      (st = upload(ctx, &P->d_rr, rr.data(), sizeof(RowRun) * rr.size())) != WVL_OK ||
      (st = upload(ctx, &P->d_wk, P->lay.wk.data(), sizeof(SfWork) * nsf)) != WVL_OK ||
      (st = upload(ctx, &P->d_foff, foff.data(), sizeof(int64_t) * (nsf + 1))) != WVL_OK) {
    wvl_plan_destroy(P);
    return st;
  }
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    wvl_plan_destroy(P);
    return hip_fail(ctx, "plan upload", "hipStreamSynchronize", e);
  }
  if (workspace_bytes) *workspace_bytes = (size_t)best_f64;
  *plan_out = P;
  return WVL_OK;
}

wvl_status wvl_plan_info_get(const wvl_plan* plan, wvl_plan_info* info) {
  if (!plan || !info) return fail(nullptr, WVL_EINVAL, "wvl_plan_info_get: null argument");
  *info = plan->info;
  return WVL_OK;
}

static wvl_status check_dt(wvl_ctx* ctx, wvl_dtype dt) {
  if (dt != WVL_F32 && dt != WVL_F64) return fail(ctx, WVL_EINVAL, "unknown dtype %d", (int)dt);
  return WVL_OK;
}

wvl_status wvl_uncompress(wvl_plan* P, wvl_dtype dt, const void* psi_c, void* psi_box) {
  if (!P) return fail(nullptr, WVL_EINVAL, "wvl_uncompress: null plan");
  wvl_ctx* ctx = P->ctx;
  if (check_dt(ctx, dt) != WVL_OK) return WVL_EINVAL;
  if (P->nsf > 0 && (!psi_c || !psi_box)) return fail(ctx, WVL_EINVAL, "wvl_uncompress: null buffer");
  for (int s0 = 0; s0 < P->nsf; s0 += 65535) {
    const int n = std::min(65535, P->nsf - s0);
    int64_t mv = 0;
    for (int k = s0; k < s0 + n; ++k)
      mv = std::max<int64_t>(mv, 8ll * P->h_sf[k].n[0] * P->h_sf[k].n[1] * P->h_sf[k].n[2]);
    WVL_LAUNCH(ctx, KK_GATHER,
               launch_gather(dt == WVL_F64, ctx->stream, P->d_sf, P->d_seg, P->d_rt, psi_c, psi_box,
                             s0, n, mv));
  }
  return WVL_OK;
}

wvl_status wvl_compress(wvl_plan* P, wvl_dtype dt, const void* box, void* hpsi_c) {
  if (!P) return fail(nullptr, WVL_EINVAL, "wvl_compress: null plan");
  wvl_ctx* ctx = P->ctx;
  if (check_dt(ctx, dt) != WVL_OK) return WVL_EINVAL;
  if (P->nsf > 0 && (!box || !hpsi_c)) return fail(ctx, WVL_EINVAL, "wvl_compress: null buffer");
  for (int s0 = 0; s0 < P->nsf; s0 += 65535) {
    const int n = std::min(65535, P->nsf - s0);
    int64_t mv = 0;
    for (int k = s0; k < s0 + n; ++k) {
      const SfDev& S = P->h_sf[k];
      mv = std::max<int64_t>(mv, 8ll * (S.n[0] + 2 * S.ext) * (S.n[1] + 2 * S.ext) *
                                     (S.n[2] + 2 * S.ext));
    }
    WVL_LAUNCH(ctx, KK_SCATTER,
               launch_scatter(dt == WVL_F64, ctx->stream, P->d_sf, P->d_seg, P->d_rt, box, hpsi_c,
                              s0, n, mv));
  }
  return WVL_OK;
}

// checks shared by the eager and the captured apply
static wvl_status apply_args(wvl_plan* P, wvl_dtype dt, uint32_t terms, const void* psi_c,
                             const void* pot, const void* hpsi_c, const void* workspace,
                             const char* who, bool pot_optional = false) {
  if (!P) return fail(nullptr, WVL_EINVAL, "%s: null plan", who);
  wvl_ctx* ctx = P->ctx;
  if (check_dt(ctx, dt) != WVL_OK) return WVL_EINVAL;
  if ((terms & ~(WVL_KIN | WVL_POT)) || terms == 0)
    return fail(ctx, WVL_EINVAL, "%s: terms must be a non-empty mix of WVL_KIN and WVL_POT", who);
  if (P->nsf == 0) return WVL_OK;
  if (!psi_c || !hpsi_c || !workspace)
    return fail(ctx, WVL_EINVAL, "%s: null coefficient or workspace buffer", who);
  if ((terms & WVL_POT) && !pot && !pot_optional)
    return fail(ctx, WVL_EINVAL, "%s: WVL_POT needs a potential", who);
  return WVL_OK;
}

// Enqueues the stages of chunk c on stream st.
static wvl_status apply_chunk(wvl_plan* P, size_t c, int f64, uint32_t terms, const void* psi_c,
                              const void* pot, void* hpsi_c, double* e_kin, double* e_pot,
                              void* workspace, int accumulate, hipStream_t st,
                              const double* conf = nullptr) {
  wvl_ctx* ctx = P->ctx;
  const int sz = f64 ? 8 : 4;
  const int d = f64 ? 1 : 0;
  const int nf1 = 2 * ctx->grid.n[0] + 29, nf2 = 2 * ctx->grid.n[1] + 29;
  const double fac = -2.0 / (ctx->grid.h * ctx->grid.h);   // -1/2 (2/h)^2
  const int pot_on = (terms & WVL_POT) ? 1 : 0, kin_on = (terms & WVL_KIN) ? 1 : 0;
  const ChunkDev& ch = P->lay.chunks[c];
  const SfWork* wk = P->d_wk + ch.sf0;
  double* parts = (double*)((char*)workspace + align_bytes(P->lay.elems_span * sz));
  WVL_LAUNCH(ctx, KK_UNPACK,
             launch_unpack(f64, st, P->d_sf, P->d_seg, P->d_rt, P->d_rr, psi_c, wk, ch.nsf,
                           ch.grid_u[d], ch.group_u[d], (size_t)ch.lds_u[d], workspace));
  if (pot_on) {
    WVL_LAUNCH(ctx, KK_UP_X, launch_up(f64, st, 0, wk, P->d_sf, ch.nsf, ch.grid_ux, workspace));
    WVL_LAUNCH(ctx, KK_UP_Y, launch_up(f64, st, 1, wk, P->d_sf, ch.nsf, ch.grid_uy, workspace));
    WVL_LAUNCH(ctx, KK_POT_COLUMN,
               launch_pot_column(f64, st, P->d_sf, wk, ch.sf0, ch.nsf, ch.grid_b, workspace, pot,
                                 nf1, nf2, parts, conf, 0.5 * ctx->grid.h));
    if (e_pot)
      WVL_LAUNCH(ctx, KK_FINALIZE,
                 launch_finalize(st, wk, ch.sf0, ch.nsf, parts, 0, ch.grid_b, e_pot));
  }
  if (kin_on) {
    WVL_LAUNCH(ctx, KK_KIN_XCOL, launch_kin_col(f64, st, 0, P->d_sf, wk, ch.sf0, ch.nsf,
                                                ch.grid_kx, workspace, fac, parts));
    WVL_LAUNCH(ctx, KK_KIN_YCOL, launch_kin_col(f64, st, 1, P->d_sf, wk, ch.sf0, ch.nsf,
                                                ch.grid_ky, workspace, fac, parts));
    if (P->lay.zmfma)
      WVL_LAUNCH(ctx, KK_KIN_ZCOL, launch_kin_zmfma(f64, st, P->d_sf, wk, ch.sf0, ch.nsf,
                                                    ch.grid_kz, workspace, fac, parts));
    else
      WVL_LAUNCH(ctx, KK_KIN_ZCOL, launch_kin_col(f64, st, 2, P->d_sf, wk, ch.sf0, ch.nsf,
                                                  ch.grid_kz, workspace, fac, parts));
    if (e_kin)
      WVL_LAUNCH(ctx, KK_FINALIZE,
                 launch_finalize(st, wk, ch.sf0, ch.nsf, parts, 1, ch.nblk_kin, e_kin));
  }
  if (pot_on)
    WVL_LAUNCH(ctx, KK_BACK_Y,
               launch_back_y(f64, st, P->d_sf, wk, ch.sf0, ch.nsf, ch.grid_by, workspace));
  // the x down pass, the kinetic parts and the compression onto the output
  // pattern in one kernel
  WVL_LAUNCH(ctx, KK_BACK_X,
             launch_back_out(f64, st, P->d_sf, P->d_seg, P->d_rt, P->d_rr, wk, ch.sf0, ch.nsf,
                             ch.grid_bx, workspace, hpsi_c, pot_on, kin_on, accumulate));
  return WVL_OK;
}

static wvl_status apply_impl(wvl_plan* P, wvl_dtype dt, uint32_t terms, const void* psi_c,
                             const void* pot, void* hpsi_c, double* e_kin, double* e_pot,
                             void* workspace, int accumulate, const char* who,
                             const double* conf = nullptr) {
  wvl_status st = apply_args(P, dt, terms, psi_c, pot, hpsi_c, workspace, who, conf != nullptr);
  if (st != WVL_OK || P->nsf == 0) return st;
  for (size_t c = 0; c < P->lay.chunks.size(); ++c)
    if ((st = apply_chunk(P, c, dt == WVL_F64, terms, psi_c, pot, hpsi_c, e_kin, e_pot, workspace,
                          accumulate, P->ctx->stream, conf)) != WVL_OK)
      return st;
  return WVL_OK;
}

wvl_status wvl_apply_local_ham(wvl_plan* plan, wvl_dtype dt, uint32_t terms, const void* psi_c,
                               const void* pot, void* hpsi_c, double* e_kin, double* e_pot,
                               void* workspace) {
  return apply_impl(plan, dt, terms, psi_c, pot, hpsi_c, e_kin, e_pot, workspace, 0,
                    "wvl_apply_local_ham");
}

}  // extern "C"

wvl_status wvl::apply_in_workspace(wvl_plan* P, wvl_dtype dt, uint32_t terms, const void* psi_c,
                                   const void* pot, void* hpsi_c, double* e_kin, double* e_pot,
                                   void* workspace, size_t cap, const char* who) {
  if (!P) return fail(nullptr, WVL_EINVAL, "%s: null plan", who);
  if (check_dt(P->ctx, dt) != WVL_OK) return WVL_EINVAL;
  const int64_t need = dt == WVL_F64 ? P->info.workspace_f64 : P->info.workspace_f32;
  if (P->nsf > 0 && need > (int64_t)cap)
    return fail(P->ctx, WVL_EINVAL,
                "%s: the plan needs a workspace of %lld bytes for %s, the static one holds %zu; "
                "create the plan with a smaller max_workspace_bytes",
                who, (long long)need, dt == WVL_F64 ? "WVL_F64" : "WVL_F32", cap);
  return apply_impl(P, dt, terms, psi_c, pot, hpsi_c, e_kin, e_pot, workspace, 0, who);
}

wvl_status wvl::plan_error(wvl_plan* P, wvl_status st, const char* msg) {
  return fail(P ? P->ctx : nullptr, st, "%s", msg);
}

void* wvl::plan_stream(const wvl_plan* P) { return P ? (void*)P->ctx->stream : nullptr; }

extern "C" {

wvl_status wvl_apply_local_ham_conf(wvl_plan* plan, wvl_dtype dt, uint32_t terms,
                                    const void* psi_c, const void* pot, const double* conf,
                                    void* hpsi_c, double* e_kin, double* e_pot, void* workspace) {
  if (plan && !(terms & WVL_POT))
    return fail(plan->ctx, WVL_EINVAL, "wvl_apply_local_ham_conf: the confinement needs WVL_POT");
  if (plan && plan->nsf > 0 && !conf)
    return fail(plan->ctx, WVL_EINVAL, "wvl_apply_local_ham_conf: null prefactors");
  return apply_impl(plan, dt, terms, psi_c, pot, hpsi_c, e_kin, e_pot, workspace, 0,
                    "wvl_apply_local_ham_conf", conf);
}

wvl_status wvl_kinetic(wvl_plan* plan, wvl_dtype dt, const void* psi_c, void* hpsi_c,
                       double* e_kin, void* workspace) {
  return apply_impl(plan, dt, WVL_KIN, psi_c, nullptr, hpsi_c, e_kin, nullptr, workspace, 1,
                    "wvl_kinetic");
}

// rows whose S/H pairs are interleaved by ket (see ensure_pattern)
constexpr int kPairGroup = 8;

static wvl_status ensure_pattern(wvl_plan* P, int ket_out) {
  wvl_ctx* ctx = P->ctx;
  PatternCache& pc = P->pat[ket_out];
  if (pc.ready) return WVL_OK;
  const int nsf = P->nsf;
  int64_t* d_count = nullptr;
  std::vector<int64_t> cnt(nsf), rowptr(nsf + 1, 0);
  if (nsf > 0) {
    WVL_HIP(ctx, hipMalloc((void**)&d_count, sizeof(int64_t) * nsf));
    int e;
    const char* call = "launch of pattern (count)";
    {
      Trace tr(ctx, KK_PATTERN);
      e = launch_pattern(ctx->stream, P->d_sf, P->d_seg, P->d_rt, nsf, ket_out, d_count, nullptr,
                         nullptr);
    }
    if (e == 0) {
      call = "hipMemcpyAsync";
      e = (int)hipMemcpyAsync(cnt.data(), d_count, sizeof(int64_t) * nsf, hipMemcpyDeviceToHost,
                              ctx->stream);
    }
    if (e == 0) {
      call = "hipStreamSynchronize";
      e = (int)hipStreamSynchronize(ctx->stream);
    }
    (void)hipFree(d_count);
    if (e != 0) return hip_fail(ctx, "sparsity pattern count", call, (hipError_t)e);
  }
  for (int a = 0; a < nsf; ++a) rowptr[a + 1] = rowptr[a] + cnt[a];
  const int64_t nnz = rowptr[nsf];
  std::vector<int32_t> row(nnz);
  for (int a = 0; a < nsf; ++a)
    for (int64_t q = rowptr[a]; q < rowptr[a + 1]; ++q) row[q] = a;
  wvl_status st;
  if ((st = upload(ctx, &pc.d_rowptr, rowptr.data(), sizeof(int64_t) * (nsf + 1))) != WVL_OK)
    return st;
  if ((st = upload(ctx, &pc.d_row, row.data(), sizeof(int32_t) * nnz)) != WVL_OK) {
    free_pattern(pc);
    return st;
  }
  if (nnz > 0) {
    hipError_t e = hipMalloc((void**)&pc.d_col, sizeof(int32_t) * nnz);
    if (e != hipSuccess) {
      free_pattern(pc);
      return fail(ctx, WVL_ENOMEM, "pattern columns: hipMalloc returned %s (%s)",
                  hipGetErrorName(e), hipGetErrorString(e));
    }
    int le;
    const char* call = "launch of pattern (fill)";
    {
      Trace tr(ctx, KK_PATTERN);
      le = launch_pattern(ctx->stream, P->d_sf, P->d_seg, P->d_rt, nsf, ket_out, nullptr,
                          pc.d_rowptr, pc.d_col);
    }
    if (le == 0) {
      call = "hipStreamSynchronize";
      le = (int)hipStreamSynchronize(ctx->stream);
    }
    if (le != 0) {
      free_pattern(pc);
      return hip_fail(ctx, "sparsity pattern fill", call, (hipError_t)le);
    }
  } else {
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
      free_pattern(pc);
      return hip_fail(ctx, "pattern upload", "hipStreamSynchronize", e);
    }
  }
  // Value pairs are processed in groups of kPairGroup rows, the rows in the
  // Morton order of their box centres and the pairs of a group ordered by
  // ket: concurrently running pairs then share the bra rows and each ket's
  // overlap in the caches (the values land at their CSR positions
  // regardless, each summed in the same order).
  if (nnz > 0) {
    if (nnz > INT32_MAX) {
      free_pattern(pc);
      return fail(ctx, WVL_EUNSUPPORTED, "pattern with %lld pairs exceeds 2^31", (long long)nnz);
    }
    std::vector<std::pair<uint32_t, int>> key(nsf);
    for (int a = 0; a < nsf; ++a) {
      const SfDev& S = P->h_sf[a];
      key[a] = {morton3((uint32_t)(S.lo[0] + S.n[0] / 2), (uint32_t)(S.lo[1] + S.n[1] / 2),
                        (uint32_t)(S.lo[2] + S.n[2] / 2)), a};
    }
    std::sort(key.begin(), key.end());
    std::vector<int32_t> col(nnz);
    const char* call = "hipMemcpyAsync";
    hipError_t ce = hipMemcpyAsync(col.data(), pc.d_col, sizeof(int32_t) * nnz,
                                   hipMemcpyDeviceToHost, ctx->stream);
    if (ce == hipSuccess) {
      call = "hipStreamSynchronize";
      ce = hipStreamSynchronize(ctx->stream);
    }
    if (ce != hipSuccess) {
      free_pattern(pc);
      return hip_fail(ctx, "pattern columns", call, ce);
    }
    std::vector<int32_t> order;
    order.reserve(nnz);
    std::vector<std::pair<int32_t, int32_t>> grp;   // (ket, CSR position)
    for (int c0 = 0; c0 < nsf; c0 += kPairGroup) {
      grp.clear();
      for (int c = c0; c < std::min(nsf, c0 + kPairGroup); ++c) {
        const int a = key[c].second;
        for (int64_t q = rowptr[a]; q < rowptr[a + 1]; ++q) grp.emplace_back(col[q], (int32_t)q);
      }
      std::stable_sort(grp.begin(), grp.end(),
                       [](const std::pair<int32_t, int32_t>& x,
                          const std::pair<int32_t, int32_t>& y) { return x.first < y.first; });
      for (const auto& e : grp) order.push_back(e.second);
    }
    if ((st = upload(ctx, &pc.d_order, order.data(), sizeof(int32_t) * nnz)) != WVL_OK) {
      free_pattern(pc);
      return st;
    }
    // the overlap of a function with itself: S_ab = S_ba, so only the pairs
    // a <= b are summed and each value is written to both positions
    if (!ket_out) {
      std::vector<int32_t> ou, mu;
      ou.reserve(nnz / 2 + nsf);
      mu.reserve(nnz / 2 + nsf);
      bool sym = true;
      for (int64_t s = 0; s < nnz && sym; ++s) {
        const int32_t k = order[s], a = row[k], b = col[k];
        if (a > b) continue;
        int32_t m = -1;
        if (a != b) {
          const auto e = col.begin() + rowptr[b + 1];
          const auto it = std::lower_bound(col.begin() + rowptr[b], e, a);
          if (it == e || *it != a)
            sym = false;
          else
            m = (int32_t)(it - col.begin());
        }
        ou.push_back(k);
        mu.push_back(m);
      }
      if (sym && (st = upload(ctx, &pc.d_order_u, ou.data(), sizeof(int32_t) * ou.size())) ==
                     WVL_OK)
        st = upload(ctx, &pc.d_mirror_u, mu.data(), sizeof(int32_t) * mu.size());
      if (st != WVL_OK) {
        free_pattern(pc);
        return st;
      }
      pc.nnz_u = sym ? (int64_t)ou.size() : 0;
    }
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
      free_pattern(pc);
      return hip_fail(ctx, "pattern order upload", "hipStreamSynchronize", e);
    }
  }
  pc.nnz = nnz;
  pc.ready = true;
  return WVL_OK;
}

wvl_status wvl_sparse_overlap(wvl_plan* P, const void* bra_c, int ket_is_output, const void* ket_c,
                              wvl_dtype dt, int64_t* nnz, int64_t* rowptr, int32_t* col,
                              double* val) {
  if (!P) return fail(nullptr, WVL_EINVAL, "wvl_sparse_overlap: null plan");
  wvl_ctx* ctx = P->ctx;
  if (check_dt(ctx, dt) != WVL_OK) return WVL_EINVAL;
  if (ket_is_output != 0 && ket_is_output != 1)
    return fail(ctx, WVL_EINVAL, "wvl_sparse_overlap: ket_is_output must be 0 or 1");
  wvl_status st = ensure_pattern(P, ket_is_output);
  if (st != WVL_OK) return st;
  const PatternCache& pc = P->pat[ket_is_output];
  if (nnz) *nnz = pc.nnz;
  if (rowptr)
    WVL_HIP(ctx, hipMemcpyAsync(rowptr, pc.d_rowptr, sizeof(int64_t) * (P->nsf + 1),
                                hipMemcpyDeviceToDevice, ctx->stream));
  if (col && pc.nnz)
    WVL_HIP(ctx, hipMemcpyAsync(col, pc.d_col, sizeof(int32_t) * pc.nnz, hipMemcpyDeviceToDevice,
                                ctx->stream));
  if (val && pc.nnz) {
    if (!bra_c || !ket_c) return fail(ctx, WVL_EINVAL, "wvl_sparse_overlap: null bra or ket");
    const bool half = !ket_is_output && bra_c == ket_c && pc.nnz_u > 0;
    WVL_LAUNCH(ctx, ket_is_output ? KK_SPARSE_H : KK_SPARSE_S,
               launch_sparse_values(dt == WVL_F64, ctx->stream, P->d_sf, P->d_seg, P->d_rt,
                                    P->d_rr, ket_is_output, bra_c, ket_c, pc.d_row, pc.d_col,
                                    half ? pc.d_order_u : pc.d_order,
                                    half ? pc.d_mirror_u : nullptr, half ? pc.nnz_u : pc.nnz,
                                    val));
  }
  return WVL_OK;
}

wvl_status wvl_synthesize(wvl_plan* P, wvl_dtype dt, const void* psi_c, void* fine,
                          void* workspace) {
  if (!P) return fail(nullptr, WVL_EINVAL, "wvl_synthesize: null plan");
  wvl_ctx* ctx = P->ctx;
  if (check_dt(ctx, dt) != WVL_OK) return WVL_EINVAL;
  if (P->nsf == 0) return WVL_OK;
  if (!psi_c || !fine || !workspace) return fail(ctx, WVL_EINVAL, "wvl_synthesize: null buffer");
  const int f64 = dt == WVL_F64 ? 1 : 0;
  for (size_t c = 0; c < P->lay.chunks.size(); ++c) {
    const ChunkDev& ch = P->lay.chunks[c];
    const SfWork* wk = P->d_wk + ch.sf0;
    hipStream_t st = ctx->stream;
    WVL_LAUNCH(ctx, KK_UNPACK,
               launch_unpack(f64, st, P->d_sf, P->d_seg, P->d_rt, P->d_rr, psi_c, wk, ch.nsf,
                             ch.grid_u[f64], ch.group_u[f64], (size_t)ch.lds_u[f64], workspace));
    WVL_LAUNCH(ctx, KK_UP_X, launch_up(f64, st, 0, wk, P->d_sf, ch.nsf, ch.grid_ux, workspace));
    WVL_LAUNCH(ctx, KK_UP_Y, launch_up(f64, st, 1, wk, P->d_sf, ch.nsf, ch.grid_uy, workspace));
    WVL_LAUNCH(ctx, KK_UP_Z, launch_up_z(f64, st, wk, P->d_sf, ch.nsf, ch.grid_b, workspace,
                                         P->d_foff, fine));
  }
  return WVL_OK;
}

// functions whose fine box meets each k_dens_tile tile, increasing index
static wvl_status ensure_cover(wvl_plan* P) {
  if (P->d_cptr) return WVL_OK;
  wvl_ctx* ctx = P->ctx;
  int gf[3], nt[3];
  for (int a = 0; a < 3; ++a) {
    gf[a] = 2 * ctx->grid.n[a] + 29;
    nt[a] = (gf[a] + kDensTile[a] - 1) / kDensTile[a];
  }
  const int64_t ntile = (int64_t)nt[0] * nt[1] * nt[2];
  if (ntile > INT32_MAX) return fail(ctx, WVL_EUNSUPPORTED, "density: fine grid too large");
  std::vector<int64_t> cptr(ntile + 1, 0);
  std::vector<int32_t> csf;
  for (int pass = 0; pass < 2; ++pass) {
    std::vector<int64_t> pos;
    if (pass == 1) {
      for (int64_t t = 0; t < ntile; ++t) cptr[t + 1] += cptr[t];
      pos.assign(cptr.begin(), cptr.end() - 1);
      csf.resize(cptr[ntile]);
    }
    for (int k = 0; k < P->nsf; ++k) {
      const SfDev& S = P->h_sf[k];
      int t0[3], t1[3];
      for (int a = 0; a < 3; ++a) {
        t0[a] = (2 * S.lo[a]) / kDensTile[a];
        t1[a] = (2 * S.lo[a] + 2 * S.n[a] + 28) / kDensTile[a];
      }
      for (int z = t0[2]; z <= t1[2]; ++z)
        for (int y = t0[1]; y <= t1[1]; ++y)
          for (int x = t0[0]; x <= t1[0]; ++x) {
            const int64_t t = ((int64_t)z * nt[1] + y) * nt[0] + x;
            if (pass == 0)
              ++cptr[t + 1];
            else
              csf[pos[t]++] = k;
          }
    }
  }
  int64_t maxc = 0;
  for (int64_t t = 0; t < ntile; ++t) maxc = std::max(maxc, cptr[t + 1] - cptr[t]);
  if (maxc > kDensMaxCover)
    return fail(ctx, WVL_EUNSUPPORTED,
                "density: %lld fine boxes meet one tile (at most %d are supported)",
                (long long)maxc, kDensMaxCover);
  if (P->nsf >= (1 << 24))   // the tile kernel's lookup keys hold 24-bit indices
    return fail(ctx, WVL_EUNSUPPORTED, "density: more than 2^24 - 1 functions");
  // FP32: the tiles of at most kDensChunkOne functions first (a launch of
  // their own, with less LDS per workgroup), then the others.  FP64 (chunks of 64, so
  // about half the tiles need two) runs all tiles in one launch, which
  // measured faster.
  std::vector<int32_t> tord[2];
  for (int d = 0; d < 2; ++d) {
    tord[d].reserve(ntile);
    P->dens_one[d] = 0;
    if (d == 1) {
      for (int64_t t = 0; t < ntile; ++t) tord[d].push_back((int32_t)t);
      continue;
    }
    for (int pass = 0; pass < 2; ++pass)
      for (int64_t t = 0; t < ntile; ++t)
        if ((cptr[t + 1] - cptr[t] <= kDensChunkOne) == (pass == 0)) tord[d].push_back((int32_t)t);
    for (int64_t t = 0; t < ntile; ++t) P->dens_one[d] += cptr[t + 1] - cptr[t] <= kDensChunkOne;
  }
  auto drop = [&]() {
    for (void** p : {(void**)&P->d_cptr, (void**)&P->d_csf, (void**)&P->d_tord[0],
                     (void**)&P->d_tord[1]})
      if (*p) {
        (void)hipFree(*p);
        *p = nullptr;
      }
  };
  wvl_status st;
  // d_cptr last: it marks the lists as ready
  if ((st = upload(ctx, &P->d_csf, csf.data(), sizeof(int32_t) * csf.size())) != WVL_OK ||
      (st = upload(ctx, &P->d_tord[0], tord[0].data(), sizeof(int32_t) * tord[0].size())) !=
          WVL_OK ||
      (st = upload(ctx, &P->d_tord[1], tord[1].data(), sizeof(int32_t) * tord[1].size())) !=
          WVL_OK ||
      (st = upload(ctx, &P->d_cptr, cptr.data(), sizeof(int64_t) * cptr.size())) != WVL_OK) {
    drop();
    return st;
  }
  if (hipError_t e = hipStreamSynchronize(ctx->stream); e != hipSuccess) {
    drop();
    return hip_fail(ctx, "density tile lists upload", "hipStreamSynchronize", e);
  }
  return WVL_OK;
}

wvl_status wvl_density(wvl_plan* P, wvl_dtype dt, const void* fine, const int64_t* k_rowptr,
                       const int32_t* k_col, const double* k_val, int64_t k_nnz, void* rho,
                       void* work) {
  if (!P) return fail(nullptr, WVL_EINVAL, "wvl_density: null plan");
  wvl_ctx* ctx = P->ctx;
  if (check_dt(ctx, dt) != WVL_OK) return WVL_EINVAL;
  if (k_nnz < 0) return fail(ctx, WVL_EINVAL, "wvl_density: k_nnz < 0");
  if (!rho) return fail(ctx, WVL_EINVAL, "wvl_density: null rho");
  (void)work;
  if (P->nsf > 0 && (!fine || !k_rowptr || (k_nnz > 0 && (!k_col || !k_val))))
    return fail(ctx, WVL_EINVAL, "wvl_density: null buffer");
  wvl_status st = ensure_cover(P);
  if (st != WVL_OK) return st;
  const int f64 = dt == WVL_F64 ? 1 : 0;
  int gf[3];
  for (int a = 0; a < 3; ++a) gf[a] = 2 * ctx->grid.n[a] + 29;
  WVL_LAUNCH(ctx, KK_DENS_TILE,
             launch_dens_tile(f64, ctx->stream, P->d_sf, P->d_foff, fine, k_rowptr, k_col, k_val,
                              k_nnz, P->d_cptr, P->d_csf, P->d_tord[f64], P->dens_one[f64], gf,
                              rho));
  return WVL_OK;
}

// ---------------------------------------------------------------------------
// Fermi operator expansion (Sec. IV.B, App. B)
// ---------------------------------------------------------------------------

// transpose positions in the S pattern, and the S entries' positions (and
// their transposes') in the H pattern
static wvl_status ensure_foe_maps(wvl_plan* P) {
  PatternCache& S = P->pat[0];
  if (S.maxdeg > 0) return WVL_OK;   // set once every map is on the device
  wvl_ctx* ctx = P->ctx;
  const PatternCache& Hp = P->pat[1];
  const int n = P->nsf;
  std::vector<int64_t> srp(n + 1), hrp(n + 1);
  std::vector<int32_t> scol(S.nnz), hcol(Hp.nnz);
  WVL_HIP(ctx, hipMemcpyAsync(srp.data(), S.d_rowptr, sizeof(int64_t) * (n + 1),
                              hipMemcpyDeviceToHost, ctx->stream));
  WVL_HIP(ctx, hipMemcpyAsync(hrp.data(), Hp.d_rowptr, sizeof(int64_t) * (n + 1),
                              hipMemcpyDeviceToHost, ctx->stream));
  if (S.nnz)
    WVL_HIP(ctx, hipMemcpyAsync(scol.data(), S.d_col, sizeof(int32_t) * S.nnz,
                                hipMemcpyDeviceToHost, ctx->stream));
  if (Hp.nnz)
    WVL_HIP(ctx, hipMemcpyAsync(hcol.data(), Hp.d_col, sizeof(int32_t) * Hp.nnz,
                                hipMemcpyDeviceToHost, ctx->stream));
  WVL_HIP(ctx, hipStreamSynchronize(ctx->stream));
  auto find = [](const std::vector<int64_t>& rp, const std::vector<int32_t>& cl, int i,
                 int j) -> int64_t {
    const auto b = cl.begin() + rp[i], e = cl.begin() + rp[i + 1];
    const auto it = std::lower_bound(b, e, j);
    return (it != e && *it == j) ? (int64_t)(it - cl.begin()) : -1;
  };
  std::vector<int64_t> tpos(S.nnz), hpos(S.nnz), htpos(S.nnz), dpos(n);
  int maxdeg = 0;
  for (int i = 0; i < n; ++i) maxdeg = std::max(maxdeg, (int)(srp[i + 1] - srp[i]));
  if (maxdeg > kFoeMaxDeg || S.nnz > INT32_MAX || n > kFoeMaxCol)
    return fail(ctx, WVL_EUNSUPPORTED,
                "wvl_foe: overlap pattern with %d entries in a row (at most %d), %lld in all or "
                "%d rows (at most %d)",
                maxdeg, kFoeMaxDeg, (long long)S.nnz, n, kFoeMaxCol);
  for (int i = 0; i < n; ++i) {
    dpos[i] = find(srp, scol, i, i);
    if (dpos[i] < 0)
      return fail(ctx, WVL_EUNSUPPORTED, "wvl_foe: row %d of the overlap pattern has no diagonal",
                  i);
  }
  for (int i = 0; i < n; ++i)
    for (int64_t p = srp[i]; p < srp[i + 1]; ++p) {
      const int j = scol[p];
      tpos[p] = find(srp, scol, j, i);
      hpos[p] = find(hrp, hcol, i, j);
      htpos[p] = find(hrp, hcol, j, i);
      if (tpos[p] < 0 || hpos[p] < 0 || htpos[p] < 0)
        return fail(ctx, WVL_EUNSUPPORTED,
                    "wvl_foe: overlap pattern not symmetric or not inside the H pattern");
    }
  // product work of row i: the entries of the rows k it holds
  std::vector<int64_t> work(n, 0);
  std::vector<int32_t> rows(n);
  for (int i = 0; i < n; ++i) {
    rows[i] = i;
    for (int64_t p = srp[i]; p < srp[i + 1]; ++p) work[i] += srp[scol[p] + 1] - srp[scol[p]];
  }
  std::stable_sort(rows.begin(), rows.end(),
                   [&](int32_t a, int32_t b) { return work[a] > work[b]; });
  // buffers of an earlier call that failed part way
  auto drop = [](auto*& q) {
    if (q) (void)hipFree(q);
    q = nullptr;
  };
  drop(S.d_foe_rows);
  drop(S.d_tpos);
  drop(S.d_hpos);
  drop(S.d_htpos);
  drop(S.d_dpos);
  wvl_status st;
  if ((st = upload(ctx, &S.d_foe_rows, rows.data(), sizeof(int32_t) * rows.size())) != WVL_OK ||
      (st = upload(ctx, &S.d_tpos, tpos.data(), sizeof(int64_t) * tpos.size())) != WVL_OK ||
      (st = upload(ctx, &S.d_hpos, hpos.data(), sizeof(int64_t) * hpos.size())) != WVL_OK ||
      (st = upload(ctx, &S.d_htpos, htpos.data(), sizeof(int64_t) * htpos.size())) != WVL_OK ||
      (st = upload(ctx, &S.d_dpos, dpos.data(), sizeof(int64_t) * dpos.size())) != WVL_OK)
    return st;
  WVL_HIP(ctx, hipStreamSynchronize(ctx->stream));
  S.maxdeg = maxdeg;
  return WVL_OK;
}

// wvl_foe scratch: 9 matrices on P (or 7 + npl with every T^i kept), the
// traces, four reduction slots (and the coefficients)
static size_t foe_scratch_bytes(int64_t nnz, int npl, bool keep) {
  return keep ? 8 * ((size_t)(npl + 7) * nnz + 2 * (size_t)npl + 6)
              : 8 * ((size_t)9 * nnz + (size_t)npl + 5);
}

wvl_status wvl_foe(wvl_plan* P, const double* s_val, const double* h_val, int32_t npl,
                   double delta, double n_occ, double eps_min, double eps_max, double* k_val,
                   double* mu_out, double* e_bs_out, void* scratch, size_t scratch_bytes) {
  if (!P) return fail(nullptr, WVL_EINVAL, "wvl_foe: null plan");
  wvl_ctx* ctx = P->ctx;
  const int n = P->nsf;
  if (npl < 1) return fail(ctx, WVL_EINVAL, "wvl_foe: npl < 1");
  if (!(delta > 0.0) || !std::isfinite(delta)) return fail(ctx, WVL_EINVAL, "wvl_foe: delta");
  if (!(n_occ > 0.0) || !(n_occ < n)) return fail(ctx, WVL_EINVAL, "wvl_foe: n_occ not in (0, nsf)");
  if (!s_val || !h_val || !k_val || !scratch)
    return fail(ctx, WVL_EINVAL, "wvl_foe: null buffer");
  if (!std::isfinite(eps_min) || !std::isfinite(eps_max))
    return fail(ctx, WVL_EINVAL, "wvl_foe: spectral bounds not finite");
  wvl_status st;
  if ((st = ensure_pattern(P, 0)) != WVL_OK || (st = ensure_pattern(P, 1)) != WVL_OK ||
      (st = ensure_foe_maps(P)) != WVL_OK)
    return st;
  const PatternCache& pc = P->pat[0];
  const int64_t nnz = pc.nnz;
  if (scratch_bytes < foe_scratch_bytes(nnz, npl, false))
    return fail(ctx, WVL_EINVAL, "wvl_foe: scratch of %zu bytes, at least %zu needed",
                scratch_bytes, foe_scratch_bytes(nnz, npl, false));
  // with room for every T^i, pass 2 sums the kept matrices instead of
  // running the recursion again
  const bool keep = scratch_bytes >= foe_scratch_bytes(nnz, npl, true);
  hipStream_t s = ctx->stream;
  const int64_t* rp = pc.d_rowptr;
  const int32_t* cl = pc.d_col;
  const int32_t* rw = pc.d_row;
  const int64_t* tp = pc.d_tpos;
  double* w = (double*)scratch;
  // matrices on P: six, then T^0 .. T^npl (kept) or three T^i in turn; the
  // traces, four reduction slots, the coefficients (kept)
  double *Ss = w, *Sh = w + nnz, *Hs = w + 2 * nnz, *X = w + 3 * nnz, *Ht = w + 4 * nnz;
  double* Kp = w + 5 * nnz;
  double* Tall = w + 6 * nnz;
  double* tr = w + (keep ? npl + 7 : 9) * nnz;
  double* red = tr + npl + 1;
  double* cf = red + 4;
  auto Tm = [&](int i) { return Tall + (keep ? i : i % 3) * nnz; };
  int lognb = 5;
  while ((1 << lognb) < pc.maxdeg) ++lognb;
  // C = al (A B)|_P (+ be D)
  auto mm = [&](double al, const double* A, const double* B, double be, const double* D,
                double* C) {
    return launch_foe_mm(s, n, pc.d_foe_rows, rp, cl, al, A, B, be, D, C, lognb, pc.maxdeg);
  };
  auto axpby = [&](double a, const double* x, double b, const double* y, double d, double* o) {
    return launch_foe_axpby(s, nnz, a, x, b, y, rw, cl, d, o);
  };
  // S and H on the overlap pattern, symmetric parts (they are symmetric in
  // exact arithmetic); S^-1/2 ~ (3 I - S) / 2, the first-order Taylor form
  WVL_LAUNCH(ctx, KK_FOE, launch_foe_sym(s, nnz, tp, s_val, Ss));
  WVL_LAUNCH(ctx, KK_FOE, axpby(-0.5, Ss, 0.0, nullptr, 1.5, Sh));
  WVL_LAUNCH(ctx, KK_FOE, launch_foe_gather(s, nnz, pc.d_hpos, h_val, X));
  WVL_LAUNCH(ctx, KK_FOE, launch_foe_gather(s, nnz, pc.d_htpos, h_val, Ht));
  WVL_LAUNCH(ctx, KK_FOE, axpby(0.5, X, 0.5, Ht, 0.0, Hs));
  // spectral bounds: Gershgorin discs of S^-1/2 H S^-1/2 unless given
  // (Sh and Hs are symmetric: they are their own transposes)
  if (eps_min >= eps_max) {
    WVL_LAUNCH(ctx, KK_FOE, mm(1.0, Sh, Hs, 0.0, nullptr, X));
    WVL_LAUNCH(ctx, KK_FOE, mm(1.0, X, Sh, 0.0, nullptr, Tm(0)));
    WVL_LAUNCH(ctx, KK_FOE, launch_foe_sym(s, nnz, tp, Tm(0), Ht));
    // X and T^0 are free here, and each holds nnz >= n doubles
    WVL_LAUNCH(ctx, KK_FOE, launch_foe_gersh(s, n, rp, cl, Ht, X, Tm(0), red));
    double b[2];
    WVL_HIP(ctx, hipMemcpyAsync(b, red, sizeof b, hipMemcpyDeviceToHost, s));
    WVL_HIP(ctx, hipStreamSynchronize(s));
    eps_min = b[0];
    eps_max = b[1];
    if (!(eps_max > eps_min)) eps_max = eps_min + 1.0;
  }
  const double sigma = 2.0 / (eps_max - eps_min), tau = 0.5 * (eps_min + eps_max);
  // H~ = sigma (H - tau S), then H~' = S^-1/2 H~ S^-1/2 (symmetric part)
  WVL_LAUNCH(ctx, KK_FOE, axpby(sigma, Hs, -sigma * tau, Ss, 0.0, Hs));
  WVL_LAUNCH(ctx, KK_FOE, mm(1.0, Sh, Hs, 0.0, nullptr, X));
  WVL_LAUNCH(ctx, KK_FOE, mm(1.0, X, Sh, 0.0, nullptr, Tm(0)));
  WVL_LAUNCH(ctx, KK_FOE, launch_foe_sym(s, nnz, tp, Tm(0), Ht));
  // Spectrum guard: with the Taylor S^-1/2, S^-1/2 S S^-1/2 is not I, so
  // H~' can reach outside [-1, 1] even for exact bounds, and T^i then grows
  // like cosh(i acosh|x|).  When its Gershgorin discs [a, b] do, the
  // recursion runs on X = (H~' - c I) / r with [c - r, c + r] =
  // [min(a, -1), max(b, 1)], and f is taken at (r x + c) / sigma + tau:
  // the effective scale sigma / r and shift tau + c / sigma.
  double gc = 0.0, gr = 1.0;
  {
    WVL_LAUNCH(ctx, KK_FOE, launch_foe_gersh(s, n, rp, cl, Ht, X, Tm(0), red));
    double b[2];
    WVL_HIP(ctx, hipMemcpyAsync(b, red, sizeof b, hipMemcpyDeviceToHost, s));
    WVL_HIP(ctx, hipStreamSynchronize(s));
    if (!std::isfinite(b[0]) || !std::isfinite(b[1]))
      return fail(ctx, WVL_EINVAL, "wvl_foe: S or H holds values that are not finite");
    if (b[0] < -1.0 || b[1] > 1.0) {
      const double glo = std::min(b[0], -1.0), ghi = std::max(b[1], 1.0);
      gc = 0.5 * (glo + ghi);
      gr = 0.5 * (ghi - glo);
      WVL_LAUNCH(ctx, KK_FOE, axpby(1.0 / gr, Ht, 0.0, nullptr, -gc / gr, Tm(0)));
      WVL_LAUNCH(ctx, KK_FOE, axpby(1.0, Tm(0), 0.0, nullptr, 0.0, Ht));
    }
  }
  const double sig_f = sigma / gr, tau_f = tau + gc / sigma;
  // pass 1: traces of the Chebyshev matrices T^0 .. T^npl
  auto start = [&]() -> wvl_status {
    WVL_LAUNCH(ctx, KK_FOE, axpby(0.0, nullptr, 0.0, nullptr, 1.0, Tm(0)));
    WVL_LAUNCH(ctx, KK_FOE, axpby(1.0, Ht, 0.0, nullptr, 0.0, Tm(1)));
    return WVL_OK;
  };
  auto trace = [&](int i) { return launch_foe_trace(s, n, pc.d_dpos, Tm(i), 0, 1, tr, i); };
  if ((st = start()) != WVL_OK) return st;
  if (!keep) {
    WVL_LAUNCH(ctx, KK_FOE, trace(0));
    WVL_LAUNCH(ctx, KK_FOE, trace(1));
  }
  for (int j = 1; j < npl; ++j) {
    WVL_LAUNCH(ctx, KK_FOE_MM, mm(2.0, Ht, Tm(j), -1.0, Tm(j - 1), Tm(j + 1)));
    if (!keep) WVL_LAUNCH(ctx, KK_FOE, trace(j + 1));
  }
  if (keep) WVL_LAUNCH(ctx, KK_FOE, launch_foe_trace(s, n, pc.d_dpos, Tall, nnz, npl + 1, tr, 0));
  std::vector<double> trh(npl + 1);
  WVL_HIP(ctx, hipMemcpyAsync(trh.data(), tr, sizeof(double) * (npl + 1), hipMemcpyDeviceToHost,
                              s));
  WVL_HIP(ctx, hipStreamSynchronize(s));
  // chemical potential: Tr K'(mu) = c_0/2 Tr T^0 + sum_i c_i Tr T^i = n_occ,
  // increasing in mu; bisection
  if (!P->foe_coef || P->foe_coef->npl != npl) {
    P->foe_coef.reset(new (std::nothrow) FoeCoef(npl));
    if (!P->foe_coef) return fail(ctx, WVL_ENOMEM, "wvl_foe: host allocation failed");
  }
  const FoeCoef& coefficients = *P->foe_coef;
  std::vector<double> coef, g;
  coefficients.weights(trh, &g);
  auto trace_at = [&](double mu) { return coefficients.trace(g, sig_f, tau_f, mu, delta); };
  double lo = (gc - gr) / sigma + tau - 20.0 * delta, hi = (gc + gr) / sigma + tau + 20.0 * delta;
  for (int it = 0; it < 200 && hi - lo > 1e-13 * std::max(1.0, std::fabs(lo) + std::fabs(hi));
       ++it) {
    const double mid = 0.5 * (lo + hi);
    if (trace_at(mid) < n_occ)
      lo = mid;
    else
      hi = mid;
  }
  const double mu = 0.5 * (lo + hi);
  coefficients(sig_f, tau_f, mu, delta, &coef);
  // pass 2: K' = c_0/2 I + sum_i c_i T^i(H~')
  if (keep) {
    // the host vector must outlive the copy: wait for it before going on
    WVL_HIP(ctx, hipMemcpyAsync(cf, coef.data(), sizeof(double) * (npl + 1),
                                hipMemcpyHostToDevice, s));
    WVL_HIP(ctx, hipStreamSynchronize(s));
    WVL_LAUNCH(ctx, KK_FOE, launch_foe_series(s, nnz, npl, cf, Tall, rw, cl, Kp));
  } else {
    WVL_LAUNCH(ctx, KK_FOE, axpby(coef[1], Ht, 0.0, nullptr, 0.5 * coef[0], Kp));
    if ((st = start()) != WVL_OK) return st;
    for (int j = 1; j < npl; ++j) {
      WVL_LAUNCH(ctx, KK_FOE_MM, mm(2.0, Ht, Tm(j), -1.0, Tm(j - 1), Tm(j + 1)));
      WVL_LAUNCH(ctx, KK_FOE, axpby(1.0, Kp, coef[j + 1], Tm(j + 1), 0.0, Kp));
    }
  }
  // K = S^-1/2 K' S^-1/2 (symmetric part); E_BS = Tr(K H~) / sigma + tau Tr(K S)
  WVL_LAUNCH(ctx, KK_FOE, mm(1.0, Sh, Kp, 0.0, nullptr, X));
  WVL_LAUNCH(ctx, KK_FOE, mm(1.0, X, Sh, 0.0, nullptr, Tm(0)));
  WVL_LAUNCH(ctx, KK_FOE, launch_foe_sym(s, nnz, tp, Tm(0), k_val));
  WVL_LAUNCH(ctx, KK_FOE, launch_foe_dot(s, nnz, k_val, Hs, X, red, 2));
  WVL_LAUNCH(ctx, KK_FOE, launch_foe_dot(s, nnz, k_val, Ss, X, red, 3));
  double e2[2];
  WVL_HIP(ctx, hipMemcpyAsync(e2, red + 2, sizeof e2, hipMemcpyDeviceToHost, s));
  WVL_HIP(ctx, hipStreamSynchronize(s));
  if (mu_out) *mu_out = mu;
  if (e_bs_out) *e_bs_out = e2[0] / sigma + tau * e2[1];
  return WVL_OK;
}

// ---------------------------------------------------------------------------
// support-function gradient (Eq. (gradient), Sec. IV.A)
// ---------------------------------------------------------------------------

static size_t gradient_scratch_bytes(int64_t nnz) { return 8 * (size_t)7 * (size_t)nnz; }

wvl_status wvl_gradient(wvl_plan* P, wvl_dtype dt, const double* s_val, const double* h_val,
                        const double* k_val, const void* psi_c, const void* hpsi_c, void* g_c,
                        void* scratch, size_t scratch_bytes) {
  if (!P) return fail(nullptr, WVL_EINVAL, "wvl_gradient: null plan");
  wvl_ctx* ctx = P->ctx;
  if (check_dt(ctx, dt) != WVL_OK) return WVL_EINVAL;
  if (P->nsf == 0) return WVL_OK;
  if (!s_val || !h_val || !k_val || !psi_c || !hpsi_c || !g_c || !scratch)
    return fail(ctx, WVL_EINVAL, "wvl_gradient: null buffer");
  wvl_status st;
  if ((st = ensure_pattern(P, 0)) != WVL_OK || (st = ensure_pattern(P, 1)) != WVL_OK ||
      (st = ensure_foe_maps(P)) != WVL_OK)
    return st;
  const PatternCache& pc = P->pat[0];
  const int64_t nnz = pc.nnz;
  if (scratch_bytes < gradient_scratch_bytes(nnz))
    return fail(ctx, WVL_EINVAL, "wvl_gradient: scratch of %zu bytes, at least %zu needed",
                scratch_bytes, gradient_scratch_bytes(nnz));
  hipStream_t s = ctx->stream;
  const int n = P->nsf;
  double* w = (double*)scratch;
  double *Ss = w, *Hp = w + nnz, *A = w + 2 * nnz, *X = w + 3 * nnz, *Lam = w + 4 * nnz;
  double *Si = w + 5 * nnz, *M = w + 6 * nnz;
  int lognb = 5;
  while ((1 << lognb) < pc.maxdeg) ++lognb;
  auto mm = [&](const double* L, const double* R, double* C) {
    return launch_foe_mm(s, n, pc.d_foe_rows, pc.d_rowptr, pc.d_col, 1.0, L, R, 0.0, nullptr, C,
                         lognb, pc.maxdeg);
  };
  // the matrices on the overlap pattern P, every product truncated to P:
  // A = S K; Lambda = (H K) S; M = 1/2 (2 I - S) (Lambda + Lambda^T)
  WVL_LAUNCH(ctx, KK_FOE, launch_foe_sym(s, nnz, pc.d_tpos, s_val, Ss));
  WVL_LAUNCH(ctx, KK_FOE, launch_foe_gather(s, nnz, pc.d_hpos, h_val, Hp));
  WVL_LAUNCH(ctx, KK_FOE_MM, mm(Ss, k_val, A));
  WVL_LAUNCH(ctx, KK_FOE_MM, mm(Hp, k_val, X));
  WVL_LAUNCH(ctx, KK_FOE_MM, mm(X, Ss, Lam));
  WVL_LAUNCH(ctx, KK_FOE, launch_foe_sym(s, nnz, pc.d_tpos, Lam, X));   // (Lambda + Lambda^T) / 2
  WVL_LAUNCH(ctx, KK_FOE,
             launch_foe_axpby(s, nnz, -1.0, Ss, 0.0, nullptr, pc.d_row, pc.d_col, 2.0, Si));
  WVL_LAUNCH(ctx, KK_FOE_MM, mm(Si, X, M));
  // g_a = L^a [sum_d A_ad H phi_d - M_ad phi_d]
  for (int s0 = 0; s0 < n; s0 += 65535) {
    const int cnt = std::min(65535, n - s0);
    WVL_LAUNCH(ctx, KK_GRADIENT,
               launch_grad_rows(dt == WVL_F64, s, P->d_sf, P->d_seg, P->d_rt, P->d_rr,
                                pc.d_rowptr, pc.d_col, A, M, psi_c, hpsi_c, s0, cnt, g_c));
  }
  return WVL_OK;
}

wvl_status wvl_update(wvl_plan* P, wvl_dtype dt, double eta, const void* hpsi_c,
                      const double* h_val, void* psi_c) {
  if (!P) return fail(nullptr, WVL_EINVAL, "wvl_update: null plan");
  wvl_ctx* ctx = P->ctx;
  if (check_dt(ctx, dt) != WVL_OK) return WVL_EINVAL;
  if (P->nsf == 0) return WVL_OK;
  if (!hpsi_c || !h_val || !psi_c) return fail(ctx, WVL_EINVAL, "wvl_update: null buffer");
  if (!P->in_sub_out)
    return fail(ctx, WVL_EINVAL, "wvl_update: an input pattern is not inside its output pattern");
  if (!std::isfinite(eta)) return fail(ctx, WVL_EINVAL, "wvl_update: eta is not finite");
  wvl_status st = ensure_pattern(P, 1);
  if (st != WVL_OK) return st;
  const PatternCache& pc = P->pat[1];
  for (int s0 = 0; s0 < P->nsf; s0 += 65535) {
    const int n = std::min(65535, P->nsf - s0);
    WVL_LAUNCH(ctx, KK_UPDATE,
               launch_update(dt == WVL_F64, ctx->stream, P->d_sf, P->d_seg, P->d_rt, eta, hpsi_c,
                             pc.d_rowptr, pc.d_col, h_val, psi_c, s0, n, P->max_in_segs, 0,
                             nullptr, nullptr));
  }
  return WVL_OK;
}

wvl_status wvl_precondition(wvl_plan* P, wvl_dtype dt, const void* g_c, const double* conf,
                            const double* eps, int32_t niter, void* x_c, void* workspace,
                            void* scratch) {
  if (!P) return fail(nullptr, WVL_EINVAL, "wvl_precondition: null plan");
  wvl_ctx* ctx = P->ctx;
  if (check_dt(ctx, dt) != WVL_OK) return WVL_EINVAL;
  if (niter < 0) return fail(ctx, WVL_EINVAL, "wvl_precondition: niter < 0");
  if (P->nsf == 0) return WVL_OK;
  if (!g_c || !x_c || !workspace || !scratch || !eps)
    return fail(ctx, WVL_EINVAL, "wvl_precondition: null buffer");
  if (!P->in_sub_out)
    return fail(ctx, WVL_EINVAL,
                "wvl_precondition: an input pattern is not inside its output pattern");
  const int f64 = dt == WVL_F64, sz = f64 ? 8 : 4;
  char* base = (char*)scratch;
  void* r = base;                   base += align_bytes(P->info.in_coefs * sz);
  void* p = base;                   base += align_bytes(P->info.in_coefs * sz);
  void* ap_in = base;               base += align_bytes(P->info.in_coefs * sz);
  void* ap_out = base;              base += align_bytes(P->info.out_coefs * sz);
  double* rr = (double*)base;       base += align_bytes(8ll * P->nsf);
  double* pap = (double*)base;      base += align_bytes(8ll * P->nsf);
  double* rrn = (double*)base;
  const uint32_t terms = WVL_KIN | (conf ? WVL_POT : 0);
  hipStream_t st = ctx->stream;
  for (int s0 = 0; s0 < P->nsf; s0 += 65535) {
    const int n = std::min(65535, P->nsf - s0);
    WVL_LAUNCH(ctx, KK_UPDATE, launch_cg_init(f64, st, P->d_sf, g_c, x_c, r, p, s0, n));
    WVL_LAUNCH(ctx, KK_UPDATE, launch_sf_dot(f64, st, P->d_sf, r, r, rr, s0, n));
  }
  for (int it = 0; it < niter; ++it) {
    // A p = P_L (T + C) P_L p - min(eps, 0) p
    wvl_status s = apply_impl(P, dt, terms, p, nullptr, ap_out, nullptr, nullptr, workspace, 0,
                              "wvl_precondition", conf);
    if (s != WVL_OK) return s;
    for (int s0 = 0; s0 < P->nsf; s0 += 65535) {
      const int n = std::min(65535, P->nsf - s0);
      WVL_LAUNCH(ctx, KK_UPDATE,
                 launch_update(f64, st, P->d_sf, P->d_seg, P->d_rt, 0.0, ap_out, nullptr, nullptr,
                               nullptr, p, s0, n, P->max_in_segs, 1, eps, ap_in));
      WVL_LAUNCH(ctx, KK_UPDATE, launch_sf_dot(f64, st, P->d_sf, p, ap_in, pap, s0, n));
      WVL_LAUNCH(ctx, KK_UPDATE,
                 launch_cg_xr(f64, st, P->d_sf, rr, pap, p, ap_in, x_c, r, s0, n));
      WVL_LAUNCH(ctx, KK_UPDATE, launch_sf_dot(f64, st, P->d_sf, r, r, rrn, s0, n));
      WVL_LAUNCH(ctx, KK_UPDATE, launch_cg_p(f64, st, P->d_sf, rr, rrn, r, p, s0, n));
    }
  }
  return WVL_OK;
}

// Captures the apply (and optional S/H values) into G.  Chunks with
// disjoint workspace go to parallel branches.
static wvl_status capture_step(wvl_plan* P, wvl_dtype dt, uint32_t terms, const void* psi_c,
                               const void* pot, void* hpsi_c, double* e_kin, double* e_pot,
                               void* workspace, double* s_val, double* h_val, wvl_graph* G) {
  wvl_ctx* ctx = P->ctx;
  const int f64 = dt == WVL_F64;
  const size_t nch = P->lay.chunks.size();
  // kernels are loaded lazily on first use; a load (which also uploads the
  // constant filter tables) must not happen inside the capture
  int pe = preload_kernels();
  if (pe == 0) pe = preload_fused_kernels();
  if (pe != 0)
    return hip_fail(ctx, "graph capture", "kernel preload (hipFuncGetAttributes)",
                    (hipError_t)pe);
  const size_t nbr = P->lay.disjoint ? std::min<size_t>(nch, 4) : 0;
  // streams[0] is the capture origin (the context's stream may be the
  // legacy default stream, which cannot be captured); 1.. are branches
  while (P->streams.size() < nbr + 1) {
    hipStream_t st = nullptr;
    WVL_HIP(ctx, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    P->streams.push_back(st);
  }
  std::vector<hipEvent_t>& ev = G->events;
  auto cleanup = [&]() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    ev.clear();
  };
  for (size_t k = 0; k < nbr + 1; ++k) {
    hipEvent_t e = nullptr;
    if (hipError_t he = hipEventCreateWithFlags(&e, hipEventDisableTiming); he != hipSuccess) {
      cleanup();
      return hip_fail(ctx, "graph capture", "hipEventCreateWithFlags", he);
    }
    ev.push_back(e);
  }
  const bool prof = ctx->prof;
  ctx->prof = false;   // no tracing events inside a graph
  hipStream_t cs = P->streams[0];
  hipError_t he = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  wvl_status st = he == hipSuccess ? WVL_OK
                                   : hip_fail(ctx, "graph capture", "hipStreamBeginCapture", he);
  // fork/join steps: the first failing call ends the capture with its name
  auto step = [&](hipError_t e, const char* call) {
    if (st == WVL_OK && e != hipSuccess) st = hip_fail(ctx, "graph capture", call, e);
  };
  if (st == WVL_OK && P->nsf > 0) {
    if (nbr > 0) {
      // fork: every branch waits for the capture origin
      step(hipEventRecord(ev[0], cs), "hipEventRecord (fork)");
      for (size_t b = 0; st == WVL_OK && b < nbr; ++b)
        step(hipStreamWaitEvent(P->streams[b + 1], ev[0], 0), "hipStreamWaitEvent (fork)");
      for (size_t c = 0; st == WVL_OK && c < nch; ++c)
        st = apply_chunk(P, c, f64, terms, psi_c, pot, hpsi_c, e_kin, e_pot, workspace, 0,
                         P->streams[1 + c % nbr]);
      // join
      for (size_t b = 0; st == WVL_OK && b < nbr; ++b) {
        step(hipEventRecord(ev[b + 1], P->streams[b + 1]), "hipEventRecord (join)");
        if (st == WVL_OK) step(hipStreamWaitEvent(cs, ev[b + 1], 0), "hipStreamWaitEvent (join)");
      }
    } else {
      for (size_t c = 0; st == WVL_OK && c < nch; ++c)
        st = apply_chunk(P, c, f64, terms, psi_c, pot, hpsi_c, e_kin, e_pot, workspace, 0, cs);
    }
    for (int ket_out = 0; st == WVL_OK && ket_out < 2; ++ket_out) {
      double* val = ket_out ? h_val : s_val;
      const PatternCache& pc = P->pat[ket_out];
      if (!val || pc.nnz == 0) continue;
      // S = <psi|psi> is symmetric: half the pairs, each written twice
      const bool half = !ket_out && pc.nnz_u > 0;
      const int e = launch_sparse_values(f64, cs, P->d_sf, P->d_seg, P->d_rt, P->d_rr, ket_out,
                                         psi_c, ket_out ? hpsi_c : psi_c, pc.d_row, pc.d_col,
                                         half ? pc.d_order_u : pc.d_order,
                                         half ? pc.d_mirror_u : nullptr,
                                         half ? pc.nnz_u : pc.nnz, val);
      if (e != 0) st = hip_fail(ctx, "graph capture", "launch of sparse_values", (hipError_t)e);
    }
  }
  hipGraph_t g = nullptr;
  if (he == hipSuccess) {
    const hipError_t ee = hipStreamEndCapture(cs, &g);
    if (st == WVL_OK && ee != hipSuccess)
      st = hip_fail(ctx, "graph capture", "hipStreamEndCapture", ee);
  }
  ctx->prof = prof;
  if (st != WVL_OK) {
    if (g) (void)hipGraphDestroy(g);
    cleanup();
    return st;
  }
  hipGraphExec_t x = nullptr;
  he = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (he != hipSuccess) {
    (void)hipGraphDestroy(g);
    cleanup();
    return hip_fail(ctx, "graph capture", "hipGraphInstantiate", he);
  }
  G->plan = P;
  G->graph = g;
  G->exec = x;
  G->layout_version = P->layout_version;
  return WVL_OK;
}

wvl_status wvl_graph_create(wvl_plan* P, wvl_dtype dt, uint32_t terms, const void* psi_c,
                            const void* pot, void* hpsi_c, double* e_kin, double* e_pot,
                            void* workspace, double* s_val, double* h_val, wvl_graph** graph) {
  if (!graph) return fail(P ? P->ctx : nullptr, WVL_EINVAL, "wvl_graph_create: null graph pointer");
  *graph = nullptr;
  wvl_status st = apply_args(P, dt, terms, psi_c, pot, hpsi_c, workspace, "wvl_graph_create");
  if (st != WVL_OK) return st;
  if ((s_val || h_val) && P->nsf > 0 && !psi_c)
    return fail(P->ctx, WVL_EINVAL, "wvl_graph_create: S/H values need psi_c");
  if (s_val && (st = ensure_pattern(P, 0)) != WVL_OK) return st;
  if (h_val && (st = ensure_pattern(P, 1)) != WVL_OK) return st;
  wvl_graph* G = new (std::nothrow) wvl_graph;
  if (!G) return fail(P->ctx, WVL_ENOMEM, "wvl_graph_create: out of host memory");
  st = capture_step(P, dt, terms, psi_c, pot, hpsi_c, e_kin, e_pot, workspace, s_val, h_val, G);
  if (st != WVL_OK) {
    delete G;
    return st;
  }
  *graph = G;
  return WVL_OK;
}

wvl_status wvl_graph_launch(wvl_graph* G) {
  if (!G || !G->plan) return fail(nullptr, WVL_EINVAL, "wvl_graph_launch: null graph");
  wvl_ctx* ctx = G->plan->ctx;
  if (G->layout_version != G->plan->layout_version)
    return fail(ctx, WVL_EINVAL, "wvl_graph_launch: the plan's layout changed since the capture");
  WVL_HIP(ctx, hipGraphLaunch(G->exec, ctx->stream));
  return WVL_OK;
}

void wvl_graph_destroy(wvl_graph* G) {
  if (!G) return;
  if (G->exec) (void)hipGraphExecDestroy(G->exec);
  if (G->graph) (void)hipGraphDestroy(G->graph);
  for (hipEvent_t e : G->events) (void)hipEventDestroy(e);
  delete G;
}

static wvl_status set_layout(wvl_plan* P, Layout&& L) {
  wvl_ctx* ctx = P->ctx;
  P->lay = std::move(L);
  P->info.chunks = (int64_t)P->lay.chunks.size();
  ++P->layout_version;
  WVL_HIP(ctx, hipMemcpyAsync(P->d_wk, P->lay.wk.data(), sizeof(SfWork) * P->nsf,
                              hipMemcpyHostToDevice, ctx->stream));
  WVL_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return WVL_OK;
}

wvl_status wvl_plan_set_schedule(wvl_plan* P, int32_t nbins, int32_t kin_mfma) {
  if (!P) return fail(nullptr, WVL_EINVAL, "wvl_plan_set_schedule: null plan");
  if (nbins < 1 || (kin_mfma != 0 && kin_mfma != 1))
    return fail(P->ctx, WVL_EINVAL, "wvl_plan_set_schedule: nbins >= 1, kin_mfma 0 or 1");
  Layout L;
  std::string err;
  if (!make_layout(P, nbins, kin_mfma != 0, &L, &err))
    return fail(P->ctx, WVL_EUNSUPPORTED, "%s", err.c_str());
  if (L.bytes(4) > P->ws_cap[0] || L.bytes(8) > P->ws_cap[1])
    return fail(P->ctx, WVL_EINVAL,
                "wvl_plan_set_schedule: this schedule needs more workspace than the plan reported");
  return set_layout(P, std::move(L));
}

wvl_status wvl_plan_autotune(wvl_plan* P, wvl_dtype dt, uint32_t terms, const void* psi_c,
                             const void* pot, void* hpsi_c, void* workspace, int32_t reps,
                             wvl_tune_point* tried, int32_t max_tried, int32_t* ntried,
                             wvl_tune_point* best) {
  wvl_status st = apply_args(P, dt, terms, psi_c, pot, hpsi_c, workspace, "wvl_plan_autotune");
  if (st != WVL_OK) return st;
  wvl_ctx* ctx = P->ctx;
  if (reps < 1) return fail(ctx, WVL_EINVAL, "wvl_plan_autotune: reps must be >= 1");
  if (ntried) *ntried = 0;
  if (P->nsf == 0) return WVL_OK;
  const int sz = dt == WVL_F64 ? 8 : 4;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  WVL_HIP(ctx, hipEventCreate(&e0));
  if (hipError_t he = hipEventCreate(&e1); he != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(ctx, "wvl_plan_autotune", "hipEventCreate", he);
  }
  wvl_tune_point top{0, 0, 1e300};
  int n = 0;
  for (int zm = 0; zm < 2; ++zm)
  for (int nb : kTuneBins) {
    Layout L;
    std::string err;
    if (!make_layout(P, nb, zm != 0, &L, &err) || L.bytes(sz) > P->ws_cap[sz == 8]) continue;
    if ((st = set_layout(P, std::move(L))) != WVL_OK) break;
    // warm-up, then `reps` timed eager applies of this layout
    if ((st = apply_impl(P, dt, terms, psi_c, pot, hpsi_c, nullptr, nullptr, workspace, 0,
                         "wvl_plan_autotune")) != WVL_OK)
      break;
    const char* call = "hipEventRecord";
    hipError_t he = hipEventRecord(e0, ctx->stream);
    for (int r = 0; he == hipSuccess && st == WVL_OK && r < reps; ++r)
      st = apply_impl(P, dt, terms, psi_c, pot, hpsi_c, nullptr, nullptr, workspace, 0,
                      "wvl_plan_autotune");
    if (st != WVL_OK) break;
    if (he == hipSuccess) he = hipEventRecord(e1, ctx->stream);
    if (he == hipSuccess) {
      call = "hipEventSynchronize";
      he = hipEventSynchronize(e1);
    }
    float ms = 0.f;
    if (he == hipSuccess) {
      call = "hipEventElapsedTime";
      he = hipEventElapsedTime(&ms, e0, e1);
    }
    if (he != hipSuccess) {
      st = hip_fail(ctx, "wvl_plan_autotune", call, he);
      break;
    }
    const wvl_tune_point pt{nb, zm, (double)ms / reps};
    if (tried && n < max_tried) tried[n] = pt;
    ++n;
    if (pt.ms < top.ms) top = pt;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != WVL_OK) return st;
  if (ntried) *ntried = n;
  if (n == 0) return fail(ctx, WVL_EUNSUPPORTED, "wvl_plan_autotune: no candidate fits");
  Layout L;
  std::string err;
  if (!make_layout(P, top.nbins, top.kin_mfma != 0, &L, &err))
    return fail(ctx, WVL_EUNSUPPORTED, "%s", err.c_str());
  if ((st = set_layout(P, std::move(L))) != WVL_OK) return st;
  if (best) *best = top;
  return WVL_OK;
}

}  // extern "C"

// HIP kernels for gfx950 (MI355X): local Hamiltonian on batched localization
// regions, and sparse overlap / Hamiltonian matrix elements.
//
// Operator factorization used here (exactly equal, in exact arithmetic, to
// L' (T + R^T W^T V W R) L of the paper's Sec. III.B):
//   potential:  per axis, synthesis followed by the magic filter is one
//               stride-2 upsampling filter C_b (b = scaling/wavelet channel,
//               31 taps); the adjoint chain (transposed magic filter then
//               analysis) is the matching stride-2 downsampling with C_b.
//               Three up passes lead to the fine real-space grid, the
//               potential multiplies there, three down passes come back.
//   kinetic:    the second-derivative filter at h/2 seen from the coarse
//               two-level basis, K_ab = R^T a R along each axis (29 taps,
//               2x2 channels), applied directly on the coarse box.
// Each pass is one launch over every support function of a chunk
// (blockIdx.y = function); threads map to output points, x fastest, so
// global loads and stores along x are coalesced for every axis.
#include <hip/hip_runtime.h>

#include "wvl_filters.h"
#include "wvl_internal.h"

namespace wvl {

__constant__ double cC64[2][31] = {WVL_C0_F64, WVL_C1_F64};
__constant__ float cC32[2][31] = {WVL_C0_F32, WVL_C1_F32};
__constant__ double cK64[2][2][29] = {{WVL_K00_F64, WVL_K01_F64}, {WVL_K10_F64, WVL_K11_F64}};
__constant__ float cK32[2][2][29] = {{WVL_K00_F32, WVL_K01_F32}, {WVL_K10_F32, WVL_K11_F32}};
__constant__ double cKD64[2] = WVL_KD_F64;

template <typename T>
__device__ __forceinline__ T ctab(int b, int n);
template <>
__device__ __forceinline__ double ctab<double>(int b, int n) { return cC64[b][n]; }
template <>
__device__ __forceinline__ float ctab<float>(int b, int n) { return cC32[b][n]; }
template <typename T>
__device__ __forceinline__ T ktab(int a, int b, int n);
template <>
__device__ __forceinline__ double ktab<double>(int a, int b, int n) { return cK64[a][b][n]; }
template <>
__device__ __forceinline__ float ktab<float>(int a, int b, int n) { return cK32[a][b][n]; }

constexpr int TPB = 256;

__device__ __forceinline__ int nr_of(int n) { return 2 * n + 29; }

// deterministic block sum of one double per thread (blockDim.x == TPB)
__device__ double block_sum(double v) {
  __shared__ double red[TPB];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = TPB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------------------
// compressed <-> dense
// ---------------------------------------------------------------------------

// Uncompress: thread per dense point of the input box [8][n2][n1][n0].
template <typename T>
__global__ __launch_bounds__(TPB) void k_gather(const SfDev* __restrict__ sfs,
                                                const wvl_seg* __restrict__ seg,
                                                const int32_t* __restrict__ rt,
                                                const T* __restrict__ psi, T* __restrict__ dst,
                                                const SfWork* __restrict__ wk, int sf0,
                                                int use_work) {
  const int s = blockIdx.y;
  const SfDev& sf = sfs[sf0 + s];
  const int n0 = sf.n[0], n1 = sf.n[1], n2 = sf.n[2];
  const int64_t vol = 8ll * n0 * n1 * n2;
  const int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (idx >= vol) return;
  const int x = (int)(idx % n0);
  int64_t t = idx / n0;
  const int y = (int)(t % n1);
  t /= n1;
  const int z = (int)(t % n2);
  const int c = (int)(t / n2);
  const int pat = c == 0 ? 0 : 1;
  const int64_t r = (int64_t)z * n1 + y;
  const int32_t s0 = rt[sf.rt[pat] + r], s1 = rt[sf.rt[pat] + r + 1];
  const int gx = sf.lo[0] + x;
  T v = T(0);
  for (int q = s0; q < s1; ++q) {
    const wvl_seg g = seg[q];
    if (gx >= g.i1s && gx <= g.i1e) {
      const int64_t k = g.off + (gx - g.i1s);
      v = c == 0 ? psi[sf.cin + k] : psi[sf.cin + sf.n_c + (int64_t)(c - 1) * sf.n_f + k];
      break;
    }
  }
  T* out = use_work ? dst + wk[s].c8 : dst + sf.box_in;
  out[idx] = v;
}

// Compress onto the output pattern: thread per dense point of the output box.
template <typename T>
__global__ __launch_bounds__(TPB) void k_scatter(const SfDev* __restrict__ sfs,
                                                 const wvl_seg* __restrict__ seg,
                                                 const int32_t* __restrict__ rt,
                                                 const T* __restrict__ src, T* __restrict__ out,
                                                 const SfWork* __restrict__ wk, int sf0,
                                                 int use_work, int accumulate) {
  const int s = blockIdx.y;
  const SfDev& sf = sfs[sf0 + s];
  const int e = sf.ext;
  const int n0 = sf.n[0] + 2 * e, n1 = sf.n[1] + 2 * e, n2 = sf.n[2] + 2 * e;
  const int64_t vol = 8ll * n0 * n1 * n2;
  const int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (idx >= vol) return;
  const int x = (int)(idx % n0);
  int64_t t = idx / n0;
  const int y = (int)(t % n1);
  t /= n1;
  const int z = (int)(t % n2);
  const int c = (int)(t / n2);
  const int pat = c == 0 ? 2 : 3;
  const int64_t r = (int64_t)z * n1 + y;
  const int32_t s0 = rt[sf.rt[pat] + r], s1 = rt[sf.rt[pat] + r + 1];
  const int gx = sf.lo[0] - e + x;
  for (int q = s0; q < s1; ++q) {
    const wvl_seg g = seg[q];
    if (gx >= g.i1s && gx <= g.i1e) {
      const int64_t k = g.off + (gx - g.i1s);
      const int64_t o = c == 0 ? sf.cout + k : sf.cout + sf.on_c + (int64_t)(c - 1) * sf.on_f + k;
      const T* in = use_work ? src + wk[s].o8 : src + sf.box_out;
      const T v = in[idx];
      out[o] = accumulate ? out[o] + v : v;
      return;
    }
  }
}

// ---------------------------------------------------------------------------
// potential part: up passes (coarse two-level -> fine real space)
// ---------------------------------------------------------------------------

// Pass along axis AX: out(l) = sum_i C_0[l-2i] in_{2c}(i) + C_1[l-2i] in_{2c+1}(i)
// Input dims: axes < AX fine (2n+29), axes >= AX coarse (n).  With WITHV the
// output is multiplied by the potential and the partial sums of V f^2 are
// written per block.
template <typename T, int AX, bool WITHV>
__global__ __launch_bounds__(TPB) void k_up(const SfDev* __restrict__ sfs,
                                            const SfWork* __restrict__ wk, int sf0,
                                            T* __restrict__ ws, const T* __restrict__ pot, int nf1,
                                            int nf2, double* __restrict__ epart) {
  const int s = blockIdx.y;
  const SfDev& sf = sfs[sf0 + s];
  const SfWork& w = wk[s];
  const int n[3] = {sf.n[0], sf.n[1], sf.n[2]};
  int id[3], od[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    id[a] = a < AX ? nr_of(n[a]) : n[a];
    od[a] = a <= AX ? nr_of(n[a]) : n[a];
  }
  const int och = 4 >> AX;
  const int64_t vol = (int64_t)och * od[0] * od[1] * od[2];
  const int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x;
  double eacc = 0.0;
  if (idx < vol) {
    const int x = (int)(idx % od[0]);
    int64_t t = idx / od[0];
    const int y = (int)(t % od[1]);
    t /= od[1];
    const int z = (int)(t % od[2]);
    const int c = (int)(t / od[2]);
    const T* in = ws + (AX == 0 ? w.c8 : AX == 1 ? w.a1 : w.a2);
    T* out = ws + (AX == 0 ? w.a1 : AX == 1 ? w.a2 : w.g);
    const int64_t chvol = (int64_t)id[0] * id[1] * id[2];
    const int p = AX == 0 ? x : AX == 1 ? y : z;
    const int64_t stride = AX == 0 ? 1 : AX == 1 ? id[0] : (int64_t)id[0] * id[1];
    const int64_t base = (AX == 0 ? ((int64_t)z * id[1] + y) * id[0]
                          : AX == 1 ? (int64_t)z * id[1] * id[0] + x
                                    : (int64_t)y * id[0] + x);
    const T* in0 = in + (int64_t)(2 * c) * chvol + base;
    const T* in1 = in0 + chvol;
    const int N = n[AX];
    const int ilo = max(0, (p - 29) >> 1);
    const int ihi = min(N - 1, p >> 1);
    T acc = T(0);
    for (int i = ilo; i <= ihi; ++i) {
      const int ci = p - 2 * i;
      acc += ctab<T>(0, ci) * in0[i * stride] + ctab<T>(1, ci) * in1[i * stride];
    }
    if (WITHV) {
      const int64_t gi = ((int64_t)(2 * sf.lo[2] + z) * nf2 + (2 * sf.lo[1] + y)) * nf1 +
                         (2 * sf.lo[0] + x);
      const T v = pot[gi];
      eacc = (double)v * (double)acc * (double)acc;
      acc = v * acc;
    }
    out[idx] = acc;
  }
  if (WITHV) {
    const double b = block_sum(eacc);
    if (threadIdx.x == 0) epart[w.epart + blockIdx.x] = b;
  }
}

// ---------------------------------------------------------------------------
// potential part: down passes (fine real space -> coarse two-level, L' box)
// ---------------------------------------------------------------------------

// Pass along axis AX: out_{2c+b}(i) = sum_l C_b[l-2i] in_c(l), i in [-e, n+e).
// Input dims: axes <= AX fine, axes > AX output coarse (n+2e).
template <typename T, int AX, bool ACC>
__global__ __launch_bounds__(TPB) void k_down(const SfDev* __restrict__ sfs,
                                              const SfWork* __restrict__ wk, int sf0,
                                              T* __restrict__ ws) {
  const int s = blockIdx.y;
  const SfDev& sf = sfs[sf0 + s];
  const SfWork& w = wk[s];
  const int e = sf.ext;
  int id[3], od[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int nr = nr_of(sf.n[a]), no = sf.n[a] + 2 * e;
    id[a] = a > AX ? no : nr;
    od[a] = a >= AX ? no : nr;
  }
  const int och = 2 << (2 - AX);
  const int64_t vol = (int64_t)och * od[0] * od[1] * od[2];
  const int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (idx >= vol) return;
  const int x = (int)(idx % od[0]);
  int64_t t = idx / od[0];
  const int y = (int)(t % od[1]);
  t /= od[1];
  const int z = (int)(t % od[2]);
  const int co = (int)(t / od[2]);
  const int c = co >> 1, b = co & 1;
  const T* in = ws + (AX == 2 ? w.g : AX == 1 ? w.b1 : w.b2);
  T* out = ws + (AX == 2 ? w.b1 : AX == 1 ? w.b2 : w.o8);
  const int64_t chvol = (int64_t)id[0] * id[1] * id[2];
  const int p = AX == 0 ? x : AX == 1 ? y : z;
  const int64_t stride = AX == 0 ? 1 : AX == 1 ? id[0] : (int64_t)id[0] * id[1];
  const int64_t base = (AX == 0 ? ((int64_t)z * id[1] + y) * id[0]
                        : AX == 1 ? (int64_t)z * id[1] * id[0] + x
                                  : (int64_t)y * id[0] + x);
  const T* src = in + (int64_t)c * chvol + base;
  const int nr = id[AX];
  const int two_i = 2 * (p - e);  // 2 i, i = p - e
  const int qlo = max(0, two_i), qhi = min(nr - 1, two_i + 30);
  T acc = T(0);
  for (int q = qlo; q <= qhi; ++q) acc += ctab<T>(b, q - two_i) * src[q * stride];
  if (ACC) acc += out[idx];
  out[idx] = acc;
}

// ---------------------------------------------------------------------------
// kinetic part on the coarse box
// ---------------------------------------------------------------------------

// out_c(i) (+)= fac * sum_j sum_b K_{a b}[j] in_{c_b}(i + j) along AX, with a
// the output channel's bit for AX and c_b the input channel with that bit b.
// FP32: off-diagonal taps accumulate in FP32, the scaling channel in the
// difference form sum_{j != 0} K_j (x_{i+j} - x_i) (its filter sums to zero
// exactly, not after rounding); the diagonal terms and the factor
// fac = -1/2 (2/h)^2 are applied in FP64 before the one final rounding, so
// that no FP32 tap rounding biases <phi|T|phi>.
template <typename T, int AX, bool ACC>
__global__ __launch_bounds__(TPB) void k_kin(const SfDev* __restrict__ sfs,
                                             const SfWork* __restrict__ wk, int sf0,
                                             T* __restrict__ ws, double fac) {
  const int s = blockIdx.y;
  const SfDev& sf = sfs[sf0 + s];
  const SfWork& w = wk[s];
  const int e = sf.ext;
  const int n[3] = {sf.n[0], sf.n[1], sf.n[2]};
  const int od[3] = {n[0] + 2 * e, n[1] + 2 * e, n[2] + 2 * e};
  const int64_t vol = 8ll * od[0] * od[1] * od[2];
  const int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (idx >= vol) return;
  const int x = (int)(idx % od[0]);
  int64_t t = idx / od[0];
  const int y = (int)(t % od[1]);
  t /= od[1];
  const int z = (int)(t % od[2]);
  const int c = (int)(t / od[2]);
  const int ic[3] = {x - e, y - e, z - e};
  T* out = ws + w.o8;
  bool inside = true;
#pragma unroll
  for (int a = 0; a < 3; ++a)
    if (a != AX && (ic[a] < 0 || ic[a] >= n[a])) inside = false;
  T res = T(0);
  if (inside) {
    const T* in = ws + w.c8;
    const int64_t chvol = (int64_t)n[0] * n[1] * n[2];
    const int a = (c >> AX) & 1;
    const int c0 = c & ~(1 << AX), c1 = c | (1 << AX);
    const int64_t stride = AX == 0 ? 1 : AX == 1 ? n[0] : (int64_t)n[0] * n[1];
    const int64_t base = AX == 0 ? ((int64_t)ic[2] * n[1] + ic[1]) * n[0]
                         : AX == 1 ? (int64_t)ic[2] * n[1] * n[0] + ic[0]
                                   : (int64_t)ic[1] * n[0] + ic[0];
    const T* in0 = in + (int64_t)c0 * chvol + base;
    const T* in1 = in + (int64_t)c1 * chvol + base;
    const int i = ic[AX], N = n[AX];
    const int jlo = max(-14, -i), jhi = min(14, N - 1 - i);
    if (sizeof(T) == 4) {
      const bool in_box = i >= 0 && i < N;
      const T self = in_box ? in0[i * stride] : T(0);
      const T self1 = in_box ? in1[i * stride] : T(0);
      T acc = T(0);
      for (int j = jlo; j <= min(jhi, -1); ++j)
        acc += ktab<T>(a, 0, j + 14) * (in0[(i + j) * stride] - self) +
               ktab<T>(a, 1, j + 14) * in1[(i + j) * stride];
      for (int j = max(jlo, 1); j <= jhi; ++j)
        acc += ktab<T>(a, 0, j + 14) * (in0[(i + j) * stride] - self) +
               ktab<T>(a, 1, j + 14) * in1[(i + j) * stride];
      // taps whose input lies outside the box still carry the -self term
      T outside = T(0);
      for (int j = -14; j < jlo; ++j) outside += ktab<T>(a, 0, j + 14);
      for (int j = jhi + 1; j <= 14; ++j) outside += ktab<T>(a, 0, j + 14);
      acc -= outside * self;
      const double r = (double)acc + cKD64[a] * (double)self + cK64[a][1][14] * (double)self1;
      res = (T)(fac * r);
    } else {
      double acc = 0.0;
      for (int j = jlo; j <= jhi; ++j)
        acc += cK64[a][0][j + 14] * (double)in0[(i + j) * stride] +
               cK64[a][1][j + 14] * (double)in1[(i + j) * stride];
      res = (T)(fac * acc);
    }
  }
  if (ACC) res += out[idx];
  out[idx] = res;
}

// e_kin partials: sum over the input box of C8 * O8 (O8 holding T C8 only)
template <typename T>
__global__ __launch_bounds__(TPB) void k_ekin(const SfDev* __restrict__ sfs,
                                              const SfWork* __restrict__ wk, int sf0,
                                              const T* __restrict__ ws,
                                              double* __restrict__ kpart) {
  const int s = blockIdx.y;
  const SfDev& sf = sfs[sf0 + s];
  const SfWork& w = wk[s];
  const int e = sf.ext;
  const int n0 = sf.n[0], n1 = sf.n[1], n2 = sf.n[2];
  const int64_t vol = 8ll * n0 * n1 * n2;
  const int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x;
  double v = 0.0;
  if (idx < vol) {
    const int x = (int)(idx % n0);
    int64_t t = idx / n0;
    const int y = (int)(t % n1);
    t /= n1;
    const int z = (int)(t % n2);
    const int c = (int)(t / n2);
    const int m0 = n0 + 2 * e, m1 = n1 + 2 * e, m2 = n2 + 2 * e;
    const int64_t o = (((int64_t)c * m2 + z + e) * m1 + y + e) * m0 + x + e;
    v = (double)ws[w.c8 + idx] * (double)ws[w.o8 + o];
  }
  const double b = block_sum(v);
  if (threadIdx.x == 0) kpart[w.kpart + blockIdx.x] = b;
}

// one block per function: fixed-order sum of its partials
__global__ __launch_bounds__(TPB) void k_finalize(const SfWork* __restrict__ wk, int sf0,
                                                  const double* __restrict__ parts, int which,
                                                  int nblk, double* __restrict__ out) {
  const int s = blockIdx.x;
  const int64_t off = which == 0 ? wk[s].epart : wk[s].kpart;
  double v = 0.0;
  for (int i = threadIdx.x; i < nblk; i += TPB) v += parts[off + i];
  const double b = block_sum(v);
  if (threadIdx.x == 0) out[sf0 + s] = b;
}

template <typename T>
__global__ __launch_bounds__(TPB) void k_fill(T* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i < n) p[i] = T(0);
}

// ---------------------------------------------------------------------------
// sparse pattern and values
// ---------------------------------------------------------------------------

struct PatBox {
  int ox, oy, oz, bx, by;  // pattern box origin and row extents
};

__device__ __forceinline__ PatBox pat_box(const SfDev& s, int out) {
  const int e = out ? s.ext : 0;
  return PatBox{s.lo[0] - e, s.lo[1] - e, s.lo[2] - e, s.n[0] + 2 * e, s.n[1] + 2 * e};
}

__device__ __forceinline__ bool bb_meet(const int32_t* a, const int32_t* b) {
  return a[0] <= a[1] && b[0] <= b[1] && a[0] <= b[1] && b[0] <= a[1] && a[2] <= b[3] &&
         b[2] <= a[3] && a[4] <= b[5] && b[4] <= a[5];
}

// does the input coarse pattern of A share a point with B's pattern?
__device__ bool coarse_intersect(const SfDev& A, const SfDev& B, int ket_out,
                                 const wvl_seg* __restrict__ seg,
                                 const int32_t* __restrict__ rt) {
  const int32_t* bb = ket_out ? B.bb_out : B.bb_in;
  const int y0 = max(A.bb_in[2], bb[2]), y1 = min(A.bb_in[3], bb[3]);
  const int z0 = max(A.bb_in[4], bb[4]), z1 = min(A.bb_in[5], bb[5]);
  const PatBox pb = pat_box(B, ket_out);
  const int pB = ket_out ? 2 : 0;
  for (int z = z0; z <= z1; ++z) {
    for (int y = y0; y <= y1; ++y) {
      const int64_t ra = (int64_t)(z - A.lo[2]) * A.n[1] + (y - A.lo[1]);
      const int64_t rb = (int64_t)(z - pb.oz) * pb.by + (y - pb.oy);
      int qa = rt[A.rt[0] + ra], qa1 = rt[A.rt[0] + ra + 1];
      int qb = rt[B.rt[pB] + rb], qb1 = rt[B.rt[pB] + rb + 1];
      while (qa < qa1 && qb < qb1) {
        const wvl_seg sa = seg[qa], sb = seg[qb];
        if (sa.i1e < sb.i1s) {
          ++qa;
        } else if (sb.i1e < sa.i1s) {
          ++qb;
        } else {
          return true;
        }
      }
    }
  }
  return false;
}

// one 64-lane wavefront per row a; count (rowptr == NULL) or fill columns
__global__ __launch_bounds__(64) void k_pattern(const SfDev* __restrict__ sfs,
                                                const wvl_seg* __restrict__ seg,
                                                const int32_t* __restrict__ rt, int nsf,
                                                int ket_out, int64_t* __restrict__ count,
                                                const int64_t* __restrict__ rowptr,
                                                int32_t* __restrict__ col) {
  const int a = blockIdx.x;
  const int lane = threadIdx.x;
  const SfDev& A = sfs[a];
  int64_t n = 0;
  for (int b0 = 0; b0 < nsf; b0 += 64) {
    const int b = b0 + lane;
    bool hit = false;
    if (b < nsf) {
      const SfDev& B = sfs[b];
      if (bb_meet(A.bb_in, ket_out ? B.bb_out : B.bb_in))
        hit = coarse_intersect(A, B, ket_out, seg, rt);
    }
    const unsigned long long m = __ballot(hit);
    if (rowptr != nullptr && hit) {
      const int before = __popcll(m & ((1ull << lane) - 1ull));
      col[rowptr[a] + n + before] = b;
    }
    n += __popcll(m);
  }
  if (rowptr == nullptr && lane == 0) count[a] = n;
}

// one wavefront per nonzero; lanes take rows of the overlap box in a fixed
// order, partial sums combine in a fixed shuffle tree
template <typename T>
__global__ __launch_bounds__(64) void k_sparse_values(const SfDev* __restrict__ sfs,
                                                      const wvl_seg* __restrict__ seg,
                                                      const int32_t* __restrict__ rt, int ket_out,
                                                      const T* __restrict__ bra,
                                                      const T* __restrict__ ket,
                                                      const int32_t* __restrict__ rowi,
                                                      const int32_t* __restrict__ coli,
                                                      double* __restrict__ val) {
  const int64_t k = blockIdx.x;
  const int lane = threadIdx.x;
  const SfDev& A = sfs[rowi[k]];
  const SfDev& B = sfs[coli[k]];
  const int32_t* bb = ket_out ? B.bb_out : B.bb_in;
  const int y0 = max(A.bb_in[2], bb[2]), y1 = min(A.bb_in[3], bb[3]);
  const int z0 = max(A.bb_in[4], bb[4]), z1 = min(A.bb_in[5], bb[5]);
  const PatBox pb = pat_box(B, ket_out);
  const int pc = ket_out ? 2 : 0, pf = ket_out ? 3 : 1;
  const int64_t bc = ket_out ? B.cout : B.cin;
  const int64_t bnc = ket_out ? B.on_c : B.n_c, bnf = ket_out ? B.on_f : B.n_f;
  const int ny = y1 - y0 + 1;
  const int nrows = (y1 >= y0 && z1 >= z0) ? ny * (z1 - z0 + 1) : 0;
  double acc = 0.0;
  for (int r = lane; r < nrows; r += 64) {
    const int y = y0 + r % ny, z = z0 + r / ny;
    const int64_t ra = (int64_t)(z - A.lo[2]) * A.n[1] + (y - A.lo[1]);
    const int64_t rb = (int64_t)(z - pb.oz) * pb.by + (y - pb.oy);
    for (int fine = 0; fine < 2; ++fine) {
      int qa = rt[A.rt[fine] + ra], qa1 = rt[A.rt[fine] + ra + 1];
      const int pB = fine ? pf : pc;
      int qb = rt[B.rt[pB] + rb], qb1 = rt[B.rt[pB] + rb + 1];
      while (qa < qa1 && qb < qb1) {
        const wvl_seg sa = seg[qa], sb = seg[qb];
        const int x0 = max(sa.i1s, sb.i1s), x1 = min(sa.i1e, sb.i1e);
        if (x0 <= x1) {
          if (!fine) {
            const T* pa = bra + A.cin + sa.off + (x0 - sa.i1s);
            const T* pk = ket + bc + sb.off + (x0 - sb.i1s);
            for (int x = 0; x <= x1 - x0; ++x) acc += (double)pa[x] * (double)pk[x];
          } else {
            for (int comp = 0; comp < 7; ++comp) {
              const T* pa = bra + A.cin + A.n_c + comp * A.n_f + sa.off + (x0 - sa.i1s);
              const T* pk = ket + bc + bnc + comp * bnf + sb.off + (x0 - sb.i1s);
              for (int x = 0; x <= x1 - x0; ++x) acc += (double)pa[x] * (double)pk[x];
            }
          }
        }
        if (sa.i1e < sb.i1e) ++qa; else ++qb;
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (lane == 0) val[k] = acc;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static inline dim3 grid2(int64_t maxvol, int nsf) {
  return dim3((unsigned)((maxvol + TPB - 1) / TPB), (unsigned)nsf);
}

int launch_gather(int f64, void* stream, const SfDev* sf, const wvl_seg* seg, const int32_t* rt,
                  const void* psi, void* box, const SfWork* wk, int sf0, int nsf, int64_t maxvol,
                  int use_work) {
  if (nsf == 0 || maxvol == 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  if (f64)
    hipLaunchKernelGGL(k_gather<double>, grid2(maxvol, nsf), dim3(TPB), 0, st, sf, seg, rt,
                       (const double*)psi, (double*)box, wk, sf0, use_work);
  else
    hipLaunchKernelGGL(k_gather<float>, grid2(maxvol, nsf), dim3(TPB), 0, st, sf, seg, rt,
                       (const float*)psi, (float*)box, wk, sf0, use_work);
  return (int)hipGetLastError();
}

int launch_scatter(int f64, void* stream, const SfDev* sf, const wvl_seg* seg, const int32_t* rt,
                   const void* box, void* out, const SfWork* wk, int sf0, int nsf, int64_t maxvol,
                   int use_work, int accumulate) {
  if (nsf == 0 || maxvol == 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  if (f64)
    hipLaunchKernelGGL(k_scatter<double>, grid2(maxvol, nsf), dim3(TPB), 0, st, sf, seg, rt,
                       (const double*)box, (double*)out, wk, sf0, use_work, accumulate);
  else
    hipLaunchKernelGGL(k_scatter<float>, grid2(maxvol, nsf), dim3(TPB), 0, st, sf, seg, rt,
                       (const float*)box, (float*)out, wk, sf0, use_work, accumulate);
  return (int)hipGetLastError();
}

template <typename T>
static void up_t(hipStream_t st, int axis, const SfDev* sf, const SfWork* wk, int sf0, int nsf,
                 int64_t maxvol, T* ws, const T* pot, int nf1, int nf2, double* epart) {
  const dim3 g = grid2(maxvol, nsf);
  if (axis == 0)
    hipLaunchKernelGGL((k_up<T, 0, false>), g, dim3(TPB), 0, st, sf, wk, sf0, ws, pot, nf1, nf2,
                       epart);
  else if (axis == 1)
    hipLaunchKernelGGL((k_up<T, 1, false>), g, dim3(TPB), 0, st, sf, wk, sf0, ws, pot, nf1, nf2,
                       epart);
  else
    hipLaunchKernelGGL((k_up<T, 2, true>), g, dim3(TPB), 0, st, sf, wk, sf0, ws, pot, nf1, nf2,
                       epart);
}

int launch_up(int f64, void* stream, int axis, const SfDev* sf, const SfWork* wk, int sf0, int nsf,
              int64_t maxvol, void* ws, const void* pot, int nf1, int nf2, double* epart,
              int nblk) {
  (void)nblk;
  if (nsf == 0 || maxvol == 0) return 0;
  if (f64)
    up_t<double>((hipStream_t)stream, axis, sf, wk, sf0, nsf, maxvol, (double*)ws,
                 (const double*)pot, nf1, nf2, epart);
  else
    up_t<float>((hipStream_t)stream, axis, sf, wk, sf0, nsf, maxvol, (float*)ws,
                (const float*)pot, nf1, nf2, epart);
  return (int)hipGetLastError();
}

template <typename T>
static void down_t(hipStream_t st, int axis, const SfDev* sf, const SfWork* wk, int sf0, int nsf,
                   int64_t maxvol, T* ws, int acc) {
  const dim3 g = grid2(maxvol, nsf);
  if (axis == 2)
    hipLaunchKernelGGL((k_down<T, 2, false>), g, dim3(TPB), 0, st, sf, wk, sf0, ws);
  else if (axis == 1)
    hipLaunchKernelGGL((k_down<T, 1, false>), g, dim3(TPB), 0, st, sf, wk, sf0, ws);
  else if (acc)
    hipLaunchKernelGGL((k_down<T, 0, true>), g, dim3(TPB), 0, st, sf, wk, sf0, ws);
  else
    hipLaunchKernelGGL((k_down<T, 0, false>), g, dim3(TPB), 0, st, sf, wk, sf0, ws);
}

int launch_down(int f64, void* stream, int axis, const SfDev* sf, const SfWork* wk, int sf0,
                int nsf, int64_t maxvol, void* ws, int accumulate) {
  if (nsf == 0 || maxvol == 0) return 0;
  if (f64)
    down_t<double>((hipStream_t)stream, axis, sf, wk, sf0, nsf, maxvol, (double*)ws, accumulate);
  else
    down_t<float>((hipStream_t)stream, axis, sf, wk, sf0, nsf, maxvol, (float*)ws, accumulate);
  return (int)hipGetLastError();
}

template <typename T>
static void kin_t(hipStream_t st, int axis, const SfDev* sf, const SfWork* wk, int sf0, int nsf,
                  int64_t maxvol, T* ws, int acc, double fac) {
  const dim3 g = grid2(maxvol, nsf);
#define WVL_KIN_CASE(AXV)                                                                   \
  if (axis == AXV) {                                                                        \
    if (acc)                                                                                \
      hipLaunchKernelGGL((k_kin<T, AXV, true>), g, dim3(TPB), 0, st, sf, wk, sf0, ws, fac);  \
    else                                                                                    \
      hipLaunchKernelGGL((k_kin<T, AXV, false>), g, dim3(TPB), 0, st, sf, wk, sf0, ws, fac); \
  }
  WVL_KIN_CASE(0)
  WVL_KIN_CASE(1)
  WVL_KIN_CASE(2)
#undef WVL_KIN_CASE
}

int launch_kin(int f64, void* stream, int axis, const SfDev* sf, const SfWork* wk, int sf0,
               int nsf, int64_t maxvol, void* ws, int accumulate, double fac) {
  if (nsf == 0 || maxvol == 0) return 0;
  if (f64)
    kin_t<double>((hipStream_t)stream, axis, sf, wk, sf0, nsf, maxvol, (double*)ws, accumulate,
                  fac);
  else
    kin_t<float>((hipStream_t)stream, axis, sf, wk, sf0, nsf, maxvol, (float*)ws, accumulate,
                 fac);
  return (int)hipGetLastError();
}

int launch_fill(int f64, void* stream, void* ptr, int64_t n) {
  if (n == 0) return 0;
  const dim3 g((unsigned)((n + TPB - 1) / TPB));
  if (f64)
    hipLaunchKernelGGL(k_fill<double>, g, dim3(TPB), 0, (hipStream_t)stream, (double*)ptr, n);
  else
    hipLaunchKernelGGL(k_fill<float>, g, dim3(TPB), 0, (hipStream_t)stream, (float*)ptr, n);
  return (int)hipGetLastError();
}

int launch_ekin_partials(int f64, void* stream, const SfDev* sf, const SfWork* wk, int sf0,
                         int nsf, int64_t maxvol, void* ws, double* kpart, int nblk) {
  (void)nblk;
  if (nsf == 0 || maxvol == 0) return 0;
  if (f64)
    hipLaunchKernelGGL(k_ekin<double>, grid2(maxvol, nsf), dim3(TPB), 0, (hipStream_t)stream, sf,
                       wk, sf0, (const double*)ws, kpart);
  else
    hipLaunchKernelGGL(k_ekin<float>, grid2(maxvol, nsf), dim3(TPB), 0, (hipStream_t)stream, sf,
                       wk, sf0, (const float*)ws, kpart);
  return (int)hipGetLastError();
}

int launch_finalize(void* stream, const SfWork* wk, int sf0, int nsf, const double* parts,
                    int which, int nblk, double* out) {
  if (nsf == 0) return 0;
  hipLaunchKernelGGL(k_finalize, dim3(nsf), dim3(TPB), 0, (hipStream_t)stream, wk, sf0, parts,
                     which, nblk, out);
  return (int)hipGetLastError();
}

int launch_pattern(void* stream, const SfDev* sf, const wvl_seg* seg, const int32_t* rt, int nsf,
                   int ket_out, int64_t* count, const int64_t* rowptr, int32_t* col) {
  if (nsf == 0) return 0;
  hipLaunchKernelGGL(k_pattern, dim3(nsf), dim3(64), 0, (hipStream_t)stream, sf, seg, rt, nsf,
                     ket_out, count, rowptr, col);
  return (int)hipGetLastError();
}

int launch_sparse_values(int f64, void* stream, const SfDev* sf, const wvl_seg* seg,
                         const int32_t* rt, int ket_out, const void* bra, const void* ket,
                         const int32_t* row, const int32_t* col, int64_t nnz, double* val) {
  if (nnz == 0) return 0;
  if (f64)
    hipLaunchKernelGGL(k_sparse_values<double>, dim3((unsigned)nnz), dim3(64), 0,
                       (hipStream_t)stream, sf, seg, rt, ket_out, (const double*)bra,
                       (const double*)ket, row, col, val);
  else
    hipLaunchKernelGGL(k_sparse_values<float>, dim3((unsigned)nnz), dim3(64), 0,
                       (hipStream_t)stream, sf, seg, rt, ket_out, (const float*)bra,
                       (const float*)ket, row, col, val);
  return (int)hipGetLastError();
}

}  // namespace wvl

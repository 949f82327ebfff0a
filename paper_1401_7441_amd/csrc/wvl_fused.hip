// Fused local-Hamiltonian kernels for gfx950 (MI355X).
//
// The operator factorization is the one of wvl_kernels.hip (potential term as
// stride-2 up passes C_b = synthesis then magic filter, potential multiply,
// stride-2 down passes; kinetic term as the coarse two-level filters
// K_ab = R^T a R), but the separable passes are grouped by where their data
// can live:
//   k_unpack     one coarse plane of one component: uncompress through the
//                compact row runs, write the dense box in two layouts (C8 x
//                fastest, C8X y fastest) for the other kernels.
//   k_up_x       one coarse row per thread, streaming along x: the x up pass
//                (synthesis and magic filter in one 31-tap filter) into GX
//                through 32-wide LDS stages.
//   k_up_y       one fine column per thread, streaming along y: the y up
//                pass from GX into G1.
//   k_pot_column one fine (x, y) column per thread, streaming along z with
//                register rings: up pass z, potential multiply (FP64 energy
//                partials), down pass z -> G2.  Every input is read once.
//   k_kin_col    one coarse column per thread (along x, y or z): that axis'
//                part of the kinetic term with a 32-slot register window,
//                and that part's share of <phi|T|phi>.
//   k_back_y     one fine (channel, z', x) column per thread, streaming along
//                y: the y down pass; 16-wide LDS stages transpose the result
//                so that y' is the fastest axis of the x down pass' input.
//   k_back_out   one output (z', y', channel) row per thread, streaming along
//                x: the x down pass plus the three kinetic parts; each
//                wave's 16 rows x 8 components are staged 16 x' at a time in
//                LDS and written straight onto the compressed output pattern.
// Register ring slots are compile-time constants after unrolling by the ring
// period, so the rings stay in VGPRs.
#include <hip/hip_runtime.h>

#include "wvl_filters.h"
#include "wvl_internal.h"

namespace wvl {

__constant__ double fC64[2][31] = {WVL_C0_F64, WVL_C1_F64};
__constant__ float fC32[2][31] = {WVL_C0_F32, WVL_C1_F32};
__constant__ double fK64[2][2][29] = {{WVL_K00_F64, WVL_K01_F64}, {WVL_K10_F64, WVL_K11_F64}};
__constant__ float fK32[2][2][29] = {{WVL_K00_F32, WVL_K01_F32}, {WVL_K10_F32, WVL_K11_F32}};
__constant__ double fKD64[2] = WVL_KD_F64;

// LDS row stride of the 16-wide output stages: element (j, lane) at
// j * kSP + lane; the flush reads (j = lane & 15, row = 4 it + lane >> 4),
// whose banks 4 j + row are all distinct
constexpr int kSP = 68;

// Register prefetch of the streaming passes: with distance PF > 0 the loads
// of step q + PF are issued at step q into a ring of PF registers (slot
// q mod PF, a compile-time constant after unrolling), so a step's inputs
// have been in flight for PF steps when it uses them instead of costing one
// load latency per step.  Prefetched indices are clamped into the stream, so
// every load is in bounds; values of steps outside the stream are replaced by
// zeros where they are used, so results do not depend on PF.  PF = 0 loads
// at the step itself.  The distances per pass and precision are the fastest
// of {0, 4, 8} measured on gfx950 (more VGPRs can cost more occupancy than
// the prefetch gains).
template <typename T> constexpr int pf_up_x() { return sizeof(T) == 8 ? 8 : 0; }
template <typename T> constexpr int pf_up_y() { return 8; }
template <typename T> constexpr int pf_pot() { return sizeof(T) == 8 ? 4 : 0; }
template <typename T, int AX> constexpr int pf_kin() {
  return sizeof(T) == 8 ? (AX == 1 ? 4 : 0) : (AX == 1 ? 8 : 4);
}
template <typename T> constexpr int pf_back_y() { return sizeof(T) == 8 ? 0 : 8; }
constexpr int kPfBackQ = 8, kPfBackK = 4;   // k_back_out: Q pairs, kinetic parts
constexpr int pf_slots(int pf) { return pf > 0 ? pf : 1; }
// element min(max(i, 0), n - 1) of a stream with the given stride (n >= 1)
template <typename T>
__device__ __forceinline__ T ld_clamp(const T* p, int i, int n, int64_t stride) {
  return p[(int64_t)min(max(i, 0), n - 1) * stride];
}

template <typename T>
__device__ __forceinline__ T Ct(int b, int n);
template <>
__device__ __forceinline__ double Ct<double>(int b, int n) { return fC64[b][n]; }
template <>
__device__ __forceinline__ float Ct<float>(int b, int n) { return fC32[b][n]; }
template <typename T>
__device__ __forceinline__ T Kt(int a, int b, int n);
template <>
__device__ __forceinline__ double Kt<double>(int a, int b, int n) { return fK64[a][b][n]; }
template <>
__device__ __forceinline__ float Kt<float>(int a, int b, int n) { return fK32[a][b][n]; }

// deterministic block sum: a fixed shuffle tree inside each 64-lane wave,
// then the wave sums in order (result valid in thread 0)
__device__ double block_sum_any(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __shared__ double part[16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) part[wv] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) r += part[k];
  __syncthreads();
  return r;
}

// value of component c (0 = scaling, 1..7 wavelets) of function sf at the
// global coarse point (gx, row r of its input box); 0 off the pattern
template <typename T>
__device__ __forceinline__ T coef_at(const SfDev& sf, const wvl_seg* __restrict__ seg,
                                     const int32_t* __restrict__ rt, const T* __restrict__ psi,
                                     int c, int64_t r, int gx) {
  const int pat = c == 0 ? 0 : 1;
  const int32_t s0 = rt[sf.rt[pat] + r], s1 = rt[sf.rt[pat] + r + 1];
  for (int q = s0; q < s1; ++q) {
    const wvl_seg g = seg[q];
    if (gx >= g.i1s && gx <= g.i1e) {
      const int64_t k = g.off + (gx - g.i1s);
      return c == 0 ? psi[sf.cin + k] : psi[sf.cin + sf.n_c + 7 * k + (c - 1)];
    }
  }
  return T(0);
}

// ---------------------------------------------------------------------------
// k_unpack: block = (function, group of G components, input plane z)
// ---------------------------------------------------------------------------
// Uncompress one coarse plane of G components (G = 8, 4, 2 or 1: as many as
// the plane's LDS stage fits; the host picks it per chunk) through the
// compact row runs (one record per row; rows with several runs walk the
// segments), then write each twice: C8[c][z][y][x] (x fastest) and
// C8X[c][z][x][y] (y fastest), both with consecutive threads on consecutive
// addresses.  With G = 8 a thread reads the seven wavelets of its point, which
// are consecutive in the compressed layout, in one block.
template <typename T>
__global__ __launch_bounds__(256) void k_unpack(const SfDev* __restrict__ sfs,
                                                const wvl_seg* __restrict__ seg,
                                                const int32_t* __restrict__ rt,
                                                const RowRun* __restrict__ rr,
                                                const T* __restrict__ psi,
                                                const SfWork* __restrict__ wk,
                                                T* __restrict__ ws, int G) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* pl = reinterpret_cast<T*>(smem_raw);   // [G][N1][N0 + 1]
  const SfWork& w = wk[blockIdx.y];
  const SfDev& sf = sfs[w.id];
  const int N0 = sf.n[0], N1 = sf.n[1], N2 = sf.n[2];
  const int ng = 8 / G;
  const int cg = blockIdx.x % ng, z = blockIdx.x / ng;
  if (z >= N2) return;   // uniform over the block
  const int c0 = cg * G;                      // first component of the group
  const int ld = N0 + 1, pls = N1 * ld;       // LDS row and plane strides
  const int np = N0 * N1;
  const int cf0 = max(c0, 1), cf1 = c0 + G;   // wavelet components of the group
  const int64_t fbase = sf.cin + sf.n_c;      // fine point k at fbase + 7 k
  for (int idx = threadIdx.x; idx < np; idx += 256) {
    const int y = idx / N0, x = idx - y * N0;
    const int64_t r = (int64_t)z * N1 + y;
    const int gx = sf.lo[0] + x;
    T* const o = pl + y * ld + x;
    if (c0 == 0) {   // scaling coefficients
      const RowRun run = rr[sf.rr[0] + r];
      T v = T(0);
      if (run.len == kMultiRun) {
        v = coef_at<T>(sf, seg, rt, psi, 0, r, gx);
      } else {
        const int dx = gx - (int)run.x0;
        if (dx >= 0 && dx < (int)run.len) v = psi[sf.cin + run.off + dx];
      }
      o[0] = v;
    }
    if (cf0 < cf1) {   // wavelets
      const RowRun run = rr[sf.rr[1] + r];
      if (run.len == kMultiRun) {
        for (int c = cf0; c < cf1; ++c) o[(c - c0) * pls] = coef_at<T>(sf, seg, rt, psi, c, r, gx);
      } else {
        const int dx = gx - (int)run.x0;
        const bool in = dx >= 0 && dx < (int)run.len;
        const T* f = psi + fbase + 7 * (int64_t)(in ? run.off + dx : 0);
        for (int c = cf0; c < cf1; ++c) o[(c - c0) * pls] = in ? f[c - 1] : T(0);
      }
    }
  }
  __syncthreads();
  const int64_t plane = (int64_t)np;
  for (int idx = threadIdx.x; idx < G * np; idx += 256) {
    const int c = idx / np, rem = idx - c * np;
    const int y = rem / N0, x = rem - y * N0;
    ws[w.c8 + ((int64_t)(c0 + c) * N2 + z) * plane + rem] = pl[c * pls + y * ld + x];
  }
  for (int idx = threadIdx.x; idx < G * np; idx += 256) {
    const int c = idx / np, rem = idx - c * np;
    const int x = rem / N1, y = rem - x * N1;
    ws[w.c8x + ((int64_t)(c0 + c) * N2 + z) * plane + rem] = pl[c * pls + y * ld + x];
  }
}

// ---------------------------------------------------------------------------
// k_up_x: thread = one coarse row (channel pair, z, y), streaming along x
// ---------------------------------------------------------------------------
// The two components c = a1 + 2 a2 + 4 a3 (a1 = 0, 1) of channel pair
// ch = a2 + 2 a3 are read from C8X (y across the lanes); fine points p = 2q,
// 2q+1 (f_p = sum_i C_a1[p - 2i] x_a1(i), i = q-15..q) come out of a 16-slot
// ring.  Every 32 fine points are staged in LDS and written to
// GX[ch][z][y][px] (px fastest), 2 rows x 32 points per store.
constexpr int kSPX = 66;   // stage stride: banks 2 j + row parity are distinct
template <typename T>
__global__ __launch_bounds__(64) void k_up_x(const SfDev* __restrict__ sfs,
                                             const SfWork* __restrict__ wk,
                                             T* __restrict__ ws) {
  __shared__ T st[32 * kSPX];
  const SfWork& w = wk[blockIdx.y];
  const SfDev& sf = sfs[w.id];
  const int N0 = sf.n[0], N1 = sf.n[1], N2 = sf.n[2];
  const int R0 = 2 * N0 + 29;
  const int nrow = 4 * N2 * N1;
  const int row0 = blockIdx.x * 64;
  if (row0 >= nrow) return;   // uniform over the block
  const int lane = threadIdx.x;
  const int row = row0 + lane;
  const bool active = row < nrow;
  const int y = active ? row % N1 : 0;
  const int t = active ? row / N1 : 0;
  const int z = t % N2, ch = t / N2;
  const int64_t plane = (int64_t)N0 * N1;
  const int c0 = 2 * (ch & 1) + 4 * (ch >> 1);
  const T* in0 = ws + w.c8x + ((int64_t)c0 * N2 + z) * plane + y;        // [c][z][x][y]
  const T* in1 = in0 + (int64_t)N2 * plane;                               // component c0 + 1
  const int obase = active ? row * R0 : -1;                               // GX row start
  T* gx = ws + w.gx;
  constexpr int PF = pf_up_x<T>();
  T xs[16], xd[16], f0[pf_slots(PF)], f1[pf_slots(PF)];
#pragma unroll
  for (int k = 0; k < 16; ++k) xs[k] = xd[k] = T(0);
#pragma unroll
  for (int d = 0; d < PF; ++d) {
    f0[d] = ld_clamp(in0, d, N0, N1);
    f1[d] = ld_clamp(in1, d, N0, N1);
  }
  const int qend = N0 + 14;
  for (int q0 = 0; q0 <= qend; q0 += 16) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int q = q0 + u, sp = u % pf_slots(PF);
      const bool ok = active && q < N0;
      if constexpr (PF > 0) {
        xs[u] = ok ? f0[sp] : T(0);
        xd[u] = ok ? f1[sp] : T(0);
        f0[sp] = ld_clamp(in0, q + PF, N0, N1);
        f1[sp] = ld_clamp(in1, q + PF, N0, N1);
      } else {
        xs[u] = ok ? in0[(int64_t)q * N1] : T(0);
        xd[u] = ok ? in1[(int64_t)q * N1] : T(0);
      }
      T fe = T(0), fo = T(0);
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int sl = (u - k) & 15;
        fe += Ct<T>(0, 2 * k) * xs[sl] + Ct<T>(1, 2 * k) * xd[sl];
        if (k < 15) fo += Ct<T>(0, 2 * k + 1) * xs[sl] + Ct<T>(1, 2 * k + 1) * xd[sl];
      }
      st[(2 * u) * kSPX + lane] = fe;
      st[(2 * u + 1) * kSPX + lane] = fo;
    }
    // flush px = 2 q0 + j, j = 0..31
    __syncthreads();
    const int j = lane & 31;
    const int px = 2 * q0 + j;
    const bool okp = px < R0;
#pragma unroll 4
    for (int it = 0; it < 32; ++it) {
      const int rl = 2 * it + (lane >> 5);
      const int ob = __shfl(obase, rl, 64);
      if (okp && ob >= 0) gx[ob + px] = st[j * kSPX + rl];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// k_up_y: thread = one fine column (a3, z, px), streaming along y
// ---------------------------------------------------------------------------
// Reads GX[a2 + 2 a3][z][y][px] for a2 = 0, 1 (px across the lanes) and
// writes G1[a3][z][py][px] for py = 2q, 2q+1 from a 16-slot ring.
template <typename T>
__global__ __launch_bounds__(256) void k_up_y(const SfDev* __restrict__ sfs,
                                              const SfWork* __restrict__ wk,
                                              T* __restrict__ ws) {
  const SfWork& w = wk[blockIdx.y];
  const SfDev& sf = sfs[w.id];
  const int N0 = sf.n[0], N1 = sf.n[1], N2 = sf.n[2];
  const int R0 = 2 * N0 + 29, R1 = 2 * N1 + 29;
  const int64_t ncol = 2ll * N2 * R0;                 // columns (a3, z, px), px fastest
  const int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (col >= ncol) return;
  const int px = (int)(col % R0);
  const int64_t t = col / R0;
  const int z = (int)(t % N2), a3 = (int)(t / N2);
  const int64_t gxc = (int64_t)N2 * N1 * R0;          // GX channel stride
  const T* in0 = ws + w.gx + ((int64_t)(2 * a3) * N2 + z) * N1 * R0 + px;   // a2 = 0
  const T* in1 = in0 + gxc;                                                   // a2 = 1
  T* out = ws + w.g1 + ((int64_t)a3 * N2 + z) * ((int64_t)R1 * R0) + px;
  // (out moves forward as the stream advances)
  constexpr int PF = pf_up_y<T>();
  static_assert(PF > 0, "k_up_y streams through its prefetch ring");
  T xs[16], xd[16], f0[PF], f1[PF];
#pragma unroll
  for (int k = 0; k < 16; ++k) xs[k] = xd[k] = T(0);
#pragma unroll
  for (int d = 0; d < PF; ++d) {
    f0[d] = ld_clamp(in0, d, N1, R0);
    f1[d] = ld_clamp(in1, d, N1, R0);
  }
  const int qend = N1 + 14;
  const int64_t gstep = 16 * (int64_t)R0;   // out advances by 16 coarse rows per block
  for (int q0 = 0; q0 <= qend; q0 += 16, out += 2 * gstep) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int q = q0 + u, sp = u % PF;
      const T v0 = f0[sp], v1 = f1[sp];
      f0[sp] = ld_clamp(in0, q + PF, N1, R0);
      f1[sp] = ld_clamp(in1, q + PF, N1, R0);
      if (q <= qend) {
        xs[u] = q < N1 ? v0 : T(0);
        xd[u] = q < N1 ? v1 : T(0);
        T fe = T(0), fo = T(0);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const int sl = (u - k) & 15;
          fe += Ct<T>(0, 2 * k) * xs[sl] + Ct<T>(1, 2 * k) * xd[sl];
          if (k < 15) fo += Ct<T>(0, 2 * k + 1) * xs[sl] + Ct<T>(1, 2 * k + 1) * xd[sl];
        }
        out[(2 * u) * R0] = fe;
        if (2 * q + 1 < R1) out[(2 * u + 1) * R0] = fo;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// k_up_z: thread = one fine (x, y) column, streaming along z
// ---------------------------------------------------------------------------
// Reads G1[a3][z][py][px] for a3 = 0, 1 and writes the function's values on
// its fine box, FINE[pz][py][px] (fine point p of an axis at global fine
// index 2 lo + p), for pz = 2q, 2q+1 from a 16-slot ring: the last step of
// the synthesis to real space.
template <typename T>
__global__ __launch_bounds__(256) void k_up_z(const SfDev* __restrict__ sfs,
                                              const SfWork* __restrict__ wk,
                                              const T* __restrict__ ws,
                                              const int64_t* __restrict__ fine_off,
                                              T* __restrict__ fine) {
  const SfWork& w = wk[blockIdx.y];
  const SfDev& sf = sfs[w.id];
  const int N0 = sf.n[0], N1 = sf.n[1], N2 = sf.n[2];
  const int R0 = 2 * N0 + 29, R1 = 2 * N1 + 29, R2 = 2 * N2 + 29;
  const int64_t plane = (int64_t)R1 * R0;
  const int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (col >= plane) return;
  const T* in0 = ws + w.g1 + col;                 // a3 = 0
  const T* in1 = in0 + (int64_t)N2 * plane;       // a3 = 1
  T* out = fine + fine_off[w.id] + col;
  constexpr int PF = pf_up_y<T>();   // the same stream shape as k_up_y
  T xs[16], xd[16], f0[PF], f1[PF];
#pragma unroll
  for (int k = 0; k < 16; ++k) xs[k] = xd[k] = T(0);
#pragma unroll
  for (int d = 0; d < PF; ++d) {
    f0[d] = ld_clamp(in0, d, N2, plane);
    f1[d] = ld_clamp(in1, d, N2, plane);
  }
  const int qend = N2 + 14;
  for (int q0 = 0; q0 <= qend; q0 += 16, out += 32 * plane) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int q = q0 + u, sp = u % PF;
      const T v0 = f0[sp], v1 = f1[sp];
      f0[sp] = ld_clamp(in0, q + PF, N2, plane);
      f1[sp] = ld_clamp(in1, q + PF, N2, plane);
      if (q <= qend) {
        xs[u] = q < N2 ? v0 : T(0);
        xd[u] = q < N2 ? v1 : T(0);
        T fe = T(0), fo = T(0);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const int sl = (u - k) & 15;
          fe += Ct<T>(0, 2 * k) * xs[sl] + Ct<T>(1, 2 * k) * xd[sl];
          if (k < 15) fo += Ct<T>(0, 2 * k + 1) * xs[sl] + Ct<T>(1, 2 * k + 1) * xd[sl];
        }
        out[(2 * u) * plane] = fe;
        if (2 * q + 1 < R2) out[(2 * u + 1) * plane] = fo;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// k_pot_column: thread = one fine (x, y) column of one function
// ---------------------------------------------------------------------------
// Streaming over coarse z index q: input pair x(q) arrives, fine points
// p = 2q, 2q+1 are produced (f_p = sum_i C_b[p - 2i] x_b(i), i = q-15..q),
// multiplied by V, and scattered into the output accumulators of coarse
// i' = q-15..q (out_b(i') += C_b[p - 2i'] g_p); i' = q-15 is then complete.
template <typename T>
__global__ __launch_bounds__(256) void k_pot_column(const SfDev* __restrict__ sfs,
                                                    const SfWork* __restrict__ wk, int sf0,
                                                    T* __restrict__ ws, const T* __restrict__ pot,
                                                    int nf1, int nf2,
                                                    double* __restrict__ epart,
                                                    const double* __restrict__ conf, double hh) {
  const SfWork& w = wk[blockIdx.y];
  const SfDev& sf = sfs[w.id];
  // confining potential a |r - R|^4 (a = 0: none); fine point p of an axis
  // sits at (2 lo + p - 14) h/2
  const double ca = conf ? conf[w.id] : 0.0;
  const int N0 = sf.n[0], N1 = sf.n[1], N2 = sf.n[2], e = sf.ext;
  const int R0 = 2 * N0 + 29, R1 = 2 * N1 + 29, R2 = 2 * N2 + 29;
  const int O2 = N2 + 2 * e;
  const int64_t ncol = (int64_t)R0 * R1;
  const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double eacc = 0.0;
  if (col < ncol) {
    const int px = (int)(col % R0), py = (int)(col / R0);
    const T* in0 = ws + w.g1 + col;
    const T* in1 = in0 + (int64_t)N2 * ncol;
    T* out0 = ws + w.g2 + col;
    T* out1 = out0 + (int64_t)O2 * ncol;
    const int64_t vstride = (int64_t)nf1 * nf2;
    // no potential array: V = 0 (the confinement alone)
    const T* vp = pot ? pot + ((int64_t)(2 * sf.lo[2]) * nf2 + (2 * sf.lo[1] + py)) * nf1 +
                            (2 * sf.lo[0] + px)
                      : nullptr;
    const double cdx = (double)(2 * sf.lo[0] + px - 14) * hh - sf.c[0];
    const double cdy = (double)(2 * sf.lo[1] + py - 14) * hh - sf.c[1];
    const double cxy = cdx * cdx + cdy * cdy;
    const double cz0 = (double)(2 * sf.lo[2] - 14) * hh - sf.c[2];
    constexpr int PF = pf_pot<T>(), NS = pf_slots(PF);
    T xs[16], xd[16], a0[16], a1[16], f0[NS], f1[NS], fve[NS], fvo[NS];
#pragma unroll
    for (int k = 0; k < 16; ++k) xs[k] = xd[k] = a0[k] = a1[k] = T(0);
#pragma unroll
    for (int d = 0; d < PF; ++d) {
      f0[d] = ld_clamp(in0, d, N2, ncol);
      f1[d] = ld_clamp(in1, d, N2, ncol);
      fve[d] = vp ? ld_clamp(vp, 2 * d, R2, vstride) : T(0);
      fvo[d] = vp ? ld_clamp(vp, 2 * d + 1, R2, vstride) : T(0);
    }
    if (e == 16) {  // coarse i' = -16 lies beyond the filter reach
      out0[0] = T(0);
      out1[0] = T(0);
    }
    const int qend = N2 - 1 + e + 15;
    for (int q0 = 0; q0 <= qend; q0 += 16) {
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int q = q0 + u, sp = u % NS;
        T v0 = T(0), v1 = T(0), pve = T(0), pvo = T(0);
        if constexpr (PF > 0) {
          v0 = f0[sp];
          v1 = f1[sp];
          pve = fve[sp];
          pvo = fvo[sp];
          f0[sp] = ld_clamp(in0, q + PF, N2, ncol);
          f1[sp] = ld_clamp(in1, q + PF, N2, ncol);
          if (vp) {
            fve[sp] = ld_clamp(vp, 2 * (q + PF), R2, vstride);
            fvo[sp] = ld_clamp(vp, 2 * (q + PF) + 1, R2, vstride);
          }
        }
        if (q <= qend) {
        if constexpr (PF == 0) {
          const int p = 2 * q;
          v0 = q < N2 ? in0[(int64_t)q * ncol] : T(0);
          v1 = q < N2 ? in1[(int64_t)q * ncol] : T(0);
          pve = (vp && p < R2) ? vp[(int64_t)p * vstride] : T(0);
          pvo = (vp && p + 1 < R2) ? vp[(int64_t)(p + 1) * vstride] : T(0);
        }
        xs[u] = q < N2 ? v0 : T(0);
        xd[u] = q < N2 ? v1 : T(0);
        T fe = T(0), fo = T(0);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const int sl = (u - k) & 15;
          fe += Ct<T>(0, 2 * k) * xs[sl] + Ct<T>(1, 2 * k) * xd[sl];
          if (k < 15) fo += Ct<T>(0, 2 * k + 1) * xs[sl] + Ct<T>(1, 2 * k + 1) * xd[sl];
        }
        const int p = 2 * q;
        T ve = (vp && p < R2) ? pve : T(0);
        T vo = (vp && p + 1 < R2) ? pvo : T(0);
        if (ca != 0.0) {
          const double dze = cz0 + (double)p * hh, dzo = dze + hh;
          const double re = cxy + dze * dze, ro = cxy + dzo * dzo;
          ve = (T)((double)ve + ca * re * re);
          vo = (T)((double)vo + ca * ro * ro);
        }
        eacc += (double)ve * (double)fe * (double)fe + (double)vo * (double)fo * (double)fo;
        const T ge = ve * fe, go = vo * fo;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const int sl = (u - k) & 15;
          a0[sl] += Ct<T>(0, 2 * k) * ge;
          a1[sl] += Ct<T>(1, 2 * k) * ge;
          if (k < 15) {
            a0[sl] += Ct<T>(0, 2 * k + 1) * go;
            a1[sl] += Ct<T>(1, 2 * k + 1) * go;
          }
        }
        // i' = q - 15 is complete
        const int sl = (u + 1) & 15;
        const int pp = q - 15 + e;
        if (pp >= 0 && pp < O2) {
          out0[(int64_t)pp * ncol] = a0[sl];
          out1[(int64_t)pp * ncol] = a1[sl];
        }
        a0[sl] = T(0);
        a1[sl] = T(0);
        }
      }
    }
  }
  const double b = block_sum_any(eacc);
  if (threadIdx.x == 0) epart[w.epart + blockIdx.x] = b;
}

// ---------------------------------------------------------------------------
// k_kin_col: thread = coarse column of a component pair along axis AX of the
// input box
// ---------------------------------------------------------------------------
// out_a(i') = fac sum_j sum_b K_ab[j] x_b(i'+j) for i' = -e .. N+e-1, where
// x_b is the component whose AX bit is b; the window holds x(i-28..i) when
// output i' = i - 14 is formed.  Each block also leaves the partial
// sum_{i' in box} x_a(i') out_a(i') of <phi|T|phi> in its e_kin slot.
// Inputs and outputs:
//   AX = 0: c8x [c][z][x][y] -> ox[8][N2][O0][N1]   (256 threads, y fastest)
//   AX = 1: c8  [c][z][y][x] -> oy[8][N2][N0][O1]   (64 threads, one column
//           per lane along x; every 16 outputs are staged in LDS and written
//           out 4 columns x 16 consecutive y' per store, y' fastest; rows
//           qrow_stride(O1) apart and windows at y' = 16 m, so that each
//           store is one whole aligned piece of a row)
//   AX = 2: c8x [c][z][x][y] -> oz[8][O2][N0][N1]   (256 threads, y fastest)
// (FP32, y axis: the register allocator is asked for 3 waves per SIMD, which
// costs a few spilled values and measured 7% faster than the 2 waves its
// 184 VGPRs allow)
template <typename T, int AX>
__global__ __launch_bounds__(AX == 1 ? 64 : 256)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && AX == 1 ? 3 : 1))) void k_kin_col(
    const SfDev* __restrict__ sfs, const SfWork* __restrict__ wk, int sf0, T* __restrict__ ws,
    double fac, double* __restrict__ kpart) {
  __shared__ T st[AX == 1 ? 2 * 16 * kSP : 1];   // AX = 1: [a][16 outputs][kSP]
  const SfWork& w = wk[blockIdx.y];
  const SfDev& sf = sfs[w.id];
  const int N0 = sf.n[0], N1 = sf.n[1], N2 = sf.n[2], e = sf.ext;
  const int64_t plane = (int64_t)N0 * N1;
  const int NA = AX == 2 ? N2 : AX == 1 ? N1 : N0;
  const int OA = NA + 2 * e;
  const int64_t ncol = AX == 2 ? plane : AX == 1 ? (int64_t)N0 * N2 : (int64_t)N1 * N2;
  const int64_t idx0 = (int64_t)blockIdx.x * blockDim.x;
  if (idx0 >= 4 * ncol) return;   // whole block beyond this function's columns
  // this axis' first e_kin slot, counted on the function's own box
  const int slot0 = AX == 0 ? 0
                  : AX == 1 ? kin_blocks(0, N0, N1, N2)
                            : kin_blocks(0, N0, N1, N2) + kin_blocks(1, N0, N1, N2);
  const int64_t idx = idx0 + threadIdx.x;
  const bool active = idx < 4 * ncol;
  const int pr = active ? (int)(idx / ncol) : 0;
  const int64_t col = active ? idx % ncol : 0;
  // component with AX bit b: AX = 0 -> b + 2 pr (pr = a2 + 2 a3);
  // AX = 1 -> a1 + 2b + 4 a3 (pr = a1 + 2 a3); AX = 2 -> pr + 4b (pr = a1 + 2 a2)
  const int cb0 = AX == 2 ? pr : AX == 1 ? (pr & 1) + 4 * (pr >> 1) : 2 * pr;
  const int cb1 = AX == 2 ? pr + 4 : AX == 1 ? cb0 + 2 : cb0 + 1;
  int64_t ibase, obase, istride, ostride;
  if (AX == 2) {          // column (x, y), y fastest
    ibase = col;
    istride = plane;
    obase = col;
    ostride = plane;
  } else if (AX == 1) {   // column (x, z), x fastest
    const int x = (int)(col % N0), z = (int)(col / N0);
    ibase = (int64_t)z * plane + x;
    istride = N0;
    obase = ((int64_t)z * N0 + x) * qrow_stride(OA);
    ostride = 1;
  } else {                // column (y, z), y fastest
    const int y = (int)(col % N1), z = (int)(col / N1);
    ibase = (int64_t)z * plane + y;
    istride = N1;
    obase = (int64_t)z * OA * N1 + y;
    ostride = N1;
  }
  const int64_t icomp = (int64_t)N2 * plane;                          // component size
  const int64_t ocomp = AX == 2 ? (int64_t)OA * plane : AX == 1 ? (int64_t)N2 * N0 * qrow_stride(OA)
                                                                : (int64_t)N2 * OA * N1;
  const T* inb = ws + (AX == 1 ? w.c8 : w.c8x);
  const T* in0 = inb + cb0 * icomp + ibase;
  const T* in1 = inb + cb1 * icomp + ibase;
  T* outb = ws + (AX == 2 ? w.oz : AX == 1 ? w.oy : w.ox);
  T* out0 = outb + cb0 * ocomp + obase;
  T* out1 = outb + cb1 * ocomp + obase;
  const int lane = threadIdx.x;
  // AX = 1: where this lane's column starts in the output (-1: no column)
  const int colbase0 = active ? (int)(out0 - outb) : -1;   // < 8 N2 N0 O1
  const int colbase1 = active ? (int)(out1 - outb) : -1;
  // the scaling-channel window in double: its differences are then exact
  constexpr int PF = pf_kin<T, AX>(), NS = pf_slots(PF);
  double x0[32];
  T x1[32], f0[NS], f1[NS];
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    x0[k] = 0.0;
    x1[k] = T(0);
  }
  double eacc = 0.0;
  const int istart = 14 - e;           // emits i' = -e first
  const int iend = NA - 1 + e + 14;    // emits i' = NA - 1 + e last
  const int ilo = istart - 28;
  // first window: the largest i0 <= ilo with i0 = 14 - e (mod 16), so that
  // the staged outputs (AX = 1) start at y' = 16 m
  const int i0first = ilo - ((((ilo - (14 - e)) % 16) + 16) % 16);
#pragma unroll
  for (int d = 0; d < PF; ++d) {
    f0[d] = ld_clamp(in0, i0first + d, NA, istride);
    f1[d] = ld_clamp(in1, i0first + d, NA, istride);
  }
  for (int i0 = i0first; i0 <= iend; i0 += 32) {
#pragma unroll
    for (int u = 0; u < 32; ++u) {
      const int i = i0 + u, sp = u % NS;
      const bool ok = active && i >= 0 && i < NA;
      if constexpr (PF > 0) {
        x0[u] = ok ? (double)f0[sp] : 0.0;
        x1[u] = ok ? f1[sp] : T(0);
        f0[sp] = ld_clamp(in0, i + PF, NA, istride);
        f1[sp] = ld_clamp(in1, i + PF, NA, istride);
      } else {
        x0[u] = ok ? (double)in0[(int64_t)i * istride] : 0.0;
        x1[u] = ok ? in1[(int64_t)i * istride] : T(0);
      }
      if (i >= istart && i <= iend) {
        const int ip = i - 14;            // output coarse index i'
        const int sc = (u + 18) & 31;     // slot of x(i') = x(i - 14)
        double r0, r1;
        if (sizeof(T) == 4) {
          // scaling-channel taps in the difference form with FP64 taps,
          // summed in double (the differences of FP32 values are exact
          // there), completed by the row sums D_a; wavelet taps in FP32
          double s0 = 0.0, s1 = 0.0;
          T w0 = T(0), w1 = T(0);
#pragma unroll
          for (int t = 0; t < 29; ++t) {
            if (t == 14) continue;
            const int sl = (u + 4 + t) & 31;    // x(i - 28 + t) = x(i' + t - 14)
            const double d0 = x0[sl] - x0[sc];
            s0 += fK64[0][0][t] * d0;
            s1 += fK64[1][0][t] * d0;
            w0 += Kt<T>(0, 1, t) * x1[sl];
            w1 += Kt<T>(1, 1, t) * x1[sl];
          }
          const double c0 = x0[sc], c1 = (double)x1[sc];
          r0 = fac * ((s0 + (double)w0) + fKD64[0] * c0 + fK64[0][1][14] * c1);
          r1 = fac * ((s1 + (double)w1) + fKD64[1] * c0 + fK64[1][1][14] * c1);
        } else {
          double s0 = 0.0, s1 = 0.0;
#pragma unroll
          for (int t = 0; t < 29; ++t) {
            const int sl = (u + 4 + t) & 31;
            s0 += fK64[0][0][t] * (double)x0[sl] + fK64[0][1][t] * (double)x1[sl];
            s1 += fK64[1][0][t] * (double)x0[sl] + fK64[1][1][t] * (double)x1[sl];
          }
          r0 = fac * s0;
          r1 = fac * s1;
        }
        if (ip >= 0 && ip < NA) eacc += x0[sc] * r0 + (double)x1[sc] * r1;
        const int pp = ip + e;
        if (AX == 1) {
          st[(u & 15) * kSP + lane] = (T)r0;
          st[(16 + (u & 15)) * kSP + lane] = (T)r1;
        } else if (active) {
          out0[(int64_t)pp * ostride] = (T)r0;
          out1[(int64_t)pp * ostride] = (T)r1;
        }
      }
      if (AX == 1 && (u & 15) == 15) {
        // outputs pp = i0 + (u - 15) + j - 14 + e, j = 0..15, of the 64
        // columns (those with 0 <= pp < OA were formed above): 4 columns x
        // 16 consecutive y' per store
        __syncthreads();
        const int j = lane & 15;
        const int pp = i0 + (u - 15) + j - 14 + e;
        const bool okp = pp >= 0 && pp < OA;
#pragma unroll
        for (int it = 0; it < 16; ++it) {
          const int cl = it * 4 + (lane >> 4);
          const int b0c = __shfl(colbase0, cl, 64), b1c = __shfl(colbase1, cl, 64);
          if (okp && b0c >= 0) {
            outb[b0c + pp] = st[j * kSP + cl];
            outb[b1c + pp] = st[(16 + j) * kSP + cl];
          }
        }
        __syncthreads();
      }
    }
  }
  const double bs = block_sum_any(eacc);
  if (threadIdx.x == 0) kpart[w.kpart + slot0 + blockIdx.x] = bs;
}

// ---------------------------------------------------------------------------
// k_kin_zmfma: the z part of the kinetic term as banded-Toeplitz matrix
// products on the FP64 matrix cores (v_mfma_f64_16x16x4f64)
// ---------------------------------------------------------------------------
// Wave = 16 consecutive (x, y) columns of one component pair pr = a1 + 2 a2
// of one function; it walks the output z' in tiles of 16.  For output
// channel a (component pr + 4 a) and a tile starting at z'0:
//   D_a[r][c] = sum_b sum_k A_ab[r][k] X_b[z'0 - e - 14 + k][c],
//   A_ab[r][k] = K_ab[k - r] for 0 <= k - r <= 28 (else 0), k = 0..43,
// i.e. 11 steps of k = 4 per input channel b: 22 MFMAs per output channel
// (58 useful of 88 multiply-adds per output).  The same products as the
// stencil of k_kin_col<T, 2>, in another order, summed in double for both
// element types (FP32 inputs enter exactly).  Lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16] of a step and holds D[l / 16 + 4 j][l % 16] in
// element j (the FP64 form interleaves the rows; checked on the device).  Block = 4 waves; its e_kin slot gets
// the sum of x_a(z) D_a over the outputs inside the box, in a fixed order.
typedef double wvl_d4 __attribute__((ext_vector_type(4)));

template <typename T>
__global__ __launch_bounds__(256) void k_kin_zmfma(const SfDev* __restrict__ sfs,
                                                   const SfWork* __restrict__ wk, int sf0,
                                                   T* __restrict__ ws, double fac,
                                                   double* __restrict__ kpart) {
  const SfWork& w = wk[blockIdx.y];
  const SfDev& sf = sfs[w.id];
  const int N0 = sf.n[0], N1 = sf.n[1], N2 = sf.n[2], e = sf.ext;
  const int64_t plane = (int64_t)N0 * N1;
  const int OA = N2 + 2 * e;
  const int ngrp = (int)((plane + 15) / 16);            // 16-column groups per pair
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int item = blockIdx.x * 4 + wv;                  // (pair, group)
  if (blockIdx.x * 4 >= 4 * ngrp) return;                // uniform over the block
  const int slot0 = kin_blocks(0, N0, N1, N2) + kin_blocks(1, N0, N1, N2);
  double eacc = 0.0;
  if (item < 4 * ngrp) {
    const int pr = item / ngrp, grp = item - pr * ngrp;
    const int64_t icomp = (int64_t)N2 * plane, ocomp = (int64_t)OA * plane;
    const int rsel = lane & 15, ksel = lane >> 4;
    const int64_t col = (int64_t)grp * 16 + rsel;        // this lane's column (B and D)
    const bool colok = col < plane;
    const T* in0 = ws + w.c8x + (int64_t)pr * icomp + col;          // b = 0
    const T* in1 = in0 + 4 * icomp;                                  // b = 1 (component + 4)
    T* out0 = ws + w.oz + (int64_t)pr * ocomp + col;
    T* out1 = out0 + 4 * ocomp;
    // A operands of the 11 k-steps, per (a, b): K_ab[4 s + ksel - rsel]
    double Ak[2][2][11];
#pragma unroll
    for (int s = 0; s < 11; ++s) {
      const int t = 4 * s + ksel - rsel;
      const bool ok = t >= 0 && t <= 28;
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) Ak[a][b][s] = ok ? fac * fK64[a][b][ok ? t : 0] : 0.0;
    }
    for (int z0 = 0; z0 < OA; z0 += 16) {
      const int zin0 = z0 - e - 14;
      wvl_d4 d0 = {0.0, 0.0, 0.0, 0.0}, d1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < 11; ++s) {
        const int zi = zin0 + 4 * s + ksel;
        const bool ok = colok && zi >= 0 && zi < N2;
        const double x0 = ok ? (double)in0[(int64_t)zi * plane] : 0.0;
        const double x1 = ok ? (double)in1[(int64_t)zi * plane] : 0.0;
        d0 = __builtin_amdgcn_mfma_f64_16x16x4f64(Ak[0][0][s], x0, d0, 0, 0, 0);
        d1 = __builtin_amdgcn_mfma_f64_16x16x4f64(Ak[1][0][s], x0, d1, 0, 0, 0);
        d0 = __builtin_amdgcn_mfma_f64_16x16x4f64(Ak[0][1][s], x1, d0, 0, 0, 0);
        d1 = __builtin_amdgcn_mfma_f64_16x16x4f64(Ak[1][1][s], x1, d1, 0, 0, 0);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int zp = z0 + ksel + 4 * j;
        if (!colok || zp >= OA) continue;
        out0[(int64_t)zp * plane] = (T)d0[j];
        out1[(int64_t)zp * plane] = (T)d1[j];
        const int z = zp - e;
        if (z >= 0 && z < N2)
          eacc += (double)in0[(int64_t)z * plane] * d0[j] + (double)in1[(int64_t)z * plane] * d1[j];
      }
    }
  }
  const double bs = block_sum_any(eacc);
  if (threadIdx.x == 0) kpart[w.kpart + slot0 + blockIdx.x] = bs;
}

// ---------------------------------------------------------------------------
// k_back_y: block = (function, 64 consecutive fine columns (a3, z', px))
// ---------------------------------------------------------------------------
// Thread = fine column px of G2[a3][z'][.][px], streaming along y: fine pair
// p = 2q, 2q+1 arrives and is scattered into the accumulators of coarse
// i' = q-15..q (out_b(i') += C_b[p - 2i'] g_p, b = a2); i' = q-15 is then
// complete.  Every 16 results are staged in LDS and written out as
// Q[a2 + 2 a3][z'][px][y'] (y' fastest, rows qrow_stride(O1) apart), 4
// columns x 16 y' per store.  The stream starts up to 15 steps early (zero
// inputs) so that every window is y' = 16 m .. 16 m + 15: each store is then
// one whole aligned piece of a row.
template <typename T>
__global__ __launch_bounds__(64) void k_back_y(const SfDev* __restrict__ sfs,
                                               const SfWork* __restrict__ wk, int sf0,
                                               T* __restrict__ ws) {
  __shared__ T st[2 * 16 * kSP];
  const SfWork& w = wk[blockIdx.y];
  const SfDev& sf = sfs[w.id];
  const int N0 = sf.n[0], N1 = sf.n[1], N2 = sf.n[2], e = sf.ext;
  const int R0 = 2 * N0 + 29, R1 = 2 * N1 + 29;
  const int O1 = N1 + 2 * e, O2 = N2 + 2 * e;
  const int64_t ncols = 2ll * O2 * R0;           // columns (a3, z', px), px fastest
  const int64_t col0 = (int64_t)blockIdx.x * 64;
  if (col0 >= ncols) return;
  const int lane = threadIdx.x;
  const int64_t col = col0 + lane;
  const bool active = col < ncols;
  // G2[a3][z'][py][px]: column (a3, z', px) starts at (a3 O2 + z') R1 R0 + px
  const int64_t slab = active ? col / R0 : 0;     // a3 * O2 + z'
  const int px = active ? (int)(col % R0) : 0;
  const T* in = ws + w.g2 + slab * R1 * R0 + px;
  // Q[a2 + 2 a3][z'][px][y']: start of this column's y' run for a2 = 0
  const int a3 = (int)(slab / O2), zp = (int)(slab - (int64_t)a3 * O2);
  const int QS = qrow_stride(O1);
  const int qcol = active ? ((2 * a3 * O2 + zp) * R0 + px) * QS : -1;
  const int qa = O2 * R0 * QS;                      // a2 stride (< 2^31 elements)
  T* qo = ws + w.q;
  if (e == 16 && active) {  // coarse i' = -16 lies beyond the filter reach
    qo[qcol] = T(0);
    qo[qa + qcol] = T(0);
  }
  constexpr int PF = pf_back_y<T>();
  T a0[16], a1[16], fe_[pf_slots(PF)], fo_[pf_slots(PF)];
#pragma unroll
  for (int k = 0; k < 16; ++k) a0[k] = a1[k] = T(0);
  // first window y' = q0s - 15 + e: a multiple of 16 at or below 0
  const int ph = (15 - e) & 15;
  const int q0s = ph > 0 ? ph - 16 : 0;
#pragma unroll
  for (int d = 0; d < PF; ++d) {
    fe_[d] = ld_clamp(in, 2 * (q0s + d), R1, R0);
    fo_[d] = ld_clamp(in, 2 * (q0s + d) + 1, R1, R0);
  }
  const int qend = N1 + e + 14;
  for (int q0 = q0s; q0 <= qend; q0 += 16) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int q = q0 + u, sp = u % pf_slots(PF);
      T ve = T(0), vo = T(0);
      if constexpr (PF > 0) {
        ve = fe_[sp];
        vo = fo_[sp];
        fe_[sp] = ld_clamp(in, 2 * (q + PF), R1, R0);
        fo_[sp] = ld_clamp(in, 2 * (q + PF) + 1, R1, R0);
      }
      if (q <= qend) {
        const int p = 2 * q;
        if constexpr (PF == 0) {
          ve = (active && p >= 0 && p < R1) ? in[(int64_t)p * R0] : T(0);
          vo = (active && p >= 0 && p + 1 < R1) ? in[(int64_t)(p + 1) * R0] : T(0);
        }
        const T ge = (active && p >= 0 && p < R1) ? ve : T(0);
        const T go = (active && p >= 0 && p + 1 < R1) ? vo : T(0);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const int sl = (u - k) & 15;
          a0[sl] += Ct<T>(0, 2 * k) * ge;
          a1[sl] += Ct<T>(1, 2 * k) * ge;
          if (k < 15) {
            a0[sl] += Ct<T>(0, 2 * k + 1) * go;
            a1[sl] += Ct<T>(1, 2 * k + 1) * go;
          }
        }
        const int sl = (u + 1) & 15;
        st[u * kSP + lane] = a0[sl];          // y' = q - 15 + e
        st[(16 + u) * kSP + lane] = a1[sl];
        a0[sl] = T(0);
        a1[sl] = T(0);
      }
    }
    // flush y' = q0 - 15 + e + j, j = 0..15
    __syncthreads();
    const int j = lane & 15;
    const int yp = q0 - 15 + e + j;
    const bool oky = yp >= 0 && yp < O1 && q0 + j <= qend;
#pragma unroll
    for (int it = 0; it < 16; ++it) {
      const int cl = it * 4 + (lane >> 4);
      const int qc = __shfl(qcol, cl, 64);
      if (oky && qc >= 0) {
        qo[qc + yp] = st[j * kSP + cl];
        qo[qa + qc + yp] = st[(16 + j) * kSP + cl];
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// k_back_out: block = (function, kBackOutRows output rows (y', z')), streaming along x
// ---------------------------------------------------------------------------
// Block = 4 kBackOutRows threads = output rows (y', z') x the 4 channel pairs
// ch = a2 + 2 a3 (thread t: row t / 4, ch = t % 4), rows in (z', y') order,
// so that one wave holds all 8 components of its 16 rows.  Thread = output
// row (y', z') of channel ch, components c = a1 + 2 a2 + 4 a3 (a1 = 0, 1).
// Streaming along x: fine pair p = 2q, 2q+1 of Q[ch][z'][p][y'] is scattered
// into the potential accumulators of coarse i' = q-15..q; i' = q-15 is then
// complete and gets the x, y and z kinetic parts (from k_kin_col).  Every
// 16 x' the block's values [component][x'][row] are staged in LDS and written
// straight to the compressed output: per row and pattern, the points of its
// run that fall in the window are contiguous in the output (scaling values
// one per point, wavelets seven per point), so the window's runs of each row
// (first and last window index, output point index; from the row's single
// run or, for rows with several, its segments) make the stores consecutive.
// The dense output box and a separate compression pass are not needed.
constexpr int kBoRows = kBackOutRows, kBoThreads = 4 * kBackOutRows;
constexpr uint32_t kBoGroup = 8;   // row blocks per XCD run (a power of two)
// Orders a wave's LDS accesses across the lanes of that wave (LDS requests of
// one wave are served in order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// A 16-point window of a row meets at most 16 segments of a pattern (each
// holds at least one point; segments may touch).
constexpr int kBoRuns = 16;
template <typename T>
__global__ __launch_bounds__(kBoThreads) void k_back_out(const SfDev* __restrict__ sfs,
                                                  const wvl_seg* __restrict__ seg,
                                                  const int32_t* __restrict__ rt,
                                                  const RowRun* __restrict__ rr,
                                                  const SfWork* __restrict__ wk, int sf0,
                                                  const T* __restrict__ ws, T* __restrict__ out,
                                                  int pot_on, int kin_on, int accumulate) {
  constexpr int SR = kBoRows + 1;                   // LDS stride of one (component, x') row
  __shared__ T st[8 * 16 * SR];                     // [component][x' in window][row]
  // per pattern (scaling, wavelets) and row, the runs in the window: window
  // indices [js, je) and the point index (within the pattern) of js
  __shared__ int8_t od_js[2][kBoRuns][kBoRows], od_je[2][kBoRuns][kBoRows];
  __shared__ int32_t od_o[2][kBoRuns][kBoRows];
  __shared__ int32_t od_n[2][kBoRows];
  // XCD-aware order: the 8 XCDs take blocks round-robin; each run of
  // kBoGroup consecutive row blocks (logical order: rows fastest, then
  // functions) goes to one XCD, whose L2 then serves the cache lines of Q
  // and of the kinetic parts that neighbouring row blocks share
  uint32_t lb = blockIdx.x + blockIdx.y * gridDim.x;
  if (lb < ((gridDim.x * gridDim.y) & ~(8u * kBoGroup - 1u))) {
    const uint32_t x = lb & 7, sl = lb >> 3;
    lb = kBoGroup * (8 * (sl / kBoGroup) + x) + sl % kBoGroup;
  }
  const int bxl = (int)(lb % gridDim.x), byl = (int)(lb / gridDim.x);
  const SfWork& w = wk[byl];
  const SfDev& sf = sfs[w.id];
  const int N0 = sf.n[0], N1 = sf.n[1], N2 = sf.n[2], e = sf.ext;
  const int R0 = 2 * N0 + 29;
  const int O0 = N0 + 2 * e, O1 = N1 + 2 * e, O2 = N2 + 2 * e;
  const int64_t nout = (int64_t)O1 * O2;
  const int64_t r0 = (int64_t)bxl * kBoRows;
  if (r0 >= nout) return;   // uniform over the block
  const int tid = threadIdx.x;
  const int rl = tid >> 2, ch = tid & 3;
  const int64_t orw = r0 + rl;
  const bool active = orw < nout;
  const int zp = active ? (int)(orw / O1) : 0, yp = active ? (int)(orw % O1) : 0;
  const int a2 = ch & 1, a3 = ch >> 1;
  const int z = zp - e, y = yp - e;
  const bool zin = kin_on && z >= 0 && z < N2;
  const bool yin = y >= 0 && y < N1;
  const int64_t plane = (int64_t)N0 * N1;
  // Wave wv computes, stages and writes rows 16 wv .. 16 wv + 15 on its own
  // (all 8 components of a row sit in one wave), so the waves of a block
  // never wait for each other.  Lanes 0..31 describe (pattern lane / 16,
  // row 16 wv + lane % 16).
  const int lane = tid & 63, wv = tid >> 6;
  const int drow = 16 * wv + (lane & 15), dpat = (lane >> 4) & 1;
  RowRun myrun{0, 0, 0};
  int64_t mygrow = -1;   // the row's index in the pattern's row table, -1: none
  if (lane < 32) {
    const int64_t r = r0 + drow;
    if (r < nout) {
      mygrow = sf.rt[2 + dpat] + r;
      myrun = rr[sf.rr[2 + dpat] + r];
    }
  }
  const int xg0 = sf.lo[0] - e;   // global x of x' = 0
  // runs of the window x' = xw + j, jlo <= j < jhi
  auto describe = [&](int xw, int jlo, int jhi) {
    if (lane >= 32) return;
    int n = 0;
    auto add = [&](int gx0, int len, int64_t off) {   // run [gx0, gx0 + len) from point off
      const int b = gx0 - xg0 - xw;                     // its window index
      const int js = max(jlo, b), je = min(jhi, b + len);
      if (js < je && n < kBoRuns) {
        od_js[dpat][n][drow] = (int8_t)js;
        od_je[dpat][n][drow] = (int8_t)je;
        od_o[dpat][n][drow] = (int32_t)(off + (js - b));
        ++n;
      }
    };
    if (mygrow >= 0 && myrun.len != 0) {
      if (myrun.len != kMultiRun) {
        add(myrun.x0, myrun.len, myrun.off);
      } else {
        for (int q = rt[mygrow]; q < rt[mygrow + 1]; ++q)
          add(seg[q].i1s, seg[q].i1e - seg[q].i1s + 1, seg[q].off);
      }
    }
    od_n[dpat][drow] = n;
  };
  const int QS = qrow_stride(O1);
  const T* qin = ws + w.q + ((int64_t)(ch * O2 + zp) * R0) * QS + yp;
  const int c0 = 2 * a2 + 4 * a3, c1 = c0 + 1;
  const int64_t comp_x = (int64_t)N2 * O0 * N1, comp_y = (int64_t)N2 * N0 * QS;
  const int64_t comp_z = (int64_t)O2 * plane;
  const T* oxp = ws + w.ox + ((int64_t)(zin ? z : 0) * O0) * N1 + (yin ? y : 0);  // [c][z][x'][y]
  const T* oyp = ws + w.oy + (int64_t)(zin ? z : 0) * N0 * QS + yp;   // [c][z][x][y'], rows QS apart
  const T* ozp = ws + w.oz + (int64_t)zp * plane + (yin ? y : 0);                // [c][z'][x][y]
  T* const outc = out + sf.cout;
  T* const outf = out + sf.cout + sf.on_c;
  auto put = [&](T* o, T v) { *o = accumulate ? *o + v : v; };
  // writes the described runs from the staged values (vals false: zeros, for
  // points no filter reaches); wave wv writes rows 16 wv .. 16 wv + 15
  auto flush = [&](bool vals) {
    // scaling values: 4 rows of 16 lanes per pass
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = 16 * wv + 4 * i + (lane >> 4), j = lane & 15;
      const int n = od_n[0][r];
      for (int u = 0; u < n; ++u) {
        const int js = od_js[0][u][r];
        if (j >= js && j < od_je[0][u][r]) {
          put(outc + od_o[0][u][r] + (j - js), vals ? st[j * SR + r] : T(0));
          break;
        }
      }
    }
    // wavelets: one run at a time, seven consecutive outputs per point
    for (int i = 0; i < 16; ++i) {
      const int r = 16 * wv + i;
      const int n = __builtin_amdgcn_readfirstlane(od_n[1][r]);
      for (int u = 0; u < n; ++u) {
        const int js = __builtin_amdgcn_readfirstlane(od_js[1][u][r]);
        const int n7 = 7 * (__builtin_amdgcn_readfirstlane(od_je[1][u][r]) - js);
        T* const ob = outf + 7 * (int64_t)__builtin_amdgcn_readfirstlane(od_o[1][u][r]);
        for (int t = lane; t < n7; t += 64) {
          const int jj = t / 7, c = t - 7 * jj + 1;
          put(ob + t, vals ? st[(c * 16 + js + jj) * SR + r] : T(0));
        }
      }
    }
  };
  if (e == 16) {   // coarse i' = -16 lies beyond every filter's reach
    describe(0, 0, 1);
    wave_lds_sync();
    flush(false);
    wave_lds_sync();
  }
  T p0[16], p1[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) p0[k] = p1[k] = T(0);
  // prefetch rings: Q pairs kPfBackQ steps ahead, the kinetic parts (x part
  // at x' = q - 15 + e, y and z parts at i' = q - 15) kPfBackK steps ahead
  const T* const ox0 = oxp + c0 * comp_x;
  const T* const ox1 = oxp + c1 * comp_x;
  const T* const oy0 = oyp + c0 * comp_y;
  const T* const oy1 = oyp + c1 * comp_y;
  const T* const oz0 = ozp + c0 * comp_z;
  const T* const oz1 = ozp + c1 * comp_z;
  T fe_[kPfBackQ], fo_[kPfBackQ], kx0[kPfBackK], kx1[kPfBackK], ky0[kPfBackK], ky1[kPfBackK],
      kz0[kPfBackK], kz1[kPfBackK];
  auto fetch_q = [&](int q, int s) {
    fe_[s] = ld_clamp(qin, 2 * q, R0, QS);
    fo_[s] = ld_clamp(qin, 2 * q + 1, R0, QS);
  };
  auto fetch_k = [&](int q, int s) {
    kx0[s] = ld_clamp(ox0, q - 15 + e, O0, N1);
    kx1[s] = ld_clamp(ox1, q - 15 + e, O0, N1);
    ky0[s] = ld_clamp(oy0, q - 15, N0, QS);
    ky1[s] = ld_clamp(oy1, q - 15, N0, QS);
    kz0[s] = ld_clamp(oz0, q - 15, N0, N1);
    kz1[s] = ld_clamp(oz1, q - 15, N0, N1);
  };
  if (pot_on) {
#pragma unroll
    for (int d = 0; d < kPfBackQ; ++d) fetch_q(d, d);
  }
  if (kin_on) {
#pragma unroll
    for (int d = 0; d < kPfBackK; ++d) fetch_k(d, d);
  }
  const int qend = N0 + e + 14;
  for (int q0 = 0; q0 <= qend; q0 += 16) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int q = q0 + u, sp = u % kPfBackQ, sk = u % kPfBackK;
      if (q > qend) continue;
      const T vx0 = kx0[sk], vx1 = kx1[sk], vy0 = ky0[sk], vy1 = ky1[sk];
      const T vz0 = kz0[sk], vz1 = kz1[sk];
      if (kin_on) fetch_k(q + kPfBackK, sk);
      if (pot_on) {
        const int p = 2 * q;
        const T ge = (active && p < R0) ? fe_[sp] : T(0);
        const T go = (active && p + 1 < R0) ? fo_[sp] : T(0);
        fetch_q(q + kPfBackQ, sp);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const int sl = (u - k) & 15;
          p0[sl] += Ct<T>(0, 2 * k) * ge;
          p1[sl] += Ct<T>(1, 2 * k) * ge;
          if (k < 15) {
            p0[sl] += Ct<T>(0, 2 * k + 1) * go;
            p1[sl] += Ct<T>(1, 2 * k + 1) * go;
          }
        }
      }
      // i' = q - 15 is complete
      const int ip = q - 15;
      const int xp = ip + e;
      const int ps = (u + 1) & 15;
      T v0 = p0[ps], v1 = p1[ps];
      p0[ps] = T(0);
      p1[ps] = T(0);
      if (active && kin_on && xp >= 0 && xp < O0) {
        const bool xin = ip >= 0 && ip < N0;
        if (zin && yin) {            // x part: ox[c][z][x'][y]
          v0 += vx0;
          v1 += vx1;
        }
        if (xin) {
          T k0 = T(0), k1 = T(0);
          if (zin) {                 // y part: oy[c][z][x][y']
            k0 += vy0;
            k1 += vy1;
          }
          if (yin) {                 // z part: oz[c][z'][x][y]
            k0 += vz0;
            k1 += vz1;
          }
          v0 += k0;
          v1 += k1;
        }
      }
      st[(c0 * 16 + u) * SR + rl] = v0;
      st[(c1 * 16 + u) * SR + rl] = v1;
    }
    // window x' = q0 - 15 + e + j, j = 0..15: the part inside [0, O0) with
    // q = q0 + j <= qend
    const int xw = q0 - 15 + e;
    describe(xw, max(0, -xw), min(16, min(O0 - xw, qend - q0 + 1)));
    wave_lds_sync();
    flush(true);
    wave_lds_sync();
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

// Loads the code objects of every kernel an apply may launch (and with them
// the filter tables in constant memory), so that no lazy load happens while
// a stream is being captured.
int preload_fused_kernels() {
  const void* fns[] = {
      (const void*)k_unpack<float>,         (const void*)k_unpack<double>,
      (const void*)k_up_z<float>,           (const void*)k_up_z<double>,
      (const void*)k_up_x<float>,           (const void*)k_up_x<double>,
      (const void*)k_up_y<float>,           (const void*)k_up_y<double>,
      (const void*)k_pot_column<float>,     (const void*)k_pot_column<double>,
      (const void*)k_kin_col<float, 0>,     (const void*)k_kin_col<float, 1>,
      (const void*)k_kin_col<float, 2>,     (const void*)k_kin_col<double, 0>,
      (const void*)k_kin_col<double, 1>,    (const void*)k_kin_col<double, 2>,
      (const void*)k_back_y<float>,         (const void*)k_back_y<double>,
      (const void*)k_back_out<float>,       (const void*)k_back_out<double>,
      (const void*)k_kin_zmfma<float>,      (const void*)k_kin_zmfma<double>};
  for (const void* f : fns) {
    hipFuncAttributes a;
    const hipError_t e = hipFuncGetAttributes(&a, f);
    if (e != hipSuccess) return (int)e;
  }
  return 0;
}

int launch_unpack(int f64, void* stream, const SfDev* sf, const wvl_seg* seg, const int32_t* rt,
                  const RowRun* rr, const void* psi, const SfWork* wk, int nsf, int gridx,
                  int group, size_t lds, void* ws) {
  if (nsf == 0 || gridx == 0) return 0;
  if (group != 1 && group != 2 && group != 4 && group != 8) return (int)hipErrorInvalidValue;
  const dim3 g((unsigned)gridx, (unsigned)nsf);
  if (f64)
    hipLaunchKernelGGL(k_unpack<double>, g, dim3(256), lds, (hipStream_t)stream, sf, seg, rt, rr,
                       (const double*)psi, wk, (double*)ws, group);
  else
    hipLaunchKernelGGL(k_unpack<float>, g, dim3(256), lds, (hipStream_t)stream, sf, seg, rt, rr,
                       (const float*)psi, wk, (float*)ws, group);
  return (int)hipGetLastError();
}

int launch_up(int f64, void* stream, int axis, const SfWork* wk, const SfDev* sf, int nsf,
              int gridx, void* ws) {
  if (nsf == 0 || gridx == 0) return 0;
  const dim3 g((unsigned)gridx, (unsigned)nsf);
  hipStream_t st = (hipStream_t)stream;
  if (axis == 0) {
    if (f64)
      hipLaunchKernelGGL(k_up_x<double>, g, dim3(64), 0, st, sf, wk, (double*)ws);
    else
      hipLaunchKernelGGL(k_up_x<float>, g, dim3(64), 0, st, sf, wk, (float*)ws);
  } else {
    if (f64)
      hipLaunchKernelGGL(k_up_y<double>, g, dim3(256), 0, st, sf, wk, (double*)ws);
    else
      hipLaunchKernelGGL(k_up_y<float>, g, dim3(256), 0, st, sf, wk, (float*)ws);
  }
  return (int)hipGetLastError();
}

int launch_up_z(int f64, void* stream, const SfWork* wk, const SfDev* sf, int nsf, int gridx,
                const void* ws, const int64_t* fine_off, void* fine) {
  if (nsf == 0) return 0;
  const dim3 g((unsigned)gridx, (unsigned)nsf);
  if (f64)
    hipLaunchKernelGGL(k_up_z<double>, g, dim3(256), 0, (hipStream_t)stream, sf, wk,
                       (const double*)ws, fine_off, (double*)fine);
  else
    hipLaunchKernelGGL(k_up_z<float>, g, dim3(256), 0, (hipStream_t)stream, sf, wk,
                       (const float*)ws, fine_off, (float*)fine);
  return (int)hipGetLastError();
}

int launch_pot_column(int f64, void* stream, const SfDev* sf, const SfWork* wk, int sf0, int nsf,
                      int gridx, void* ws, const void* pot, int nf1, int nf2, double* epart,
                      const double* conf, double hh) {
  if (nsf == 0 || gridx == 0) return 0;
  const dim3 g((unsigned)gridx, (unsigned)nsf);
  if (f64)
    hipLaunchKernelGGL(k_pot_column<double>, g, dim3(256), 0, (hipStream_t)stream, sf, wk, sf0,
                       (double*)ws, (const double*)pot, nf1, nf2, epart, conf, hh);
  else
    hipLaunchKernelGGL(k_pot_column<float>, g, dim3(256), 0, (hipStream_t)stream, sf, wk, sf0,
                       (float*)ws, (const float*)pot, nf1, nf2, epart, conf, hh);
  return (int)hipGetLastError();
}

int launch_kin_zmfma(int f64, void* stream, const SfDev* sf, const SfWork* wk, int sf0, int nsf,
                     int gridx, void* ws, double fac, double* kpart) {
  if (nsf == 0 || gridx == 0) return 0;
  const dim3 g((unsigned)gridx, (unsigned)nsf);
  if (f64)
    hipLaunchKernelGGL(k_kin_zmfma<double>, g, dim3(256), 0, (hipStream_t)stream, sf, wk, sf0,
                       (double*)ws, fac, kpart);
  else
    hipLaunchKernelGGL(k_kin_zmfma<float>, g, dim3(256), 0, (hipStream_t)stream, sf, wk, sf0,
                       (float*)ws, fac, kpart);
  return (int)hipGetLastError();
}

int launch_kin_col(int f64, void* stream, int axis, const SfDev* sf, const SfWork* wk, int sf0,
                   int nsf, int gridx, void* ws, double fac, double* kpart) {
  if (nsf == 0 || gridx == 0) return 0;
  const dim3 g((unsigned)gridx, (unsigned)nsf);
  hipStream_t st = (hipStream_t)stream;
  if (f64) {
    double* w = (double*)ws;
    if (axis == 2)
      hipLaunchKernelGGL((k_kin_col<double, 2>), g, dim3(256), 0, st, sf, wk, sf0, w, fac, kpart);
    else if (axis == 1)
      hipLaunchKernelGGL((k_kin_col<double, 1>), g, dim3(64), 0, st, sf, wk, sf0, w, fac, kpart);
    else
      hipLaunchKernelGGL((k_kin_col<double, 0>), g, dim3(256), 0, st, sf, wk, sf0, w, fac, kpart);
  } else {
    float* w = (float*)ws;
    if (axis == 2)
      hipLaunchKernelGGL((k_kin_col<float, 2>), g, dim3(256), 0, st, sf, wk, sf0, w, fac, kpart);
    else if (axis == 1)
      hipLaunchKernelGGL((k_kin_col<float, 1>), g, dim3(64), 0, st, sf, wk, sf0, w, fac, kpart);
    else
      hipLaunchKernelGGL((k_kin_col<float, 0>), g, dim3(256), 0, st, sf, wk, sf0, w, fac, kpart);
  }
  return (int)hipGetLastError();
}

int launch_back_y(int f64, void* stream, const SfDev* sf, const SfWork* wk, int sf0, int nsf,
                  int gridx, void* ws) {
  if (nsf == 0 || gridx == 0) return 0;
  const dim3 g((unsigned)gridx, (unsigned)nsf);
  if (f64)
    hipLaunchKernelGGL(k_back_y<double>, g, dim3(64), 0, (hipStream_t)stream, sf, wk, sf0,
                       (double*)ws);
  else
    hipLaunchKernelGGL(k_back_y<float>, g, dim3(64), 0, (hipStream_t)stream, sf, wk, sf0,
                       (float*)ws);
  return (int)hipGetLastError();
}

int launch_back_out(int f64, void* stream, const SfDev* sf, const wvl_seg* seg, const int32_t* rt,
                    const RowRun* rr, const SfWork* wk, int sf0, int nsf, int gridx,
                    const void* ws, void* out, int pot_on, int kin_on, int accumulate) {
  if (nsf == 0 || gridx == 0) return 0;
  const dim3 g((unsigned)gridx, (unsigned)nsf);
  if (f64)
    hipLaunchKernelGGL(k_back_out<double>, g, dim3(kBoThreads), 0, (hipStream_t)stream, sf, seg, rt, rr,
                       wk, sf0, (const double*)ws, (double*)out, pot_on, kin_on, accumulate);
  else
    hipLaunchKernelGGL(k_back_out<float>, g, dim3(kBoThreads), 0, (hipStream_t)stream, sf, seg, rt, rr,
                       wk, sf0, (const float*)ws, (float*)out, pot_on, kin_on, accumulate);
  return (int)hipGetLastError();
}

}  // namespace wvl

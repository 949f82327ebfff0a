// Fused local-Hamiltonian kernels for gfx950 (MI355X).
//
// The operator factorization is the one of wvl_kernels.hip (potential term as
// stride-2 up passes C_b = synthesis then magic filter, potential multiply,
// stride-2 down passes; kinetic term as the coarse two-level filters
// K_ab = R^T a R), but the separable passes are grouped by where their data
// can live:
//   k_fwd_plane  one input z-plane: gather from the compressed segments into
//                LDS, up pass x, up pass y -> fine (x, y) plane in global G1;
//                also the dense coarse plane C8 for the kinetic kernels.
//   k_pot_column one fine (x, y) column per thread, streaming along z with
//                register rings: up pass z, potential multiply (FP64 energy
//                partials), down pass z -> G2.  Every input is read once.
//   k_kin_zcol   one coarse (x, y, component pair) column per thread: the
//                z-part of the kinetic term with a 32-slot register window.
//   k_back_plane one output z-plane (row tile): down pass y and x from LDS,
//                plus the x/y kinetic parts and the z part, e_kin partials,
//                and the compress step straight into the output pattern.
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
      return c == 0 ? psi[sf.cin + k] : psi[sf.cin + sf.n_c + (int64_t)(c - 1) * sf.n_f + k];
    }
  }
  return T(0);
}

// ---------------------------------------------------------------------------
// k_fwd_plane: block = (function, input plane z, channel a3, row tile)
// ---------------------------------------------------------------------------
// LDS: A[4][ny][N0] (components a1 + 2 a2 of channel a3, input rows iy0..iy1),
//      B[2][ny][R0] (after the x up pass, channel a2).
// Output G1[a3][z][py][px], py in the tile [py0, py1), px in [0, R0).
template <typename T>
__global__ __launch_bounds__(256) void k_fwd_plane(const SfDev* __restrict__ sfs,
                                                   const wvl_seg* __restrict__ seg,
                                                   const int32_t* __restrict__ rt,
                                                   const T* __restrict__ psi,
                                                   const SfWork* __restrict__ wk, int sf0,
                                                   T* __restrict__ ws, int tile_rows, int up_on) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const SfDev& sf = sfs[sf0 + blockIdx.y];
  const SfWork& w = wk[blockIdx.y];
  const int N0 = sf.n[0], N1 = sf.n[1], N2 = sf.n[2];
  const int R0 = 2 * N0 + 29, R1 = 2 * N1 + 29;
  const int ntile = (R1 + tile_rows - 1) / tile_rows;
  int bx = blockIdx.x;
  const int tile = bx % ntile;
  bx /= ntile;
  const int a3 = bx & 1;
  const int z = bx >> 1;
  if (z >= N2) return;
  const int py0 = tile * tile_rows, py1 = min(R1, py0 + tile_rows);
  const int iy0 = max(0, (py0 - 29) >> 1), iy1 = min(N1 - 1, (py1 - 1) >> 1);
  const int ny = iy1 - iy0 + 1;
  T* A = sm;
  T* B = A + 4 * ny * N0;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int64_t plane = (int64_t)N0 * N1;
  // 1. gather components of channel a3 on rows iy0..iy1 (and, tile 0 only,
  //    the dense coarse plane of every row for the kinetic kernels)
  for (int idx = tid; up_on && idx < 4 * ny * N0; idx += nth) {
    const int x = idx % N0;
    const int t = idx / N0;
    const int yy = t % ny, c4 = t / ny;
    const int c = c4 + 4 * a3;
    A[idx] = coef_at<T>(sf, seg, rt, psi, c, (int64_t)z * N1 + iy0 + yy, sf.lo[0] + x);
  }
  if (tile == 0) {
    T* c8 = ws + w.c8;
    for (int idx = tid; idx < 4 * N1 * N0; idx += nth) {
      const int x = idx % N0;
      const int t = idx / N0;
      const int y = t % N1, c4 = t / N1;
      const int c = c4 + 4 * a3;
      c8[((int64_t)c * N2 + z) * plane + (int64_t)y * N0 + x] =
          coef_at<T>(sf, seg, rt, psi, c, (int64_t)z * N1 + y, sf.lo[0] + x);
    }
  }
  if (!up_on) return;
  __syncthreads();
  // 2. up pass x: B[a2][yy][px], px = 2q (16 taps) and 2q+1 (15 taps) share
  //    the inputs i = q-15..q
  const int Q0 = N0 + 15;
  for (int idx = tid; idx < 2 * ny * Q0; idx += nth) {
    const int q = idx % Q0;
    const int t = idx / Q0;
    const int yy = t % ny, a2 = t / ny;
    const T* s = A + (2 * a2) * ny * N0 + yy * N0;
    const T* d = s + ny * N0;
    T fe = T(0), fo = T(0);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int i = q - k;
      if (i >= 0 && i < N0) {
        const T sv = s[i], dv = d[i];
        fe += Ct<T>(0, 2 * k) * sv + Ct<T>(1, 2 * k) * dv;
        if (k < 15) fo += Ct<T>(0, 2 * k + 1) * sv + Ct<T>(1, 2 * k + 1) * dv;
      }
    }
    T* o = B + a2 * ny * R0 + yy * R0;
    o[2 * q] = fe;
    if (2 * q + 1 < R0) o[2 * q + 1] = fo;
  }
  __syncthreads();
  // 3. up pass y into global: rows py = 2q, 2q+1 of the tile
  T* g1 = ws + w.g1 + ((int64_t)a3 * N2 + z) * ((int64_t)R0 * R1);
  const int qy0 = py0 >> 1, qy1 = (py1 + 1) >> 1;
  const int nq = qy1 - qy0;
  for (int idx = tid; idx < nq * R0; idx += nth) {
    const int px = idx % R0;
    const int q = qy0 + idx / R0;
    T fe = T(0), fo = T(0);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int i = q - k;
      if (i >= iy0 && i <= iy1) {
        const T sv = B[(i - iy0) * R0 + px], dv = B[ny * R0 + (i - iy0) * R0 + px];
        fe += Ct<T>(0, 2 * k) * sv + Ct<T>(1, 2 * k) * dv;
        if (k < 15) fo += Ct<T>(0, 2 * k + 1) * sv + Ct<T>(1, 2 * k + 1) * dv;
      }
    }
    const int pe = 2 * q, po = 2 * q + 1;
    if (pe >= py0 && pe < py1) g1[(int64_t)pe * R0 + px] = fe;
    if (po >= py0 && po < py1) g1[(int64_t)po * R0 + px] = fo;
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
                                                    double* __restrict__ epart) {
  const SfDev& sf = sfs[sf0 + blockIdx.y];
  const SfWork& w = wk[blockIdx.y];
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
    const T* vp = pot + ((int64_t)(2 * sf.lo[2]) * nf2 + (2 * sf.lo[1] + py)) * nf1 +
                  (2 * sf.lo[0] + px);
    T xs[16], xd[16], a0[16], a1[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) xs[k] = xd[k] = a0[k] = a1[k] = T(0);
    if (e == 16) {  // coarse i' = -16 lies beyond the filter reach
      out0[0] = T(0);
      out1[0] = T(0);
    }
    const int qend = N2 - 1 + e + 15;
    for (int q0 = 0; q0 <= qend; q0 += 16) {
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int q = q0 + u;
        if (q <= qend) {
        xs[u] = q < N2 ? in0[(int64_t)q * ncol] : T(0);
        xd[u] = q < N2 ? in1[(int64_t)q * ncol] : T(0);
        T fe = T(0), fo = T(0);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const int sl = (u - k) & 15;
          fe += Ct<T>(0, 2 * k) * xs[sl] + Ct<T>(1, 2 * k) * xd[sl];
          if (k < 15) fo += Ct<T>(0, 2 * k + 1) * xs[sl] + Ct<T>(1, 2 * k + 1) * xd[sl];
        }
        const int p = 2 * q;
        const T ve = p < R2 ? vp[(int64_t)p * vstride] : T(0);
        const T vo = p + 1 < R2 ? vp[(int64_t)(p + 1) * vstride] : T(0);
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
// k_kin_zcol: thread = coarse column (x, y) of component pair p = a1 + 2 a2
// ---------------------------------------------------------------------------
// out_a(i') = fac sum_j sum_b K_ab[j] x_b(i'+j), x_b = component p + 4b; the
// window holds x(i-28..i) when output i' = i - 14 is formed.
template <typename T>
__global__ __launch_bounds__(256) void k_kin_zcol(const SfDev* __restrict__ sfs,
                                                  const SfWork* __restrict__ wk, int sf0,
                                                  T* __restrict__ ws, double fac) {
  const SfDev& sf = sfs[sf0 + blockIdx.y];
  const SfWork& w = wk[blockIdx.y];
  const int N0 = sf.n[0], N1 = sf.n[1], N2 = sf.n[2], e = sf.ext;
  const int O2 = N2 + 2 * e;
  const int64_t plane = (int64_t)N0 * N1;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 4 * plane) return;
  const int pr = (int)(idx / plane);
  const int64_t xy = idx % plane;
  const T* in0 = ws + w.c8 + (int64_t)pr * N2 * plane + xy;
  const T* in1 = ws + w.c8 + (int64_t)(pr + 4) * N2 * plane + xy;
  T* out0 = ws + w.oz + (int64_t)pr * O2 * plane + xy;
  T* out1 = ws + w.oz + (int64_t)(pr + 4) * O2 * plane + xy;
  T x0[32], x1[32];
#pragma unroll
  for (int k = 0; k < 32; ++k) x0[k] = x1[k] = T(0);
  const int istart = 14 - e;           // emits i' = -e first
  const int iend = N2 - 1 + e + 14;    // emits i' = N2 - 1 + e last
  const int ilo = istart - 28;
  const int i0first = (ilo >= 0) ? (ilo & ~31) : -(((-ilo) + 31) & ~31);
  for (int i0 = i0first; i0 <= iend; i0 += 32) {
#pragma unroll
    for (int u = 0; u < 32; ++u) {
      const int i = i0 + u;
      if (i > iend) continue;
      const bool ok = i >= 0 && i < N2;
      x0[u] = ok ? in0[(int64_t)i * plane] : T(0);
      x1[u] = ok ? in1[(int64_t)i * plane] : T(0);
      if (i >= istart) {
        const int ip = i - 14;            // output coarse index i'
        const int sc = (u + 18) & 31;     // slot of x(i') = x(i - 14)
        T r0, r1;
        if (sizeof(T) == 4) {
          T s0 = T(0), s1 = T(0);
#pragma unroll
          for (int t = 0; t < 29; ++t) {
            if (t == 14) continue;
            const int sl = (u + 4 + t) & 31;    // x(i - 28 + t) = x(i' + t - 14)
            const T d0 = x0[sl] - x0[sc];
            s0 += Kt<T>(0, 0, t) * d0 + Kt<T>(0, 1, t) * x1[sl];
            s1 += Kt<T>(1, 0, t) * d0 + Kt<T>(1, 1, t) * x1[sl];
          }
          const double c0 = (double)x0[sc], c1 = (double)x1[sc];
          r0 = (T)(fac * ((double)s0 + fKD64[0] * c0 + fK64[0][1][14] * c1));
          r1 = (T)(fac * ((double)s1 + fKD64[1] * c0 + fK64[1][1][14] * c1));
        } else {
          double s0 = 0.0, s1 = 0.0;
#pragma unroll
          for (int t = 0; t < 29; ++t) {
            const int sl = (u + 4 + t) & 31;
            s0 += fK64[0][0][t] * (double)x0[sl] + fK64[0][1][t] * (double)x1[sl];
            s1 += fK64[1][0][t] * (double)x0[sl] + fK64[1][1][t] * (double)x1[sl];
          }
          r0 = (T)(fac * s0);
          r1 = (T)(fac * s1);
        }
        const int pp = ip + e;
        out0[(int64_t)pp * plane] = r0;
        out1[(int64_t)pp * plane] = r1;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// k_back_plane: block = (function, output plane z', channel a3, row tile)
// ---------------------------------------------------------------------------
// LDS: P[nq][R0] (G2 plane rows q0..q1), Q[2][T][R0] (after the y down pass,
//      channel a2), Cin[4][nyi][N0] (input plane z = z' - e, rows yi0..yi1,
//      components a1 + 2 a2 of channel a3).
// threads per block of k_back_plane: FP64 keeps one wave per SIMD per block so
// that its accumulators fit without spilling
template <typename T>
constexpr int back_threads() { return sizeof(T) == 8 ? 256 : 512; }

template <typename T>
__global__ __launch_bounds__(back_threads<T>()) void k_back_plane(
    const SfDev* __restrict__ sfs, const wvl_seg* __restrict__ seg,
    const int32_t* __restrict__ rt, const SfWork* __restrict__ wk, int sf0,
    const T* __restrict__ ws, T* __restrict__ out, int tile_rows, double fac, int pot_on,
    int kin_on, int accumulate, double* __restrict__ kpart) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const SfDev& sf = sfs[sf0 + blockIdx.y];
  const SfWork& w = wk[blockIdx.y];
  const int N0 = sf.n[0], N1 = sf.n[1], N2 = sf.n[2], e = sf.ext;
  const int R0 = 2 * N0 + 29, R1 = 2 * N1 + 29;
  const int O0 = N0 + 2 * e, O1 = N1 + 2 * e, O2 = N2 + 2 * e;
  const int ntile = (O1 + tile_rows - 1) / tile_rows;
  int bx = blockIdx.x;
  const int tile = bx % ntile;
  bx /= ntile;
  const int a3 = bx & 1;
  const int zp = bx >> 1;
  const int tid = threadIdx.x, nth = blockDim.x;
  if (zp >= O2) {
    if (tid == 0) kpart[w.kpart + blockIdx.x] = 0.0;
    return;
  }
  const int y0 = tile * tile_rows, y1 = min(O1, y0 + tile_rows);
  const int ty = y1 - y0;
  const int z = zp - e;
  const bool zin = kin_on && z >= 0 && z < N2;
  // P rows: q in [2(y0-e), 2(y1-1-e)+30] within [0, R1)
  const int q0 = max(0, 2 * (y0 - e)), q1 = min(R1 - 1, 2 * (y1 - 1 - e) + 30);
  const int nq = max(0, q1 - q0 + 1);
  const int yi0 = max(0, y0 - e - 14), yi1 = min(N1 - 1, y1 - 1 - e + 14);
  const int nyi = zin ? max(0, yi1 - yi0 + 1) : 0;
  T* P = sm;
  T* Qb = P + (pot_on ? nq * R0 : 0);
  T* Cin = Qb + (pot_on ? 2 * ty * R0 : 0);
  const int64_t ncol = (int64_t)R0 * R1;
  const int64_t plane = (int64_t)N0 * N1;
  if (pot_on) {
    const T* g2 = ws + w.g2 + ((int64_t)a3 * O2 + zp) * ncol;
    for (int idx = tid; idx < nq * R0; idx += nth) P[idx] = g2[(int64_t)q0 * R0 + idx];
  }
  if (nyi > 0) {
    for (int idx = tid; idx < 4 * nyi * N0; idx += nth) {
      const int x = idx % N0;
      const int t = idx / N0;
      const int yy = t % nyi, c4 = t / nyi;
      Cin[idx] = ws[w.c8 + ((int64_t)(c4 + 4 * a3) * N2 + z) * plane + (int64_t)(yi0 + yy) * N0 + x];
    }
  }
  __syncthreads();
  if (pot_on) {
    // down pass y: Qb[a2][yy][px] = sum_q C_a2[q - 2i'] P[q][px]; a thread makes
    // rows yy, yy+1 of both channels a2 from the 33 inputs q = 2i'..2i'+32
    const int npair = (ty + 1) >> 1;
    for (int idx = tid; idx < npair * R0; idx += nth) {
      const int px = idx % R0;
      const int yy = 2 * (idx / R0);
      const int two_i = 2 * (y0 + yy - e);
      T r[2][2] = {{T(0), T(0)}, {T(0), T(0)}};   // [a2][row]
#pragma unroll
      for (int t = 0; t < 33; ++t) {
        const int q = two_i + t;
        const T v = (q >= q0 && q <= q1) ? P[(q - q0) * R0 + px] : T(0);
#pragma unroll
        for (int a2 = 0; a2 < 2; ++a2) {
          if (t <= 30) r[a2][0] += Ct<T>(a2, t) * v;
          if (t >= 2) r[a2][1] += Ct<T>(a2, t - 2) * v;
        }
      }
#pragma unroll
      for (int a2 = 0; a2 < 2; ++a2) {
        Qb[(a2 * ty + yy) * R0 + px] = r[a2][0];
        if (yy + 1 < ty) Qb[(a2 * ty + yy + 1) * R0 + px] = r[a2][1];
      }
    }
    __syncthreads();
  }
  // outputs: a thread makes columns xo, xo+1 of row yy for all four components
  // c4 = a1 + 2 a2 of channel a3, so every filter index is a compile-time constant
  const int npx = (O0 + 1) >> 1;
  double kacc = 0.0;
  for (int idx = tid; idx < ty * npx; idx += nth) {
    const int xp = idx % npx, yy = idx / npx;
    const int yo = y0 + yy;           // output row within the grown box
    const int iy = yo - e;            // input-box row
    const int xo0 = 2 * xp;
    const int ix0 = xo0 - e;
    T val[4][2];
#pragma unroll
    for (int c4 = 0; c4 < 4; ++c4) val[c4][0] = val[c4][1] = T(0);
    if (pot_on) {
      const int two_i = 2 * ix0;
#pragma unroll
      for (int a2 = 0; a2 < 2; ++a2) {
        const T* qrow = Qb + (a2 * ty + yy) * R0;
#pragma unroll
        for (int t = 0; t < 33; ++t) {
          const int q = two_i + t;
          const T v = (q >= 0 && q < R0) ? qrow[q] : T(0);
#pragma unroll
          for (int a1 = 0; a1 < 2; ++a1) {
            if (t <= 30) val[a1 + 2 * a2][0] += Ct<T>(a1, t) * v;
            if (t >= 2) val[a1 + 2 * a2][1] += Ct<T>(a1, t - 2) * v;
          }
        }
      }
    }
    T kin[4][2];
#pragma unroll
    for (int c4 = 0; c4 < 4; ++c4) kin[c4][0] = kin[c4][1] = T(0);
    if (zin) {
      // x part (rows inside the input box): inputs x = ix0 - 14 .. ix0 + 15 are
      // streamed once and folded into both columns h and both channels a1
      if (iy >= 0 && iy < N1) {
#pragma unroll
        for (int a2 = 0; a2 < 2; ++a2) {
          const T* r0p = Cin + ((0 + 2 * a2) * nyi + (iy - yi0)) * N0;
          const T* r1p = Cin + ((1 + 2 * a2) * nyi + (iy - yi0)) * N0;
          T s0[2], s1[2];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int x = ix0 + h;
            const bool ok = x >= 0 && x < N0;
            s0[h] = ok ? r0p[x] : T(0);
            s1[h] = ok ? r1p[x] : T(0);
          }
          T acc[2][2] = {{T(0), T(0)}, {T(0), T(0)}};   // [a1][h]
#pragma unroll
          for (int t = 0; t < 30; ++t) {
            const int x = ix0 - 14 + t;
            const bool ok = x >= 0 && x < N0;
            const T v0 = ok ? r0p[x] : T(0);
            const T v1 = ok ? r1p[x] : T(0);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const int tt = t - h;
              if (tt < 0 || tt > 28) continue;
              if (sizeof(T) == 4) {
                if (tt == 14) continue;
                const T d0 = v0 - s0[h];
#pragma unroll
                for (int a1 = 0; a1 < 2; ++a1)
                  acc[a1][h] += Kt<T>(a1, 0, tt) * d0 + Kt<T>(a1, 1, tt) * v1;
              } else {
#pragma unroll
                for (int a1 = 0; a1 < 2; ++a1)
                  acc[a1][h] += Kt<T>(a1, 0, tt) * v0 + Kt<T>(a1, 1, tt) * v1;
              }
            }
          }
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int a1 = 0; a1 < 2; ++a1) {
              if (sizeof(T) == 4)
                kin[a1 + 2 * a2][h] += (T)(fac * ((double)acc[a1][h] + fKD64[a1] * (double)s0[h] +
                                                  fK64[a1][1][14] * (double)s1[h]));
              else
                kin[a1 + 2 * a2][h] += (T)(fac * (double)acc[a1][h]);
            }
        }
      }
      // y part (columns inside the input box): inputs y = iy - 14 .. iy + 14
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int ix = ix0 + h;
        if (ix < 0 || ix >= N0) continue;
        const bool iny = iy >= 0 && iy < N1;
#pragma unroll
        for (int a1 = 0; a1 < 2; ++a1) {
          const T* c0p = Cin + (a1 * nyi - yi0) * N0 + ix;         // a2 = 0 input
          const T* c1p = Cin + ((a1 + 2) * nyi - yi0) * N0 + ix;   // a2 = 1 input
          const T s0 = iny ? c0p[iy * N0] : T(0);
          const T s1 = iny ? c1p[iy * N0] : T(0);
          T acc[2] = {T(0), T(0)};   // [a2]
#pragma unroll
          for (int t = 0; t < 29; ++t) {
            const int y = iy - 14 + t;
            const bool ok = y >= 0 && y < N1;
            const T v0 = ok ? c0p[y * N0] : T(0);
            const T v1 = ok ? c1p[y * N0] : T(0);
            if (sizeof(T) == 4) {
              if (t == 14) continue;
              const T d0 = v0 - s0;
#pragma unroll
              for (int a2 = 0; a2 < 2; ++a2) acc[a2] += Kt<T>(a2, 0, t) * d0 + Kt<T>(a2, 1, t) * v1;
            } else {
#pragma unroll
              for (int a2 = 0; a2 < 2; ++a2) acc[a2] += Kt<T>(a2, 0, t) * v0 + Kt<T>(a2, 1, t) * v1;
            }
          }
#pragma unroll
          for (int a2 = 0; a2 < 2; ++a2) {
            if (sizeof(T) == 4)
              kin[a1 + 2 * a2][h] += (T)(fac * ((double)acc[a2] + fKD64[a2] * (double)s0 +
                                                fK64[a2][1][14] * (double)s1));
            else
              kin[a1 + 2 * a2][h] += (T)(fac * (double)acc[a2]);
          }
        }
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int xo = xo0 + h;
      if (xo >= O0) continue;
      const int ix = xo - e;
      const bool inbox = kin_on && ix >= 0 && ix < N0 && iy >= 0 && iy < N1;
      const int gx = sf.lo[0] - e + xo;
#pragma unroll
      for (int c4 = 0; c4 < 4; ++c4) {
        const int c = c4 + 4 * a3;
        T k = kin[c4][h];
        if (inbox) {
          // z part, computed by k_kin_zcol for every output plane
          k += ws[w.oz + ((int64_t)c * O2 + zp) * plane + (int64_t)iy * N0 + ix];
          if (zin) kacc += (double)Cin[(c4 * nyi + (iy - yi0)) * N0 + ix] * (double)k;
        }
        const T v = val[c4][h] + k;
        // compress: the output pattern row (yo, zp) of component c
        const int pat = c == 0 ? 2 : 3;
        const int64_t r = (int64_t)zp * O1 + yo;
        const int32_t s0 = rt[sf.rt[pat] + r], s1 = rt[sf.rt[pat] + r + 1];
        for (int qq = s0; qq < s1; ++qq) {
          const wvl_seg g = seg[qq];
          if (gx >= g.i1s && gx <= g.i1e) {
            const int64_t kk = g.off + (gx - g.i1s);
            const int64_t o =
                c == 0 ? sf.cout + kk : sf.cout + sf.on_c + (int64_t)(c - 1) * sf.on_f + kk;
            out[o] = accumulate ? out[o] + v : v;
            break;
          }
        }
      }
    }
  }
  const double b = block_sum_any(kacc);
  if (tid == 0) kpart[w.kpart + blockIdx.x] = b;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

int launch_fwd_plane(int f64, void* stream, const SfDev* sf, const wvl_seg* seg,
                     const int32_t* rt, const void* psi, const SfWork* wk, int sf0, int nsf,
                     int gridx, int tile_rows, size_t lds, void* ws, int up_on) {
  if (nsf == 0 || gridx == 0) return 0;
  const dim3 g((unsigned)gridx, (unsigned)nsf);
  if (f64)
    hipLaunchKernelGGL(k_fwd_plane<double>, g, dim3(256), lds, (hipStream_t)stream, sf, seg, rt,
                       (const double*)psi, wk, sf0, (double*)ws, tile_rows, up_on);
  else
    hipLaunchKernelGGL(k_fwd_plane<float>, g, dim3(256), lds, (hipStream_t)stream, sf, seg, rt,
                       (const float*)psi, wk, sf0, (float*)ws, tile_rows, up_on);
  return (int)hipGetLastError();
}

int launch_pot_column(int f64, void* stream, const SfDev* sf, const SfWork* wk, int sf0, int nsf,
                      int gridx, void* ws, const void* pot, int nf1, int nf2, double* epart) {
  if (nsf == 0 || gridx == 0) return 0;
  const dim3 g((unsigned)gridx, (unsigned)nsf);
  if (f64)
    hipLaunchKernelGGL(k_pot_column<double>, g, dim3(256), 0, (hipStream_t)stream, sf, wk, sf0,
                       (double*)ws, (const double*)pot, nf1, nf2, epart);
  else
    hipLaunchKernelGGL(k_pot_column<float>, g, dim3(256), 0, (hipStream_t)stream, sf, wk, sf0,
                       (float*)ws, (const float*)pot, nf1, nf2, epart);
  return (int)hipGetLastError();
}

int launch_kin_zcol(int f64, void* stream, const SfDev* sf, const SfWork* wk, int sf0, int nsf,
                    int gridx, void* ws, double fac) {
  if (nsf == 0 || gridx == 0) return 0;
  const dim3 g((unsigned)gridx, (unsigned)nsf);
  if (f64)
    hipLaunchKernelGGL(k_kin_zcol<double>, g, dim3(256), 0, (hipStream_t)stream, sf, wk, sf0,
                       (double*)ws, fac);
  else
    hipLaunchKernelGGL(k_kin_zcol<float>, g, dim3(256), 0, (hipStream_t)stream, sf, wk, sf0,
                       (float*)ws, fac);
  return (int)hipGetLastError();
}

int launch_back_plane(int f64, void* stream, const SfDev* sf, const wvl_seg* seg,
                      const int32_t* rt, const SfWork* wk, int sf0, int nsf, int gridx,
                      int tile_rows, size_t lds, const void* ws, void* out, double fac, int pot_on,
                      int kin_on, int accumulate, double* kpart) {
  if (nsf == 0 || gridx == 0) return 0;
  const dim3 g((unsigned)gridx, (unsigned)nsf);
  if (f64)
    hipLaunchKernelGGL(k_back_plane<double>, g, dim3(back_threads<double>()), lds, (hipStream_t)stream, sf, seg, rt,
                       wk, sf0, (const double*)ws, (double*)out, tile_rows, fac, pot_on, kin_on,
                       accumulate, kpart);
  else
    hipLaunchKernelGGL(k_back_plane<float>, g, dim3(back_threads<float>()), lds, (hipStream_t)stream, sf, seg, rt,
                       wk, sf0, (const float*)ws, (float*)out, tile_rows, fac, pot_on, kin_on,
                       accumulate, kpart);
  return (int)hipGetLastError();
}

}  // namespace wvl

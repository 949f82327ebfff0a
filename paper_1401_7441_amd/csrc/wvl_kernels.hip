// HIP kernels for gfx950 (MI355X): the dense-box <-> compressed copies of the
// standalone uncompress / compress entry points, fixed-order energy sums, and
// the sparse overlap / Hamiltonian matrix elements.  The local Hamiltonian
// itself runs in the fused kernels of wvl_fused.hip.
#include <hip/hip_runtime.h>

#include "wvl_internal.h"

namespace wvl {

constexpr int TPB = 256;

// deterministic block sum of one double per thread: a fixed shuffle tree in
// each 64-lane wave, then the wave sums in order
__device__ double block_sum(double v) {
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

// ---------------------------------------------------------------------------
// compressed <-> dense
// ---------------------------------------------------------------------------

// Uncompress: thread per dense point of the input box [8][n2][n1][n0].
template <typename T>
__global__ __launch_bounds__(TPB) void k_gather(const SfDev* __restrict__ sfs,
                                                const wvl_seg* __restrict__ seg,
                                                const int32_t* __restrict__ rt,
                                                const T* __restrict__ psi, T* __restrict__ dst,
                                                int sf0) {
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
      v = c == 0 ? psi[sf.cin + k] : psi[sf.cin + sf.n_c + 7 * k + (c - 1)];
      break;
    }
  }
  dst[sf.box_in + idx] = v;
}

// Compress onto the output pattern: thread per dense point of the output box.
template <typename T>
__global__ __launch_bounds__(TPB) void k_scatter(const SfDev* __restrict__ sfs,
                                                 const wvl_seg* __restrict__ seg,
                                                 const int32_t* __restrict__ rt,
                                                 const T* __restrict__ src, T* __restrict__ out,
                                                 int sf0) {
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
      const int64_t o = c == 0 ? sf.cout + k : sf.cout + sf.on_c + 7 * k + (c - 1);
      out[o] = src[sf.box_out + idx];
      return;
    }
  }
}

// one block per function: fixed-order sum of its partials
__global__ __launch_bounds__(TPB) void k_finalize(const SfWork* __restrict__ wk, int sf0,
                                                  const double* __restrict__ parts, int which,
                                                  int nblk, double* __restrict__ out) {
  const int s = blockIdx.x;
  const int64_t off = which == 0 ? wk[s].epart : wk[s].kpart;
  if (which == 1) nblk = (int)wk[s].nkpart;   // only the function's own slots
  double v = 0.0;
  for (int i = threadIdx.x; i < nblk; i += TPB) v += parts[off + i];
  const double b = block_sum(v);
  if (threadIdx.x == 0) out[wk[s].id] = b;
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

// one wavefront per nonzero (a, b), in two phases per batch of 64 rows of the
// box where both patterns may meet.  Phase 1: lane r resolves row r (row
// tables, segment lists) to the first overlapping run of each kind (scaling /
// wavelet) and keeps it in LDS; further runs of the same row, which sphere
// patterns never produce, are summed by that lane directly.  Phase 2: four
// 16-lane groups stream the kept runs with contiguous loads.  Every lane's
// partial sum and the final shuffle tree have an order fixed by the pair.
// mirror (may be NULL): for the pair at processing position s, the CSR
// position that receives the same value as well (the transposed pair of a
// symmetric matrix), or -1.
template <typename T>
__device__ __forceinline__ double run_dot(const T* __restrict__ pa, const T* __restrict__ pk,
                                          int n) {
  double acc = 0.0;
  for (int x = 0; x < n; ++x) acc += (double)pa[x] * (double)pk[x];
  return acc;
}

template <typename T>
__global__ __launch_bounds__(64) void k_sparse_values(const SfDev* __restrict__ sfs,
                                                      const wvl_seg* __restrict__ seg,
                                                      const int32_t* __restrict__ rt,
                                                      const RowRun* __restrict__ rr, int ket_out,
                                                      const T* __restrict__ bra,
                                                      const T* __restrict__ ket,
                                                      const int32_t* __restrict__ rowi,
                                                      const int32_t* __restrict__ coli,
                                                      const int32_t* __restrict__ order,
                                                      const int32_t* __restrict__ mirror,
                                                      int64_t nnz, double* __restrict__ val) {
  __shared__ int64_t ea[2][64], eb[2][64];   // run start offsets (bra, ket) per kind
  __shared__ int32_t el[2][64];              // run lengths (0: none)
  // Workgroups are dealt to the 8 XCDs in turn: block b runs on XCD b % 8.
  // Each XCD walks its own contiguous eighth of the processing order, so the
  // pairs resident on one XCD share rows (and, rows being in spatial order,
  // most of their kets) in that XCD's L2.
  const int64_t per = (nnz + 7) / 8;
  const int64_t s = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (s >= nnz) return;
  const int64_t k = order[s];
  const int lane = threadIdx.x;
  const int grp = lane >> 4, gl = lane & 15;
  const SfDev& A = sfs[rowi[k]];
  const SfDev& B = sfs[coli[k]];
  const int32_t* bb = ket_out ? B.bb_out : B.bb_in;
  const int y0 = max(A.bb_in[2], bb[2]), y1 = min(A.bb_in[3], bb[3]);
  const int z0 = max(A.bb_in[4], bb[4]), z1 = min(A.bb_in[5], bb[5]);
  const PatBox pb = pat_box(B, ket_out);
  const int pc = ket_out ? 2 : 0, pf = ket_out ? 3 : 1;
  const int64_t bc = ket_out ? B.cout : B.cin;
  const int64_t bnc = ket_out ? B.on_c : B.n_c;
  const int ny = y1 - y0 + 1;
  const int nrows = (y1 >= y0 && z1 >= z0) ? ny * (z1 - z0 + 1) : 0;
  double acc = 0.0;
  for (int r0 = 0; r0 < nrows; r0 += 64) {
    // phase 1
    const int r = r0 + lane;
#pragma unroll
    for (int fine = 0; fine < 2; ++fine) {
      el[fine][lane] = 0;
      if (r < nrows) {
        const int y = y0 + r % ny, z = z0 + r / ny;
        const int64_t ra = (int64_t)(z - A.lo[2]) * A.n[1] + (y - A.lo[1]);
        const int64_t rb = (int64_t)(z - pb.oz) * pb.by + (y - pb.oy);
        const int pB = fine ? pf : pc;
        // compact row runs: one 8-byte record per row and side
        const RowRun wa = rr[A.rr[fine] + ra], wb = rr[B.rr[pB] + rb];
        if (wa.len == 0 || wb.len == 0) continue;
        if (wa.len != kMultiRun && wb.len != kMultiRun) {
          const int x0 = max((int)wa.x0, (int)wb.x0);
          const int x1 = min((int)wa.x0 + wa.len, (int)wb.x0 + wb.len) - 1;
          if (x0 <= x1) {
            // fine points hold their seven wavelets contiguously
            const int sc = fine ? 7 : 1;
            ea[fine][lane] = A.cin + (fine ? A.n_c : 0) + sc * (wa.off + (x0 - wa.x0));
            eb[fine][lane] = bc + (fine ? bnc : 0) + sc * (wb.off + (x0 - wb.x0));
            el[fine][lane] = sc * (x1 - x0 + 1);
          }
          continue;
        }
        // a row with several runs on either side: merge the segment lists
        int qa = rt[A.rt[fine] + ra];
        const int qa1 = rt[A.rt[fine] + ra + 1];
        int qb = rt[B.rt[pB] + rb];
        const int qb1 = rt[B.rt[pB] + rb + 1];
        bool first = true;
        while (qa < qa1 && qb < qb1) {
          const wvl_seg sa = seg[qa], sb = seg[qb];
          const int x0 = max(sa.i1s, sb.i1s), x1 = min(sa.i1e, sb.i1e);
          if (x0 <= x1) {
            const int sc = fine ? 7 : 1;
            const int64_t oa = A.cin + (fine ? A.n_c : 0) + sc * (sa.off + (x0 - sa.i1s));
            const int64_t ob = bc + (fine ? bnc : 0) + sc * (sb.off + (x0 - sb.i1s));
            if (first) {
              ea[fine][lane] = oa;
              eb[fine][lane] = ob;
              el[fine][lane] = sc * (x1 - x0 + 1);
              first = false;
            } else {
              acc += run_dot<T>(bra + oa, ket + ob, sc * (x1 - x0 + 1));
            }
          }
          if (sa.i1e < sb.i1e) ++qa; else ++qb;
        }
      }
    }
    __syncthreads();
    // phase 2
    const int nb = min(64, nrows - r0);
    // each run (coarse, or fine with the seven wavelets of its points) is
    // one contiguous stretch on both sides
    for (int q = grp; q < nb; q += 4) {
#pragma unroll
      for (int fine = 0; fine < 2; ++fine) {
        const int l = el[fine][q];
        const T* pa = bra + ea[fine][q];
        const T* pk = ket + eb[fine][q];
        // FP64: four positions of the lane loaded before they are added, in
        // the order x, x + 16, x + 32, x + 48 (the order of the plain loop);
        // FP32 runs faster with one (fewer requests in flight per CU)
        constexpr int U = sizeof(T) == 8 ? 4 : 1;
        for (int x = gl; x < l; x += 16 * U) {
          T va[U], vk[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const bool in = x + 16 * u < l;
            va[u] = in ? pa[x + 16 * u] : T(0);
            vk[u] = in ? pk[x + 16 * u] : T(0);
          }
#pragma unroll
          for (int u = 0; u < U; ++u)
            if (x + 16 * u < l) acc += (double)va[u] * (double)vk[u];
        }
      }
    }
    __syncthreads();
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (lane == 0) {
    val[k] = acc;
    if (mirror != nullptr && mirror[s] >= 0) val[mirror[s]] = acc;
  }
}

// ---------------------------------------------------------------------------
// density rho(r) = sum_ab phi_a(r) K^ab phi_b(r) on the fine grid
// ---------------------------------------------------------------------------
// One workgroup of eight waves per tile of 16 x 4 x 1 fine-grid points (lane =
// point in every wave).  The functions whose fine box meets the tile (its
// cover, increasing index) are taken in chunks of C: the values phi_a(r) of
// an i-chunk and a j-chunk are staged in LDS (0 outside a box).  Wave w takes
// the functions a = i-chunk entries w, w + 8, ...: it scans the kernel row a
// for the columns b in the j-chunk (an LDS hash of the chunk), kept in row
// order, and accumulates
//   rho_w(r) += phi_a(r) sum_{b in row a, j-chunk} K[q] phi_b(r);
// rho(r) is then rho_0 + rho_1 + ... + rho_7.  The order of every sum is
// fixed by the tile's cover and K.  Columns outside [0, nsf) never match;
// positions outside [0, knnz) are skipped.
constexpr int kDensWaves = 8;

// orders a wave's LDS writes before its other lanes' reads (and the reads
// before the next writes)
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int LNB>
__device__ __forceinline__ int dens_bucket(int b) {
  return (int)(((uint32_t)b * 2654435761u) >> (32 - LNB));
}

// position of function b in a bucket of (function << 8 | position), or -1
__device__ __forceinline__ int dens_match(uint4 v, int b) {
  const uint32_t ub = (uint32_t)b;
  int p = -1;
  if ((v.x >> 8) == ub) p = (int)(v.x & 255u);
  if ((v.y >> 8) == ub) p = (int)(v.y & 255u);
  if ((v.z >> 8) == ub) p = (int)(v.z & 255u);
  if ((v.w >> 8) == ub) p = (int)(v.w & 255u);
  return p;
}

// ONE: every tile of the launch has at most C functions (one chunk; in FP32
// kDensChunkOne), and the second chunk buffer is left out, the cover list and
// the hash sized to one chunk (more workgroups fit in a CU's LDS)
template <typename T, bool ONE>
__global__ __launch_bounds__(64 * kDensWaves) void k_dens_tile(
    const SfDev* __restrict__ sfs, const int64_t* __restrict__ foff, const T* __restrict__ fine,
    const int64_t* __restrict__ krow, const int32_t* __restrict__ kcol,
    const double* __restrict__ kval, int64_t knnz, const int64_t* __restrict__ cptr,
    const int32_t* __restrict__ csf, const int32_t* __restrict__ tord, int64_t tbase, int tx,
    int ty, int g0, int g1, int g2, T* __restrict__ rho) {
  // functions per staged chunk
  constexpr int C = ONE && sizeof(T) == 4 ? kDensChunkOne : kDensChunk[sizeof(T) == 4 ? 0 : 1];
  constexpr int LNB = ONE ? 7 : 8;   // log2 of the hash buckets
  constexpr int NBK = 1 << LNB;
  __shared__ T vi[C * 64], vj[ONE ? 1 : C * 64];
  __shared__ int32_t cov[ONE ? C : kDensMaxCover];
  __shared__ int32_t lj[kDensWaves][64];
  __shared__ double lk[kDensWaves][64];
  // the j-chunk's functions by index: NBK buckets of four slots
  // (function << 8 | position in the chunk)
  __shared__ uint4 hb[NBK];
  uint32_t* hslot = reinterpret_cast<uint32_t*>(hb);
  double (*red)[64] = lk;   // the final reduction reuses lk
  static_assert(C <= 256 && 4 * NBK >= 2 * C, "chunk positions need 8 bits, the hash room");
  const int tile = tord[tbase + blockIdx.x];
  const int ix = tile % tx, iy = (tile / tx) % ty, iz = tile / (tx * ty);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int gx = ix * kDensTile[0] + (lane & 15);
  const int gy = iy * kDensTile[1] + (lane >> 4);
  const int gz = iz;
  const bool inside = gx < g0 && gy < g1 && gz < g2;
  const int64_t c0 = cptr[tile];
  const int m = (int)(cptr[tile + 1] - c0);
  for (int i = tid; i < m; i += 64 * kDensWaves) cov[i] = csf[c0 + i];
  // phi_a at this lane's point, 0 outside a's fine box
  auto value = [&](int a) -> T {
    const SfDev& A = sfs[a];
    const int px = gx - 2 * A.lo[0], py = gy - 2 * A.lo[1], pz = gz - 2 * A.lo[2];
    const int R0 = 2 * A.n[0] + 29, R1 = 2 * A.n[1] + 29, R2 = 2 * A.n[2] + 29;
    if (!inside || px < 0 || px >= R0 || py < 0 || py >= R1 || pz < 0 || pz >= R2) return T(0);
    return fine[foff[a] + ((int64_t)pz * R1 + py) * R0 + px];
  };
  double acc = 0.0;
  __syncthreads();
  for (int ic = 0; ic < m; ic += C) {
    const int ni = min(C, m - ic);
    for (int i = wave; i < ni; i += kDensWaves) vi[i * 64 + lane] = value(cov[ic + i]);
    for (int jc = 0; jc < m; jc += C) {
      const int nj = min(C, m - jc);
      const T* vb = vi;
      if (!ONE && jc != ic) {
        for (int j = wave; j < nj; j += kDensWaves) vj[j * 64 + lane] = value(cov[jc + j]);
        vb = vj;
      }
      for (int h = tid; h < 4 * NBK; h += 64 * kDensWaves) hslot[h] = 0xFFFFFFFFu;
      __syncthreads();
      // 4 NBK slots > nj: every insertion finds a free slot, every lookup a
      // bucket that is not full
      if (tid < nj) {
        const int b = cov[jc + tid];
        const uint32_t key = ((uint32_t)b << 8) | (uint32_t)tid;
        for (int bk = dens_bucket<LNB>(b);; bk = (bk + 1) & (NBK - 1)) {
          int c = 0;
          while (c < 4 && atomicCAS(&hslot[4 * bk + c], 0xFFFFFFFFu, key) != 0xFFFFFFFFu) ++c;
          if (c < 4) break;
        }
      }
      __syncthreads();
      const int blo = cov[jc], bhi = cov[jc + nj - 1];
      // the wave's rows i = wave, wave + 8, ..; the next row's bounds and
      // the next 64 kernel entries are loaded while the current ones are
      // used (the sums keep their order)
      int i = wave;
      int64_t q0 = 0, q1 = 0;
      if (i < ni) {
        const int a = cov[ic + i];
        q0 = max((int64_t)0, krow[a]);
        q1 = min(knnz, krow[a + 1]);
      }
      while (i < ni) {
        const int inx = i + kDensWaves;
        int64_t n0 = 0, n1 = 0;
        if (inx < ni) {
          const int an = cov[ic + inx];
          n0 = krow[an];
          n1 = krow[an + 1];
        }
        double u = 0.0;
        int bn = -1;
        double kn = 0.0;
        if (q0 + lane < q1) {
          bn = kcol[q0 + lane];
          kn = kval[q0 + lane];
        }
        for (int64_t qq = q0; qq < q1; qq += 64) {
          const int b = bn;
          const double kb = kn;
          bn = -1;
          kn = 0.0;
          if (qq + 64 + lane < q1) {
            bn = kcol[qq + 64 + lane];
            kn = kval[qq + 64 + lane];
          }
          int j = -1;
          double kq = 0.0;
          if (b >= blo && b <= bhi) {   // b's position in the j-chunk, if any
            int bk = dens_bucket<LNB>(b);
            uint4 v = hb[bk];
            int p = dens_match(v, b);
            while (p < 0 && v.w != 0xFFFFFFFFu) {
              bk = (bk + 1) & (NBK - 1);
              v = hb[bk];
              p = dens_match(v, b);
            }
            if (p >= 0) {
              j = p;
              kq = kb;
            }
          }
          const unsigned long long hit = __ballot(j >= 0);
          if (j >= 0) {
            const int pos = __popcll(hit & ((1ull << lane) - 1ull));
            lj[wave][pos] = j;
            lk[wave][pos] = kq;
          }
          wave_sync();
          const int cnt = __popcll(hit);
#pragma unroll 4
          for (int t = 0; t < cnt; ++t) u += lk[wave][t] * (double)vb[lj[wave][t] * 64 + lane];
          wave_sync();
        }
        acc += (double)vi[i * 64 + lane] * u;
        i = inx;
        q0 = max((int64_t)0, n0);
        q1 = min(knnz, n1);
      }
      __syncthreads();   // vi / vj, the hash and lk no longer read
    }
  }
  red[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && inside) {
    double r = red[0][lane];
    for (int w = 1; w < kDensWaves; ++w) r += red[w][lane];
    rho[((int64_t)gz * g1 + gy) * g0 + gx] = (T)r;
  }
}

// ---------------------------------------------------------------------------
// Fermi operator expansion: matrices on one symmetric pattern P (CSR, sorted
// columns, diagonal present), values in double
// ---------------------------------------------------------------------------

// C = alpha (A B)|_P + beta D, one workgroup of W waves per row i of P,
// rows taken in the order `rows` gives (longest work first).  Row i's
// columns go into an LDS hash table of 2^lognb buckets of four 32-bit slots,
// each slot (column << 10 | position in the row); a bucket fills from its
// first slot, and a full one spills into the next.  Wave w takes the k of
// row i with index t = w, w + W, .. in increasing order; its lanes walk row
// k of B in parts of 256 / NH entries, NH parts a step, and add A_ik B_kj to
// the wave's accumulator of that part's slot when j is in row i.  The next
// step's entries of B are loaded while the current ones are added.  The
// accumulators are summed in (wave, slot) order at the end, so every entry's
// sum has a fixed order.  D may be NULL
// (beta ignored).  Needs columns below 2^21 and rows of at most 1024
// entries; LDS: W NH + 2 doubles per row entry (maxdeg) and 16 bytes per
// bucket.
constexpr uint32_t kFoeEmpty = 0xFFFFFFFFu;

__device__ __forceinline__ int foe_bucket(int j, int lognb) {
  return (int)(((uint32_t)j * 2654435761u) >> (32 - lognb));
}

// position of column j in a bucket, or -1
__device__ __forceinline__ int foe_match(uint4 v, int j) {
  const uint32_t uj = (uint32_t)j;
  int p = -1;
  if ((v.x >> 10) == uj) p = (int)(v.x & 1023u);
  if ((v.y >> 10) == uj) p = (int)(v.y & 1023u);
  if ((v.z >> 10) == uj) p = (int)(v.z & 1023u);
  if ((v.w >> 10) == uj) p = (int)(v.w & 1023u);
  return p;
}

template <int W, int NH>
__global__ __launch_bounds__(64 * W) void k_foe_mm(
    const int32_t* __restrict__ rows, const int64_t* __restrict__ rowptr,
    const int32_t* __restrict__ col, double alpha,
    const double* __restrict__ A, const double* __restrict__ B, double beta,
    const double* __restrict__ D, double* __restrict__ C, int lognb, int maxdeg) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* acc = reinterpret_cast<double*>(smem_raw);   // [W][NH][maxdeg]
  double* av = acc + (size_t)W * NH * maxdeg;           // A_ik, [maxdeg]
  int* kst = reinterpret_cast<int*>(av + maxdeg);       // start of row k in B
  int* kdg = kst + maxdeg;                              // length of row k
  uint4* bucket = reinterpret_cast<uint4*>(kdg + maxdeg);   // [nb]
  uint32_t* slot = reinterpret_cast<uint32_t*>(bucket);
  constexpr int nt = 64 * W;
  constexpr int QW = 256 / NH;   // entries of a row k per part
  constexpr int UH = 4 / NH;     // 64-lane slots per part
  const int nb = 1 << lognb;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int i = rows[blockIdx.x];
  const int64_t r0 = rowptr[i];
  const int deg = (int)(rowptr[i + 1] - r0);
  for (int h = tid; h < 4 * nb; h += nt) slot[h] = kFoeEmpty;
  for (int p = tid; p < deg; p += nt) {
    const int k = col[r0 + p];
    const int64_t k0 = rowptr[k];
    kst[p] = (int)k0;
    kdg[p] = (int)(rowptr[k + 1] - k0);
    av[p] = A[r0 + p];
#pragma unroll
    for (int w = 0; w < W * NH; ++w) acc[(size_t)w * maxdeg + p] = 0.0;
  }
  __syncthreads();
  // 4 nb slots > deg: every insertion finds a free slot, every lookup a
  // bucket that is not full
  for (int p = tid; p < deg; p += nt) {
    const int j = col[r0 + p];
    const uint32_t key = ((uint32_t)j << 10) | (uint32_t)p;
    for (int b = foe_bucket(j, lognb);; b = (b + 1) & (nb - 1)) {
      int c = 0;
      while (c < 4 && atomicCAS(&slot[4 * b + c], kFoeEmpty, key) != kFoeEmpty) ++c;
      if (c < 4) break;
    }
  }
  __syncthreads();
  double* my = acc + (size_t)wave * NH * maxdeg;   // the wave's NH accumulators
  // the wave's parts in order: (t, q0) for t = wave, wave + W, .. and
  // q0 = 0, QW, .. below the length of row k; a step takes NH parts, part h
  // on the 64-lane slots h UH .. h UH + UH - 1 and into accumulator h
  int qt = wave, qq = 0;
  auto next = [&](int& k0, int& kd, int& q0, double& a) {
    if (qt >= deg) {
      k0 = 0;
      kd = 0;
      q0 = 0;
      a = 0.0;
      return;
    }
    k0 = kst[qt];
    kd = kdg[qt];
    q0 = qq;
    a = av[qt];
    qq += QW;
    if (qq >= kd) {
      qt += W;
      qq = 0;
    }
  };
  // column -1: none
  auto load = [&](const int (&k0)[NH], const int (&kd)[NH], const int (&q0)[NH], int (&jj)[4],
                  double (&bb)[4]) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int h = u / UH;
      const int q = q0[h] + 64 * (u % UH) + lane;
      jj[u] = q < kd[h] ? col[k0[h] + q] : -1;
      bb[u] = q < kd[h] ? B[k0[h] + q] : 0.0;
    }
  };
  // the four lookups, the four accumulator reads and the four writes are
  // issued together: within a part the columns (one row of B) are distinct,
  // and parts add into accumulators of their own
  auto add = [&](const int (&jj)[4], const double (&bb)[4], const double (&a)[NH]) {
    int b[4];
    uint4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      b[u] = foe_bucket(jj[u], lognb);
      v[u] = bucket[b[u]];
    }
    int p[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      p[u] = foe_match(v[u], jj[u]);
      while (p[u] < 0 && jj[u] >= 0 && v[u].w != kFoeEmpty) {
        b[u] = (b[u] + 1) & (nb - 1);
        v[u] = bucket[b[u]];
        p[u] = foe_match(v[u], jj[u]);
      }
    }
    double o[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) o[u] = my[(size_t)(u / UH) * maxdeg + (p[u] >= 0 ? p[u] : 0)];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (p[u] >= 0) my[(size_t)(u / UH) * maxdeg + p[u]] = o[u] + a[u / UH] * bb[u];
  };
  int steps = 0;
  for (int t = wave; t < deg; t += W) steps += (kdg[t] + QW - 1) / QW;
  steps = (steps + NH - 1) / NH;
  int k0[NH], kd[NH], q0[NH];
  double a[NH];
#pragma unroll
  for (int h = 0; h < NH; ++h) next(k0[h], kd[h], q0[h], a[h]);
  int jj[4];
  double bb[4];
  load(k0, kd, q0, jj, bb);
  // the next step's entries of B load while the current ones are added
  for (; steps > 0; --steps) {
    double an[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) next(k0[h], kd[h], q0[h], an[h]);
    int jn[4];
    double bn[4];
    load(k0, kd, q0, jn, bn);
    add(jj, bb, a);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      jj[u] = jn[u];
      bb[u] = bn[u];
    }
#pragma unroll
    for (int h = 0; h < NH; ++h) a[h] = an[h];
  }
  __syncthreads();
  for (int p = tid; p < deg; p += nt) {
    double v = acc[p];
#pragma unroll
    for (int w = 1; w < W * NH; ++w) v += acc[(size_t)w * maxdeg + p];
    C[r0 + p] = D ? alpha * v + beta * D[r0 + p] : alpha * v;
  }
}

// v = a x + b y (+ d on the diagonal), each term only when present; the one
// expression both k_foe_axpby and k_foe_series evaluate
__device__ __forceinline__ double foe_lin(bool hx, double a, double x, bool hy, double b,
                                          double y, bool diag, double d) {
  double v = 0.0;
  if (hx) v += a * x;
  if (hy) v += b * y;
  if (diag) v += d;
  return v;
}

// elementwise on P: out = a X + b Y (+ d on the diagonal when row != NULL)
__global__ __launch_bounds__(TPB) void k_foe_axpby(int64_t nnz, double a,
                                                   const double* __restrict__ X, double b,
                                                   const double* __restrict__ Y,
                                                   const int32_t* __restrict__ row,
                                                   const int32_t* __restrict__ col, double d,
                                                   double* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (p >= nnz) return;
  out[p] = foe_lin(X != nullptr, a, X ? X[p] : 0.0, Y != nullptr, b, Y ? Y[p] : 0.0,
                   row && row[p] == col[p], d);
}

// the Chebyshev series on P from the kept matrices T^0 .. T^npl (T^j at
// T + j nnz): out = c_0 / 2 I + c_1 T^1, then out += c_j T^j for j = 2 ..
// npl, term by term as k_foe_axpby adds them when the matrices are
// recomputed (same values, bit for bit)
__global__ __launch_bounds__(TPB) void k_foe_series(int64_t nnz, int npl,
                                                    const double* __restrict__ c,
                                                    const double* __restrict__ T,
                                                    const int32_t* __restrict__ row,
                                                    const int32_t* __restrict__ col,
                                                    double* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (p >= nnz) return;
  const bool diag = row[p] == col[p];
  double v = foe_lin(true, c[1], T[nnz + p], false, 0.0, 0.0, diag, 0.5 * c[0]);
  for (int j = 2; j <= npl; ++j)
    v = foe_lin(true, 1.0, v, true, c[j], T[(int64_t)j * nnz + p], diag, 0.0);
  out[p] = v;
}

// symmetric part on P: out = (X + X^T) / 2
__global__ __launch_bounds__(TPB) void k_foe_sym(int64_t nnz, const int64_t* __restrict__ tpos,
                                                 const double* __restrict__ X,
                                                 double* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (p >= nnz) return;
  out[p] = 0.5 * (X[p] + X[tpos[p]]);
}

// out = values of X (on pattern Q) at the positions qpos of P's entries
__global__ __launch_bounds__(TPB) void k_foe_gather(int64_t nnz, const int64_t* __restrict__ qpos,
                                                    const double* __restrict__ X,
                                                    double* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (p >= nnz) return;
  out[p] = X[qpos[p]];
}

// one block: out[slot] = sum_p X[p] Y[p] over P, in a fixed order
// block b of nblk: part[b] = sum of X[p] Y[p] over its contiguous chunk of
// the entries; then one block: out[slot] = part[0] + .. + part[nblk - 1]
// (both sums in fixed orders)
__global__ __launch_bounds__(TPB) void k_foe_dot(int64_t nnz, int64_t chunk,
                                                 const double* __restrict__ X,
                                                 const double* __restrict__ Y,
                                                 double* __restrict__ part) {
  const int64_t p0 = (int64_t)blockIdx.x * chunk;
  const int64_t p1 = min(nnz, p0 + chunk);
  double v = 0.0;
  for (int64_t p = p0 + threadIdx.x; p < p1; p += TPB) v += X[p] * Y[p];
  const double s = block_sum(v);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(TPB) void k_foe_sum(int n, const double* __restrict__ part,
                                                 double* __restrict__ out, int slot) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += TPB) v += part[i];
  const double s = block_sum(v);
  if (threadIdx.x == 0) out[slot] = s;
}

// block b: out[slot + b] = trace of X + b stride, its diagonal entries at
// dpos[0..n), in a fixed order
__global__ __launch_bounds__(TPB) void k_foe_trace(int n, const int64_t* __restrict__ dpos,
                                                   const double* __restrict__ X, int64_t stride,
                                                   double* __restrict__ out, int slot) {
  const double* Xb = X + (int64_t)blockIdx.x * stride;
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += TPB) v += Xb[dpos[i]];
  const double s = block_sum(v);
  if (threadIdx.x == 0) out[slot + blockIdx.x] = s;
}

// Gershgorin discs of X: one wave per row i (four rows per block) sums
// r_i = sum_{j != i} |X_ij| over the lanes in a fixed tree and writes
// lo[i] = X_ii - r_i, hi[i] = X_ii + r_i
__global__ __launch_bounds__(TPB) void k_foe_gersh_rows(int nrow,
                                                        const int64_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ col,
                                                        const double* __restrict__ X,
                                                        double* __restrict__ lo,
                                                        double* __restrict__ hi) {
  const int i = blockIdx.x * (TPB / 64) + (int)(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= nrow) return;
  double dgl = 0.0, r = 0.0;
  for (int64_t q = rowptr[i] + lane; q < rowptr[i + 1]; q += 64) {
    if (col[q] == i)
      dgl = X[q];
    else
      r += fabs(X[q]);
  }
  for (int o = 32; o > 0; o >>= 1) {
    r += __shfl_xor(r, o, 64);
    dgl += __shfl_xor(dgl, o, 64);   // one lane holds the diagonal, the others 0
  }
  if (lane == 0) {
    lo[i] = dgl - r;
    hi[i] = dgl + r;
  }
}

// one block: out[0] = min_i lo[i], out[1] = max_i hi[i]
__global__ __launch_bounds__(TPB) void k_foe_gersh(int nrow, const double* __restrict__ lo,
                                                   const double* __restrict__ hi,
                                                   double* __restrict__ out) {
  __shared__ double sl[TPB], sh[TPB];
  double l = 1e300, h = -1e300;
  for (int i = threadIdx.x; i < nrow; i += TPB) {
    l = fmin(l, lo[i]);
    h = fmax(h, hi[i]);
  }
  sl[threadIdx.x] = l;
  sh[threadIdx.x] = h;
  __syncthreads();
  for (int s = TPB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sl[threadIdx.x] = fmin(sl[threadIdx.x], sl[threadIdx.x + s]);
      sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sl[0];
    out[1] = sh[0];
  }
}

// ---------------------------------------------------------------------------
// support-function update: psi <- psi - eta (P_L hpsi - H_aa psi)
// ---------------------------------------------------------------------------
// Block = 64 consecutive input segments of one function (coarse blocks, then
// fine).  Every input segment lies inside one maximal output segment (the
// input pattern is contained in the output pattern), so each segment maps
// affinely into H psi; the map is found once per segment and staged in LDS.
constexpr int kUpdSegs = 64;
// mode 0 (update):   psi <- psi - eta (P_L hpsi - H_aa psi)      (out = psi)
// mode 1 (restrict): out <- P_L hpsi - min(shift_a, 0) psi
template <typename T>
__global__ __launch_bounds__(256) void k_update(const SfDev* __restrict__ sfs,
                                                const wvl_seg* __restrict__ seg,
                                                const int32_t* __restrict__ rt, double eta,
                                                const T* __restrict__ hpsi,
                                                const int64_t* __restrict__ hrow,
                                                const int32_t* __restrict__ hcol,
                                                const double* __restrict__ hval,
                                                T* __restrict__ psi, int sf0, int mode,
                                                const double* __restrict__ shift,
                                                T* __restrict__ out) {
  __shared__ int s_in[kUpdSegs + 1];     // coefficient offset relative to the first segment
  __shared__ int64_t s_out[kUpdSegs];    // H psi index of the segment's first point
  __shared__ double s_diag;
  const int a = sf0 + blockIdx.y;
  const SfDev& sf = sfs[a];
  const int64_t nrows = (int64_t)sf.n[1] * sf.n[2];
  const int cb0 = rt[sf.rt[0]], ce0 = rt[sf.rt[0] + nrows];
  const int fb0 = rt[sf.rt[1]], fe0 = rt[sf.rt[1] + nrows];
  const int nbc = (ce0 - cb0 + kUpdSegs - 1) / kUpdSegs;
  const int nbf = (fe0 - fb0 + kUpdSegs - 1) / kUpdSegs;
  int bx = blockIdx.x;
  const bool fine = bx >= nbc;
  if (fine) bx -= nbc;
  if (bx >= (fine ? nbf : nbc)) return;   // uniform over the block
  const int sA = (fine ? fb0 : cb0) + bx * kUpdSegs;
  const int nseg = min(kUpdSegs, (fine ? fe0 : ce0) - sA);
  const int tid = threadIdx.x;
  const int64_t off0 = seg[sA].off;
  const PatBox ob = pat_box(sf, 1);
  if (tid < nseg) {
    const wvl_seg g = seg[sA + tid];
    s_in[tid] = (int)(g.off - off0);
    if (tid == nseg - 1) s_in[nseg] = (int)(g.off - off0) + (g.i1e - g.i1s + 1);
    const int64_t r = (int64_t)(g.i3 - ob.oz) * ob.by + (g.i2 - ob.oy);
    const int pat = fine ? 3 : 2;
    int64_t o = -1;
    for (int q = rt[sf.rt[pat] + r]; q < rt[sf.rt[pat] + r + 1]; ++q) {
      const wvl_seg h = seg[q];
      if (g.i1s >= h.i1s && g.i1s <= h.i1e) {
        o = h.off + (g.i1s - h.i1s);
        break;
      }
    }
    s_out[tid] = o;   // always found: the plan checks input inside output
  }
  if (tid == 0) {
    if (mode == 0) {  // H_aa: the diagonal entry of row a
      int64_t lo = hrow[a], hi = hrow[a + 1] - 1;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (hcol[mid] < a) lo = mid + 1; else hi = mid;
      }
      s_diag = hval[lo];
    } else {
      s_diag = shift ? fmin(shift[a], 0.0) : 0.0;
    }
  }
  __syncthreads();
  const int total = s_in[nseg];
  const double d = s_diag;
  const int cfirst = fine ? 1 : 0, clast = fine ? 7 : 0;
  for (int k = tid; k < total; k += 256) {
    int lo = 0, hi = nseg - 1;   // last segment with s_in <= k
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_in[mid] <= k) lo = mid; else hi = mid - 1;
    }
    if (s_out[lo] < 0) continue;   // not reached: the host checks input inside output
    const int64_t oi = s_out[lo] + (k - s_in[lo]);
    for (int c = cfirst; c <= clast; ++c) {
      const int64_t i = sf.cin + (c == 0 ? off0 + k : sf.n_c + 7 * (off0 + k) + (c - 1));
      const int64_t o = sf.cout + (c == 0 ? oi : sf.on_c + 7 * oi + (c - 1));
      const double x = (double)psi[i];
      if (mode == 0)
        psi[i] = (T)(x - eta * ((double)hpsi[o] - d * x));
      else
        out[i] = (T)((double)hpsi[o] - d * x);
    }
  }
}

// ---------------------------------------------------------------------------
// per-function vector algebra for the preconditioner (input layout: each
// function's coefficients are contiguous); one block per function, fixed
// summation order
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(TPB) void k_sf_dot(const SfDev* __restrict__ sfs,
                                                const T* __restrict__ a,
                                                const T* __restrict__ b, double* __restrict__ out,
                                                int sf0) {
  const SfDev& sf = sfs[sf0 + blockIdx.x];
  const int64_t n = sf.n_c + 7 * sf.n_f;
  double v = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += TPB) v += (double)a[sf.cin + i] * (double)b[sf.cin + i];
  const double r = block_sum(v);
  if (threadIdx.x == 0) out[sf0 + blockIdx.x] = r;
}

// one conjugate-gradient step after Ap and pAp = <p|Ap> are known:
//   al = rr / pAp (0 when pAp <= 0 or rr = 0);  x += al p;  r -= al Ap
template <typename T>
__global__ __launch_bounds__(TPB) void k_cg_xr(const SfDev* __restrict__ sfs,
                                               const double* __restrict__ rr,
                                               const double* __restrict__ pap,
                                               const T* __restrict__ p, const T* __restrict__ ap,
                                               T* __restrict__ x, T* __restrict__ r, int sf0) {
  const int a = sf0 + blockIdx.x;
  const SfDev& sf = sfs[a];
  const double al = (pap[a] > 0.0 && rr[a] > 0.0) ? rr[a] / pap[a] : 0.0;
  const int64_t n = sf.n_c + 7 * sf.n_f;
  for (int64_t i = threadIdx.x; i < n; i += TPB) {
    const int64_t k = sf.cin + i;
    x[k] = (T)((double)x[k] + al * (double)p[k]);
    r[k] = (T)((double)r[k] - al * (double)ap[k]);
  }
}

//   be = rr_new / rr (0 when rr = 0);  p = r + be p;  rr <- rr_new
template <typename T>
__global__ __launch_bounds__(TPB) void k_cg_p(const SfDev* __restrict__ sfs,
                                              double* __restrict__ rr,
                                              const double* __restrict__ rr_new,
                                              const T* __restrict__ r, T* __restrict__ p,
                                              int sf0) {
  const int a = sf0 + blockIdx.x;
  const SfDev& sf = sfs[a];
  const double be = rr[a] > 0.0 ? rr_new[a] / rr[a] : 0.0;
  const int64_t n = sf.n_c + 7 * sf.n_f;
  for (int64_t i = threadIdx.x; i < n; i += TPB) {
    const int64_t k = sf.cin + i;
    p[k] = (T)((double)r[k] + be * (double)p[k]);
  }
  __syncthreads();
  if (threadIdx.x == 0) rr[a] = rr_new[a];
}

// x = 0, r = p = -g over every function's coefficients
template <typename T>
__global__ __launch_bounds__(TPB) void k_cg_init(const SfDev* __restrict__ sfs,
                                                 const T* __restrict__ g, T* __restrict__ x,
                                                 T* __restrict__ r, T* __restrict__ p, int sf0) {
  const SfDev& sf = sfs[sf0 + blockIdx.x];
  const int64_t n = sf.n_c + 7 * sf.n_f;
  for (int64_t i = threadIdx.x; i < n; i += TPB) {
    const int64_t k = sf.cin + i;
    x[k] = T(0);
    r[k] = -g[k];
    p[k] = -g[k];
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// gradient: g_a = L^a [ sum_d A_ad H|phi_d> - sum_d M_ad |phi_d> ] over row a
// of the overlap pattern (Eq. (gradient), Sec. IV.A, localized as Sec. III.A)
// ---------------------------------------------------------------------------
// Block = function a (four waves), the neighbours d of row a staged in LDS
// (their box rows, row-table bases and coefficient offsets, A_ad and M_ad),
// kGradNb at a time.  Wave w takes the rows w, w + 4, ... of a's input box;
// for each segment of a row (the scaling coefficients of the coarse pattern,
// then the seven wavelets of each point of the fine pattern) lane j owns the
// elements j, j + 64, ... and sums, over the neighbours in CSR order, the
// values of H|phi_d> and |phi_d> at its point (0 where d's pattern lacks
// it), in double; each element of g_a is written once, by its owner.
constexpr int kGradNb = 256;

struct GradNb {
  int32_t in_y0, in_z0, in_by, in_nz;       // input box rows: origin, rows per plane, planes
  int32_t out_y0, out_z0, out_by, out_nz;   // output box rows
  int64_t rr_in[2], rr_out[2];              // RowRun bases (coarse, fine)
  int64_t rt_in[2], rt_out[2];              // row-table bases (coarse, fine)
  int64_t cin, cout, n_c, on_c;
  double a, m;
};

// index of global point gx in row r of a pattern (RowRun base rrb, row-table
// base rtb), or -1
__device__ __forceinline__ int64_t grad_find(const RowRun* __restrict__ rr,
                                             const int32_t* __restrict__ rt,
                                             const wvl_seg* __restrict__ seg, int64_t rrb,
                                             int64_t rtb, int64_t r, int gx) {
  const RowRun w = rr[rrb + r];
  if (w.len == 0) return -1;
  if (w.len != kMultiRun)
    return (gx >= (int)w.x0 && gx < (int)w.x0 + (int)w.len) ? (int64_t)w.off + gx - w.x0 : -1;
  for (int q = rt[rtb + r], q1 = rt[rtb + r + 1]; q < q1; ++q) {
    const wvl_seg g = seg[q];
    if (gx >= g.i1s && gx <= g.i1e) return g.off + (gx - g.i1s);
  }
  return -1;
}

template <typename T>
__global__ __launch_bounds__(256) void k_grad_rows(const SfDev* __restrict__ sfs,
                                                   const wvl_seg* __restrict__ seg,
                                                   const int32_t* __restrict__ rt,
                                                   const RowRun* __restrict__ rr,
                                                   const int64_t* __restrict__ rowptr,
                                                   const int32_t* __restrict__ col,
                                                   const double* __restrict__ av,
                                                   const double* __restrict__ mv,
                                                   const T* __restrict__ psi,
                                                   const T* __restrict__ hpsi, int sf0,
                                                   T* __restrict__ g) {
  __shared__ GradNb nb[kGradNb];
  const int a = sf0 + blockIdx.x;
  const SfDev& A = sfs[a];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int N1 = A.n[1], N2 = A.n[2];
  const int64_t nrows = (int64_t)N1 * N2;
  const int64_t q0 = rowptr[a], q1 = rowptr[a + 1];
  // neighbours in batches of kGradNb: each element's sum runs over the
  // batches in order, the first batch writing g and the next ones adding to
  // it (an element has the same owner, lane and wave, in every batch; rows of
  // more than kGradNb entries round once per batch)
  const int64_t nbatch = max((int64_t)1, (q1 - q0 + kGradNb - 1) / kGradNb);
  for (int64_t bi = 0; bi < nbatch; ++bi) {
    const int64_t b0 = q0 + bi * kGradNb;
    const int nn = (int)max((int64_t)0, min((int64_t)kGradNb, q1 - b0));
    __syncthreads();
    for (int t = threadIdx.x; t < nn; t += 256) {
      const int d = col[b0 + t];
      const SfDev& D = sfs[d];
      GradNb x;
      const int e = D.ext;
      x.in_y0 = D.lo[1]; x.in_z0 = D.lo[2]; x.in_by = D.n[1]; x.in_nz = D.n[2];
      x.out_y0 = D.lo[1] - e; x.out_z0 = D.lo[2] - e; x.out_by = D.n[1] + 2 * e;
      x.out_nz = D.n[2] + 2 * e;
      x.rr_in[0] = D.rr[0]; x.rr_in[1] = D.rr[1]; x.rr_out[0] = D.rr[2]; x.rr_out[1] = D.rr[3];
      x.rt_in[0] = D.rt[0]; x.rt_in[1] = D.rt[1]; x.rt_out[0] = D.rt[2]; x.rt_out[1] = D.rt[3];
      x.cin = D.cin; x.cout = D.cout; x.n_c = D.n_c; x.on_c = D.on_c;
      x.a = av[b0 + t];
      x.m = mv[b0 + t];
      nb[t] = x;
    }
    __syncthreads();
    for (int64_t r = wv; r < nrows; r += 4) {
      const int y = A.lo[1] + (int)(r % N1), z = A.lo[2] + (int)(r / N1);
#pragma unroll
      for (int fine = 0; fine < 2; ++fine) {
        const int per = fine ? 7 : 1;
        const int64_t abase = A.cin + (fine ? A.n_c : 0);
        for (int q = rt[A.rt[fine] + r], qe = rt[A.rt[fine] + r + 1]; q < qe; ++q) {
          const wvl_seg sa = seg[q];
          const int len = per * (sa.i1e - sa.i1s + 1);
          for (int j0 = 0; j0 < len; j0 += 64) {
            const int j = j0 + lane;
            const bool own = j < len;
            const int pt = own ? j / per : 0;
            const int comp = own ? j - per * pt : 0;
            const int gx = sa.i1s + pt;
            double acc = 0.0;
            for (int t = 0; t < nn; ++t) {
              const GradNb& x = nb[t];
              // H phi_d on d's output pattern
              const int ry = y - x.out_y0, rz = z - x.out_z0;
              if (ry >= 0 && ry < x.out_by && rz >= 0 && rz < x.out_nz && x.a != 0.0) {
                const int64_t k = own ? grad_find(rr, rt, seg, x.rr_out[fine], x.rt_out[fine],
                                                  (int64_t)rz * x.out_by + ry, gx)
                                      : -1;
                if (k >= 0) acc += x.a * (double)hpsi[x.cout + (fine ? x.on_c : 0) + per * k + comp];
              }
              // phi_d on d's input pattern
              const int sy = y - x.in_y0, sz = z - x.in_z0;
              if (sy >= 0 && sy < x.in_by && sz >= 0 && sz < x.in_nz && x.m != 0.0) {
                const int64_t k = own ? grad_find(rr, rt, seg, x.rr_in[fine], x.rt_in[fine],
                                                  (int64_t)sz * x.in_by + sy, gx)
                                      : -1;
                if (k >= 0) acc -= x.m * (double)psi[x.cin + (fine ? x.n_c : 0) + per * k + comp];
              }
            }
            if (own) {
              T* o = g + abase + per * sa.off + j;
              *o = bi == 0 ? (T)acc : (T)((double)*o + acc);
            }
          }
        }
      }
    }
  }
}

static inline dim3 grid2(int64_t maxvol, int nsf) {
  return dim3((unsigned)((maxvol + TPB - 1) / TPB), (unsigned)nsf);
}

// Loads the code objects of the kernels a captured step may launch.
int preload_kernels() {
  const void* fns[] = {(const void*)k_finalize, (const void*)k_sparse_values<float>,
                       (const void*)k_sparse_values<double>, (const void*)k_update<float>,
                       (const void*)k_update<double>, (const void*)k_sf_dot<float>,
                       (const void*)k_sf_dot<double>, (const void*)k_dens_tile<float, true>,
                       (const void*)k_dens_tile<float, false>,
                       (const void*)k_dens_tile<double, true>,
                       (const void*)k_dens_tile<double, false>, (const void*)k_grad_rows<float>,
                       (const void*)k_grad_rows<double>};
  for (const void* f : fns) {
    hipFuncAttributes a;
    const hipError_t e = hipFuncGetAttributes(&a, f);
    if (e != hipSuccess) return (int)e;
  }
  return 0;
}

int launch_gather(int f64, void* stream, const SfDev* sf, const wvl_seg* seg, const int32_t* rt,
                  const void* psi, void* box, int sf0, int nsf, int64_t maxvol) {
  if (nsf == 0 || maxvol == 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  if (f64)
    hipLaunchKernelGGL(k_gather<double>, grid2(maxvol, nsf), dim3(TPB), 0, st, sf, seg, rt,
                       (const double*)psi, (double*)box, sf0);
  else
    hipLaunchKernelGGL(k_gather<float>, grid2(maxvol, nsf), dim3(TPB), 0, st, sf, seg, rt,
                       (const float*)psi, (float*)box, sf0);
  return (int)hipGetLastError();
}

int launch_scatter(int f64, void* stream, const SfDev* sf, const wvl_seg* seg, const int32_t* rt,
                   const void* box, void* out, int sf0, int nsf, int64_t maxvol) {
  if (nsf == 0 || maxvol == 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  if (f64)
    hipLaunchKernelGGL(k_scatter<double>, grid2(maxvol, nsf), dim3(TPB), 0, st, sf, seg, rt,
                       (const double*)box, (double*)out, sf0);
  else
    hipLaunchKernelGGL(k_scatter<float>, grid2(maxvol, nsf), dim3(TPB), 0, st, sf, seg, rt,
                       (const float*)box, (float*)out, sf0);
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
                         const int32_t* rt, const RowRun* rr, int ket_out, const void* bra,
                         const void* ket, const int32_t* row, const int32_t* col,
                         const int32_t* order, const int32_t* mirror, int64_t nnz, double* val) {
  if (nnz == 0) return 0;
  const unsigned nblk = (unsigned)(8 * ((nnz + 7) / 8));
  if (f64)
    hipLaunchKernelGGL(k_sparse_values<double>, dim3(nblk), dim3(64), 0, (hipStream_t)stream, sf,
                       seg, rt, rr, ket_out, (const double*)bra, (const double*)ket, row, col,
                       order, mirror, nnz, val);
  else
    hipLaunchKernelGGL(k_sparse_values<float>, dim3(nblk), dim3(64), 0, (hipStream_t)stream, sf,
                       seg, rt, rr, ket_out, (const float*)bra, (const float*)ket, row, col,
                       order, mirror, nnz, val);
  return (int)hipGetLastError();
}

int launch_dens_tile(int f64, void* stream, const SfDev* sf, const int64_t* foff,
                     const void* fine, const int64_t* krow, const int32_t* kcol,
                     const double* kval, int64_t knnz, const int64_t* cptr, const int32_t* csf,
                     const int32_t* tord, int64_t n_one, const int* gf, void* rho) {
  const int tx = (gf[0] + kDensTile[0] - 1) / kDensTile[0];
  const int ty = (gf[1] + kDensTile[1] - 1) / kDensTile[1];
  const int tz = (gf[2] + kDensTile[2] - 1) / kDensTile[2];
  const int64_t ntile = (int64_t)tx * ty * tz;
  const dim3 blk(64 * kDensWaves);
  hipStream_t st = (hipStream_t)stream;
  for (int one = 1; one >= 0; --one) {
    const int64_t base = one ? 0 : n_one, n = one ? n_one : ntile - n_one;
    if (n == 0) continue;
    const dim3 g((unsigned)n);
    if (f64 && one)
      hipLaunchKernelGGL((k_dens_tile<double, true>), g, blk, 0, st, sf, foff,
                         (const double*)fine, krow, kcol, kval, knnz, cptr, csf, tord, base, tx,
                         ty, gf[0], gf[1], gf[2], (double*)rho);
    else if (f64)
      hipLaunchKernelGGL((k_dens_tile<double, false>), g, blk, 0, st, sf, foff,
                         (const double*)fine, krow, kcol, kval, knnz, cptr, csf, tord, base, tx,
                         ty, gf[0], gf[1], gf[2], (double*)rho);
    else if (one)
      hipLaunchKernelGGL((k_dens_tile<float, true>), g, blk, 0, st, sf, foff,
                         (const float*)fine, krow, kcol, kval, knnz, cptr, csf, tord, base, tx,
                         ty, gf[0], gf[1], gf[2], (float*)rho);
    else
      hipLaunchKernelGGL((k_dens_tile<float, false>), g, blk, 0, st, sf, foff,
                         (const float*)fine, krow, kcol, kval, knnz, cptr, csf, tord, base, tx,
                         ty, gf[0], gf[1], gf[2], (float*)rho);
  }
  return (int)hipGetLastError();
}

static inline dim3 grid1(int64_t n) { return dim3((unsigned)((n + TPB - 1) / TPB)); }

int launch_foe_mm(void* stream, int nrow, const int32_t* rows, const int64_t* rowptr,
                  const int32_t* col, double alpha, const double* A, const double* B, double beta,
                  const double* D, double* C, int lognb, int maxdeg) {
  if (nrow == 0) return 0;
  // rows of at most 256 entries: two rows of B (128 entries each) per step
  const int w = maxdeg <= kFoeMaxDeg / 2 ? 8 : 4;
  const int nh = maxdeg <= kFoeMaxDeg / 4 ? 2 : 1;
  const size_t lds = (size_t)maxdeg * 8 * (w * nh + 2) + ((size_t)16 << lognb);
  const dim3 g((unsigned)nrow), blk(64 * w);
  hipStream_t st = (hipStream_t)stream;
  if (nh == 2)
    hipLaunchKernelGGL((k_foe_mm<8, 2>), g, blk, lds, st, rows, rowptr, col, alpha, A, B, beta,
                       D, C, lognb, maxdeg);
  else if (w == 8)
    hipLaunchKernelGGL((k_foe_mm<8, 1>), g, blk, lds, st, rows, rowptr, col, alpha, A, B, beta,
                       D, C, lognb, maxdeg);
  else
    hipLaunchKernelGGL((k_foe_mm<4, 1>), g, blk, lds, st, rows, rowptr, col, alpha, A, B, beta,
                       D, C, lognb, maxdeg);
  return (int)hipGetLastError();
}

int launch_foe_axpby(void* stream, int64_t nnz, double a, const double* X, double b,
                     const double* Y, const int32_t* row, const int32_t* col, double d,
                     double* out) {
  if (nnz == 0) return 0;
  hipLaunchKernelGGL(k_foe_axpby, grid1(nnz), dim3(TPB), 0, (hipStream_t)stream, nnz, a, X, b, Y,
                     row, col, d, out);
  return (int)hipGetLastError();
}

int launch_foe_sym(void* stream, int64_t nnz, const int64_t* tpos, const double* X, double* out) {
  if (nnz == 0) return 0;
  hipLaunchKernelGGL(k_foe_sym, grid1(nnz), dim3(TPB), 0, (hipStream_t)stream, nnz, tpos, X, out);
  return (int)hipGetLastError();
}

int launch_foe_gather(void* stream, int64_t nnz, const int64_t* qpos, const double* X,
                      double* out) {
  if (nnz == 0) return 0;
  hipLaunchKernelGGL(k_foe_gather, grid1(nnz), dim3(TPB), 0, (hipStream_t)stream, nnz, qpos, X,
                     out);
  return (int)hipGetLastError();
}

int launch_foe_dot(void* stream, int64_t nnz, const double* X, const double* Y, double* part,
                   double* out, int slot) {
  const int nblk = (int)std::min<int64_t>(256, std::max<int64_t>(1, (nnz + 2047) / 2048));
  const int64_t chunk = (nnz + nblk - 1) / nblk;
  hipLaunchKernelGGL(k_foe_dot, dim3(nblk), dim3(TPB), 0, (hipStream_t)stream, nnz, chunk, X, Y,
                     part);
  hipLaunchKernelGGL(k_foe_sum, dim3(1), dim3(TPB), 0, (hipStream_t)stream, nblk, part, out, slot);
  return (int)hipGetLastError();
}

int launch_foe_trace(void* stream, int n, const int64_t* dpos, const double* X, int64_t stride,
                     int count, double* out, int slot) {
  if (count == 0) return 0;
  hipLaunchKernelGGL(k_foe_trace, dim3((unsigned)count), dim3(TPB), 0, (hipStream_t)stream, n,
                     dpos, X, stride, out, slot);
  return (int)hipGetLastError();
}

int launch_foe_series(void* stream, int64_t nnz, int npl, const double* c, const double* T,
                      const int32_t* row, const int32_t* col, double* out) {
  if (nnz == 0) return 0;
  hipLaunchKernelGGL(k_foe_series, grid1(nnz), dim3(TPB), 0, (hipStream_t)stream, nnz, npl, c, T,
                     row, col, out);
  return (int)hipGetLastError();
}

int launch_foe_gersh(void* stream, int nrow, const int64_t* rowptr, const int32_t* col,
                     const double* X, double* lo, double* hi, double* out) {
  if (nrow == 0) return 0;
  const int rows = TPB / 64;
  hipLaunchKernelGGL(k_foe_gersh_rows, dim3((unsigned)((nrow + rows - 1) / rows)), dim3(TPB), 0,
                     (hipStream_t)stream, nrow, rowptr, col, X, lo, hi);
  hipLaunchKernelGGL(k_foe_gersh, dim3(1), dim3(TPB), 0, (hipStream_t)stream, nrow, lo, hi, out);
  return (int)hipGetLastError();
}

int launch_update(int f64, void* stream, const SfDev* sf, const wvl_seg* seg, const int32_t* rt,
                  double eta, const void* hpsi, const int64_t* hrow, const int32_t* hcol,
                  const double* hval, void* psi, int sf0, int nsf, int64_t maxsegs, int mode,
                  const double* shift, void* out) {
  if (nsf == 0) return 0;
  const dim3 g((unsigned)(maxsegs / kUpdSegs + 2), (unsigned)nsf);
  if (f64)
    hipLaunchKernelGGL(k_update<double>, g, dim3(256), 0, (hipStream_t)stream, sf, seg, rt, eta,
                       (const double*)hpsi, hrow, hcol, hval, (double*)psi, sf0, mode, shift,
                       (double*)out);
  else
    hipLaunchKernelGGL(k_update<float>, g, dim3(256), 0, (hipStream_t)stream, sf, seg, rt, eta,
                       (const float*)hpsi, hrow, hcol, hval, (float*)psi, sf0, mode, shift,
                       (float*)out);
  return (int)hipGetLastError();
}

int launch_sf_dot(int f64, void* stream, const SfDev* sf, const void* a, const void* b,
                  double* out, int sf0, int nsf) {
  if (nsf == 0) return 0;
  if (f64)
    hipLaunchKernelGGL(k_sf_dot<double>, dim3(nsf), dim3(TPB), 0, (hipStream_t)stream, sf,
                       (const double*)a, (const double*)b, out, sf0);
  else
    hipLaunchKernelGGL(k_sf_dot<float>, dim3(nsf), dim3(TPB), 0, (hipStream_t)stream, sf,
                       (const float*)a, (const float*)b, out, sf0);
  return (int)hipGetLastError();
}

int launch_cg_init(int f64, void* stream, const SfDev* sf, const void* g, void* x, void* r,
                   void* p, int sf0, int nsf) {
  if (nsf == 0) return 0;
  if (f64)
    hipLaunchKernelGGL(k_cg_init<double>, dim3(nsf), dim3(TPB), 0, (hipStream_t)stream, sf,
                       (const double*)g, (double*)x, (double*)r, (double*)p, sf0);
  else
    hipLaunchKernelGGL(k_cg_init<float>, dim3(nsf), dim3(TPB), 0, (hipStream_t)stream, sf,
                       (const float*)g, (float*)x, (float*)r, (float*)p, sf0);
  return (int)hipGetLastError();
}

int launch_cg_xr(int f64, void* stream, const SfDev* sf, const double* rr, const double* pap,
                 const void* p, const void* ap, void* x, void* r, int sf0, int nsf) {
  if (nsf == 0) return 0;
  if (f64)
    hipLaunchKernelGGL(k_cg_xr<double>, dim3(nsf), dim3(TPB), 0, (hipStream_t)stream, sf, rr,
                       pap, (const double*)p, (const double*)ap, (double*)x, (double*)r, sf0);
  else
    hipLaunchKernelGGL(k_cg_xr<float>, dim3(nsf), dim3(TPB), 0, (hipStream_t)stream, sf, rr, pap,
                       (const float*)p, (const float*)ap, (float*)x, (float*)r, sf0);
  return (int)hipGetLastError();
}

int launch_cg_p(int f64, void* stream, const SfDev* sf, double* rr, const double* rr_new,
                const void* r, void* p, int sf0, int nsf) {
  if (nsf == 0) return 0;
  if (f64)
    hipLaunchKernelGGL(k_cg_p<double>, dim3(nsf), dim3(TPB), 0, (hipStream_t)stream, sf, rr,
                       rr_new, (const double*)r, (double*)p, sf0);
  else
    hipLaunchKernelGGL(k_cg_p<float>, dim3(nsf), dim3(TPB), 0, (hipStream_t)stream, sf, rr,
                       rr_new, (const float*)r, (float*)p, sf0);
  return (int)hipGetLastError();
}

int launch_grad_rows(int f64, void* stream, const SfDev* sf, const wvl_seg* seg,
                     const int32_t* rt, const RowRun* rr, const int64_t* rowptr,
                     const int32_t* col, const double* av, const double* mv, const void* psi,
                     const void* hpsi, int sf0, int nsf, void* g) {
  if (nsf == 0) return 0;
  if (f64)
    hipLaunchKernelGGL(k_grad_rows<double>, dim3((unsigned)nsf), dim3(256), 0, (hipStream_t)stream,
                       sf, seg, rt, rr, rowptr, col, av, mv, (const double*)psi,
                       (const double*)hpsi, sf0, (double*)g);
  else
    hipLaunchKernelGGL(k_grad_rows<float>, dim3((unsigned)nsf), dim3(256), 0, (hipStream_t)stream,
                       sf, seg, rt, rr, rowptr, col, av, mv, (const float*)psi,
                       (const float*)hpsi, sf0, (float*)g);
  return (int)hipGetLastError();
}

}  // namespace wvl

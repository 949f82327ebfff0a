// Internal structures shared by the host plan (wvl_host.cpp) and the HIP
// kernels (wvl_kernels.hip).  Not part of the public ABI.
#pragma once

#include <stdint.h>

#include "../../include/wvl.h"

namespace wvl {

// Per support function, device resident.  Boxes use local indices:
// input coarse i in [0, n), fine real-space l in [-14, 2n+14] stored at
// l + 14, output coarse i in [-ext, n+ext) stored at i + ext.
struct SfDev {
  double c[3];        // localization centre (bohr), for the confining potential
  int32_t lo[3];
  int32_t n[3];
  int32_t ext;
  int32_t pad0;
  int64_t cin;        // input coefficient offset (elements)
  int64_t cout;       // output coefficient offset
  int64_t n_c, n_f, on_c, on_f;
  int64_t box_in;     // dense input box offset (wvl_uncompress)
  int64_t box_out;    // dense output box offset (wvl_compress)
  // row tables: for pattern p (0 in-coarse, 1 in-fine, 2 out-coarse,
  // 3 out-fine) entry rt[p] + r .. rt[p] + r + 1 bounds the segments of box
  // row r = (i3 - oz) * by + (i2 - oy), as indices into the segment array.
  int64_t rt[4];
  // tight bounding boxes (x0, x1, y0, y1, z0, z1) of the input and output
  // coarse patterns, global indices (empty pattern: x0 > x1).
  int32_t bb_in[6];
  int32_t bb_out[6];
  // compact row runs: for pattern p, RowRun entry rr[p] + r describes box
  // row r (same row numbering as rt)
  int64_t rr[4];
};

// One box row of a pattern: its single run [x0, x0 + len) starting at
// coefficient `off` of the pattern; len 0 = empty row, kMultiRun = several
// runs (walk the segments through the row table instead).
struct RowRun {
  uint16_t x0, len;
  int32_t off;
};
constexpr uint16_t kMultiRun = 0xFFFF;

// k_back_out: output rows (y', z') per block, 16 per wave (one wave per block
// measured fastest: the waves share no LDS, more blocks fit a CU)
constexpr int kBackOutRows = 16;

// Workspace offsets (elements of the compute type) of one support function
// in the workspace (R = 2N + 29, O = N + 2 ext).  The plan keeps these
// records in its processing order (functions sorted by box size, cut into
// chunks); kernels find the function's SfDev through `id`.
//   c8   dense input box, x fastest      [8][N2][N1][N0]
//   c8x  dense input box, y fastest      [8][N2][N0][N1]
//   g1   after the x, y up passes        [2][N2][R1][R0]
//   g2   after the z column pass         [2][O2][R1][R0]
//   q    after the y down pass           [4][O2][R0][O1]   (channel a2 + 2 a3)
//   ox   x part of the kinetic term      [8][N2][O0][N1]
//   oy   y part of the kinetic term      [8][N2][N0][O1]
//   oz   z part of the kinetic term      [8][O2][N0][N1]
//   gx   after the x up pass             [4][N2][N1][R0]   (channel a2 + 2 a3)
struct SfWork {
  int64_t id;         // the function's index in the plan (SfDev array, outputs)
  int64_t c8, c8x, g1, g2, q, ox, oy, oz, gx;
  int64_t epart;      // offset (in doubles) of its e_pot partials
  int64_t kpart;      // offset (in doubles) of its e_kin partials
  int64_t nkpart;     // number of e_kin partials: its own k_kin_col blocks
};

// e_kin partial slots of one function: the blocks of k_kin_col along x, then
// y, then z, counted on the function's own box (so that the summation order
// does not depend on the other functions of the chunk)
// (the z part by k_kin_zmfma when zmfma: one block per 16 columns)
// row stride (elements) of Q[ch][z'][px][y'], the y analysis output: O1
// rounded up to 16, so that the 16-value chunks k_back_y writes (aligned by
// its window phase) are whole 64-byte (FP32) or 128-byte (FP64) pieces
__host__ __device__ inline int qrow_stride(int o1) { return (o1 + 15) & ~15; }
__host__ __device__ inline int kin_blocks(int axis, int n0, int n1, int n2, bool zmfma = false) {
  return axis == 0 ? (4 * n1 * n2 + 255) / 256
         : axis == 1 ? (4 * n0 * n2 + 63) / 64
         : zmfma ? (n0 * n1 + 15) / 16 : (4 * n0 * n1 + 255) / 256;
}

// per-chunk launch geometry of the fused kernels, for dtype d (0 f32, 1 f64)
struct ChunkDev {
  int32_t sf0, nsf;                // positions [sf0, sf0 + nsf) of the processing order
  int64_t maxbox_in;               // largest dense input box (elements)
  int32_t grid_u[2], group_u[2];   // k_unpack: (8 / group) blocks per input z
  int32_t grid_ux, grid_uy;        // k_up_x, k_up_y
  int64_t lds_u[2];
  int32_t grid_b;                  // k_pot_column
  int32_t grid_kx, grid_ky, grid_kz;   // k_kin_col (x, y, z)
  int32_t grid_by;                 // k_back_y
  int32_t grid_bx;                 // k_back_out
  int32_t nblk_pot, nblk_kin;      // partial slots per function
};

// the apply of wvl_apply_local_ham on a workspace of `cap` bytes that the
// caller vouches for (wvl_host.cpp); rejects plans that need more
wvl_status apply_in_workspace(wvl_plan* plan, wvl_dtype dt, uint32_t terms, const void* psi_c,
                              const void* pot, void* hpsi_c, double* e_kin, double* e_pot,
                              void* workspace, size_t cap, const char* who);
// records an error on the plan's context (or the thread's, for a NULL plan)
wvl_status plan_error(wvl_plan* plan, wvl_status st, const char* msg);
// the HIP stream of the plan's context
void* plan_stream(const wvl_plan* plan);

// load every kernel's code object before a stream capture (hipError_t as int)
int preload_kernels();         // wvl_kernels.hip
int preload_fused_kernels();   // wvl_fused.hip

// launchers implemented in wvl_kernels.hip; all return hipError_t as int
int launch_gather(int f64, void* stream, const SfDev* sf, const wvl_seg* seg, const int32_t* rt,
                  const void* psi, void* box, int sf0, int nsf, int64_t maxvol);
int launch_scatter(int f64, void* stream, const SfDev* sf, const wvl_seg* seg, const int32_t* rt,
                   const void* box, void* out, int sf0, int nsf, int64_t maxvol);
int launch_fill(int f64, void* stream, void* ptr, int64_t n);
int launch_unpack(int f64, void* stream, const SfDev* sf, const wvl_seg* seg, const int32_t* rt,
                  const RowRun* rr, const void* psi, const SfWork* wk, int nsf, int gridx,
                  int group, size_t lds, void* ws);
int launch_up(int f64, void* stream, int axis, const SfWork* wk, const SfDev* sf, int nsf,
              int gridx, void* ws);
int launch_up_z(int f64, void* stream, const SfWork* wk, const SfDev* sf, int nsf, int gridx,
                const void* ws, const int64_t* fine_off, void* fine);
// density: tiles of 16 x 4 x 1 fine-grid points (one 64-lane workgroup each)
// with the functions whose fine box meets them (at most kDensMaxCover)
// with the functions whose fine box meets them (at most kDensMaxCover),
// staged kDensChunk[FP32, FP64] functions at a time.  tord lists the tiles:
// first the n_one with at most kDensChunkOne functions (FP32), then the
// others.
constexpr int kDensTile[3] = {16, 4, 1};
constexpr int kDensMaxCover = 1024;
constexpr int kDensChunk[2] = {128, 64};
constexpr int kDensChunkOne = 120;   // FP32 tiles of one chunk (four workgroups per CU)
int launch_dens_tile(int f64, void* stream, const SfDev* sf, const int64_t* foff,
                     const void* fine, const int64_t* krow, const int32_t* kcol,
                     const double* kval, int64_t knnz, const int64_t* cptr, const int32_t* csf,
                     const int32_t* tord, int64_t n_one, const int* gf, void* rho);
int launch_pot_column(int f64, void* stream, const SfDev* sf, const SfWork* wk, int sf0, int nsf,
                      int gridx, void* ws, const void* pot, int nf1, int nf2, double* epart,
                      const double* conf, double hh);
// the z part of the kinetic term on the FP64 matrix cores (banded Toeplitz)
int launch_kin_zmfma(int f64, void* stream, const SfDev* sf, const SfWork* wk, int sf0, int nsf,
                     int gridx, void* ws, double fac, double* kpart);
int launch_kin_col(int f64, void* stream, int axis, const SfDev* sf, const SfWork* wk, int sf0,
                   int nsf, int gridx, void* ws, double fac, double* kpart);
int launch_back_y(int f64, void* stream, const SfDev* sf, const SfWork* wk, int sf0, int nsf,
                  int gridx, void* ws);
int launch_back_out(int f64, void* stream, const SfDev* sf, const wvl_seg* seg, const int32_t* rt,
                    const RowRun* rr, const SfWork* wk, int sf0, int nsf, int gridx,
                    const void* ws, void* out, int pot_on, int kin_on, int accumulate);
int launch_finalize(void* stream, const SfWork* wk, int sf0, int nsf, const double* parts,
                    int which, int nblk, double* out);
int launch_pattern(void* stream, const SfDev* sf, const wvl_seg* seg, const int32_t* rt, int nsf,
                   int ket_out, int64_t* count, const int64_t* rowptr, int32_t* col);
// Fermi operator expansion on a symmetric CSR pattern (row: row of each
// entry, tpos: position of the transposed entry).  foe_mm: one workgroup per
// row, 8 waves when no row has more than kFoeMaxDeg / 2 entries, else 4
// (and two rows of B a step when none has more than kFoeMaxDeg / 4);
// rows of at most kFoeMaxDeg entries, columns below kFoeMaxCol, entries
// addressed with 32-bit offsets; 2^lognb hash buckets of 16 bytes, at least
// as many as the longest row has entries (maxdeg) and at least 32 (at most
// 64 KiB of LDS in all).
constexpr int kFoeMaxDeg = 1024;
constexpr int kFoeMaxCol = 1 << 21;
int launch_foe_mm(void* stream, int nrow, const int32_t* rows, const int64_t* rowptr,
                  const int32_t* col, double alpha, const double* A, const double* B, double beta,
                  const double* D, double* C, int lognb, int maxdeg);
int launch_foe_axpby(void* stream, int64_t nnz, double a, const double* X, double b,
                     const double* Y, const int32_t* row, const int32_t* col, double d,
                     double* out);
int launch_foe_sym(void* stream, int64_t nnz, const int64_t* tpos, const double* X, double* out);
int launch_foe_gather(void* stream, int64_t nnz, const int64_t* qpos, const double* X,
                      double* out);
// dot: part needs min(256, ceil(nnz / 2048)) doubles (at most nnz)
int launch_foe_dot(void* stream, int64_t nnz, const double* X, const double* Y, double* part,
                   double* out, int slot);
int launch_foe_trace(void* stream, int n, const int64_t* dpos, const double* X, int64_t stride,
                     int count, double* out, int slot);
int launch_foe_series(void* stream, int64_t nnz, int npl, const double* c, const double* T,
                      const int32_t* row, const int32_t* col, double* out);
// Gershgorin bounds: lo, hi hold nrow doubles each
int launch_foe_gersh(void* stream, int nrow, const int64_t* rowptr, const int32_t* col,
                     const double* X, double* lo, double* hi, double* out);
int launch_update(int f64, void* stream, const SfDev* sf, const wvl_seg* seg, const int32_t* rt,
                  double eta, const void* hpsi, const int64_t* hrow, const int32_t* hcol,
                  const double* hval, void* psi, int sf0, int nsf, int64_t maxsegs, int mode,
                  const double* shift, void* out);
// g_a = L^a [sum_d A_ad H phi_d - M_ad phi_d] over the rows of a CSR pattern
// (A and M in its order), one block per function a of [sf0, sf0 + nsf)
int launch_grad_rows(int f64, void* stream, const SfDev* sf, const wvl_seg* seg,
                     const int32_t* rt, const RowRun* rr, const int64_t* rowptr,
                     const int32_t* col, const double* av, const double* mv, const void* psi,
                     const void* hpsi, int sf0, int nsf, void* g);
int launch_sf_dot(int f64, void* stream, const SfDev* sf, const void* a, const void* b,
                  double* out, int sf0, int nsf);
int launch_cg_init(int f64, void* stream, const SfDev* sf, const void* g, void* x, void* r,
                   void* p, int sf0, int nsf);
int launch_cg_xr(int f64, void* stream, const SfDev* sf, const double* rr, const double* pap,
                 const void* p, const void* ap, void* x, void* r, int sf0, int nsf);
int launch_cg_p(int f64, void* stream, const SfDev* sf, double* rr, const double* rr_new,
                const void* r, void* p, int sf0, int nsf);
int launch_sparse_values(int f64, void* stream, const SfDev* sf, const wvl_seg* seg,
                         const int32_t* rt, const RowRun* rr, int ket_out, const void* bra,
                         const void* ket, const int32_t* row, const int32_t* col,
                         const int32_t* order, const int32_t* mirror, int64_t nnz, double* val);

}  // namespace wvl

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
};

// Workspace offsets (elements of the compute type) of one support function
// inside its chunk's workspace.
struct SfWork {
  int64_t c8, a1, a2, g, b1, b2, o8;
  int64_t epart;      // offset (in doubles) of its e_pot partials
  int64_t kpart;      // offset (in doubles) of its e_kin partials
};

enum Pass {
  P_GATHER = 0,  // compressed -> C8
  P_UPX, P_UPY, P_UPZ,
  P_DOWNZ, P_DOWNY, P_DOWNX,
  P_KIN,         // C8 -> O8 (any axis)
  P_SCATTER,     // O8 -> compressed
  P_NPASS
};

// one chunk of support functions processed together
struct ChunkDev {
  int32_t sf0, nsf;
  int64_t maxvol[P_NPASS];
  int32_t nblk_pot, nblk_kin;
};

// launchers implemented in wvl_kernels.hip; all return hipError_t as int
int launch_gather(int f64, void* stream, const SfDev* sf, const wvl_seg* seg, const int32_t* rt,
                  const void* psi, void* box, const SfWork* wk, int sf0, int nsf, int64_t maxvol,
                  int use_work);
int launch_scatter(int f64, void* stream, const SfDev* sf, const wvl_seg* seg, const int32_t* rt,
                   const void* box, void* out, const SfWork* wk, int sf0, int nsf, int64_t maxvol,
                   int use_work, int accumulate);
int launch_up(int f64, void* stream, int axis, const SfDev* sf, const SfWork* wk, int sf0, int nsf,
              int64_t maxvol, void* ws, const void* pot, int nf1, int nf2, double* epart,
              int nblk);
int launch_down(int f64, void* stream, int axis, const SfDev* sf, const SfWork* wk, int sf0,
                int nsf, int64_t maxvol, void* ws, int accumulate);
int launch_kin(int f64, void* stream, int axis, const SfDev* sf, const SfWork* wk, int sf0,
               int nsf, int64_t maxvol, void* ws, int accumulate, double fac);
int launch_fill(int f64, void* stream, void* ptr, int64_t n);
int launch_ekin_partials(int f64, void* stream, const SfDev* sf, const SfWork* wk, int sf0,
                         int nsf, int64_t maxvol, void* ws, double* kpart, int nblk);
int launch_finalize(void* stream, const SfWork* wk, int sf0, int nsf, const double* parts,
                    int which, int nblk, double* out);
int launch_pattern(void* stream, const SfDev* sf, const wvl_seg* seg, const int32_t* rt, int nsf,
                   int ket_out, int64_t* count, const int64_t* rowptr, int32_t* col);
int launch_sparse_values(int f64, void* stream, const SfDev* sf, const wvl_seg* seg,
                         const int32_t* rt, int ket_out, const void* bra, const void* ket,
                         const int32_t* row, const int32_t* col, int64_t nnz, double* val);

}  // namespace wvl

/*
 * wvl.h -- C ABI of the MI355X local-Hamiltonian library for linear-scaling
 * Daubechies-wavelet DFT (Mohr et al., arXiv:1401.7441).
 *
 * The library applies the local Kohn-Sham Hamiltonian (kinetic energy plus a
 * local potential) to many localized support functions, each stored
 * compressed on its own localization region, and forms the sparse overlap
 * and Hamiltonian matrices between support functions whose regions overlap.
 *
 * Problem statement followed by every call (paper sections):
 *   Sec. II.B, Eq. (Phi): two-level basis on a uniform coarse grid of spacing
 *     h with the origin in a corner; a coarse point carries one scaling
 *     function, a fine point one scaling function plus seven wavelets of the
 *     least-asymmetric Daubechies family of order 16.
 *   Sec. III: a support function keeps only the coefficients within R_cut of
 *     its centre (the projector L); Sec. III.B: H is applied as
 *     L' H L |phi> with L' the region grown by `ext` grid points (8 in the
 *     paper).
 *   Sec. II.A: S_ab = <phi_a|phi_b>, H_ab = <phi_a|H|phi_b>.
 *
 * Memory: every pointer documented as "device" is a caller-owned device
 * buffer (HIP global memory, e.g. a torch tensor's data_ptr()); the library
 * never frees caller memory.  "host" pointers are read during the call only.
 * Element type of coefficient, potential and box buffers: float for WVL_F32,
 * double for WVL_F64.  Energies and matrix values are always double.
 *
 * Asynchrony: compute calls only enqueue work on the context's stream and
 * return; results are ready after that stream is synchronized.  Exceptions:
 * wvl_plan_create (waits for its host-to-device copies) and the pattern phase
 * of wvl_sparse_overlap (returns nnz to the host, so it synchronizes).
 *
 * Errors: every call returns a wvl_status.  WVL_EINVAL means the arguments
 * were rejected before anything was launched; wvl_last_error() names the
 * offending support function or segment.  WVL_EDEVICE reports a HIP failure.
 * No C++ exception crosses this interface.
 *
 * Threading: a context is bound to one HIP stream and must not be used from
 * two threads at once; distinct contexts, with the plans created on them,
 * may be used from different threads at the same time (graph capture is
 * thread-local).  A plan may be applied any number of times; it builds its
 * sparsity patterns on first use and changes its layout only under
 * wvl_plan_autotune / wvl_plan_set_schedule, so one plan is used by one
 * thread at a time.
 */
#ifndef WVL_H
#define WVL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WVL_ABI_VERSION 1

typedef enum {
  WVL_OK = 0,
  WVL_EINVAL = -1,       /* invalid argument, nothing launched             */
  WVL_ENOMEM = -2,       /* device allocation by the library failed         */
  WVL_EDEVICE = -3,      /* a HIP call or kernel launch failed              */
  WVL_EUNSUPPORTED = -4  /* valid request this build does not support       */
} wvl_status;

typedef enum { WVL_F32 = 0, WVL_F64 = 1 } wvl_dtype;

/* terms of wvl_apply_local_ham */
enum { WVL_KIN = 1u, WVL_POT = 2u };

/* Global grid (Sec. II.B).  n[0..2] coarse points along x, y, z; coarse point
 * (i1, i2, i3) sits at h*(i1, i2, i3) bohr.  The potential lives on the fine
 * grid of 2n+29 points per axis, spacing h/2; fine point p sits at
 * (p - 14)*h/2, and is stored V[p3][p2][p1] with p1 fastest. */
typedef struct {
  double h;
  int32_t n[3];
} wvl_grid;

/* One segment: the coarse points i1 = i1s..i1e (inclusive) at fixed (i2, i3),
 * in global coarse indices.  `off` is the position of point i1s among the
 * points of its list: in the compressed layout (see wvl_locreg) the scaling
 * coefficient of coarse point i1s sits at coef_off + off, and the seven
 * wavelet coefficients of fine point i1s at coef_off + n_c + 7 off .. + 6. */
typedef struct {
  int32_t i1s, i1e, i2, i3;
  int64_t off;
} wvl_seg;

/* One localization region (Sec. III) and where its coefficients live.
 *
 * Input pattern: coarse segments seg[seg_c .. seg_c+nseg_c), fine segments
 * seg[seg_f .. seg_f+nseg_f).  Output (L') pattern: oseg_c/noseg_c and
 * oseg_f/noseg_f.  Segment lists are sorted by (i3, i2, i1s), disjoint, with
 * `off` the running sum of lengths starting at 0; every fine segment lies
 * inside a coarse segment of the same pattern.
 *
 * Input box: lo[a] .. lo[a]+dims[a]-1 per axis (inside the grid), holding the
 * input pattern.  Output box: the input box grown by `ext` on every side
 * (0 <= ext <= 16); the output pattern lies inside it and inside the grid.
 *
 * Compressed layout of the input coefficients, starting at element coef_off
 * of the batch buffer: [s: n_c][d: n_f][7] -- the scaling coefficients of
 * the n_c coarse points in segment order, then for each of the n_f fine
 * points (segment order) its seven wavelet coefficients, component
 * l = a1 + 2 a2 + 4 a3 at position l - 1 (a_d = 1: wavelet along axis d).
 * Output coefficients likewise at ocoef_off with on_c, on_f.
 *
 * center/radius/fine_radius describe the sphere the pattern was built from
 * (informational; radius <= 0 for patterns not built from a sphere). */
typedef struct {
  double center[3];
  double radius;
  double fine_radius;
  int32_t ext;
  int32_t lo[3];
  int32_t dims[3];
  int32_t pad_;
  int64_t seg_c, nseg_c, seg_f, nseg_f;
  int64_t oseg_c, noseg_c, oseg_f, noseg_f;
  int64_t coef_off, n_c, n_f;
  int64_t ocoef_off, on_c, on_f;
} wvl_locreg;

typedef struct {
  int64_t nsf;
  int64_t in_coefs;     /* elements of the input coefficient buffer       */
  int64_t out_coefs;    /* elements of the output coefficient buffer      */
  int64_t in_box;       /* elements of the dense input boxes (uncompress) */
  int64_t out_box;      /* elements of the dense output boxes (compress)  */
  int64_t workspace_f32;/* workspace bytes for WVL_F32                     */
  int64_t workspace_f64;/* workspace bytes for WVL_F64                     */
  int64_t chunks;       /* support-function chunks one apply iterates     */
  int64_t fine_box;     /* elements of all fine boxes (wvl_synthesize)    */
} wvl_plan_info;

typedef struct wvl_ctx wvl_ctx;
typedef struct wvl_plan wvl_plan;

/* Localization regions of spheres (Sec. III; host-only, no device use).
 * Coarse set of function k: grid points with
 *   (h*i1-X)^2 + (h*i2-Y)^2 + (h*i3-Z)^2 <= R*R
 * evaluated in double precision in exactly that order without contraction;
 * input box = its bounding box.  Fine set: the coarse points within
 * fine_radii[k].  Output coarse set: points within R + ext*h that lie in the
 * input box grown by ext and in the grid.  Output fine set: output coarse
 * points belonging to the union of all functions' input fine sets.
 * Coefficient offsets are laid out back to back in function order.
 *   centers: host [nsf][3]; radii, fine_radii: host [nsf]
 *   lr: host out [nsf]; segs: host out [*nsegs] or NULL
 *   nsegs: in = capacity of segs, out = segments needed.  With segs NULL or
 *   too small, fills lr's counts, sets *nsegs and returns WVL_OK only when
 *   segs was NULL (WVL_EINVAL when a non-NULL segs is too small).
 * Errors: WVL_EINVAL for h <= 0, an empty region, or radii < 0. */
wvl_status wvl_build_locregs(const wvl_grid* grid, int32_t nsf, const double* centers,
                             const double* radii, const double* fine_radii, int32_t ext,
                             wvl_locreg* lr, wvl_seg* segs, int64_t* nsegs);

/* Context bound to a grid and a HIP stream (hipStream_t; NULL = default). */
wvl_status wvl_create(wvl_ctx** ctx, const wvl_grid* grid, void* hip_stream);
void wvl_destroy(wvl_ctx* ctx);
/* Message of the last failed call on ctx (ctx NULL: of the last failed
 * context-free call on this thread).  Never NULL. */
const char* wvl_last_error(const wvl_ctx* ctx);

/* Validates and uploads a batch of localization regions (host arrays lr[nsf],
 * segs[nsegs]).  max_workspace_bytes bounds the FP64 workspace (0: no bound);
 * functions are then processed in chunks that fit.  *workspace_bytes
 * receives the FP64 workspace size (wvl_plan_info gives both dtypes). */
wvl_status wvl_plan_create(wvl_ctx* ctx, int32_t nsf, const wvl_locreg* lr, const wvl_seg* segs,
                           int64_t nsegs, size_t max_workspace_bytes, wvl_plan** plan,
                           size_t* workspace_bytes);
void wvl_plan_destroy(wvl_plan* plan);
wvl_status wvl_plan_info_get(const wvl_plan* plan, wvl_plan_info* info);

/* Uncompress (Sec. III, compressed storage): psi_c (device, input pattern
 * layout) -> psi_box (device): function k's dense box
 * [8][dims2][dims1][dims0] (component, z, y, x; x fastest) starting at the
 * running sum of 8*prod(dims) of the functions before it; zero off-pattern. */
wvl_status wvl_uncompress(wvl_plan* plan, wvl_dtype dt, const void* psi_c, void* psi_box);

/* Compress onto the output (L') pattern: box (device, function k's dense
 * output box [8][dims2+2e][dims1+2e][dims0+2e] at the running sum of their
 * sizes) -> hpsi_c (device, output layout, overwritten). */
wvl_status wvl_compress(wvl_plan* plan, wvl_dtype dt, const void* box, void* hpsi_c);

/* Local Hamiltonian (Sec. III.B): hpsi = L' (T + V) L psi for every function.
 *   terms: WVL_KIN and/or WVL_POT.
 *   psi_c: device, input layout.  pot: device global fine-grid potential
 *   (see wvl_grid), may be NULL without WVL_POT.  hpsi_c: device, output
 *   layout, overwritten.  e_kin / e_pot: device double[nsf] or NULL:
 *   <phi|T|phi> and the potential energy sum_r V f(r)^2 on the fine grid.
 *   workspace: device, at least the plan's workspace size for dt.
 * T is the exact Galerkin kinetic operator of the two-level basis; V is the
 * magic-filter quadrature of the local potential on the fine grid. */
wvl_status wvl_apply_local_ham(wvl_plan* plan, wvl_dtype dt, uint32_t terms, const void* psi_c,
                               const void* pot, void* hpsi_c, double* e_kin, double* e_pot,
                               void* workspace);

/* wvl_apply_local_ham with a confining potential per function (Sec. IV.A:
 * the quartic confinement a_a |r - R_a|^4 of the trace and hybrid modes):
 * on the fine grid the potential of function a becomes V(r) + conf[a]
 * |r - center_a|^4, with center_a = wvl_locreg.center and the fine point l
 * of an axis at (2 lo + l) h/2.  conf: device double[nsf] (0 = none for
 * that function).  terms must contain WVL_POT; e_pot then includes the
 * confinement energy.  Other arguments and errors as wvl_apply_local_ham. */
wvl_status wvl_apply_local_ham_conf(wvl_plan* plan, wvl_dtype dt, uint32_t terms,
                                    const void* psi_c, const void* pot, const double* conf,
                                    void* hpsi_c, double* e_kin, double* e_pot, void* workspace);

/* Allocation-free variant of wvl_apply_local_ham, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The workspace is a static device array
 * of WVL_STATIC_WORKSPACE_BYTES that the library holds on every GPU it runs
 * on until the process ends; the call makes no hipMalloc, hipFree or other
 * allocating call.  The plan's workspace size for dt (wvl_plan_info;
 * bounded at plan creation by max_workspace_bytes, which makes the functions
 * run in chunks that reuse one region) must not exceed it: larger plans are
 * rejected with WVL_EINVAL before anything is launched.  Every call on one
 * GPU uses the same array: calls that overlap on one GPU (two streams, two
 * threads, or one call still running on another stream) race; the array
 * keeps the last call's contents, and the apply reads nothing of it that it
 * has not written in the same call.  The GPU is the one of the context's
 * stream (the current device for the NULL stream).  Other arguments and
 * errors as wvl_apply_local_ham. */
#define WVL_STATIC_WORKSPACE_BYTES ((size_t)128 << 20)
wvl_status wvl_apply_local_ham_static(wvl_plan* plan, wvl_dtype dt, uint32_t terms,
                                      const void* psi_c, const void* pot, void* hpsi_c,
                                      double* e_kin, double* e_pot);

/* Kinetic term only (Sec. III.B, the -1/2 nabla^2 part), ACCUMULATED into
 * hpsi_c (device, output layout): hpsi += L' T L psi.  e_kin as above. */
wvl_status wvl_kinetic(wvl_plan* plan, wvl_dtype dt, const void* psi_c, void* hpsi_c,
                       double* e_kin, void* workspace);

/* Sparse overlap (ket_is_output = 0: S_ab = <phi_a|phi_b>, ket in the input
 * layout) or Hamiltonian (1: H_ab = <phi_a|H phi_b>, ket = the output of
 * wvl_apply_local_ham in the output layout) matrix (Sec. II.A).
 * Pattern: (a, b) is present when a's input coarse set shares a point with
 * b's input (S) or output (H) coarse set.  CSR, rows ascending, columns
 * ascending within a row.
 * Two phases: with rowptr, col and val all NULL the pattern is computed on
 * the device, cached in the plan, *nnz set (the call synchronizes the
 * stream).  Otherwise rowptr (device int64[nsf+1]), col (device int32[nnz])
 * and val (device double[nnz]) are filled, each optional; values are dot
 * products accumulated in double in an order fixed per pair.  For S with
 * bra_c == ket_c the pairs a <= b are summed and each value written to
 * (a, b) and (b, a); a pair's sum does not depend on which side is the bra,
 * so the values are those of the full computation, bit for bit. */
wvl_status wvl_sparse_overlap(wvl_plan* plan, const void* bra_c, int ket_is_output,
                              const void* ket_c, wvl_dtype dt, int64_t* nnz, int64_t* rowptr,
                              int32_t* col, double* val);

/* Real-space values of every support function on its fine box (Sec. II.B:
 * the two-level synthesis to the grid of spacing h/2, then the magic filter,
 * the steps the potential term of wvl_apply_local_ham starts with).  Function
 * k's box holds (2 N + 29)^3 points per its box dims N, stored
 * fine[off_k + (pz (2 N1 + 29) + py) (2 N0 + 29) + px] with off_k the sum of
 * the boxes of functions 0..k-1 (wvl_plan_info.fine_box elements in all);
 * point p of an axis sits at global fine-grid index 2 lo + p, the grid of
 * the potential.  psi_c: device, input layout; fine: device, dt; workspace
 * as for wvl_apply_local_ham.  Asynchronous on the context's stream. */
wvl_status wvl_synthesize(wvl_plan* plan, wvl_dtype dt, const void* psi_c, void* fine,
                          void* workspace);

/* Electronic density on the fine grid, Eq. (density) of Sec. II:
 *   rho(r) = sum_ab phi_a(r) K^ab phi_b(r)
 * with phi on the fine grid as wvl_synthesize writes it (fine) and the
 * density kernel K in CSR form: k_rowptr (device int64[nsf + 1]), k_col
 * (device int32[k_nnz]), k_val (device double[k_nnz]); any pattern, entries
 * summed as given (columns outside [0, nsf) and positions outside
 * [0, k_nnz) are skipped).  rho: device, dt, the global fine grid
 * [2 n2 + 29][2 n1 + 29][2 n0 + 29] (z, y, x), every point written (0 where
 * no fine box reaches).  work: unused (may be NULL).  Sums run in double
 * in an order fixed by the plan and K (per point: the functions meeting its
 * tile in increasing index, each with its row of K in stored order), so the
 * result is reproducible bitwise.  The first call builds the plan's tile
 * lists (synchronizes once).  Errors: WVL_EINVAL for null buffers or
 * k_nnz < 0; WVL_EUNSUPPORTED when more than 1024 fine boxes meet one tile
 * of 16 x 4 x 1 fine-grid points, or the plan has 2^24 or more functions. */
wvl_status wvl_density(wvl_plan* plan, wvl_dtype dt, const void* fine, const int64_t* k_rowptr,
                       const int32_t* k_col, const double* k_val, int64_t k_nnz, void* rho,
                       void* work);

/* Density kernel by the Fermi operator expansion (Sec. IV.B and App. B),
 * on the overlap pattern P of the plan (the pattern wvl_sparse_overlap
 * reports with ket_is_output = 0; every matrix below lives on P, each
 * product truncated to P):
 *   S, H      symmetric parts of the given S (on P) and H (on the H
 *             pattern, taken at P's entries);
 *   S^-1/2    ~ (3 I - S) / 2, the first-order Taylor expansion;
 *   H~ = sigma (H - tau S), sigma = 2 / (eps_max - eps_min),
 *             tau = (eps_min + eps_max) / 2;
 *   H~' = S^-1/2 H~ S^-1/2;  K' = c_0/2 I + sum_{i=1..npl} c_i T^i(H~'),
 *             T^i by the Chebyshev recursion, c_i the Chebyshev coefficients
 *             on [-1, 1] of f = (1 - erf((eps - mu) / delta)) / 2;
 *   mu        such that Tr K' = n_occ (bisection: the traces of the T^i are
 *             taken once; K' then sums the kept T^i with the final
 *             coefficients, or, in the smaller scratch, forms them again);
 *   K = S^-1/2 K' S^-1/2;  E_BS = Tr(K H~) / sigma + tau Tr(K S).
 * The symmetric part is taken after each two-sided product, since the
 * truncation breaks the symmetry the exact product has.  Spectrum guard:
 * with the Taylor S^-1/2, H~' can reach outside [-1, 1] even for exact
 * bounds (the recursion would then grow without bound); when the Gershgorin
 * discs [a, b] of H~' do, the recursion runs on (H~' - c I) / r with
 * [c - r, c + r] = [min(a, -1), max(b, 1)] and f is taken at
 * (r x + c) / sigma + tau, which leaves p an approximation of f(H~' / sigma
 * + tau).  Inside [-1, 1] nothing changes.
 *   s_val:   device double[nnz of P], S values (wvl_sparse_overlap order)
 *   h_val:   device double[nnz of the H pattern], H values
 *   npl:     expansion degree (>= 1); delta: width of the Fermi function
 *            (> 0); n_occ: the target trace, in (0, nsf)
 *   eps_min, eps_max: spectral bounds of H c = eps S c; eps_min >= eps_max
 *            asks for Gershgorin bounds of S^-1/2 H S^-1/2
 *   k_val:   device double[nnz of P], the kernel K
 *   mu, e_bs: host, the chemical potential and the band-structure energy
 *            (either may be NULL)
 *   scratch, scratch_bytes: device buffer and its size: at least
 *            8 ((npl + 7) nnz + 2 npl + 6) bytes keeps every T^i (one
 *            recursion); at least 8 (9 nnz + npl + 5) bytes runs the
 *            recursion twice.  Both give the same values, bit for bit.
 * All arithmetic is in double, sums in fixed orders (bitwise reproducible).
 * Synchronizes (the traces and bounds come back to the host).  Errors:
 * WVL_EINVAL for bad parameters, null buffers, a scratch below the smaller
 * size, or S and H that make H~' not finite; WVL_EUNSUPPORTED when P is
 * not symmetric, not inside the H pattern, lacks a diagonal entry, has a
 * row of more than 1024 entries, or the plan has more than 2^21 functions. */
wvl_status wvl_foe(wvl_plan* plan, const double* s_val, const double* h_val, int32_t npl,
                   double delta, double n_occ, double eps_min, double eps_max, double* k_val,
                   double* mu, double* e_bs, void* scratch, size_t scratch_bytes);

/* Gradient of the support functions, Eq. (gradient) of Sec. IV.A, in the
 * energy mode (band-structure energy Omega = sum_ab K^ab H_ab, K fixed),
 * localized as in Sec. III.A (g_a <- L^a g_a):
 *   g_a = L^a [ sum_d A_ad H|phi_d> - sum_d M_ad |phi_d> ],
 *   A = S K,  M = 1/2 S^-1 (Lambda + Lambda^T),  Lambda = H K S,
 * with S^-1 taken by its first-order Taylor expansion 2 I - S, every matrix on
 * the overlap pattern P (the pattern wvl_sparse_overlap reports with
 * ket_is_output = 0; H read at P's entries; S by its symmetric part), every
 * product truncated to P, and the sums over the functions d of row a of P.
 *   s_val:  device double[nnz of P], S values
 *   h_val:  device double[nnz of the H pattern], H values
 *   k_val:  device double[nnz of P], the density kernel (e.g. from wvl_foe)
 *   psi_c:  device, input layout; hpsi_c: device, output layout (the result
 *           of wvl_apply_local_ham)
 *   g_c:    device, input layout, overwritten with the gradients
 *   scratch, scratch_bytes: device buffer of at least 56 nnz(P) bytes
 * Matrix arithmetic in double; each gradient element summed over its row's
 * functions in CSR order in double and rounded once (rows of more than 256
 * entries: once per 256).  Asynchronous, except that the first call builds
 * the patterns and their maps (synchronizes).  Errors: WVL_EINVAL for null
 * buffers or a small scratch; WVL_EUNSUPPORTED as wvl_foe for patterns it
 * cannot take. */
wvl_status wvl_gradient(wvl_plan* plan, wvl_dtype dt, const double* s_val, const double* h_val,
                        const double* k_val, const void* psi_c, const void* hpsi_c, void* g_c,
                        void* scratch, size_t scratch_bytes);

/* Support-function update step (the localized gradient step of Sec. III.A
 * and IV.A, reduced to a fixed step length):
 *   psi_a <- psi_a - eta (P_La (H psi)_a - H_aa psi_a)
 * for every function a, where P_La keeps the coefficients of H psi on a's
 * input pattern and H_aa is the diagonal entry of row a of the Hamiltonian
 * matrix.  hpsi_c: device, output layout (the result of
 * wvl_apply_local_ham); h_val: device double[nnz], the H values in the CSR
 * order wvl_sparse_overlap(ket_is_output = 1) reports; psi_c: device, input
 * layout, updated in place (arithmetic in double, one rounding per value).
 * Builds the H pattern if needed (synchronizes once).  Errors: WVL_EINVAL for
 * null buffers, a non-finite eta, or a plan whose input pattern is not inside
 * its output pattern. */
wvl_status wvl_update(wvl_plan* plan, wvl_dtype dt, double eta, const void* hpsi_c,
                      const double* h_val, void* psi_c);

/* Preconditioning of support-function gradients (Sec. IV.A, Eq.
 * (precond)): for every function a, approximately solve
 *   (-1/2 nabla^2 + conf[a] |r - R_a|^4 - eps[a]) x_a = -g_a
 * on its localization region (operator restricted to the input pattern on
 * both sides: P_L (T + C) P_L - eps), by `niter` conjugate-gradient steps
 * from x = 0.  eps values above 0 are taken as 0, so that the operator stays
 * positive definite; a function whose residual vanishes stops moving.
 *   g_c:   device, input layout (the localized gradient)
 *   conf:  device double[nsf] confinement prefactors, or NULL (kinetic only)
 *   eps:   device double[nsf] (the approximate Lagrange multipliers)
 *   x_c:   device, input layout, overwritten with the preconditioned gradient
 *   workspace: as for wvl_apply_local_ham
 *   scratch:   device, at least 3 align(in_coefs sz) + align(out_coefs sz)
 *              + 3 align(8 nsf) bytes, align(n) = n rounded up to 256 and
 *              sz the size of the compute type
 * Per-function scalars and dot products are in double, in a fixed order.
 * Errors as wvl_apply_local_ham; WVL_EINVAL for niter < 0 or a plan whose
 * input pattern is not inside its output pattern. */
wvl_status wvl_precondition(wvl_plan* plan, wvl_dtype dt, const void* g_c, const double* conf,
                            const double* eps, int32_t niter, void* x_c, void* workspace,
                            void* scratch);

/* Batching of uneven boxes (Sec. III.B: each function is worked on inside
 * its own localization region only).  A plan sorts the functions by box
 * volume and cuts them into bins; every bin runs each stage as one launch
 * over all its functions.  Without a workspace bound the bins use disjoint
 * workspace regions and are independent.
 *
 * wvl_graph_create captures one step into a HIP graph: the local-H apply of
 * every function (independent bins as parallel branches, on streams the plan
 * owns), then, when s_val / h_val are non-NULL, the overlap values (bra =
 * ket = psi_c) and the Hamiltonian values (bra psi_c, ket hpsi_c) on the
 * plan's patterns, in the CSR order wvl_sparse_overlap reports.  Arguments
 * are those of wvl_apply_local_ham; every buffer must stay valid while the
 * graph lives.  Patterns are built before the capture (this synchronizes).
 * wvl_graph_launch enqueues the graph on the context's stream; results are
 * bitwise identical to the eager calls.  A graph taken before
 * wvl_plan_autotune changed the plan's layout is rejected (WVL_EINVAL).
 * Errors: WVL_EINVAL for bad arguments, WVL_EDEVICE for HIP failures. */
typedef struct wvl_graph wvl_graph;
wvl_status wvl_graph_create(wvl_plan* plan, wvl_dtype dt, uint32_t terms, const void* psi_c,
                            const void* pot, void* hpsi_c, double* e_kin, double* e_pot,
                            void* workspace, double* s_val, double* h_val, wvl_graph** graph);
wvl_status wvl_graph_launch(wvl_graph* graph);
void wvl_graph_destroy(wvl_graph* graph);

/* Autotuner over the plan's schedule: for every bin count in
 * {1, 2, 3, 4, 6, 8} (functions sorted by box volume, cut into that many
 * launches per stage) and both forms of the kinetic term's z part (the
 * register-window stencil on the vector units, or banded-Toeplitz products
 * on the FP64 matrix cores), runs the apply `reps` times (after one warm-up)
 * and keeps the fastest layout.  Buffers as for wvl_apply_local_ham (hpsi_c is overwritten; the
 * workspace is the size wvl_plan_create reported, which covers every
 * candidate).  tried (host, may be NULL) receives up to max_tried points,
 * *ntried the number timed, *best the chosen one.  Synchronous; the plan
 * must not be in use on another stream meanwhile.  A change of bin count
 * alone leaves later results bitwise unchanged; the matrix-core z part sums
 * in another order and agrees with the vector form to the parity
 * tolerances. */
typedef struct {
  int32_t nbins;      /* bins of the size-sorted functions */
  int32_t kin_mfma;   /* 1: z part of the kinetic term on the matrix cores */
  double ms;          /* mean duration of one apply */
} wvl_tune_point;
wvl_status wvl_plan_autotune(wvl_plan* plan, wvl_dtype dt, uint32_t terms, const void* psi_c,
                             const void* pot, void* hpsi_c, void* workspace, int32_t reps,
                             wvl_tune_point* tried, int32_t max_tried, int32_t* ntried,
                             wvl_tune_point* best);

/* Sets the plan's schedule directly (a point wvl_plan_autotune tries): nbins
 * bins of the size-sorted functions, kin_mfma 1 for the z part of the
 * kinetic term on the matrix cores.  Synchronous; graphs captured before are
 * rejected afterwards.  Results agree with every other schedule to the
 * parity tolerances (bitwise for a change of nbins alone).  Errors:
 * WVL_EINVAL for nbins < 1, kin_mfma outside {0, 1}, or a schedule that
 * needs more workspace than the plan reported (bins beyond 8 may). */
wvl_status wvl_plan_set_schedule(wvl_plan* plan, int32_t nbins, int32_t kin_mfma);

/* Kernel tracing.  With profiling enabled, every kernel the context launches
 * is bracketed by two HIP events recorded on the context's stream; times
 * are aggregated per kernel kind.  wvl_profile_read synchronizes the stream,
 * folds pending events into the totals and returns, for kernel kind `id`
 * (0 <= id < wvl_profile_count()), its name, launch count and summed
 * duration in milliseconds.  wvl_profile_reset clears the totals.
 * Errors: WVL_EINVAL for a NULL context or an id out of range. */
wvl_status wvl_profile_enable(wvl_ctx* ctx, int enable);
wvl_status wvl_profile_reset(wvl_ctx* ctx);
int32_t wvl_profile_count(void);
wvl_status wvl_profile_read(wvl_ctx* ctx, int32_t id, const char** name, int64_t* launches,
                            double* total_ms);

#ifdef __cplusplus
}
#endif
#endif /* WVL_H */

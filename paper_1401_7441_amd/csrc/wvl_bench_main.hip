// Native benchmark driver for the library: no Python, no torch, so that
// hardware-counter profilers can attach to it.
//
//   wvl_bench <geometry file> <f32|f64> <steps> <warmup> [copy MiB]
//
// The geometry file holds localization centres and radii (written by the
// seeded input generator); coefficients and the potential are filled with a
// deterministic pattern of the right shape (their values do not change the
// work done).  A step is one local-Hamiltonian apply over every function plus
// the overlap and Hamiltonian matrix values on their resident patterns.  With
// a copy size, one plain device-to-device copy kernel of that size runs first
// (a known-traffic reference for the memory counters).  With WVL_BENCH_FOE
// set to a degree, one Fermi-operator-expansion call on synthetic S and H of
// the step's patterns follows (its kernels then appear in counter runs).
// Prints one JSON line.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/wvl.h"

#define HIPCHECK(x)                                                                   \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess) {                                                           \
      fprintf(stderr, "%s:%d: %s\n", __FILE__, __LINE__, hipGetErrorString(e_));      \
      exit(3);                                                                        \
    }                                                                                 \
  } while (0)
#define WCHECK(ctx, x)                                                                \
  do {                                                                                \
    wvl_status s_ = (x);                                                              \
    if (s_ != WVL_OK) {                                                               \
      fprintf(stderr, "%s:%d: status %d: %s\n", __FILE__, __LINE__, (int)s_,          \
              wvl_last_error(ctx));                                                   \
      exit(4);                                                                        \
    }                                                                                 \
  } while (0)

__global__ void k_copy(const float4* __restrict__ a, float4* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

template <typename T>
static void fill_pattern(std::vector<T>& v, uint64_t seed) {
  uint64_t s = seed * 0x9E3779B97F4A7C15ull + 1;
  for (size_t i = 0; i < v.size(); ++i) {
    s ^= s << 13;
    s ^= s >> 7;
    s ^= s << 17;
    v[i] = (T)(((double)(s >> 11) / 9007199254740992.0 - 0.5) * 0.02);
  }
}

template <typename T>
static int run(const char* path, int steps, int warmup, int copy_mib) {
  FILE* f = fopen(path, "rb");
  if (!f) { fprintf(stderr, "cannot open %s\n", path); return 2; }
  int32_t hdr[6];
  double h;
  if (fread(hdr, 4, 6, f) != 6 || fread(&h, 8, 1, f) != 1) { fprintf(stderr, "bad header\n"); return 2; }
  const int nsf = hdr[0];
  std::vector<double> cen(3 * (size_t)nsf), rad(nsf), frad(nsf);
  if (fread(cen.data(), 8, cen.size(), f) != cen.size() || fread(rad.data(), 8, nsf, f) != (size_t)nsf ||
      fread(frad.data(), 8, nsf, f) != (size_t)nsf) {
    fprintf(stderr, "short geometry file\n");
    return 2;
  }
  fclose(f);
  wvl_grid g{};
  g.h = h;
  g.n[0] = hdr[1]; g.n[1] = hdr[2]; g.n[2] = hdr[3];
  const int ext = hdr[4];

  if (copy_mib > 0) {   // reference copy of known size
    const int64_t n4 = (int64_t)copy_mib * (1 << 20) / 16;
    float4 *a, *b;
    HIPCHECK(hipMalloc(&a, n4 * 16));
    HIPCHECK(hipMalloc(&b, n4 * 16));
    HIPCHECK(hipMemset(a, 0, n4 * 16));
    hipLaunchKernelGGL(k_copy, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, 0, a, b, n4);
    HIPCHECK(hipDeviceSynchronize());
    HIPCHECK(hipFree(a));
    HIPCHECK(hipFree(b));
  }

  std::vector<wvl_locreg> lr(nsf);
  int64_t nsegs = 0;
  WCHECK(nullptr, wvl_build_locregs(&g, nsf, cen.data(), rad.data(), frad.data(), ext, lr.data(),
                                    nullptr, &nsegs));
  std::vector<wvl_seg> segs(nsegs);
  WCHECK(nullptr, wvl_build_locregs(&g, nsf, cen.data(), rad.data(), frad.data(), ext, lr.data(),
                                    segs.data(), &nsegs));
  hipStream_t st;
  HIPCHECK(hipStreamCreate(&st));
  wvl_ctx* ctx = nullptr;
  WCHECK(nullptr, wvl_create(&ctx, &g, st));
  wvl_plan* plan = nullptr;
  size_t wsb = 0;
  WCHECK(ctx, wvl_plan_create(ctx, nsf, lr.data(), segs.data(), nsegs, 0, &plan, &wsb));
  wvl_plan_info info{};
  WCHECK(ctx, wvl_plan_info_get(plan, &info));
  const wvl_dtype dt = sizeof(T) == 8 ? WVL_F64 : WVL_F32;
  const int64_t ws_bytes = sizeof(T) == 8 ? info.workspace_f64 : info.workspace_f32;
  const int64_t nf = (int64_t)(2 * g.n[0] + 29) * (2 * g.n[1] + 29) * (2 * g.n[2] + 29);

  std::vector<T> hpsi(info.in_coefs), hpot(nf);
  fill_pattern(hpsi, 1);
  for (int64_t i = 0; i < nf; ++i) hpot[i] = (T)(-0.5 - 0.25 * std::cos(0.001 * (double)i));
  T *psi, *pot, *out;
  void* ws;
  double *ek, *ep;
  HIPCHECK(hipMalloc(&psi, sizeof(T) * info.in_coefs));
  HIPCHECK(hipMalloc(&pot, sizeof(T) * nf));
  HIPCHECK(hipMalloc(&out, sizeof(T) * std::max<int64_t>(1, info.out_coefs)));
  HIPCHECK(hipMalloc(&ws, ws_bytes));
  HIPCHECK(hipMalloc(&ek, sizeof(double) * nsf));
  HIPCHECK(hipMalloc(&ep, sizeof(double) * nsf));
  HIPCHECK(hipMemcpy(psi, hpsi.data(), sizeof(T) * info.in_coefs, hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(pot, hpot.data(), sizeof(T) * nf, hipMemcpyHostToDevice));

  int64_t nnz_s = 0, nnz_h = 0;
  WCHECK(ctx, wvl_sparse_overlap(plan, psi, 0, psi, dt, &nnz_s, nullptr, nullptr, nullptr));
  WCHECK(ctx, wvl_sparse_overlap(plan, psi, 1, out, dt, &nnz_h, nullptr, nullptr, nullptr));
  int64_t *rs, *rh;
  int32_t *cs, *chh;
  double *vs, *vh;
  HIPCHECK(hipMalloc(&rs, 8 * (nsf + 1)));
  HIPCHECK(hipMalloc(&rh, 8 * (nsf + 1)));
  HIPCHECK(hipMalloc(&cs, 4 * std::max<int64_t>(1, nnz_s)));
  HIPCHECK(hipMalloc(&chh, 4 * std::max<int64_t>(1, nnz_h)));
  HIPCHECK(hipMalloc(&vs, 8 * std::max<int64_t>(1, nnz_s)));
  HIPCHECK(hipMalloc(&vh, 8 * std::max<int64_t>(1, nnz_h)));

  auto step = [&]() {
    WCHECK(ctx, wvl_apply_local_ham(plan, dt, WVL_KIN | WVL_POT, psi, pot, out, ek, ep, ws));
    int64_t n1 = nnz_s, n2 = nnz_h;
    WCHECK(ctx, wvl_sparse_overlap(plan, psi, 0, psi, dt, &n1, rs, cs, vs));
    WCHECK(ctx, wvl_sparse_overlap(plan, psi, 1, out, dt, &n2, rh, chh, vh));
  };
  for (int i = 0; i < warmup; ++i) step();
  HIPCHECK(hipStreamSynchronize(st));
  WCHECK(ctx, wvl_profile_enable(ctx, 1));
  WCHECK(ctx, wvl_profile_reset(ctx));
  const auto t0 = std::chrono::steady_clock::now();
  for (int i = 0; i < steps; ++i) step();
  HIPCHECK(hipStreamSynchronize(st));
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  // with WVL_BENCH_FOE=<npl>: one density kernel by the Fermi operator
  // expansion (after a warm-up call) on synthetic S and H of the step's
  // patterns: S = I + small symmetric terms, H symmetric, half the
  // functions occupied, Gershgorin bounds
  double foe_ms = -1.0, foe_mu = 0.0, foe_ebs = 0.0;
  if (const char* fe = getenv("WVL_BENCH_FOE")) {
    const int npl = atoi(fe);
    std::vector<int64_t> hrs(nsf + 1), hrh(nsf + 1);
    std::vector<int32_t> hcs(nnz_s), hch(nnz_h);
    HIPCHECK(hipMemcpy(hrs.data(), rs, 8 * (nsf + 1), hipMemcpyDeviceToHost));
    HIPCHECK(hipMemcpy(hrh.data(), rh, 8 * (nsf + 1), hipMemcpyDeviceToHost));
    HIPCHECK(hipMemcpy(hcs.data(), cs, 4 * nnz_s, hipMemcpyDeviceToHost));
    HIPCHECK(hipMemcpy(hch.data(), chh, 4 * nnz_h, hipMemcpyDeviceToHost));
    auto sval = [](int a, int b) { return a == b ? 1.0 : 0.01 * std::sin(0.37 * (a + 1) * (b + 1)); };
    auto hval = [](int a, int b) {
      return a == b ? -0.3 + 0.6 * std::sin(0.11 * a) : 0.05 * std::cos(0.23 * (a + 1) * (b + 1));
    };
    std::vector<double> sv(nnz_s), hv(nnz_h);
    for (int a = 0; a < nsf; ++a) {
      for (int64_t q = hrs[a]; q < hrs[a + 1]; ++q) sv[q] = sval(a, hcs[q]);
      for (int64_t q = hrh[a]; q < hrh[a + 1]; ++q) hv[q] = hval(a, hch[q]);
    }
    HIPCHECK(hipMemcpy(vs, sv.data(), 8 * nnz_s, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(vh, hv.data(), 8 * nnz_h, hipMemcpyHostToDevice));
    double* kv;
    void* scr;
    const size_t scr_bytes = 8 * ((size_t)(npl + 7) * nnz_s + 2 * npl + 6);
    HIPCHECK(hipMalloc(&kv, 8 * std::max<int64_t>(1, nnz_s)));
    HIPCHECK(hipMalloc(&scr, scr_bytes));
    WCHECK(ctx, wvl_foe(plan, vs, vh, npl, 1.0, 0.5 * nsf, 1.0, 0.0, kv, &foe_mu, &foe_ebs, scr,
                        scr_bytes));
    const auto f0 = std::chrono::steady_clock::now();
    WCHECK(ctx, wvl_foe(plan, vs, vh, npl, 1.0, 0.5 * nsf, 1.0, 0.0, kv, &foe_mu, &foe_ebs, scr,
                        scr_bytes));
    foe_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - f0).count();
    HIPCHECK(hipFree(kv));
    HIPCHECK(hipFree(scr));
  }
  printf("{\"driver\": \"wvl_bench\", \"nsf\": %d, \"dtype\": \"%s\", \"steps\": %d, \"ms_per_step\": %.4f, "
         "\"s_nnz\": %lld, \"h_nnz\": %lld, \"foe_ms\": %.4f, \"foe_mu\": %.6f, \"kernels\": {",
         nsf, sizeof(T) == 8 ? "f64" : "f32", steps, ms / std::max(1, steps), (long long)nnz_s,
         (long long)nnz_h, foe_ms, foe_mu);
  bool first = true;
  for (int k = 0; k < wvl_profile_count(); ++k) {
    const char* name;
    int64_t n;
    double tot;
    WCHECK(ctx, wvl_profile_read(ctx, k, &name, &n, &tot));
    if (!n) continue;
    printf("%s\"%s\": {\"launches\": %lld, \"avg_ms\": %.5f}", first ? "" : ", ", name, (long long)n,
           tot / n);
    first = false;
  }
  printf("}}\n");
  fflush(stdout);
  wvl_plan_destroy(plan);
  wvl_destroy(ctx);
  HIPCHECK(hipStreamDestroy(st));
  for (void* p : {(void*)psi, (void*)pot, (void*)out, ws, (void*)ek, (void*)ep, (void*)rs, (void*)rh,
                  (void*)cs, (void*)chh, (void*)vs, (void*)vh})
    HIPCHECK(hipFree(p));
  return 0;
}

int main(int argc, char** argv) {
  if (argc < 5) {
    fprintf(stderr, "usage: %s <geometry file> <f32|f64> <steps> <warmup> [copy MiB]\n", argv[0]);
    return 2;
  }
  const std::string dt = argv[2];
  const int steps = atoi(argv[3]), warmup = atoi(argv[4]);
  const int copy = argc > 5 ? atoi(argv[5]) : 0;
  if (dt == "f32") return run<float>(argv[1], steps, warmup, copy);
  if (dt == "f64") return run<double>(argv[1], steps, warmup, copy);
  fprintf(stderr, "dtype must be f32 or f64\n");
  return 2;
}

// Host driver: context set-up, multigrid hierarchy (Sec. 5.1), V-cycle, PCG
// (Sec. 5.2) and the interior-point step (Sec. 3).  All arithmetic runs in the
// kernels; the host only sequences launches and reads scalars.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "ctx.h"
#include "kernels.h"
#include "vec.h"
#include "dense.h"

namespace ipmg {

namespace {

template <typename P>
void dalloc(P*& p, size_t bytes) {
  void* q = nullptr;
  if (hipMalloc(&q, bytes ? bytes : 8) != hipSuccess) throw Error(IPMG_E_NOMEM, "device allocation failed");
  p = (P*)q;
}
template <typename P>
void dfree(P*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

// Safeguard of the Jacobi damping on every level except the coarsest:
// omega_k = min(omega, SAFE_PRODUCT / rho_k), rho_k the Rayleigh-quotient estimate of
// the largest eigenvalue of D_k^-1 A_k after POWER_STEPS power iterations.  Damped
// Jacobi diverges once omega * rho >= 2, which happens for omega = 0.6 on 3D
// elasticity and on the augmented system Z late in the interior-point run.
constexpr double SAFE_PRODUCT = 1.6;
constexpr int POWER_STEPS = 12;
// The augmented system Z: the top of the spectrum of D^-1 Z late in a 3D
// interior-point run is a cluster of element-local modes of the rank-one terms,
// which power iteration approaches slowly from below (12 steps: rho = 6.2 where
// it is about 7.9, so omega * rho > 2 and PCG broke down).
constexpr int POWER_STEPS_Z = 30;
// After a breakdown of a Newton-system solve (the V-cycle was not positive definite:
// omega * rho reached 2 because the estimate of rho came out too low), the damping
// of every level is estimated again with four times the power steps and the
// smaller product 1.2, and the solve continues from its last iterate.
constexpr int RETRY_POWER_FACTOR = 4;
constexpr double SAFE_PRODUCT_RETRY = 1.2;

// Scratch of ipmg_pcg_noalloc: the PCG work vectors and the reduction arrays of a
// solve, for callers that cannot allocate device memory.  Each GPU the library runs
// on holds its own copy until the process ends; host code reaches it only through
// the address hipGetSymbolAddress returns for that device (scratch_address).
static __device__ __align__(256) unsigned char scratch[IPMG_NOALLOC_SCRATCH_BYTES];

// Device address of this device's copy of `scratch`, looked up once per device with
// that device current (the array's name is only a host-side stand-in).
unsigned char* scratch_address() {
  static std::mutex mu;
  static unsigned char* addr[64] = {nullptr};
  int dev = 0;
  IPMG_HIP(hipGetDevice(&dev));
  IPMG_REQUIRE(dev >= 0 && dev < 64, IPMG_E_INVALID, "device index out of range");
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    IPMG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    addr[dev] = (unsigned char*)p;
  }
  return addr[dev];
}

}  // namespace

void sync(Ctx& c) { IPMG_HIP(hipStreamSynchronize(c.stream)); }

void read_scalars(Ctx& c) {
  IPMG_HIP(hipMemcpyAsync(c.hscal, c.red.scal, sizeof(double) * S_COUNT, hipMemcpyDeviceToHost, c.stream));
  IPMG_HIP(hipMemcpyAsync(c.hflags, c.red.flags, sizeof(int) * F_COUNT, hipMemcpyDeviceToHost, c.stream));
  sync(c);
}

static void ensure_z_buffers(Ctx& c) {
  if (c.h64) return;
  const Dims& d = c.fine();
  const size_t m = (size_t)d.m, n1 = (size_t)d.nslots + 1;
  dalloc(c.h64, sizeof(double) * c.nd * m);
  if (c.fp32) dalloc(c.hT, sizeof(float) * c.nd * m);
  else c.hT = c.h64;
  dalloc(c.hsbuf, sizeof(double) * m);   // h_e'v_e of the operator pass in flight
  dalloc(c.bZ64, sizeof(double) * n1);
  if (c.fp32) dalloc(c.lev[c.L - 1].bZ, sizeof(float) * n1);
  else c.lev[c.L - 1].bZ = c.bZ64;
  c.lev[c.L - 1].bZ64 = c.bZ64;
  for (int k = 0; k < c.L - 1; ++k) {
    const size_t nk = (size_t)c.lev[k].d.nslots + 1;
    dalloc(c.lev[k].bZ64, sizeof(double) * nk);
    if (c.fp32) dalloc(c.lev[k].bZ, sizeof(float) * nk);
    else c.lev[k].bZ = c.lev[k].bZ64;
  }
  dalloc(c.ipG3, sizeof(double) * m);
  dalloc(c.ipW, sizeof(double) * m);
  dalloc(c.ipSW, sizeof(double) * m);
  dalloc(c.ipDx, sizeof(double) * m);
  dalloc(c.ipDphi, sizeof(double) * m);
  dalloc(c.ipDpsi, sizeof(double) * m);
  dalloc(c.ipRhs, sizeof(double) * n1);
  dalloc(c.ipD, sizeof(double) * n1);
  dalloc(c.ipKu, sizeof(double) * n1);
}

void ctx_init(Ctx& c, const ipmg_desc& d, hipStream_t st) {
  IPMG_REQUIRE(d.dim == 2 || d.dim == 3, IPMG_E_INVALID, "dim must be 2 or 3");
  IPMG_REQUIRE(d.levels >= 1 && d.levels <= 16, IPMG_E_INVALID, "levels must be in [1, 16]");
  IPMG_REQUIRE(d.nu_pre >= 1 && d.nu_post >= 0 && d.nu_pre <= 64 && d.nu_post <= 64, IPMG_E_INVALID,
               "sweeps: need 1 <= nu_pre <= 64, 0 <= nu_post <= 64");
  IPMG_REQUIRE(d.omega > 0.0 && d.omega < 2.0, IPMG_E_INVALID, "omega must be in (0, 2)");
  IPMG_REQUIRE(d.pcg_flexible == 0 || d.pcg_flexible == 1, IPMG_E_INVALID, "pcg_flexible must be 0 or 1");
  IPMG_REQUIRE(d.E > 0.0 && d.nu > -1.0 && d.nu < 0.5, IPMG_E_INVALID, "material: E > 0, -1 < nu < 0.5");
  const int f = 1 << (d.levels - 1);
  for (int a = 0; a < d.dim; ++a) {
    IPMG_REQUIRE(d.nel[a] >= 1 && d.nel[a] <= (1 << 16), IPMG_E_INVALID, "element counts must be in [1, 65536]");
    IPMG_REQUIRE(d.nel[a] % f == 0, IPMG_E_INVALID, "element counts must be divisible by 2^(levels-1)");
  }
  c.desc = d;
  {
    int dev = 0;
    IPMG_HIP(hipGetDevice(&dev));
    IPMG_HIP(hipDeviceGetAttribute(&c.cus, hipDeviceAttributeMultiprocessorCount, dev));
  }
  c.dim = d.dim;
  c.fp32 = d.vcycle_fp32 != 0;
  c.tsz = c.fp32 ? sizeof(float) : sizeof(double);
  c.L = d.levels;
  c.stream = st;
  c.nd = d.dim * (1 << d.dim);
  c.ops = d.dim == 2 ? make_ops2d() : make_ops3d();
  c.lev.resize(c.L);
  for (int k = 0; k < c.L; ++k) {
    const int s = 1 << (c.L - 1 - k);
    c.lev[k].d = make_dims(d.dim, d.nel[0] / s, d.nel[1] / s, d.dim == 3 ? d.nel[2] / s : 1);
  }
  const Dims& fd = c.fine();
  IPMG_REQUIRE(fd.nslots < ((int64_t)1 << 31), IPMG_E_INVALID, "grid too large");
  if (const char* e = std::getenv("IPMG_STORED_COARSE")) c.coarse_from_x = e[0] != '1';
  if (const char* e = std::getenv("IPMG_UNTILED")) c.tiled2d = e[0] != '1';
  if (const char* e = std::getenv("IPMG_UNFUSED")) c.fused2d = e[0] != '1';
  if (const char* e = std::getenv("IPMG_UNSTAGED")) c.fused_staged = e[0] != '1';
  if (const char* e = std::getenv("IPMG_STAGED_MAX_NODES")) c.staged_max_nodes = std::max<int64_t>(0, std::atoll(e));
  if (const char* e = std::getenv("IPMG_NO_FOLD_PROLONG")) c.fold_prolong = e[0] != '1';
  if (const char* e = std::getenv("IPMG_NO_FOLD_SOLUTION")) c.fold_solution = e[0] != '1';
  if (const char* e = std::getenv("IPMG_NO_FOLD_RN2")) c.fold_rn2_fin = e[0] != '1';
  if (const char* e = std::getenv("IPMG_NO_FOLD_RESTRICT")) c.fold_restrict = e[0] != '1';
  if (const char* e = std::getenv("IPMG_NO_ELEM_HV")) c.elem_hv = e[0] != '1';
  if (const char* e = std::getenv("IPMG_NO_ELEM_APPLY3")) c.elem_apply3 = e[0] != '1';
  if (const char* e = std::getenv("IPMG_ELEM_APPLY3_MIN")) c.elem_apply3_min = std::max<int64_t>(0, std::atoll(e));
  if (const char* e = std::getenv("IPMG_NO_ELEM_FINE3")) c.elem_fine3 = e[0] != '1';
  if (const char* e = std::getenv("IPMG_NO_MFMA")) c.mfma = e[0] != '1';
  if (const char* e = std::getenv("IPMG_NO_LANE_SHARE")) c.lane_share = e[0] != '1';
  if (const char* e = std::getenv("IPMG_NO_JACOBI2_RESID")) c.fuse_resid = e[0] != '1';
  if (const char* e = std::getenv("IPMG_NO_PJACOBI2")) c.fuse_post = e[0] != '1';
  if (const char* e = std::getenv("IPMG_NJ32")) c.nj32 = std::atoi(e);
  if (const char* e = std::getenv("IPMG_NJ64")) c.nj64 = std::atoi(e);
  if (const char* e = std::getenv("IPMG_NJ_DIR")) c.nj_dir = std::atoi(e);
  c.power_steps = POWER_STEPS;
  c.power_steps_z = POWER_STEPS_Z;
  if (const char* e = std::getenv("IPMG_TILED_MIN_NODES")) c.tiled_min_nodes = std::max<int64_t>(0, std::atoll(e));
  c.ncoarse = (int)std::min<int64_t>(c.lev[0].d.nslots + 1, (int64_t)1 << 30);

  // reductions
  dalloc(c.red.partials, sizeof(double) * 8 * MAX_PARTIALS);
  dalloc(c.red.counter, sizeof(unsigned) * C_COUNT);
  dalloc(c.red.scal, sizeof(double) * S_COUNT);
  dalloc(c.red.flags, sizeof(int) * F_COUNT);
  IPMG_HIP(hipMemsetAsync(c.red.counter, 0, sizeof(unsigned) * C_COUNT, st));
  IPMG_HIP(hipMemsetAsync(c.red.scal, 0, sizeof(double) * S_COUNT, st));
  IPMG_HIP(hipMemsetAsync(c.red.flags, 0, sizeof(int) * F_COUNT, st));
  if (hipHostMalloc((void**)&c.hscal, sizeof(double) * S_COUNT, hipHostMallocDefault) != hipSuccess)
    throw Error(IPMG_E_NOMEM, "pinned allocation failed");
  // coherent: kernels write PCG flags into it directly
  if (hipHostMalloc((void**)&c.hflags, sizeof(int) * F_COUNT * 4, hipHostMallocCoherent) != hipSuccess)
    throw Error(IPMG_E_NOMEM, "pinned allocation failed");
  IPMG_HIP(hipEventCreate(&c.ev0));
  IPMG_HIP(hipEventCreate(&c.ev1));
  c.noalloc_scratch = scratch_address();

  // level vectors
  const int nsym = c.nd * (c.nd + 1) / 2;
  for (int k = 0; k < c.L; ++k) {
    Level& l = c.lev[k];
    const size_t n1 = (size_t)l.d.nslots + 1;
    dalloc(l.r, c.tsz * n1);
    dalloc(l.z, c.tsz * n1);
    dalloc(l.z2, c.tsz * n1);
    dalloc(l.t, c.tsz * n1);
    IPMG_HIP(hipMemsetAsync(l.z, 0, c.tsz * n1, st));
    IPMG_HIP(hipMemsetAsync(l.z2, 0, c.tsz * n1, st));
    if (k < c.L - 1) {
      dalloc(l.E64, sizeof(double) * (size_t)nsym * (size_t)l.d.m);
      if (c.fp32) dalloc(l.E, sizeof(float) * (size_t)nsym * (size_t)l.d.m);
      else l.E = l.E64;
    }
  }
  // Densities, followed by a zero pad of nx + 2 entries: kernels read an element
  // outside the grid (or a 2 x 2 block of them) there instead of branching.
  const int64_t xn = fd.m + fd.nx + 2;
  dalloc(c.x64, sizeof(double) * xn);
  IPMG_HIP(hipMemsetAsync(c.x64, 0, sizeof(double) * xn, st));
  if (c.fp32) {
    dalloc(c.xT, sizeof(float) * xn);
    IPMG_HIP(hipMemsetAsync(c.xT, 0, sizeof(float) * xn, st));
  } else {
    c.xT = c.x64;
  }
  const size_t n1 = (size_t)fd.nslots + 1;
  dalloc(c.pr, sizeof(double) * n1);
  dalloc(c.pp, sizeof(double) * n1);
  dalloc(c.pq, sizeof(double) * n1);
  dalloc(c.pt, sizeof(double) * n1);
  dalloc(c.pb, sizeof(double) * n1);
  dalloc(c.pu, sizeof(double) * n1);
  dalloc(c.pp2, sizeof(double) * n1);
  vfill(st, c.pp, 0.0, (int64_t)n1);    // the direction kernel reads p_old (times 0) on the first iteration
  vfill(st, c.pp2, 0.0, (int64_t)n1);
  dalloc(c.omega_dev, sizeof(double) * 2 * c.L);
  dalloc(c.oc_cand, sizeof(double) * OC_CAND);
  if (d.dim == 3 && c.L >= 2 && c.elem_apply3) dalloc(c.ye, c.tsz * 24 * (size_t)c.lev[c.L - 2].d.m);
  if (d.dim == 3 && c.elem_fine3) {
    dalloc(c.fine_ye64, sizeof(double) * 24 * (size_t)fd.m);
    if (c.fp32) dalloc(c.fine_ye, sizeof(float) * 24 * (size_t)fd.m);
    else c.fine_ye = c.fine_ye64;
    dalloc(c.fine_dg, c.tsz * (size_t)fd.nslots);
  }
  vfill_small(st, c.omega_dev, c.L, d.omega);

  // element matrix on the GPU, mirrored to the host and to constant memory
  double* dK0 = nullptr;
  dalloc(dK0, sizeof(double) * c.nd * c.nd);
  c.ops->element_stiffness(c, dK0);
  IPMG_HIP(hipGetLastError());
  IPMG_HIP(hipMemcpyAsync(c.K0, dK0, sizeof(double) * c.nd * c.nd, hipMemcpyDeviceToHost, st));
  sync(c);
  dfree(dK0);
  c.ops->upload_k0(c.K0);
}

void ctx_free(Ctx& c) {
  if (c.stream) (void)hipStreamSynchronize(c.stream);
  for (auto& l : c.lev) {
    dfree(l.r); dfree(l.z); dfree(l.z2); dfree(l.t);
    if (l.E != (void*)l.E64) dfree(l.E);
    l.E = nullptr;
    dfree(l.E64);
    if (l.bZ != (void*)l.bZ64 && l.bZ != (void*)c.bZ64) dfree(l.bZ);
    l.bZ = nullptr;
    if (l.bZ64 != c.bZ64) dfree(l.bZ64);
    l.bZ64 = nullptr;
  }
  if (c.xT != (void*)c.x64) dfree(c.xT);
  c.xT = nullptr;
  if (c.hT != (void*)c.h64) dfree(c.hT);
  c.hT = nullptr;
  dfree(c.x64); dfree(c.h64); dfree(c.bZ64); dfree(c.hsbuf);
  dfree(c.pr); dfree(c.pp); dfree(c.pq); dfree(c.pt); dfree(c.pb); dfree(c.pu); dfree(c.pp2);
  dfree(c.dA); dfree(c.dLi); dfree(c.dAi); dfree(c.dAif); dfree(c.dpart); dfree(c.omega_dev);
  dfree(c.red.partials); dfree(c.red.counter); dfree(c.red.scal); dfree(c.red.flags);
  dfree(c.ipG3); dfree(c.ipW); dfree(c.ipSW); dfree(c.ipDx); dfree(c.ipDphi); dfree(c.ipDpsi);
  dfree(c.ipRhs); dfree(c.ipD); dfree(c.ipKu);
  dfree(c.oc_t); dfree(c.oc_cand); dfree(c.ye); dfree(c.simp_xt); dfree(c.simp_xp);
  for (double** b : {&c.simp_cf, &c.simp_g, &c.simp_E, &c.simp_a, &c.simp_t, &c.simp_b1, &c.simp_b2, &c.simp_b3,
                     &c.simp_bcoef, &c.simp_rcoef, &c.simp_r, &c.simp_y, &c.simp_p, &c.simp_q})
    dfree(*b);
  if (c.fine_ye != (void*)c.fine_ye64) dfree(c.fine_ye);
  c.fine_ye = nullptr;
  dfree(c.fine_ye64); dfree(c.fine_dg);
  if (c.hscal) (void)hipHostFree(c.hscal);
  if (c.hflags) (void)hipHostFree(c.hflags);
  c.hscal = nullptr; c.hflags = nullptr;
  for (auto e : c.prof_ev) (void)hipEventDestroy(e);
  c.prof_ev.clear();
  c.prof_cls.clear();
  if (c.ev0) (void)hipEventDestroy(c.ev0);
  if (c.ev1) (void)hipEventDestroy(c.ev1);
  c.ev0 = c.ev1 = nullptr;
  delete c.ops;
  c.ops = nullptr;
}

void set_density(Ctx& c, const double* x) {
  const Dims& d = c.fine();
  IPMG_HIP(hipMemsetAsync(c.red.flags + F_BAD, 0, sizeof(int), c.stream));
  vcopy_positive(c.stream, x, c.x64, d.m, c.red);
  if (c.fp32) vconvert<float, double>(c.stream, c.x64, (float*)c.xT, d.m, nullptr);
  read_scalars(c);
  if (c.hflags[F_BAD]) {
    c.have_x = false;
    throw Error(IPMG_E_DOMAIN, "densities must be finite and positive");
  }
  c.have_x = true;
  c.hier_op = -1;
}

// Damping of level k from the spectral-radius estimate of D^-1 A (power iteration
// with the normalisation folded into the next step, then the Rayleigh quotient);
// everything stays on the device.
static void jacobi_damping(Ctx& c, int k, int op, int steps, double product) {
  Level& l = c.lev[k];
  const int aug = op == IPMG_OP_Z;
  c.ops->power_start(c, k, aug, l.z);
  void* v = l.z;
  void* w = l.z2;
  int sin = -1, sout = S_TMP4;
  for (int it = 0; it < steps; ++it) {
    c.ops->level(c, k, op, M_POWER, v, nullptr, w, nullptr, sout, sin, nullptr);
    std::swap(v, w);
    sin = sout;
    sout = sout == S_TMP4 ? S_TMP5 : S_TMP4;
  }
  c.ops->level(c, k, op, M_RAYLEIGH, v, nullptr, nullptr, nullptr, S_TMP6, -1, nullptr);
  vset_omega(c.stream, c.red, c.omega_dev + k, c.omega_dev + c.L + k, S_TMP6, S_TMP7, c.desc.omega, product);
}

static void ensure_dense(Ctx& c) {
  if (c.dA) return;
  const int64_t n = c.lev[0].d.nslots + 1;
  IPMG_REQUIRE(n <= DENSE_MAX_N, IPMG_E_INVALID, "coarsest level too large for the dense solve; use more levels");
  const int64_t np = dense_packed_size((int)n), nt = dense_tiles((int)n);
  dalloc(c.dA, sizeof(double) * np);
  dalloc(c.dLi, sizeof(double) * np);
  dalloc(c.dAi, sizeof(double) * np);
  if (c.fp32) dalloc(c.dAif, sizeof(float) * np);
  dalloc(c.dpart, sizeof(double) * nt * nt * DT);
}

void mg_setup(Ctx& c, int op, double* ms) {
  IPMG_REQUIRE(c.have_x, IPMG_E_STATE, "set the densities first");
  IPMG_REQUIRE(op == IPMG_OP_K || c.have_z, IPMG_E_STATE, "prepare the Newton system first");
  auto t0 = std::chrono::steady_clock::now();
  const int L = c.L;
  if (op == IPMG_OP_Z && c.fp32)
    vconvert<float, double>(c.stream, c.bZ64, (float*)c.lev[L - 1].bZ, c.fine().nslots, nullptr);
  const int nsym = c.nd * (c.nd + 1) / 2;
  for (int k = L - 1; k >= 1; --k) {
    Level& lc = c.lev[k - 1];
    c.ops->galerkin(c, k, op);                       // FP64 chain
    if (c.fp32) vconvert<float, double>(c.stream, lc.E64, (float*)lc.E, (int64_t)nsym * lc.d.m, nullptr);
    if (op == IPMG_OP_Z) {
      c.ops->restrict64(c, k, c.lev[k].bZ64, lc.bZ64);
      if (c.fp32) vconvert<float, double>(c.stream, lc.bZ64, (float*)lc.bZ, lc.d.nslots, nullptr);
    }
  }
  IPMG_HIP(hipGetLastError());
  ensure_dense(c);
  c.ops->fine_diag(c, op);
  const int steps = op == IPMG_OP_Z ? c.power_steps_z : c.power_steps;
  for (int k = 1; k < L; ++k) jacobi_damping(c, k, op, steps, SAFE_PRODUCT);
  const int n = c.lev[0].d.nslots + (op == IPMG_OP_Z ? 1 : 0);
  IPMG_HIP(hipMemsetAsync(c.red.flags + F_BAD, 0, sizeof(int), c.stream));
  dense_init(c.stream, c.dA, n, 1);
  c.ops->dense_assemble(c, op, c.dA, n);
  dense_factor_inverse(c.stream, c.dA, c.dLi, c.dAi, n, c.red, c.dAif);
  IPMG_HIP(hipGetLastError());
  read_scalars(c);
  IPMG_REQUIRE(!c.hflags[F_BAD], IPMG_E_BREAKDOWN, "coarsest operator is not positive definite");
  c.hier_op = op;
  auto t1 = std::chrono::steady_clock::now();
  if (ms) *ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
}

// V-cycle on level k: lev[k].r -> returned buffer (Algorithm MG, zero start).
// beta64 (finest level only): if not null, the last post-smoothing sweep also
// forms beta = beta64'y / rho of Algorithm PCG on the device.
// A ||r||^2 finalize left pending by pcg_iteration (c.rn2_fin_blocks) is done by
// the finest level's fused first two sweeps, else here before the first kernel.
static void rn2_fin_flush(Ctx& c, const int* gate) {
  if (!c.rn2_fin_blocks) return;
  vpcg_update_fin_nb(c.stream, c.rn2_fin_blocks, c.red, gate, c.rn2_fin_zpend);
  c.rn2_fin_blocks = 0;
}

static void* vcycle_level(Ctx& c, int op, int k, const int* gate, const double* beta64) {
  Level& l = c.lev[k];
  const int aug = op == IPMG_OP_Z;
  if (c.rn2_fin_blocks && (k == 0 || c.ops->fused_applies(c, k, op) || c.desc.nu_pre < 2)) rn2_fin_flush(c, gate);
  if (k == 0) {
    const int n = l.d.nslots + aug;
    if (c.fp32) dense_apply<float, float>(c.stream, c.dAif, c.dpart, n, (const float*)l.r, (float*)l.z, gate);
    else dense_apply<double, double>(c.stream, c.dAi, c.dpart, n, (const double*)l.r, (double*)l.z, gate);
    return l.z;
  }
  if (c.ops->fused_applies(c, k, op)) {
    c.ops->fused_down(c, k, gate);                                            // two sweeps, residual, P'
    void* vc = vcycle_level(c, op, k - 1, gate, nullptr);
    c.ops->fused_up(c, k, vc, l.z2, gate);                                    // P, two sweeps
    return l.z2;
  }
  void* cur = l.z;
  void* nxt = l.z2;
  const double* w = c.omega_dev + k;
  const bool fine = k == c.L - 1;
  const int jac = fine ? PC_FINE_JACOBI : (k == c.L - 2 ? PC_SUB_JACOBI : -1);
  int pre = 0;
  bool resid_done = false;
  if (c.desc.nu_pre >= 2) {                   // the first two sweeps in one pass (z1 not stored)
    ProfTag pt(c, fine ? PC_FINE_JACOBI2 : -1);
    if (c.desc.nu_pre == 2 && c.ops->jacobi2_resid(c, k, op, l.r, nxt, l.t, w, gate)) {
      std::swap(cur, nxt);                    // ... and the residual of their result
      pre = 2;
      resid_done = true;
    } else if (c.ops->jacobi2(c, k, op, l.r, nxt, w, gate)) {
      std::swap(cur, nxt);
      pre = 2;
    }
  }
  rn2_fin_flush(c, gate);
  if (pre == 0) {
    ProfTag pt(c, fine ? PC_FINE_JACOBI0 : -1);
    c.ops->level(c, k, op, M_JACOBI0, nullptr, l.r, cur, w, 0, -1, gate);     // pre-smoothing
    pre = 1;
  }
  for (int s = pre; s < c.desc.nu_pre; ++s) {
    ProfTag pt(c, jac);
    c.ops->level(c, k, op, M_JACOBI, cur, l.r, nxt, w, 0, -1, gate);
    std::swap(cur, nxt);
  }
  if (!resid_done) {
    ProfTag pt(c, fine ? PC_FINE_RESID : -1);
    c.ops->level(c, k, op, M_RESID, cur, l.r, l.t, nullptr, 0, -1, gate);     // restricted residual
  }
  if (c.ops->down_restricts(c, k - 1, op)) c.down_from_t = l.t;             // restricted in the next pass
  else c.ops->restrict_to(c, k, l.t, c.lev[k - 1].r, aug, gate);
  void* vc = vcycle_level(c, op, k - 1, gate, nullptr);                       // coarse correction
  IPMG_REQUIRE(!c.down_from_t, IPMG_E_STATE, "restriction left pending");
  int s0 = 0;
  if (c.desc.nu_post >= 2) {                  // solution update folded into the first post-sweep
    ProfTag pt(c, fine ? PC_FINE_PJACOBI : jac);
    if (c.desc.nu_post == 2 && c.ops->prolong_jacobi2(c, k, op, cur, vc, l.r, nxt, w, gate, beta64)) {
      std::swap(cur, nxt);                    // ... and into both post-sweeps
      s0 = 2;
    } else if (c.ops->prolong_jacobi(c, k, op, cur, vc, l.r, nxt, w, gate)) {
      std::swap(cur, nxt);
      s0 = 1;
    }
  }
  if (s0 == 0) c.ops->prolong_from(c, k, cur, vc, aug, gate);                 // solution update
  for (int s = s0; s < c.desc.nu_post; ++s) {                                 // post-smoothing
    const bool last = beta64 && s == c.desc.nu_post - 1;
    ProfTag pt(c, last ? (fine ? PC_FINE_JACOBI_BETA : -1) : jac);
    c.ops->level(c, k, op, last ? M_JACOBI_BETA : M_JACOBI, cur, l.r, nxt, w, 0, -1, gate, last ? beta64 : nullptr);
    std::swap(cur, nxt);
  }
  return cur;
}

// Work a previous call left pending when it stopped on an error is dropped.
static void clear_pending(Ctx& c) {
  c.rn2_fin_blocks = 0;
  c.down_from_t = nullptr;
}

void* vcycle(Ctx& c, int op, const int* gate) {
  clear_pending(c);
  return vcycle_level(c, op, c.L - 1, gate, nullptr);
}

void vcycle64(Ctx& c, int op, const double* r, double* z) {
  IPMG_REQUIRE(c.hier_op == op, IPMG_E_STATE, "multigrid hierarchy not set up for this operator");
  const Dims& d = c.fine();
  const int64_t n = d.nslots + (op == IPMG_OP_Z ? 1 : 0);
  vmask_copy(c.stream, r, c.pt, n, d.nslots, c.dim, d.nx1, c.red, S_TMP0);
  if (c.fp32) vconvert<float, double>(c.stream, c.pt, (float*)c.lev[c.L - 1].r, n, nullptr);
  else vconvert<double, double>(c.stream, c.pt, (double*)c.lev[c.L - 1].r, n, nullptr);
  void* y = vcycle(c, op, nullptr);
  if (c.fp32) vconvert<double, float>(c.stream, (const float*)y, z, n, nullptr);
  else vconvert<double, double>(c.stream, (const double*)y, z, n, nullptr);
  IPMG_HIP(hipGetLastError());
  sync(c);
}

// Enqueue one PCG iteration (all kernels gated on flags[F_DONE]):
//   p = -y + beta p, q = A p, alpha      (one fused kernel)
//   z += alpha p, r += alpha q, ||r||^2  (one fused kernel, sets the done flag)
//   y = M r with beta = r'y / rho fused into the last smoothing sweep.
// `first` selects beta = 0 (first step after a (re)start).
// With the fold, z += alpha p of a step is done by the next step's direction
// kernel (which reads that p anyway) and, for the last step, by vzflush.
static void pcg_iteration(Ctx& c, int op, int64_t n, const int* gate, int first) {
  const bool fold = c.ops->dir_folds_solution(c);
  c.ops->dir_apply(c, op, c.yT, c.pp, c.pp2, c.pq, first, gate, fold ? c.pu : nullptr);
  std::swap(c.pp, c.pp2);                                               // c.pp holds the new p
  void* rT = c.lev[c.L - 1].r;
  double* z = fold ? nullptr : c.pu;
  {
    ProfScope ps(c, PC_PCG_UPDATE);
    if (c.fp32)
      vpcg_update<float>(c.stream, z, c.pr, c.pp, c.pq, (float*)rT, n, c.red, gate);
    else
      vpcg_update<double>(c.stream, z, c.pr, c.pp, c.pq, (double*)rT, n, c.red, gate);
  }
  if (c.fold_rn2_fin) {                   // finalized by the V-cycle's first pass
    c.rn2_fin_blocks = vpcg_update_blocks(n);
    c.rn2_fin_zpend = fold;
  } else {
    vpcg_update_fin(c.stream, n, c.red, gate, fold);
  }
  // the finest level's last post-smoothing sweep forms beta (no sweep on a one-level
  // hierarchy: the coarsest solve is the whole V-cycle)
  const bool fused_beta = c.desc.nu_post >= 1 && c.L > 1;
  void* y = vcycle_level(c, op, c.L - 1, gate, fused_beta ? c.pr : nullptr);
  if (!fused_beta) {
    if (c.fp32) vdot_beta<float>(c.stream, c.pr, (const float*)y, n, c.red, gate);
    else vdot_beta<double>(c.stream, c.pr, (const double*)y, n, c.red, gate);
  }
  c.yT = y;
}

// r (in c.pr) -> y = M r and rho = r'y; the next iteration starts with p = -y.
static void pcg_restart_direction(Ctx& c, int op, int64_t n) {
  const int* gate = c.red.flags + F_DONE;
  void* rT = c.lev[c.L - 1].r;
  if (c.fp32) vconvert<float, double>(c.stream, c.pr, (float*)rT, n, nullptr);
  else vconvert<double, double>(c.stream, c.pr, (double*)rT, n, nullptr);
  void* y = vcycle(c, op, gate);
  if (c.fp32) vdot_store<float>(c.stream, c.pr, (const float*)y, n, c.red, S_TMP0, gate);
  else vdot_store<double>(c.stream, c.pr, (const double*)y, n, c.red, S_TMP0, gate);
  vset_rho(c.stream, c.red, S_TMP0);
  c.yT = y;
}

int pcg(Ctx& c, int op, const double* b, double* u, double rtol, int maxit, ipmg_pcg_info* info) {
  clear_pending(c);
  IPMG_REQUIRE(rtol > 0.0 && maxit >= 0, IPMG_E_INVALID, "rtol > 0 and maxit >= 0 required");
  IPMG_REQUIRE(c.have_x, IPMG_E_STATE, "set the densities first");
  double setup_ms = 0.0;
  if (c.hier_op != op) mg_setup(c, op, &setup_ms);
  auto t0 = std::chrono::steady_clock::now();
  const Dims& d = c.fine();
  const int64_t n = d.nslots + (op == IPMG_OP_Z ? 1 : 0);
  const int* gate = c.red.flags + F_DONE;
  IPMG_HIP(hipMemsetAsync(c.red.flags, 0, sizeof(int) * F_COUNT, c.stream));
  vmask_copy(c.stream, b, c.pb, n, d.nslots, c.dim, d.nx1, c.red, S_BN2);
  vmask_copy(c.stream, u, c.pu, n, d.nslots, c.dim, d.nx1, c.red, S_TMP1);
  read_scalars(c);
  IPMG_REQUIRE(!c.hflags[F_BAD], IPMG_E_DOMAIN, "right-hand side or initial guess is not finite");
  const double bn2 = c.hscal[S_BN2];
  ipmg_pcg_info inf{};
  inf.setup_ms = setup_ms;
  if (bn2 == 0.0) {
    IPMG_HIP(hipMemsetAsync(u, 0, sizeof(double) * n, c.stream));
    sync(c);
    if (info) *info = inf;
    return IPMG_OK;
  }
  // r = A u - b
  c.ops->fine_apply64(c, op, c.pu, c.pq, nullptr);
  vsub_norm(c.stream, c.pq, c.pb, c.pr, n, c.red, S_RN2);
  vset_tol(c.stream, c.red, rtol);
  vfill_small(c.stream, c.red.scal + S_FLEX, 1, c.desc.pcg_flexible ? 1.0 : 0.0);
  read_scalars(c);
  int status = IPMG_OK;
  int restarts = 0;
  double rn2 = c.hscal[S_RN2];
  bool converged = rn2 <= c.hscal[S_TOL2];
  if (!converged) pcg_restart_direction(c, op, n);
  int enq = 0;   // iterations enqueued in this pass
  while (!converged) {
    // pipeline: keep one iteration in flight while reading the previous flags
    int iters_before = 0;
    read_scalars(c);
    iters_before = c.hflags[F_ITERS];
    if (c.hflags[F_DONE] == 2) { status = IPMG_E_BREAKDOWN; break; }
    int done = 0;
    int slot = 0;
    enq = 0;
    while (iters_before + enq < maxit) {
      c.flag_dst = c.hflags + F_COUNT * (1 + slot);   // the last kernel writes the flags there ...
      c.flag_written = false;
      pcg_iteration(c, op, n, gate, enq == 0 ? 1 : 0);
      if (!c.flag_written)                               // ... or they are copied
        IPMG_HIP(hipMemcpyAsync(c.hflags + F_COUNT * (1 + slot), c.red.flags, sizeof(int) * F_COUNT,
                                hipMemcpyDeviceToHost, c.stream));
      c.flag_dst = nullptr;
      IPMG_HIP(hipEventRecord(slot ? c.ev1 : c.ev0, c.stream));
      ++enq;
      if (enq >= 2) {
        IPMG_HIP(hipEventSynchronize(slot ? c.ev0 : c.ev1));
        if (c.hflags[F_COUNT * (1 + (slot ^ 1)) + F_DONE]) { done = 1; break; }
      }
      slot ^= 1;
    }
    // A pending update belongs to the last enqueued step (any later direction
    // kernel, gated or not, applies and clears it), whose p is c.pp.
    if (c.ops->dir_folds_solution(c)) vzflush(c.stream, c.pu, c.pp, n, c.red);
    IPMG_HIP(hipGetLastError());
    read_scalars(c);
    (void)done;
    if (c.hflags[F_DONE] == 2) { status = IPMG_E_BREAKDOWN; break; }
    if (c.hflags[F_DONE] != 1) { status = IPMG_E_NOT_CONVERGED; break; }
    // confirm with the true residual; restart from it if the recurrence drifted
    c.ops->fine_apply64(c, op, c.pu, c.pq, nullptr);
    vsub_norm(c.stream, c.pq, c.pb, c.pr, n, c.red, S_RN2);
    read_scalars(c);
    if (c.hscal[S_RN2] <= c.hscal[S_TOL2]) { converged = true; break; }
    if (c.hflags[F_ITERS] >= maxit) { status = IPMG_E_NOT_CONVERGED; break; }
    ++restarts;
    vset_tol(c.stream, c.red, rtol);
    pcg_restart_direction(c, op, n);
  }
  read_scalars(c);
  const double relres_rec = std::sqrt(c.hscal[S_RN2] / bn2);
  // true residual and b'u at exit
  c.ops->fine_apply64(c, op, c.pu, c.pq, nullptr);
  vsub_norm(c.stream, c.pq, c.pb, c.pt, n, c.red, S_TMP2);
  vdot(c.stream, c.pb, c.pu, n, c.red, S_TMP3, nullptr);
  IPMG_HIP(hipMemcpyAsync(u, c.pu, sizeof(double) * n, hipMemcpyDeviceToDevice, c.stream));
  read_scalars(c);
  auto t1 = std::chrono::steady_clock::now();
  inf.iters = c.hflags[F_ITERS];
  inf.restarts = restarts;
  inf.status = status;
  inf.relres = relres_rec;
  inf.true_relres = std::sqrt(c.hscal[S_TMP2] / bn2);
  inf.bu = c.hscal[S_TMP3];
  inf.solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  if (info) *info = inf;
  return status;
}

// Layout of the allocation-free PCG's scratch: seven vectors of n_slots + 1 doubles
// (r, p, q, t, b, u, second p), then the reduction partials, the scalars, the flags
// and the counters; every part starts on a 256-byte boundary.
namespace {
struct NoallocLayout {
  size_t vec, partials, scal, flags, counter, total;
};
NoallocLayout noalloc_layout(const Ctx& c) {
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  NoallocLayout l;
  l.vec = up(sizeof(double) * ((size_t)c.fine().nslots + 1));
  l.partials = 7 * l.vec;
  l.scal = l.partials + up(sizeof(double) * 8 * MAX_PARTIALS);
  l.flags = l.scal + sizeof(double) * S_COUNT;
  l.counter = l.flags + sizeof(int) * F_COUNT;
  l.total = up(l.counter + sizeof(unsigned) * C_COUNT);
  return l;
}
}  // namespace

size_t pcg_noalloc_bytes(const Ctx& c) { return noalloc_layout(c).total; }

int pcg_noalloc(Ctx& c, int op, const double* b, double* u, double rtol, int maxit, ipmg_pcg_info* info) {
  IPMG_REQUIRE(c.have_x, IPMG_E_STATE, "set the densities first");
  IPMG_REQUIRE(c.hier_op == op, IPMG_E_STATE,
               "set up the multigrid hierarchy of this operator first (ipmg_mg_setup or a solve)");
  const NoallocLayout l = noalloc_layout(c);
  IPMG_REQUIRE(l.total <= (size_t)IPMG_NOALLOC_SCRATCH_BYTES, IPMG_E_INVALID,
               "grid too large for the scratch of the allocation-free PCG");
  IPMG_REQUIRE(c.noalloc_scratch, IPMG_E_STATE, "scratch address not set");
  unsigned char* s = c.noalloc_scratch;
  // the context's own buffers, restored however the call ends
  struct Saved {
    Ctx& c;
    double *pr, *pp, *pq, *pt, *pb, *pu, *pp2;
    Red red;
    explicit Saved(Ctx& cc)
        : c(cc), pr(cc.pr), pp(cc.pp), pq(cc.pq), pt(cc.pt), pb(cc.pb), pu(cc.pu), pp2(cc.pp2), red(cc.red) {}
    ~Saved() {
      c.pr = pr; c.pp = pp; c.pq = pq; c.pt = pt; c.pb = pb; c.pu = pu; c.pp2 = pp2;
      c.red = red;
    }
  } saved(c);
  double* v[7];
  for (int k = 0; k < 7; ++k) v[k] = (double*)(s + k * l.vec);
  c.pr = v[0]; c.pp = v[1]; c.pq = v[2]; c.pt = v[3]; c.pb = v[4]; c.pu = v[5]; c.pp2 = v[6];
  c.red.partials = (double*)(s + l.partials);
  c.red.scal = (double*)(s + l.scal);
  c.red.flags = (int*)(s + l.flags);
  c.red.counter = (unsigned*)(s + l.counter);
  // The array keeps the last call's contents: the direction kernel reads p_old
  // (times 0) on the first step, so both direction buffers start at zero, as do
  // the scalars, flags and counters (cleared with fill kernels, not memset nodes).
  const int64_t n1 = c.fine().nslots + 1;
  vfill(c.stream, c.pp, 0.0, n1);
  vfill(c.stream, c.pp2, 0.0, n1);
  vfill(c.stream, c.red.scal, 0.0, (int64_t)((l.total - l.scal) / sizeof(double)));
  IPMG_HIP(hipGetLastError());
  return pcg(c, op, b, u, rtol, maxit, info);
}

// ------------------------------------------------------------------ OC update --
void oc_update(Ctx& c, const double* u, const double* x, double V, double xbar, double q, double lam_hi,
               double tau, const double* blend, double* x_new, ipmg_oc_info* info) {
  const Dims& d = c.fine();
  if (!c.oc_t) dalloc(c.oc_t, sizeof(double) * (size_t)d.m);
  c.ops->oc_energy(c, u, x, q, c.oc_t);
  voc_init(c.stream, c.red, c.oc_cand, lam_hi);
  // trials of sequential bisection in exact arithmetic, plus two for rounding;
  // passes past the end are gated on the device
  const int trials = (int)std::ceil(std::log2(lam_hi / tau)) + 2;
  for (;;) {
    for (int p = 0; p < (trials + OC_LEVELS - 1) / OC_LEVELS; ++p)
      voc_pass(c.stream, c.oc_t, d.m, xbar, V, tau, c.oc_cand, c.red);
    IPMG_HIP(hipGetLastError());
    read_scalars(c);
    if (c.hflags[F_OCDONE]) break;
  }
  voc_apply(c.stream, c.oc_t, d.m, xbar, blend, x_new, c.red);
  IPMG_HIP(hipGetLastError());
  read_scalars(c);
  if (info) {
    info->lambda = c.hscal[S_OCLAM];
    info->volume = c.hscal[S_OCSUM];
    info->trials = (int)c.hscal[S_OCSTEPS];
  }
}

// --------------------------------------------------------------------- SIMP --
// Compliance and gradient of the SIMP model with the density filter (Sec. 9):
// x~ = W x, K^ = K(x~^p), u = K^-1 f by MG-PCG, c = f'u, grad = -W' (p x~^(p-1) o E).
int simp_compliance(Ctx& c, const double* x, const double* f, double rmin, double p, double rtol, int maxit,
                    double* u, double* grad, ipmg_pcg_info* info) {
  const Dims& d = c.fine();
  if (!c.simp_xt) dalloc(c.simp_xt, sizeof(double) * (size_t)d.m);
  if (!c.simp_xp) dalloc(c.simp_xp, sizeof(double) * (size_t)d.m);
  c.ops->filter(c, rmin, x, c.simp_xt, 0);
  c.ops->simp_pow(c, c.simp_xt, p, c.simp_xp, nullptr);
  IPMG_HIP(hipGetLastError());
  set_density(c, c.simp_xp);
  IPMG_HIP(hipMemsetAsync(u, 0, sizeof(double) * (size_t)d.nslots, c.stream));
  const int st = pcg(c, IPMG_OP_K, f, u, rtol, maxit, info);
  if (st != IPMG_OK) return st;
  c.ops->element_sens(c, u, u, 1.0, c.simp_xp);               // E_e
  c.ops->simp_pow(c, c.simp_xt, p, nullptr, c.simp_xp);        // p x~^(p-1) E
  c.ops->filter(c, rmin, c.simp_xp, grad, 1);                  // W' (...)
  vscale(c.stream, grad, -1.0, d.m);
  IPMG_HIP(hipGetLastError());
  sync(c);
  return IPMG_OK;
}

// ------------------------------------------------------- SIMP interior point --
static void ensure_simp_buffers(Ctx& c) {
  if (c.simp_cf) return;
  const Dims& d = c.fine();
  const size_t m = (size_t)d.m, n1 = (size_t)d.nslots + 1;
  if (!c.simp_xt) dalloc(c.simp_xt, sizeof(double) * m);
  if (!c.simp_xp) dalloc(c.simp_xp, sizeof(double) * m);
  for (double** b : {&c.simp_cf, &c.simp_E, &c.simp_a, &c.simp_t, &c.simp_b1, &c.simp_b2, &c.simp_b3, &c.simp_bcoef,
                     &c.simp_rcoef})
    dalloc(*b, sizeof(double) * m);
  dalloc(c.simp_g, sizeof(double) * (size_t)c.nd * m);
  for (double** b : {&c.simp_r, &c.simp_y, &c.simp_p, &c.simp_q}) dalloc(*b, sizeof(double) * n1);
}

// x~ = W x, K^ = sum x~^p K_e (set as the densities), c = p x~^(p-1).
static void simp_densities(Ctx& c, const double* x, double rmin, double pexp) {
  const Dims& d = c.fine();
  c.ops->filter(c, rmin, x, c.simp_xt, 0);
  c.ops->simp_pow(c, c.simp_xt, pexp, c.simp_xp, nullptr);
  vfill(c.stream, c.simp_cf, 1.0, d.m);
  c.ops->simp_pow(c, c.simp_xt, pexp, nullptr, c.simp_cf);
  IPMG_HIP(hipGetLastError());
  set_density(c, c.simp_xp);
}

// The SIMP Newton system at st (Sec. 9 with Sec. 2): residuals, G3 and w (ipG3,
// ipW), right-hand side (ipRhs), the exact border b = B^ D^-1 e (bZ64) and corner
// sum w (simp_corner), and the preconditioner's element-local rank-one factors
// (h64/hT) and corner (cZ).  Measures in hscal as ip_prepare.
static void simp_prepare(Ctx& c, const double* f, const ipmg_ip_params& p, double rmin, double pexp,
                         const ipmg_ip_state& st) {
  ensure_z_buffers(c);
  ensure_simp_buffers(c);
  const Dims& d = c.fine();
  c.ipV = p.V;
  simp_densities(c, st.x, rmin, pexp);
  IPMG_HIP(hipMemsetAsync(c.red.flags + F_BAD, 0, sizeof(int), c.stream));
  c.ops->simp_elem(c, st.u, c.simp_g, c.simp_E);
  vmul(c.stream, c.simp_cf, c.simp_E, c.simp_a, d.m);
  c.ops->filter(c, rmin, c.simp_a, c.simp_t, 1);                         // W'(c o E)
  c.ops->simp_design(c, c.simp_t, st.x, st.phi, st.psi, st.lam, st.s, st.r, p.xbar);
  c.ops->filter(c, rmin, c.ipW, c.simp_b1, 0);                           // W w
  vmul(c.stream, c.ipG3, c.ipW, c.simp_a, d.m);
  c.ops->filter(c, rmin, c.simp_a, c.simp_b2, 0);                        // W (G3 o w)
  c.ops->filter(c, rmin, c.ipW, c.simp_b3, 2);                           // W2 w
  c.ops->simp_coef(c, c.simp_cf, c.simp_b1, c.simp_b2, c.simp_b3, c.simp_g, c.simp_bcoef, c.simp_rcoef);
  c.ops->fine_apply64(c, IPMG_OP_K, st.u, c.ipKu, nullptr);
  c.ops->simp_nodes(c, c.ipKu, f, st.u, c.simp_g, c.simp_bcoef, c.simp_rcoef, c.ipRhs);
  IPMG_HIP(hipGetLastError());
  read_scalars(c);
  IPMG_REQUIRE(!c.hflags[F_BAD], IPMG_E_DOMAIN, "interior-point iterate left the interior or is not finite");
  c.simp_corner = c.hscal[S_TMP0];
  c.cZ = c.hscal[S_TMP7];
  c.have_z = true;
  c.hier_op = -1;
}

// y = Z^ v (n_slots + 1): K^ v_u + B^ D^-1 B^' v_u + b v_lambda, b' v_u + (sum w) v_lambda,
// with B^' v_u = W'(c o s), s_e = v_e'K0u_e, and B^ t = sum_e c_e (W t)_e K0 u_e.
static void simp_apply(Ctx& c, double rmin, const double* u, const double* v, double* y) {
  const Dims& d = c.fine();
  c.ops->fine_apply64(c, IPMG_OP_K, v, y, nullptr);
  c.ops->element_sens(c, v, u, 1.0, c.simp_a);
  vmul(c.stream, c.simp_cf, c.simp_a, c.simp_a, d.m);
  c.ops->filter(c, rmin, c.simp_a, c.simp_b1, 1);
  vmul(c.stream, c.simp_b1, c.ipW, c.simp_b1, d.m);
  c.ops->filter(c, rmin, c.simp_b1, c.simp_a, 0);
  vmul(c.stream, c.simp_cf, c.simp_a, c.simp_a, d.m);
  c.ops->simp_gather(c, c.simp_g, c.simp_a, v, y);
  vdot(c.stream, c.bZ64, v, d.nslots, c.red, S_TMP4, nullptr);
  vlam_row(c.stream, y, v, c.red, S_TMP4, c.simp_corner, d.nslots);
  IPMG_HIP(hipGetLastError());
}

// Algorithm PCG (the recurrence, stopping test and true-residual restart of pcg)
// on Z^ with the V-cycle of the prepared hierarchy, from z (from_z) or from 0.
static int simp_pcg(Ctx& c, double rmin, const double* u, const double* b, double* z, double rtol, int maxit,
                    bool from_z, ipmg_pcg_info* info) {
  const Dims& d = c.fine();
  const int64_t n1 = d.nslots + 1;
  auto t0 = std::chrono::steady_clock::now();
  auto dot = [&](const double* a, const double* bb) {
    vdot(c.stream, a, bb, n1, c.red, S_TMP5, nullptr);
    double v = 0.0;
    IPMG_HIP(hipMemcpyAsync(&v, c.red.scal + S_TMP5, sizeof(double), hipMemcpyDeviceToHost, c.stream));
    sync(c);
    return v;
  };
  double *r = c.simp_r, *y = c.simp_y, *pp = c.simp_p, *q = c.simp_q;
  ipmg_pcg_info inf{};
  const double bnorm = std::sqrt(dot(b, b));
  auto finish = [&](int status, int iters, double rel) {
    simp_apply(c, rmin, u, z, q);
    vlincomb(c.stream, q, 1.0, q, -1.0, b, n1);
    inf.iters = iters;
    inf.status = status;
    inf.relres = rel;
    inf.true_relres = bnorm > 0.0 ? std::sqrt(dot(q, q)) / bnorm : 0.0;
    inf.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
    return status;
  };
  if (!from_z) IPMG_HIP(hipMemsetAsync(z, 0, sizeof(double) * n1, c.stream));
  if (bnorm == 0.0) return finish(IPMG_OK, 0, 0.0);
  simp_apply(c, rmin, u, z, r);
  vlincomb(c.stream, r, 1.0, r, -1.0, b, n1);                 // r = A z - b
  double rel = std::sqrt(dot(r, r)) / bnorm;
  if (rel <= rtol) return finish(IPMG_OK, 0, rel);
  vcycle64(c, IPMG_OP_Z, r, y);
  vlincomb(c.stream, pp, -1.0, y, 0.0, y, n1);
  double rho = dot(r, y);
  if (!(rho > 0.0)) return finish(IPMG_E_BREAKDOWN, 0, rel);
  int iters = 0;
  while (iters < maxit) {
    simp_apply(c, rmin, u, pp, q);
    const double pq = dot(pp, q);
    if (!(pq > 0.0)) return finish(IPMG_E_BREAKDOWN, iters, rel);
    const double alpha = rho / pq;
    vlincomb(c.stream, z, 1.0, z, alpha, pp, n1);
    vlincomb(c.stream, r, 1.0, r, alpha, q, n1);
    ++iters;
    rel = std::sqrt(dot(r, r)) / bnorm;
    if (rel <= rtol) {
      simp_apply(c, rmin, u, z, q);
      vlincomb(c.stream, q, 1.0, q, -1.0, b, n1);
      if (std::sqrt(dot(q, q)) / bnorm <= rtol) return finish(IPMG_OK, iters, rel);
      ++inf.restarts;
      IPMG_HIP(hipMemcpyAsync(r, q, sizeof(double) * n1, hipMemcpyDeviceToDevice, c.stream));
      vcycle64(c, IPMG_OP_Z, r, y);
      vlincomb(c.stream, pp, -1.0, y, 0.0, y, n1);
      rho = dot(r, y);
      continue;
    }
    vcycle64(c, IPMG_OP_Z, r, y);
    const double rho_new = dot(r, y);
    if (!(rho_new > 0.0)) return finish(IPMG_E_BREAKDOWN, iters, rel);
    vlincomb(c.stream, pp, -1.0, y, rho_new / rho, pp, n1);
    rho = rho_new;
  }
  return finish(IPMG_E_NOT_CONVERGED, iters, rel);
}

int simp_ip_init(Ctx& c, const double* f, const ipmg_ip_params& p, double rmin, double pexp, ipmg_ip_state& st,
                 ipmg_pcg_info* info) {
  const Dims& d = c.fine();
  IPMG_REQUIRE(p.xbar > 0.0 && p.V > 0.0 && p.V < p.xbar * (double)d.m, IPMG_E_DOMAIN,
               "need 0 < V < m * xbar");
  ensure_simp_buffers(c);
  vfill(c.stream, st.x, p.V / (double)d.m, d.m);
  vfill(c.stream, st.phi, 1.0, d.m);
  vfill(c.stream, st.psi, 1.0, d.m);
  IPMG_HIP(hipMemsetAsync(st.u, 0, sizeof(double) * d.nslots, c.stream));
  st.lam = 1.0;
  st.s = 1.0;
  st.r = 1.0;
  simp_densities(c, st.x, rmin, pexp);
  return pcg(c, IPMG_OP_K, f, st.u, p.pcg_rtol, p.pcg_maxit, info);
}

int simp_ip_step(Ctx& c, const double* f, const ipmg_ip_params& p, double rmin, double pexp, ipmg_ip_state& st,
                 ipmg_ip_info* info) {
  const Dims& d = c.fine();
  ipmg_ip_info inf{};
  simp_prepare(c, f, p, rmin, pexp, st);
  double setup_ms = 0.0;
  mg_setup(c, IPMG_OP_Z, &setup_ms);
  ipmg_pcg_info pin{};
  int ps = simp_pcg(c, rmin, st.u, c.ipRhs, c.ipD, p.pcg_rtol, p.pcg_maxit, false, &pin);
  if (ps == IPMG_E_BREAKDOWN) {   // as ip_step: damping estimated again, continued from the last iterate
    const int first = pin.iters;
    const double first_ms = pin.solve_ms;
    for (int k = 1; k < c.L; ++k)
      jacobi_damping(c, k, IPMG_OP_Z, RETRY_POWER_FACTOR * c.power_steps_z, SAFE_PRODUCT_RETRY);
    IPMG_HIP(hipGetLastError());
    ps = simp_pcg(c, rmin, st.u, c.ipRhs, c.ipD, p.pcg_rtol, p.pcg_maxit, true, &pin);
    pin.iters += first;
    pin.solve_ms += first_ms;
    inf.pcg_retries = 1;
  }
  inf.pcg_iters = pin.iters;
  inf.pcg_status = ps;
  inf.pcg_true_relres = pin.true_relres;
  inf.setup_ms = setup_ms;
  inf.solve_ms = pin.solve_ms;
  if (ps != IPMG_OK && !(ps == IPMG_E_NOT_CONVERGED && pin.true_relres <= p.accept_rtol)) {
    if (info) *info = inf;
    return ps;
  }
  // d_x = w (B^'d_u + d_lambda - G3), B^'d_u = W'(c o s), s_e = d_u,e'K0u_e
  c.ops->element_sens(c, c.ipD, st.u, 1.0, c.simp_a);
  vmul(c.stream, c.simp_cf, c.simp_a, c.simp_a, d.m);
  c.ops->filter(c, rmin, c.simp_a, c.simp_t, 1);
  IPMG_HIP(hipMemsetAsync(c.red.flags + F_BAD, 0, sizeof(int), c.stream));
  c.ops->simp_recover(c, c.simp_t, c.ipD, st.x, st.phi, st.psi, st.s, st.r, p.xbar, p.frac, p.step_all_blocks);
  double dlam = 0.0;
  IPMG_HIP(hipMemcpyAsync(&dlam, c.ipD + d.nslots, sizeof(double), hipMemcpyDeviceToHost, c.stream));
  read_scalars(c);
  const double alpha = c.hscal[S_ALPHA];
  inf.alpha = alpha;
  if (!(alpha >= 1e-14) || !std::isfinite(dlam) || c.hflags[F_BAD]) {
    if (info) *info = inf;
    return IPMG_E_STALLED;
  }
  c.ops->ip_update(c, st.u, c.ipD, st.x, st.phi, st.psi);
  st.lam += alpha * dlam;
  simp_prepare(c, f, p, rmin, pexp, st);   // measures at the new iterate
  const double* S = c.hscal;
  const double nF1 = std::sqrt(S[S_MIN0]), nf = std::sqrt(S[S_MIN1]);
  const double nG3 = std::sqrt(S[S_TMP3]), nphi = std::sqrt(S[S_TMP4]), npsi = std::sqrt(S[S_TMP5]);
  inf.nwt = nF1 / nf + nG3 / (nphi + npsi);
  inf.compliance = S[S_MIN2];
  inf.gap = S[S_TMP6] / S[S_MIN2];
  inf.volume_res = S[S_TMP2] - p.V;
  if (!std::isfinite(inf.nwt) || !std::isfinite(inf.gap)) {
    if (info) *info = inf;
    return IPMG_E_DOMAIN;
  }
  const bool newton_ok = inf.nwt <= p.tau_nwt;
  if (p.stop_rule == 0 && newton_ok && inf.gap <= p.kkt_tol) {
    inf.converged = 1;
  } else if (newton_ok) {
    st.s *= p.sigma;
    st.r *= p.sigma;
    inf.barrier_updated = 1;
    if (p.stop_rule == 1 && std::fmax(st.s, st.r) <= p.tau_ip) inf.converged = 1;
  }
  if (info) *info = inf;
  return IPMG_OK;
}

// ------------------------------------------------------------ interior point --
int ip_init(Ctx& c, const double* f, const ipmg_ip_params& p, ipmg_ip_state& st, ipmg_pcg_info* info) {
  const Dims& d = c.fine();
  IPMG_REQUIRE(p.xbar > 0.0 && p.V > 0.0 && p.V < p.xbar * (double)d.m, IPMG_E_DOMAIN,
               "need 0 < V < m * xbar");
  vfill(c.stream, st.x, p.V / (double)d.m, d.m);
  vfill(c.stream, st.phi, 1.0, d.m);
  vfill(c.stream, st.psi, 1.0, d.m);
  IPMG_HIP(hipMemsetAsync(st.u, 0, sizeof(double) * d.nslots, c.stream));
  st.lam = 1.0;
  st.s = 1.0;
  st.r = 1.0;
  set_density(c, st.x);
  return pcg(c, IPMG_OP_K, f, st.u, p.pcg_rtol, p.pcg_maxit, info);
}

void ip_prepare(Ctx& c, const double* f, const ipmg_ip_params& p, const ipmg_ip_state& st) {
  ensure_z_buffers(c);
  set_density(c, st.x);
  c.ipV = p.V;
  IPMG_HIP(hipMemsetAsync(c.red.flags + F_BAD, 0, sizeof(int), c.stream));
  c.ops->ip_elements(c, st.u, st.x, st.phi, st.psi, st.lam, st.s, st.r, p.xbar);
  c.ops->fine_apply64(c, IPMG_OP_K, st.u, c.ipKu, nullptr);
  c.ops->ip_nodes(c, c.ipKu, f, st.u, c.ipRhs);
  IPMG_HIP(hipGetLastError());
  read_scalars(c);
  IPMG_REQUIRE(!c.hflags[F_BAD], IPMG_E_DOMAIN, "interior-point iterate left the interior or is not finite");
  c.cZ = c.hscal[S_TMP0];
  c.have_z = true;
  c.hier_op = -1;
}

int ip_step(Ctx& c, const double* f, const ipmg_ip_params& p, ipmg_ip_state& st, ipmg_ip_info* info) {
  const Dims& d = c.fine();
  ipmg_ip_info inf{};
  ip_prepare(c, f, p, st);
  double setup_ms = 0.0;
  mg_setup(c, IPMG_OP_Z, &setup_ms);
  IPMG_HIP(hipMemsetAsync(c.ipD, 0, sizeof(double) * (d.nslots + 1), c.stream));
  ipmg_pcg_info pin{};
  // A solve stopped by the iteration limit leaves its last iterate in ipD.  It is
  // taken as an inexact Newton direction (Sec. 6, stopping rule) only when its
  // true relative residual is within accept_rtol; a breakdown of the recurrence,
  // or a residual above that bound, fails the step with the state unchanged.
  int ps = pcg(c, IPMG_OP_Z, c.ipRhs, c.ipD, p.pcg_rtol, p.pcg_maxit, &pin);
  if (ps == IPMG_E_BREAKDOWN) {
    const int first = pin.iters;
    const double first_ms = pin.solve_ms;
    for (int k = 1; k < c.L; ++k)
      jacobi_damping(c, k, IPMG_OP_Z, RETRY_POWER_FACTOR * c.power_steps_z, SAFE_PRODUCT_RETRY);
    IPMG_HIP(hipGetLastError());
    ps = pcg(c, IPMG_OP_Z, c.ipRhs, c.ipD, p.pcg_rtol, p.pcg_maxit, &pin);
    pin.iters += first;
    pin.solve_ms += first_ms;
    inf.pcg_retries = 1;
  }
  inf.pcg_iters = pin.iters;
  inf.pcg_status = ps;
  inf.pcg_true_relres = pin.true_relres;
  inf.setup_ms = setup_ms;
  inf.solve_ms = pin.solve_ms;
  if (ps != IPMG_OK && !(ps == IPMG_E_NOT_CONVERGED && pin.true_relres <= p.accept_rtol)) {
    if (info) *info = inf;
    return ps;
  }
  IPMG_HIP(hipMemsetAsync(c.red.flags + F_BAD, 0, sizeof(int), c.stream));
  c.ops->ip_recover(c, c.ipD, st.x, st.phi, st.psi, st.s, st.r, p.xbar, p.frac, p.step_all_blocks);
  double dlam = 0.0;
  IPMG_HIP(hipMemcpyAsync(&dlam, c.ipD + d.nslots, sizeof(double), hipMemcpyDeviceToHost, c.stream));
  read_scalars(c);
  const double alpha = c.hscal[S_ALPHA];
  inf.alpha = alpha;
  // a non-finite entry of (d_u, d_lambda, d_x, d_phi, d_psi) sets F_BAD: the
  // comparisons of the step-length rule would skip it and leave alpha at 1
  if (!(alpha >= 1e-14) || !std::isfinite(dlam) || c.hflags[F_BAD]) {
    if (info) *info = inf;
    return IPMG_E_STALLED;
  }
  c.ops->ip_update(c, st.u, c.ipD, st.x, st.phi, st.psi);
  st.lam += alpha * dlam;
  // measures at the new iterate (same barrier parameters)
  ip_prepare(c, f, p, st);
  const double* S = c.hscal;
  const double nF1 = std::sqrt(S[S_MIN0]), nf = std::sqrt(S[S_MIN1]);
  const double nG3 = std::sqrt(S[S_TMP3]), nphi = std::sqrt(S[S_TMP4]), npsi = std::sqrt(S[S_TMP5]);
  inf.nwt = nF1 / nf + nG3 / (nphi + npsi);
  inf.compliance = S[S_MIN2];
  inf.gap = S[S_TMP6] / S[S_MIN2];
  inf.volume_res = S[S_TMP2] - p.V;
  if (!std::isfinite(inf.nwt) || !std::isfinite(inf.gap)) {
    if (info) *info = inf;
    return IPMG_E_DOMAIN;
  }
  const bool newton_ok = inf.nwt <= p.tau_nwt;
  if (p.stop_rule == 0 && newton_ok && inf.gap <= p.kkt_tol) {
    inf.converged = 1;
  } else if (newton_ok) {
    st.s *= p.sigma;
    st.r *= p.sigma;
    inf.barrier_updated = 1;
    if (p.stop_rule == 1 && std::fmax(st.s, st.r) <= p.tau_ip) inf.converged = 1;
  }
  if (info) *info = inf;
  return IPMG_OK;
}

}  // namespace ipmg

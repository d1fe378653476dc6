// Library context: grid hierarchy, device buffers and the per-dimension kernel set.
#pragma once
#include "common.h"

namespace ipmg {

struct Ctx;

// Level arrays (precision of the V-cycle, T = float or double).
struct Level {
  Dims d;
  void* r = nullptr;    // right-hand side of the level problem (n_slots + 1)
  void* z = nullptr;    // current iterate
  void* z2 = nullptr;   // Jacobi ping-pong partner
  void* t = nullptr;    // residual
  void* E = nullptr;    // coarse element matrices (NSYM * m), levels below the finest
  double* E64 = nullptr;// the same in FP64: the Galerkin chain is formed in FP64 (aliases E in FP64 mode)
  void* bZ = nullptr;   // border vector of Z on this level (n_slots)
  double* bZ64 = nullptr;// the same in FP64 (aliases bZ in FP64 mode)
};

// Kernel set of one dimension (implemented for 2 and 3 in ops2d.hip / ops3d.hip).
struct Ops {
  virtual ~Ops() {}
  virtual void element_stiffness(Ctx& c, double* dK0) = 0;           // into device buffer
  virtual void upload_k0(const double* K0) = 0;                       // host -> __constant__
  // One level pass (see LevelMode) on level lev with operator op.
  // omg: device pointer to the damping weight (Jacobi modes); sidx/sidx_in: scalar
  // slots of the mode's reductions.
  virtual void level(Ctx& c, int lev, int op, int mode, const void* v, const void* r, void* out,
                     const double* omg, int sidx, int sidx_in, const int* gate, const double* dot64 = nullptr) = 0;
  // p = -y + beta p_old; q = A p (FP64, finest level); alpha = rho / p'q on the device.
  // zs (only where dir_folds_solution): the previous step's solution update
  // zs += alpha p_old is done in the same pass when flags[F_ZPEND] is set, also
  // after the solve has stopped (gate set).
  virtual void dir_apply(Ctx& c, int op, const void* y, const double* pold, double* p, double* q, int first,
                         const int* gate, double* zs = nullptr) = 0;
  virtual bool dir_folds_solution(const Ctx& c) const = 0;
  // FP64 operator on the finest grid (PCG operator), y = A v.
  virtual void fine_apply64(Ctx& c, int op, const double* v, double* y, const int* gate) = 0;
  virtual void restrict_to(Ctx& c, int lev_f, const void* rf, void* rc, int aug, const int* gate) = 0;
  virtual void prolong_from(Ctx& c, int lev_f, void* z, const void* zc, int aug, const int* gate) = 0;
  // out = one Jacobi sweep from z2 + P zc on level lev (prolongation folded into the
  // sweep); false when that pass does not apply.
  virtual bool prolong_jacobi(Ctx& c, int lev, int op, const void* z2, const void* zc, const void* r, void* out,
                              const double* omg, const int* gate) = 0;
  // out = the first two damped-Jacobi sweeps from a zero iterate on level lev, in
  // one pass; false when that pass does not apply.
  virtual bool jacobi2(Ctx& c, int lev, int op, const void* r, void* out, const double* omg, const int* gate) = 0;
  // As jacobi2, and t = r - A out in the same pass; false when that pass does not apply.
  virtual bool jacobi2_resid(Ctx& c, int lev, int op, const void* r, void* out, void* t, const double* omg,
                             const int* gate) = 0;
  // out = z2 + P zc followed by two damped-Jacobi sweeps, in one pass (dot64: the
  // last sweep also accumulates the PCG ratio's partial sums, as M_JACOBI_BETA, and
  // its finalize follows); false when that pass does not apply.
  virtual bool prolong_jacobi2(Ctx& c, int lev, int op, const void* z2, const void* zc, const void* r, void* out,
                               const double* omg, const int* gate, const double* dot64) = 0;
  virtual void restrict64(Ctx& c, int lev_f, const double* rf, double* rc) = 0;    // border vectors
  virtual void galerkin(Ctx& c, int lev_f, int op) = 0;              // E64 of level lev_f-1
  virtual void dense_assemble(Ctx& c, int op, double* A, int n) = 0;
  virtual void power_start(Ctx& c, int lev, int aug, void* v) = 0;
  // Fused passes of level lev (see fused2d.h): false when they do not apply.
  //   down: lev.r -> z2 (into z), coarse residual (into lev-1 .r)
  //   up:   z2 (in z), coarse correction zc -> out
  virtual bool fused_applies(const Ctx& c, int lev, int op) const = 0;
  // The fused down pass of lev forms its r as P' t from the finest residual t
  // (passed in Ctx::down_from_t) instead of reading a restricted one.
  virtual bool down_restricts(const Ctx& c, int lev, int op) const = 0;
  virtual void fused_down(Ctx& c, int lev, const int* gate) = 0;
  virtual void fused_up(Ctx& c, int lev, const void* zc, void* out, const int* gate) = 0;
  virtual void element_sens(Ctx& c, const double* w, const double* u, double scale, double* g) = 0;
  // 3D finest level: the diagonal of the hierarchy's operator per DOF slot (V-cycle
  // precision), formed once per set-up (no-op elsewhere)
  virtual void fine_diag(Ctx& c, int op) = 0;
  // SIMP model (Sec. 9): the density filter (mode 0: out = W in, 1: W' in, 2: W2 in
  // with (W2)_ji = W_ji^2), and x~^p / p x~^(p-1) E
  virtual void filter(Ctx& c, double rmin, const double* in, double* out, int mode) = 0;
  virtual void simp_pow(Ctx& c, const double* xt, double p, double* xp, double* q) = 0;
  // Interior-point method on the SIMP model (Sec. 9), see the kernels in ops_impl.h:
  //   elem: g_e = K0 u_e, E_e = u_e'g_e;  design: F3 from the filtered energy term t,
  //   G3, w = 1/D (ipG3, ipW) and the sums of ip_elements;  coef: border/rhs
  //   coefficients, the lumped rank-one factors h64/hT and their corner
  //   (scal[S_TMP7]);  nodes: F1, border bZ64, right-hand side;  gather: y_u +=
  //   sum coef_e g_e + b v_lambda;  recover: d_x, d_phi, d_psi, step length.
  virtual void simp_elem(Ctx& c, const double* u, double* g, double* E) = 0;
  virtual void simp_design(Ctx& c, const double* t, const double* x, const double* phi, const double* psi,
                           double lam, double s, double r, double xbar) = 0;
  virtual void simp_coef(Ctx& c, const double* cf, const double* Ww, const double* WGw, const double* W2w,
                         const double* g, double* bcoef, double* rcoef) = 0;
  virtual void simp_nodes(Ctx& c, const double* Ku, const double* f, const double* u, const double* g,
                          const double* bcoef, const double* rcoef, double* rhs) = 0;
  virtual void simp_gather(Ctx& c, const double* g, const double* coef, const double* v, double* y) = 0;
  virtual void simp_recover(Ctx& c, const double* btdu, const double* du, const double* x, const double* phi,
                            const double* psi, double s, double r, double xbar, double frac, int all_blocks) = 0;
  // t_e = x_e (u_e'K0u_e)^q of the OC update (Sec. 4)
  virtual void oc_energy(Ctx& c, const double* u, const double* x, double q, double* t) = 0;
  // Interior point kernels (FP64).
  virtual void ip_elements(Ctx& c, const double* u, const double* x, const double* phi, const double* psi,
                           double lam, double s, double r, double xbar) = 0;
  virtual void ip_nodes(Ctx& c, const double* Ku, const double* f, const double* u, double* rhs) = 0;
  virtual void ip_recover(Ctx& c, const double* du, const double* x, const double* phi, const double* psi,
                          double s, double r, double xbar, double frac, int all_blocks) = 0;
  virtual void ip_update(Ctx& c, double* u, const double* du, double* x, double* phi, double* psi) = 0;
};

Ops* make_ops2d();
Ops* make_ops3d();

struct Ctx {
  ipmg_desc desc{};
  int dim = 2;
  bool fp32 = true;
  int L = 1;
  hipStream_t stream = nullptr;
  Ops* ops = nullptr;
  std::vector<Level> lev;      // lev[L-1] finest
  size_t tsz = 4;              // sizeof(T) of the V-cycle
  bool coarse_from_x = true;   // 2D K: first coarse level evaluated from the fine densities
  bool tiled2d = true;         // 2D level passes with register-blocked tiles
  int64_t tiled_min_nodes = (int64_t)1 << 18;  // ... on levels with at least this many nodes
  int nj32 = 4, nj64 = 2, nj_dir = 4;          // nodes per thread of the tiled passes
  bool fused2d = true;         // 2D K coarse levels: two fused launches per level
  bool fused_staged = true;    // ... with the element matrices staged in LDS (FP32 stored levels
  int64_t staged_max_nodes = (int64_t)1 << 16;  // below this size)
  int cus = 256;               // compute units of the device
  bool mfma = true;            // first coarse level's fused passes on the matrix cores (FP32)
  bool lane_share = true;      // finest-level 2D passes of K on lane-shared tiles (neighbour columns by DPP)
  bool fuse_resid = true;      // ... and the residual formed in the pass of the two sweeps from zero
  bool fuse_post = true;       // ... and the prolongation and both post-sweeps in one pass
  bool fold_solution = true;         // PCG solution update folded into the next direction kernel
  bool fold_rn2_fin = true;          // PCG ||r||^2 finalize done by the V-cycle's first pass
  bool fold_restrict = true;         // finest residual restricted inside the first coarse down pass
  const void* down_from_t = nullptr; // ... the residual, pending for that pass
  unsigned rn2_fin_blocks = 0;       // pending ||r||^2 finalize (partials of the update kernel) ...
  bool rn2_fin_zpend = false;        // ... and whether it marks z += alpha p pending
  bool fold_prolong = true;          // 2D tiled levels: prolongation folded into the first post-sweep, and
                                     // the finest level's first two pre-sweeps fused
  int power_steps = 12;        // power iterations of the damping estimate (K)
  int power_steps_z = 30;      // ... (augmented system Z)

  double K0[576] = {0};        // host copy of the element matrix
  int nd = 8;                  // DOFs per element

  // finest-level operator data
  double* x64 = nullptr;       // densities (m)
  void* xT = nullptr;          // V-cycle copy (aliases x64 in FP64 mode)
  double* h64 = nullptr;       // Z rank-one factors h_e (ND * m)
  void* hT = nullptr;
  void* hsbuf = nullptr;       // per-element h_e'v_e (m values, FP64 or FP32) for the 3D Z passes
  bool elem_hv = true;         // form h_e'v_e per element before each 3D Z pass
  double* bZ64 = nullptr;      // border of Z on the finest grid (n_slots)
  double cZ = 0.0;             // corner of Z
  bool have_x = false;
  bool have_z = false;
  int hier_op = -1;            // operator the hierarchy currently holds (-1: none)

  // PCG work vectors (FP64, n_slots + 1)
  double *pr = nullptr, *pp = nullptr, *pq = nullptr, *pt = nullptr, *pb = nullptr, *pu = nullptr;
  double* pp2 = nullptr;       // second search-direction buffer (p is double-buffered)
  void* yT = nullptr;          // level buffer holding the last preconditioned residual

  // coarsest dense solve
  int ncoarse = 0;             // dense size incl. lambda (n_slots_coarse + 1)
  double *dA = nullptr, *dLi = nullptr, *dAi = nullptr;   // packed tiles: A (then L), L^-1, A^-1
  float* dAif = nullptr;       // A^-1 rounded to FP32 (FP32 V-cycle)
  double* dpart = nullptr;     // partial sums of the dense apply

  // per-level damping on the device: omega_dev[k] = weight, omega_dev[L + k] = rho estimate
  double* omega_dev = nullptr;

  // reductions / scalars
  Red red{};
  double* hscal = nullptr;     // pinned host mirror of scal
  int* hflags = nullptr;       // pinned host mirror of flags
  // Within a PCG iteration: the pinned host slot that the iteration's last kernel
  // (the finalize of the fused PCG ratio) fills with the flags, and whether one did.
  int* flag_dst = nullptr;
  bool flag_written = false;
  int* take_flag_dst() {
    int* p = flag_dst;
    if (p) flag_written = true;
    flag_dst = nullptr;
    return p;
  }

  // interior-point scratch (FP64, m or n_slots + 1)
  double *ipG3 = nullptr, *ipW = nullptr, *ipSW = nullptr, *ipDx = nullptr, *ipDphi = nullptr, *ipDpsi = nullptr;
  double *ipRhs = nullptr, *ipD = nullptr, *ipKu = nullptr;
  double ipV = 0.0;            // volume of the current interior-point problem

  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::string err;

  // 3D stored levels: element products y_e = E_e v of the level pass in flight
  // (24 values per element of the largest stored level, V-cycle precision)
  void* ye = nullptr;
  bool elem_apply3 = true;
  // 3D finest level: element products of the pass's vector (V-cycle precision and
  // FP64, aliased in FP64 mode) and the set-up diagonal
  void* fine_ye = nullptr;
  double* fine_ye64 = nullptr;
  void* fine_dg = nullptr;
  bool elem_fine3 = true;
  int64_t elem_apply3_min = 8192;   // ... on levels with at least this many elements

  // SIMP model: filtered densities and the penalised ones (m each)
  double* simp_xt = nullptr;
  double* simp_xp = nullptr;
  // SIMP interior point (Sec. 9): c = p x~^(p-1), g_e = K0 u_e (ND x m), E, work
  // vectors on the design variables, border/rhs coefficients, PCG vectors (n_slots+1)
  double *simp_cf = nullptr, *simp_g = nullptr, *simp_E = nullptr, *simp_a = nullptr, *simp_t = nullptr;
  double *simp_b1 = nullptr, *simp_b2 = nullptr, *simp_b3 = nullptr, *simp_bcoef = nullptr, *simp_rcoef = nullptr;
  double *simp_r = nullptr, *simp_y = nullptr, *simp_p = nullptr, *simp_q = nullptr;
  double simp_corner = 0.0;    // corner of the exact Newton matrix, sum w

  // OC update: t_e = x_e E_e^q (m) and the trial multipliers of a bisection pass
  double* oc_t = nullptr;
  double* oc_cand = nullptr;

  // this device's copy of the scratch array of the allocation-free PCG entry point
  unsigned char* noalloc_scratch = nullptr;

  // kernel timing (ipmg_profile_*): HIP event pairs around every launch of the
  // selected classes; prof_tag is the class of the next level pass
  unsigned prof_mask = 0;
  int prof_tag = -1;
  int prof_used = 0;
  std::vector<hipEvent_t> prof_ev;
  std::vector<int> prof_cls;

  const Dims& fine() const { return lev[L - 1].d; }
};

// Kernel classes timed by ipmg_profile_begin (bit k of the mask selects class k).
enum ProfClass {
  PC_FINE_JACOBI = 0,       // finest level, damped-Jacobi sweep from a nonzero iterate
  PC_DIR_APPLY = 1,         // FP64 finest-level apply of the PCG direction
  PC_FINE_RESID = 2,        // finest level, residual pass
  PC_PCG_UPDATE = 3,        // fused PCG vector update
  PC_SUB_JACOBI = 4,        // first coarse level, damped-Jacobi sweep from a nonzero iterate
  PC_FINE_JACOBI0 = 5,      // finest level, first sweep from a zero iterate
  PC_FINE_JACOBI_BETA = 6,  // finest level, last sweep with the fused PCG ratio
  PC_SUB_DOWN = 7,          // first coarse level, fused pre-smoothing + residual + restriction
  PC_SUB_UP = 8,            // first coarse level, fused prolongation + post-smoothing
  // 9 and 10: reserved (no kernel records them)
  PC_FINE_PJACOBI = 11,     // finest level, prolongation folded into the first post-smoothing sweep
  PC_FINE_JACOBI2 = 12,     // finest level, the first two pre-smoothing sweeps in one pass
  PC_ELEM3 = 13,            // 3D finest level, element products of a V-cycle pass
  PC_ELEM3_DIR = 14,        // 3D finest level, element products of the FP64 direction
  PC_COUNT = 15
};

// Sets the class of the level passes enqueued in its scope.
struct ProfTag {
  Ctx& c;
  int old;
  ProfTag(Ctx& cc, int cls) : c(cc), old(cc.prof_tag) { c.prof_tag = cls; }
  ~ProfTag() { c.prof_tag = old; }
};

// Brackets the launch of one main kernel with a pair of events when its class is
// being timed (finalize kernels stay outside the bracket).
struct ProfScope {
  Ctx& c;
  bool on;
  int slot;
  ProfScope(Ctx& cc, int cls) : c(cc), on(false), slot(0) {
    if (cls >= 0 && ((c.prof_mask >> cls) & 1u) && 2 * (c.prof_used + 1) <= (int)c.prof_ev.size()) {
      on = true;
      slot = c.prof_used++;
      c.prof_cls[slot] = cls;
      (void)hipEventRecord(c.prof_ev[2 * slot], c.stream);
    }
  }
  ~ProfScope() {
    if (on) (void)hipEventRecord(c.prof_ev[2 * slot + 1], c.stream);
  }
};

// Timing of one launch by its own dispatch packet: the start and stop events of
// hipExtLaunchKernel (null when the class is not being timed).  The interval is
// the kernel's run alone, without the marker packets that a pair of hipEventRecord
// calls would place around the dispatch.
struct ProfLaunch {
  hipEvent_t t0 = nullptr, t1 = nullptr;
  ProfLaunch(Ctx& c, int cls) {
    if (cls >= 0 && ((c.prof_mask >> cls) & 1u) && 2 * (c.prof_used + 1) <= (int)c.prof_ev.size()) {
      const int slot = c.prof_used++;
      c.prof_cls[slot] = cls;
      t0 = c.prof_ev[2 * slot];
      t1 = c.prof_ev[2 * slot + 1];
    }
  }
};

// Host driver (solver.hip).
void ctx_init(Ctx& c, const ipmg_desc& d, hipStream_t st);
void ctx_free(Ctx& c);
void set_density(Ctx& c, const double* x);
void mg_setup(Ctx& c, int op, double* ms);
void* vcycle(Ctx& c, int op, const int* gate);    // lev[L-1].r -> returned level buffer
void vcycle64(Ctx& c, int op, const double* r, double* z);
int pcg(Ctx& c, int op, const double* b, double* u, double rtol, int maxit, ipmg_pcg_info* info);
// pcg with its work vectors and reduction scratch in the library's static device
// array (no allocation); needs the hierarchy of op set up.
int pcg_noalloc(Ctx& c, int op, const double* b, double* u, double rtol, int maxit, ipmg_pcg_info* info);
size_t pcg_noalloc_bytes(const Ctx& c);
void sync(Ctx& c);
void read_scalars(Ctx& c);
int ip_init(Ctx& c, const double* f, const ipmg_ip_params& p, ipmg_ip_state& st, ipmg_pcg_info* info);
void ip_prepare(Ctx& c, const double* f, const ipmg_ip_params& p, const ipmg_ip_state& st);
int ip_step(Ctx& c, const double* f, const ipmg_ip_params& p, ipmg_ip_state& st, ipmg_ip_info* info);
void oc_update(Ctx& c, const double* u, const double* x, double V, double xbar, double q, double lam_hi,
               double tau, const double* blend, double* x_new, ipmg_oc_info* info);
// Interior-point method on the SIMP model (Sec. 9): initial state (as ip_init with
// K^ in place of K) and one Newton step (as ip_step: the exact Newton matrix Z^
// applied matrix-free, PCG preconditioned by the V-cycle of the element-local
// approximation).
int simp_ip_init(Ctx& c, const double* f, const ipmg_ip_params& p, double rmin, double pexp, ipmg_ip_state& st,
                 ipmg_pcg_info* info);
int simp_ip_step(Ctx& c, const double* f, const ipmg_ip_params& p, double rmin, double pexp, ipmg_ip_state& st,
                 ipmg_ip_info* info);
int simp_compliance(Ctx& c, const double* x, const double* f, double rmin, double p, double rtol, int maxit,
                    double* u, double* grad, ipmg_pcg_info* info);

}  // namespace ipmg

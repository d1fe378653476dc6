// PCG vector kernels (Algorithm PCG, Sec. 5.2).
#include "kernels.h"
#include "vec.h"

namespace ipmg {

namespace {

constexpr int VBLOCKS = 1024;   // grid of the streaming vector kernels

inline int vgrid(int64_t n) {
  int64_t b = (n + BS - 1) / BS;
  return (int)(b < VBLOCKS ? (b < 1 ? 1 : b) : VBLOCKS);
}
// The residual update runs one entry pair per thread (2048x1024: 22.3 us against
// 23.8 us for a grid-stride loop over 1024 blocks).
constexpr int UBLOCKS = 16384;
inline int ugrid(int64_t n) {
  int64_t b = ((n + 1) / 2 + BS - 1) / BS;
  return (int)(b < UBLOCKS ? (b < 1 ? 1 : b) : UBLOCKS);
}

// Post-processing done by the last block of a reduction.
enum Fin { FIN_STORE = 0, FIN_ALPHA = 1, FIN_RN2 = 2, FIN_BETA = 3, FIN_RN2_ZPEND = 4 };

__device__ inline void finish(int fin, double tot, const Red& red, int sidx) {
  if (fin == FIN_STORE) {
    red.scal[sidx] = tot;
  } else if (fin == FIN_ALPHA) {                 // alpha = r'y / p'Ap
    red.scal[S_PQ] = tot;
    if (!(tot > 0.0) || !isfinite(tot)) {
      red.flags[F_DONE] = 2;
      red.flags[F_STATUS] = IPMG_E_BREAKDOWN;
    } else {
      red.scal[S_ALPHA] = red.scal[S_RHO] / tot;
    }
  } else if (fin == FIN_RN2 || fin == FIN_RN2_ZPEND) {   // convergence test on ||r||^2
    rn2_finish(tot, red, fin == FIN_RN2_ZPEND);
  } else if (fin == FIN_BETA) {                  // beta = r~'y~ / r'y (or Polak-Ribiere)
    if (!(tot > 0.0) || !isfinite(tot)) {
      red.flags[F_DONE] = 2;
      red.flags[F_STATUS] = IPMG_E_BREAKDOWN;
    } else {
      const double rho = red.scal[S_RHO];
      const double num = red.scal[S_FLEX] != 0.0 ? tot - (rho + red.scal[S_ALPHA] * red.scal[S_QY]) : tot;
      red.scal[S_BETA] = num / rho;
      red.scal[S_RHO] = tot;
    }
  }
}

// One-block finalize: sum the partials of the previous kernel and apply `fin`.
__global__ __launch_bounds__(BS) void k_fin1(Red red, unsigned nblocks, int fin, int sidx, const int* gate) {
  if (gate && *gate) return;
  double tot[1];
  sum_partials<1>(red, nblocks, tot);
  if (threadIdx.x == 0) finish(fin, tot[0], red, sidx);
}

template <typename TA, typename TB>
__global__ __launch_bounds__(BS) void k_dot(const TA* __restrict__ a, const TB* __restrict__ b, int64_t n,
                                            Red red, const int* gate) {
  if (gate && *gate) return;
  double s = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x; t < n; t += (int64_t)gridDim.x * BS)
    s += (double)a[t] * (double)b[t];
  const double v[1] = {s};
  block_partials<1>(v, red);
}

// z += alpha p (unless ZUPD is off: then the next direction kernel does it);
// r += alpha q; rT = (T) r; ||r||^2 -> convergence flag.
// Each thread takes pairs of entries (16-byte accesses), two pairs per step with
// all eight loads issued first, so enough bytes are in flight to stream at the
// HBM rate; an odd last entry is taken by the first thread.
template <typename T>
__device__ inline void store_pair(T* p, double a, double b) {
  if constexpr (sizeof(T) == 8) *reinterpret_cast<double2*>(p) = make_double2(a, b);
  else *reinterpret_cast<float2*>(p) = make_float2((float)a, (float)b);
}

template <typename T, bool ZUPD>
__global__ __launch_bounds__(BS) void k_pcg_update(double* __restrict__ z, double* __restrict__ r,
                                                   const double* __restrict__ p, const double* __restrict__ q,
                                                   T* __restrict__ rT, int64_t n, Red red, const int* gate) {
  if (gate && *gate) return;
  const double alpha = red.scal[S_ALPHA];
  double s0 = 0.0, s1 = 0.0;
  const int64_t np = n / 2, stride = (int64_t)gridDim.x * BS;
  double2* z2 = reinterpret_cast<double2*>(z);
  double2* r2 = reinterpret_cast<double2*>(r);
  const double2* p2 = reinterpret_cast<const double2*>(p);
  const double2* q2 = reinterpret_cast<const double2*>(q);
  int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x;
  for (; t + stride < np; t += 2 * stride) {
    const int64_t u = t + stride;
    const double2 ra = r2[t], qa = q2[t];
    const double2 rb = r2[u], qb = q2[u];
    if constexpr (ZUPD) {
      const double2 za = z2[t], pa = p2[t];
      const double2 zb = z2[u], pb = p2[u];
      z2[t] = make_double2(za.x + alpha * pa.x, za.y + alpha * pa.y);
      z2[u] = make_double2(zb.x + alpha * pb.x, zb.y + alpha * pb.y);
    }
    const double2 na = make_double2(ra.x + alpha * qa.x, ra.y + alpha * qa.y);
    const double2 nb = make_double2(rb.x + alpha * qb.x, rb.y + alpha * qb.y);
    r2[t] = na;
    r2[u] = nb;
    if (rT) {
      store_pair<T>(rT + 2 * t, na.x, na.y);
      store_pair<T>(rT + 2 * u, nb.x, nb.y);
    }
    s0 += na.x * na.x + na.y * na.y;
    s1 += nb.x * nb.x + nb.y * nb.y;
  }
  if (t < np) {
    const double2 ra = r2[t], qa = q2[t];
    if constexpr (ZUPD) {
      const double2 za = z2[t], pa = p2[t];
      z2[t] = make_double2(za.x + alpha * pa.x, za.y + alpha * pa.y);
    }
    const double2 na = make_double2(ra.x + alpha * qa.x, ra.y + alpha * qa.y);
    r2[t] = na;
    if (rT) store_pair<T>(rT + 2 * t, na.x, na.y);
    s0 += na.x * na.x + na.y * na.y;
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    const int64_t e = n - 1;
    if constexpr (ZUPD) z[e] += alpha * p[e];
    const double rn = r[e] + alpha * q[e];
    r[e] = rn;
    if (rT) rT[e] = T(rn);
    s0 += rn * rn;
  }
  const double v[1] = {s0 + s1};
  block_partials<1>(v, red);
}

// The pending solution update of the last PCG step (flags[F_ZPEND], see
// k_dir_apply2d), applied after the step loop whatever stopped it; the flag is
// cleared by the next kernel.
__global__ __launch_bounds__(BS) void k_zflush(double* __restrict__ z, const double* __restrict__ p, int64_t n,
                                               Red red) {
  if (!red.flags[F_ZPEND]) return;
  const double alpha = red.scal[S_ALPHA];
  for (int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x; t < n; t += (int64_t)gridDim.x * BS)
    z[t] += alpha * p[t];
}
__global__ void k_zclear(Red red) {
  if (threadIdx.x == 0) red.flags[F_ZPEND] = 0;
}

// p = -y + beta p  (the reading p := -y~ + beta p of Algorithm PCG).
template <typename T>
__global__ __launch_bounds__(BS) void k_pcg_dir(double* __restrict__ p, const T* __restrict__ y, int64_t n,
                                                Red red, int first, const int* gate) {
  if (gate && *gate) return;
  const double beta = first ? 0.0 : red.scal[S_BETA];
  for (int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x; t < n; t += (int64_t)gridDim.x * BS)
    p[t] = -(double)y[t] + beta * p[t];
}

// out = a - b; scal[sidx] = ||out||^2.
__global__ __launch_bounds__(BS) void k_sub_norm(const double* __restrict__ a, const double* __restrict__ b,
                                                 double* __restrict__ out, int64_t n, Red red, int sidx) {
  double s = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x; t < n; t += (int64_t)gridDim.x * BS) {
    const double o = a[t] - b[t];
    out[t] = o;
    s += o * o;
  }
  const double v[1] = {s};
  block_partials<1>(v, red);
}

// dst = src with clamped slots (nodes with i == 0) zeroed; entries beyond the
// slots (lambda) copied.  scal[sidx] = ||dst||^2, flags[F_BAD] set if non-finite.
__global__ __launch_bounds__(BS) void k_mask_copy(const double* __restrict__ src, double* __restrict__ dst,
                                                  int64_t n, int64_t nslots, int dim, int nx1, Red red, int sidx) {
  double s = 0.0;
  int bad = 0;
  for (int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x; t < n; t += (int64_t)gridDim.x * BS) {
    double v = src[t];
    if (t < nslots && ((t / dim) % nx1) == 0) v = 0.0;
    if (!isfinite(v)) bad = 1;
    dst[t] = v;
    s += v * v;
  }
  if (bad) red.flags[F_BAD] = 1;
  const double v[1] = {s};
  block_partials<1>(v, red);
}

__global__ __launch_bounds__(BS) void k_fill(double* __restrict__ dst, double value, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x; t < n; t += (int64_t)gridDim.x * BS) dst[t] = value;
}

// dst = src; flags[F_BAD] = 1 unless every entry is finite and > 0.
__global__ __launch_bounds__(BS) void k_copy_positive(const double* __restrict__ src, double* __restrict__ dst,
                                                      int64_t n, Red red) {
  int bad = 0;
  for (int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x; t < n; t += (int64_t)gridDim.x * BS) {
    const double v = src[t];
    if (!(v > 0.0) || !isfinite(v)) bad = 1;
    dst[t] = v;
  }
  if (bad) red.flags[F_BAD] = 1;
}

template <typename TD, typename TS>
__global__ __launch_bounds__(BS) void k_convert(const TS* __restrict__ src, TD* __restrict__ dst, int64_t n,
                                                const int* gate) {
  if (gate && *gate) return;
  for (int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x; t < n; t += (int64_t)gridDim.x * BS)
    dst[t] = TD(src[t]);
}

__global__ void k_set_tol(Red red, double rtol2) {
  if (threadIdx.x == 0) {
    red.scal[S_TOL2] = rtol2 * red.scal[S_BN2];
    red.flags[F_DONE] = 0;
  }
}

__global__ void k_set_rho(Red red, int sidx) {
  if (threadIdx.x == 0) {
    const double rho = red.scal[sidx];
    red.scal[S_RHO] = rho;
    if (!(rho > 0.0) || !isfinite(rho)) {
      red.flags[F_DONE] = 2;
      red.flags[F_STATUS] = IPMG_E_BREAKDOWN;
    }
  }
}

// Damping safeguard: rho = v'Av / v'Dv from scal[s_vav], scal[s_vdv];
// w[0] = min(omega, product / rho), w[1] = rho (omega kept if rho is not usable).
__global__ void k_set_omega(Red red, double* __restrict__ w, double* __restrict__ rho_out, int s_vav, int s_vdv,
                            double omega, double product) {
  if (threadIdx.x == 0) {
    const double rho = red.scal[s_vav] / red.scal[s_vdv];
    double o = omega;
    if (rho > 0.0 && isfinite(rho)) o = fmin(omega, product / rho);
    w[0] = o;
    rho_out[0] = rho;
  }
}

__global__ void k_fill_value(double* __restrict__ w, int n, double value) {
  if ((int)threadIdx.x < n) w[threadIdx.x] = value;
}

// x = x / sqrt(scal[sidx]) (power-iteration normalisation)
template <typename T>
__global__ __launch_bounds__(BS) void k_normalize(T* __restrict__ x, int64_t n, Red red, int sidx) {
  const double s = red.scal[sidx];
  const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
  for (int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x; t < n; t += (int64_t)gridDim.x * BS)
    x[t] = T((double)x[t] * inv);
}

}  // namespace

// ---------------------------------------------------------------- launchers --
void vdot(hipStream_t st, const double* a, const double* b, int64_t n, const Red& red, int sidx, const int* gate) {
  k_dot<double, double><<<vgrid(n), BS, 0, st>>>(a, b, n, red, gate);
  k_fin1<<<1, BS, 0, st>>>(red, vgrid(n), FIN_STORE, sidx, gate);
}
void vdot_alpha(hipStream_t st, const double* p, const double* q, int64_t n, const Red& red, const int* gate) {
  k_dot<double, double><<<vgrid(n), BS, 0, st>>>(p, q, n, red, gate);
  k_fin1<<<1, BS, 0, st>>>(red, vgrid(n), FIN_ALPHA, 0, gate);
}
template <typename T>
void vdot_beta(hipStream_t st, const double* r, const T* y, int64_t n, const Red& red, const int* gate) {
  k_dot<double, T><<<vgrid(n), BS, 0, st>>>(r, y, n, red, gate);
  k_fin1<<<1, BS, 0, st>>>(red, vgrid(n), FIN_BETA, 0, gate);
}
template <typename T>
void vdot_store(hipStream_t st, const double* r, const T* y, int64_t n, const Red& red, int sidx, const int* gate) {
  k_dot<double, T><<<vgrid(n), BS, 0, st>>>(r, y, n, red, gate);
  k_fin1<<<1, BS, 0, st>>>(red, vgrid(n), FIN_STORE, sidx, gate);
}
template <typename T>
void vpcg_update(hipStream_t st, double* z, double* r, const double* p, const double* q, T* rT, int64_t n,
                 const Red& red, const int* gate) {
  if (z) k_pcg_update<T, true><<<ugrid(n), BS, 0, st>>>(z, r, p, q, rT, n, red, gate);
  else k_pcg_update<T, false><<<ugrid(n), BS, 0, st>>>(z, r, p, q, rT, n, red, gate);
}
void vpcg_update_fin(hipStream_t st, int64_t n, const Red& red, const int* gate, bool zpend) {
  k_fin1<<<1, BS, 0, st>>>(red, ugrid(n), zpend ? FIN_RN2_ZPEND : FIN_RN2, 0, gate);
}
unsigned vpcg_update_blocks(int64_t n) { return (unsigned)ugrid(n); }
void vpcg_update_fin_nb(hipStream_t st, unsigned nblocks, const Red& red, const int* gate, bool zpend) {
  k_fin1<<<1, BS, 0, st>>>(red, nblocks, zpend ? FIN_RN2_ZPEND : FIN_RN2, 0, gate);
}
void vzflush(hipStream_t st, double* z, const double* p, int64_t n, const Red& red) {
  k_zflush<<<vgrid(n), BS, 0, st>>>(z, p, n, red);
  k_zclear<<<1, 64, 0, st>>>(red);
}
template <typename T>
void vpcg_dir(hipStream_t st, double* p, const T* y, int64_t n, const Red& red, int first, const int* gate) {
  k_pcg_dir<T><<<vgrid(n), BS, 0, st>>>(p, y, n, red, first, gate);
}
void vsub_norm(hipStream_t st, const double* a, const double* b, double* out, int64_t n, const Red& red, int sidx) {
  k_sub_norm<<<vgrid(n), BS, 0, st>>>(a, b, out, n, red, sidx);
  k_fin1<<<1, BS, 0, st>>>(red, vgrid(n), FIN_STORE, sidx, nullptr);
}
void vmask_copy(hipStream_t st, const double* src, double* dst, int64_t n, int64_t nslots, int dim, int nx1,
                const Red& red, int sidx) {
  k_mask_copy<<<vgrid(n), BS, 0, st>>>(src, dst, n, nslots, dim, nx1, red, sidx);
  k_fin1<<<1, BS, 0, st>>>(red, vgrid(n), FIN_STORE, sidx, nullptr);
}
template <typename TD, typename TS>
void vconvert(hipStream_t st, const TS* src, TD* dst, int64_t n, const int* gate) {
  k_convert<TD, TS><<<vgrid(n), BS, 0, st>>>(src, dst, n, gate);
}
void vset_tol(hipStream_t st, const Red& red, double rtol) { k_set_tol<<<1, 64, 0, st>>>(red, rtol * rtol); }
void vset_rho(hipStream_t st, const Red& red, int sidx) { k_set_rho<<<1, 64, 0, st>>>(red, sidx); }
template <typename T>
void vnormalize(hipStream_t st, T* x, int64_t n, const Red& red, int sidx) {
  k_normalize<T><<<vgrid(n), BS, 0, st>>>(x, n, red, sidx);
}
void vfill(hipStream_t st, double* dst, double value, int64_t n) { k_fill<<<vgrid(n), BS, 0, st>>>(dst, value, n); }

namespace {
__global__ __launch_bounds__(BS) void k_scale(double* __restrict__ v, double a, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x; t < n; t += (int64_t)gridDim.x * BS) v[t] *= a;
}
__global__ __launch_bounds__(BS) void k_mul(const double* __restrict__ a, const double* __restrict__ b,
                                            double* __restrict__ out, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x; t < n; t += (int64_t)gridDim.x * BS) out[t] = a[t] * b[t];
}
__global__ __launch_bounds__(BS) void k_lincomb(double* __restrict__ out, double a, const double* __restrict__ x,
                                                double b, const double* __restrict__ y, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x; t < n; t += (int64_t)gridDim.x * BS)
    out[t] = a * x[t] + b * y[t];
}
// y[n] = scal[sidx] + c v[n]: the lambda row of an augmented operator, b'v_u in scal.
__global__ void k_lam_row(double* __restrict__ y, const double* __restrict__ v, Red red, int sidx, double c,
                          int64_t n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) y[n] = red.scal[sidx] + c * v[n];
}
}  // namespace
void vscale(hipStream_t st, double* v, double a, int64_t n) { k_scale<<<vgrid(n), BS, 0, st>>>(v, a, n); }
void vmul(hipStream_t st, const double* a, const double* b, double* out, int64_t n) {
  k_mul<<<vgrid(n), BS, 0, st>>>(a, b, out, n);
}
void vlincomb(hipStream_t st, double* out, double a, const double* x, double b, const double* y, int64_t n) {
  k_lincomb<<<vgrid(n), BS, 0, st>>>(out, a, x, b, y, n);
}
void vlam_row(hipStream_t st, double* y, const double* v, const Red& red, int sidx, double c, int64_t n) {
  k_lam_row<<<1, 64, 0, st>>>(y, v, red, sidx, c, n);
}
void vcopy_positive(hipStream_t st, const double* src, double* dst, int64_t n, const Red& red) {
  k_copy_positive<<<vgrid(n), BS, 0, st>>>(src, dst, n, red);
}
void vset_omega(hipStream_t st, const Red& red, double* w, double* rho, int s_vav, int s_vdv, double omega,
                double product) {
  k_set_omega<<<1, 64, 0, st>>>(red, w, rho, s_vav, s_vdv, omega, product);
}
void vfill_small(hipStream_t st, double* w, int n, double value) { k_fill_value<<<1, 64, 0, st>>>(w, n, value); }

// ------------------------------------------------------------ OC bisection --
namespace {

// Trials of one pass: node 0 is the midpoint of [lo, hi]; node i has children 2i+1
// (the lower half of its interval) and 2i+2 (the upper half), each midpoint formed
// as (a + b) / 2 from its interval, exactly as sequential bisection forms it on
// that path.  One thread.
__device__ void oc_tree(double lo, double hi, double* cand) {
  double a[OC_CAND], b[OC_CAND];
  a[0] = lo;
  b[0] = hi;
  for (int i = 0; i < OC_CAND; ++i) {
    const double mid = (b[i] + a[i]) / 2.0;
    cand[i] = mid;
    if (2 * i + 2 < OC_CAND) {
      a[2 * i + 1] = a[i]; b[2 * i + 1] = mid;
      a[2 * i + 2] = mid;  b[2 * i + 2] = b[i];
    }
  }
}

__global__ void k_oc_init(Red red, double* cand, double lam_hi) {
  if (threadIdx.x != 0) return;
  red.scal[S_OCLO] = 0.0;
  red.scal[S_OCHI] = lam_hi;
  red.scal[S_OCLAM] = 0.0;
  red.scal[S_OCSTEPS] = 0.0;
  red.flags[F_OCDONE] = 0;
  oc_tree(0.0, lam_hi, cand);
}

// sum_e min(t_e / lambda_j, xbar) for every trial j of the pass.
__global__ __launch_bounds__(BS) void k_oc_sums(const double* __restrict__ t, int64_t m, double xbar,
                                                const double* __restrict__ cand, Red red) {
  if (red.flags[F_OCDONE]) return;
  double lam[OC_CAND], acc[OC_CAND];
#pragma unroll
  for (int j = 0; j < OC_CAND; ++j) {
    lam[j] = cand[j];
    acc[j] = 0.0;
  }
  for (int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x; e < m; e += (int64_t)gridDim.x * BS) {
    const double te = t[e];
#pragma unroll
    for (int j = 0; j < OC_CAND; ++j) acc[j] += fmin(te / lam[j], xbar);
  }
  // block sums, stored trial-major: partials[j * gridDim.x + block]
  __shared__ double sh[OC_CAND][BS / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < OC_CAND; ++j) {
    const double w = wave_sum(acc[j]);
    if (lane == 0) sh[j][wid] = w;
  }
  __syncthreads();
  if (threadIdx.x < OC_CAND) {
    double v = sh[threadIdx.x][0];
    for (int w = 1; w < BS / 64; ++w) v += sh[threadIdx.x][w];
    red.partials[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = v;
  }
}

// Walk the pass's trials in sequential order: while hi - lo > tau, take the node's
// midpoint, raise lo when its sum exceeds V (go to the upper half), else lower hi.
__global__ __launch_bounds__(BS) void k_oc_walk(Red red, unsigned nblocks, double V, double tau, double* cand) {
  if (red.flags[F_OCDONE]) return;
  // totals of every trial over the blocks of k_oc_sums, in a fixed order
  __shared__ double sh[OC_CAND][BS / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int j = 0; j < OC_CAND; ++j) {
    double a = 0.0;
    for (unsigned b = threadIdx.x; b < nblocks; b += BS) a += red.partials[(size_t)j * nblocks + b];
    a = wave_sum(a);
    if (lane == 0) sh[j][wid] = a;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double tot[OC_CAND];
  for (int j = 0; j < OC_CAND; ++j) {
    double v = sh[j][0];
    for (int w = 1; w < BS / 64; ++w) v += sh[j][w];
    tot[j] = v;
  }
  double lo = red.scal[S_OCLO], hi = red.scal[S_OCHI], lam = red.scal[S_OCLAM], steps = red.scal[S_OCSTEPS];
  int node = 0;
  bool done = false;
  for (int lvl = 0; lvl < OC_LEVELS; ++lvl) {
    if (!(hi - lo > tau)) { done = true; break; }
    lam = cand[node];
    steps += 1.0;
    if (tot[node] > V) {
      lo = lam;
      node = 2 * node + 2;
    } else {
      hi = lam;
      node = 2 * node + 1;
    }
  }
  if (!(hi - lo > tau)) done = true;
  red.scal[S_OCLO] = lo;
  red.scal[S_OCHI] = hi;
  red.scal[S_OCLAM] = lam;
  red.scal[S_OCSTEPS] = steps;
  if (done) red.flags[F_OCDONE] = 1;
  else oc_tree(lo, hi, cand);
}

__global__ __launch_bounds__(BS) void k_oc_apply(const double* __restrict__ t, int64_t m, double xbar,
                                                 const double* __restrict__ blend, double* __restrict__ xn, Red red) {
  const double lam = red.scal[S_OCLAM];
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x; e < m; e += (int64_t)gridDim.x * BS) {
    double v = fmin(t[e] / lam, xbar);
    if (blend) v = 0.5 * (blend[e] + v);
    xn[e] = v;
    s += v;
  }
  const double a[1] = {s};
  block_partials<1>(a, red);
}

__global__ __launch_bounds__(BS) void k_oc_apply_fin(Red red, unsigned nblocks) {
  double tot[1];
  sum_partials<1>(red, nblocks, tot);
  if (threadIdx.x == 0) red.scal[S_OCSUM] = tot[0];
}

}  // namespace

void voc_init(hipStream_t st, const Red& red, double* cand, double lam_hi) {
  k_oc_init<<<1, 64, 0, st>>>(red, cand, lam_hi);
}
void voc_pass(hipStream_t st, const double* t, int64_t m, double xbar, double V, double tau, double* cand,
              const Red& red) {
  k_oc_sums<<<vgrid(m), BS, 0, st>>>(t, m, xbar, cand, red);
  k_oc_walk<<<1, BS, 0, st>>>(red, vgrid(m), V, tau, cand);
}
void voc_apply(hipStream_t st, const double* t, int64_t m, double xbar, const double* blend, double* x_new,
               const Red& red) {
  k_oc_apply<<<vgrid(m), BS, 0, st>>>(t, m, xbar, blend, x_new, red);
  k_oc_apply_fin<<<1, BS, 0, st>>>(red, vgrid(m));
}
template void vdot_beta<float>(hipStream_t, const double*, const float*, int64_t, const Red&, const int*);
template void vdot_beta<double>(hipStream_t, const double*, const double*, int64_t, const Red&, const int*);
template void vdot_store<float>(hipStream_t, const double*, const float*, int64_t, const Red&, int, const int*);
template void vdot_store<double>(hipStream_t, const double*, const double*, int64_t, const Red&, int, const int*);
template void vpcg_update<float>(hipStream_t, double*, double*, const double*, const double*, float*, int64_t,
                                 const Red&, const int*);
template void vpcg_update<double>(hipStream_t, double*, double*, const double*, const double*, double*, int64_t,
                                  const Red&, const int*);
template void vpcg_dir<float>(hipStream_t, double*, const float*, int64_t, const Red&, int, const int*);
template void vpcg_dir<double>(hipStream_t, double*, const double*, int64_t, const Red&, int, const int*);
template void vconvert<float, double>(hipStream_t, const double*, float*, int64_t, const int*);
template void vconvert<double, float>(hipStream_t, const float*, double*, int64_t, const int*);
template void vconvert<double, double>(hipStream_t, const double*, double*, int64_t, const int*);
template void vnormalize<float>(hipStream_t, float*, int64_t, const Red&, int);
template void vnormalize<double>(hipStream_t, double*, int64_t, const Red&, int);

}  // namespace ipmg

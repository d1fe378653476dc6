// PCG vector kernels (Algorithm PCG, Sec. 5.2) and the dense coarsest-level
// solve (Cholesky factor and explicit inverse, FP64).
#include "kernels.h"
#include "vec.h"

namespace ipmg {

namespace {

constexpr int VBLOCKS = 1024;   // grid of the streaming vector kernels

inline int vgrid(int64_t n) {
  int64_t b = (n + BS - 1) / BS;
  return (int)(b < VBLOCKS ? (b < 1 ? 1 : b) : VBLOCKS);
}

// Post-processing done by the last block of a reduction.
enum Fin { FIN_STORE = 0, FIN_ALPHA = 1, FIN_RN2 = 2, FIN_BETA = 3 };

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
  } else if (fin == FIN_RN2) {                   // convergence test on ||r||^2
    red.scal[S_RN2] = tot;
    red.flags[F_ITERS] += 1;
    if (!isfinite(tot)) {
      red.flags[F_DONE] = 2;
      red.flags[F_STATUS] = IPMG_E_BREAKDOWN;
    } else if (tot <= red.scal[S_TOL2]) {
      red.flags[F_DONE] = 1;
    }
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

// z += alpha p; r += alpha q; rT = (T) r; ||r||^2 -> convergence flag.
template <typename T>
__global__ __launch_bounds__(BS) void k_pcg_update(double* __restrict__ z, double* __restrict__ r,
                                                   const double* __restrict__ p, const double* __restrict__ q,
                                                   T* __restrict__ rT, int64_t n, Red red, const int* gate) {
  if (gate && *gate) return;
  const double alpha = red.scal[S_ALPHA];
  double s = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x; t < n; t += (int64_t)gridDim.x * BS) {
    z[t] += alpha * p[t];
    const double rn = r[t] + alpha * q[t];
    r[t] = rn;
    if (rT) rT[t] = T(rn);
    s += rn * rn;
  }
  const double v[1] = {s};
  block_partials<1>(v, red);
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

// ------------------------------------------------ dense coarsest-level solve --
// Blocked Cholesky A = L L' (lower, row-major n x n, in place) and explicit inverse
// A^-1 = L^-T L^-1 on CT x CT tiles, FP64.  Only the lower triangle of A is read;
// the strict upper triangles of L and of the tiles of L^-1 are written as zero.
constexpr int CT = 32;
constexpr int CTT = 256;   // threads per tile kernel

__device__ inline int tile_rows(int n, int t0) { return n - t0 < CT ? n - t0 : CT; }

// Lower-triangular factor of the kb x kb tile in LDS (right-looking); a pivot that
// is not positive sets the breakdown flag and continues with 1.
__device__ void tile_cholesky(double (&D)[CT][CT + 1], int kb, const Red& red) {
  for (int j = 0; j < kb; ++j) {
    if (threadIdx.x == 0) {
      double d = D[j][j];
      if (!(d > 0.0) || !isfinite(d)) { red.flags[F_BAD] = 1; d = 1.0; }
      D[j][j] = sqrt(d);
    }
    __syncthreads();
    for (int r = j + 1 + threadIdx.x; r < kb; r += CTT) D[r][j] /= D[j][j];
    __syncthreads();
    for (int t = threadIdx.x; t < CT * CT; t += CTT) {
      const int r = t / CT, c = t % CT;
      if (r > j && c > j && c <= r && r < kb) D[r][c] -= D[r][j] * D[c][j];
    }
    __syncthreads();
  }
}

// Block column starting at k0: factor the diagonal tile (every block, redundantly,
// in LDS); block 0 stores it, block b > 0 solves its panel tile X L_kk' = A_ik.
__global__ __launch_bounds__(CTT) void k_chol_panel(double* __restrict__ A, int n, int k0, Red red) {
  __shared__ double D[CT][CT + 1];
  __shared__ double P[CT][CT + 1];
  const int kb = tile_rows(n, k0);
  for (int t = threadIdx.x; t < CT * CT; t += CTT) {
    const int r = t / CT, c = t % CT;
    D[r][c] = (r < kb && c <= r) ? A[(int64_t)(k0 + r) * n + k0 + c] : 0.0;
  }
  __syncthreads();
  tile_cholesky(D, kb, red);
  if (blockIdx.x == 0) {
    for (int t = threadIdx.x; t < CT * CT; t += CTT) {
      const int r = t / CT, c = t % CT;
      if (r < kb && c < kb) A[(int64_t)(k0 + r) * n + k0 + c] = c <= r ? D[r][c] : 0.0;
    }
    return;
  }
  const int i0 = k0 + kb + (blockIdx.x - 1) * CT;
  const int ib = tile_rows(n, i0);
  for (int t = threadIdx.x; t < CT * CT; t += CTT) {
    const int r = t / CT, c = t % CT;
    P[r][c] = (r < ib && c < kb) ? A[(int64_t)(i0 + r) * n + k0 + c] : 0.0;
  }
  __syncthreads();
  for (int c = 0; c < kb; ++c) {                 // column-oriented forward substitution
    for (int r = threadIdx.x; r < ib; r += CTT) P[r][c] /= D[c][c];
    __syncthreads();
    for (int t = threadIdx.x; t < CT * CT; t += CTT) {
      const int r = t / CT, c2 = t % CT;
      if (r < ib && c2 > c && c2 < kb) P[r][c2] -= P[r][c] * D[c2][c];
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < CT * CT; t += CTT) {
    const int r = t / CT, c = t % CT;
    if (r < ib && c < kb) A[(int64_t)(i0 + r) * n + k0 + c] = P[r][c];
  }
}

// Tile index pair (I, J), 0 <= J <= I, of the t-th tile of a lower block triangle.
__device__ inline void tri_pair(int t, int& I, int& J) {
  int i = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while (i * (i + 1) / 2 > t) --i;
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  I = i;
  J = t - i * (i + 1) / 2;
}

// Trailing update after block column k0: A_IJ -= L_Ik L_Jk' for the tiles of the
// lower triangle below and right of it (one block per tile).
__global__ __launch_bounds__(CTT) void k_chol_update(double* __restrict__ A, int n, int k0) {
  __shared__ double Li[CT][CT + 1];
  __shared__ double Lj[CT][CT + 1];
  int I, J;
  tri_pair((int)blockIdx.x, I, J);
  const int kb = tile_rows(n, k0);
  const int s0 = k0 + kb;
  const int i0 = s0 + I * CT, j0 = s0 + J * CT;
  const int ib = tile_rows(n, i0), jb = tile_rows(n, j0);
  for (int t = threadIdx.x; t < CT * CT; t += CTT) {
    const int r = t / CT, c = t % CT;
    Li[r][c] = (r < ib && c < kb) ? A[(int64_t)(i0 + r) * n + k0 + c] : 0.0;
    Lj[r][c] = (r < jb && c < kb) ? A[(int64_t)(j0 + r) * n + k0 + c] : 0.0;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < CT * CT; t += CTT) {
    const int r = t / CT, c = t % CT;
    if (r >= ib || c >= jb || (I == J && c > r)) continue;
    double s = 0.0;
#pragma unroll 8
    for (int k = 0; k < CT; ++k) s += Li[r][k] * Lj[c][k];
    A[(int64_t)(i0 + r) * n + j0 + c] -= s;
  }
}

// X_ii = L_ii^-1 for every diagonal tile (one block per tile; zero above the diagonal).
__global__ __launch_bounds__(CTT) void k_tri_inv_diag(const double* __restrict__ L, double* __restrict__ X, int n) {
  __shared__ double D[CT][CT + 1];
  __shared__ double Y[CT][CT + 1];
  const int i0 = blockIdx.x * CT, ib = tile_rows(n, i0);
  for (int t = threadIdx.x; t < CT * CT; t += CTT) {
    const int r = t / CT, c = t % CT;
    D[r][c] = (r < ib && c < ib) ? L[(int64_t)(i0 + r) * n + i0 + c] : 0.0;
    Y[r][c] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int k = 0; k < ib; ++k) {                 // column-oriented forward substitution on all columns
    for (int c = threadIdx.x; c < ib; c += CTT) Y[k][c] /= D[k][k];
    __syncthreads();
    for (int t = threadIdx.x; t < CT * CT; t += CTT) {
      const int r = t / CT, c = t % CT;
      if (r > k && r < ib && c < ib) Y[r][c] -= D[r][k] * Y[k][c];
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < CT * CT; t += CTT) {
    const int r = t / CT, c = t % CT;
    if (r < ib && c < ib) X[(int64_t)(i0 + r) * n + i0 + c] = c <= r ? Y[r][c] : 0.0;
  }
}

// Right-looking block forward substitution for X = L^-1 (L X = I), in place in X
// whose strictly lower tiles start at zero and whose diagonal tiles hold L_KK^-1
// (k_tri_inv_diag).  Step K: row block K, X_KJ = L_KK^-1 B_KJ for J < K
// (k_trinv_row), then B_IJ -= L_IK X_KJ for I > K, J <= K (k_trinv_update).
// Every block does one tile product, so the depth is two launches per block row.
__global__ __launch_bounds__(CTT) void k_trinv_row(double* __restrict__ X, int n, int K) {
  __shared__ double D[CT][CT + 1];
  __shared__ double Bt[CT][CT + 1];
  const int J = blockIdx.x;                          // J < K
  const int k0 = K * CT, j0 = J * CT;
  const int kb = tile_rows(n, k0);
  for (int t = threadIdx.x; t < CT * CT; t += CTT) {
    const int r = t / CT, c = t % CT;
    D[r][c] = (r < kb && c < kb) ? X[(int64_t)(k0 + r) * n + k0 + c] : 0.0;   // L_KK^-1 (lower)
    Bt[r][c] = (r < kb) ? X[(int64_t)(k0 + r) * n + j0 + c] : 0.0;            // B_KJ (J tile full)
  }
  __syncthreads();
  for (int t = threadIdx.x; t < CT * CT; t += CTT) {
    const int r = t / CT, c = t % CT;
    if (r >= kb) continue;
    double s = 0.0;
    for (int k = 0; k <= r; ++k) s += D[r][k] * Bt[k][c];
    X[(int64_t)(k0 + r) * n + j0 + c] = s;
  }
}

__global__ __launch_bounds__(CTT) void k_trinv_update(const double* __restrict__ L, double* __restrict__ X, int n,
                                                      int K) {
  __shared__ double Ta[CT][CT + 1];
  __shared__ double Tb[CT][CT + 1];
  const int I = K + 1 + (int)blockIdx.x, J = (int)blockIdx.y;    // I > K >= J
  const int i0 = I * CT, j0 = J * CT, k0 = K * CT;               // tile K is full (K < I)
  const int ib = tile_rows(n, i0);
  for (int t = threadIdx.x; t < CT * CT; t += CTT) {
    const int r = t / CT, c = t % CT;
    Ta[r][c] = (r < ib) ? L[(int64_t)(i0 + r) * n + k0 + c] : 0.0;   // L_IK
    Tb[r][c] = X[(int64_t)(k0 + r) * n + j0 + c];                     // X_KJ
  }
  __syncthreads();
  for (int t = threadIdx.x; t < CT * CT; t += CTT) {
    const int r = t / CT, c = t % CT;
    if (r >= ib) continue;
    double s = 0.0;
#pragma unroll 8
    for (int k = 0; k < CT; ++k) s += Ta[r][k] * Tb[k][c];
    X[(int64_t)(i0 + r) * n + j0 + c] -= s;
  }
}

// Strictly lower tiles of X to zero (start of the substitution).
__global__ __launch_bounds__(CTT) void k_zero_lower_tiles(double* __restrict__ X, int n) {
  const int nt = (n + CT - 1) / CT;
  const int I = blockIdx.x % nt, J = blockIdx.x / nt;
  if (J >= I) return;
  const int i0 = I * CT, j0 = J * CT, ib = tile_rows(n, i0);
  for (int t = threadIdx.x; t < CT * CT; t += CTT) {
    const int r = t / CT, c = t % CT;
    if (r < ib) X[(int64_t)(i0 + r) * n + j0 + c] = 0.0;
  }
}

// A^-1 = X' X with X = L^-1 lower triangular: tile (I, J) = sum_{K >= max(I,J)} X_KI' X_KJ.
__global__ __launch_bounds__(CTT) void k_inv_product(const double* __restrict__ X, double* __restrict__ Ai, int n) {
  __shared__ double Ta[CT][CT + 1];
  __shared__ double Tb[CT][CT + 1];
  const int nt = (n + CT - 1) / CT;
  const int I = blockIdx.x % nt, J = blockIdx.x / nt;
  const int i0 = I * CT, j0 = J * CT;
  const int ib = tile_rows(n, i0), jb = tile_rows(n, j0);
  double acc[CT * CT / CTT];
#pragma unroll
  for (int u = 0; u < CT * CT / CTT; ++u) acc[u] = 0.0;
  for (int K = I > J ? I : J; K < nt; ++K) {
    const int k0 = K * CT, kb = tile_rows(n, k0);
    __syncthreads();
    for (int t = threadIdx.x; t < CT * CT; t += CTT) {
      const int r = t / CT, c = t % CT;
      Ta[r][c] = (r < kb && c < ib) ? X[(int64_t)(k0 + r) * n + i0 + c] : 0.0;   // X_KI
      Tb[r][c] = (r < kb && c < jb) ? X[(int64_t)(k0 + r) * n + j0 + c] : 0.0;   // X_KJ
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < CT * CT / CTT; ++u) {
      const int t = threadIdx.x + u * CTT, r = t / CT, c = t % CT;
      double s = 0.0;
#pragma unroll 8
      for (int k = 0; k < CT; ++k) s += Ta[k][r] * Tb[k][c];
      acc[u] += s;
    }
  }
#pragma unroll
  for (int u = 0; u < CT * CT / CTT; ++u) {
    const int t = threadIdx.x + u * CTT, r = t / CT, c = t % CT;
    if (r < ib && c < jb) Ai[(int64_t)(i0 + r) * n + j0 + c] = acc[u];
  }
}

// zc = A^-1 rc, one wavefront per row; eight independent accumulators keep eight
// row loads in flight per lane (the matrix is streamed once per V-cycle and needs
// that many bytes outstanding to approach the HBM rate).
template <typename T>
__global__ __launch_bounds__(BS) void k_dense_solve(const double* __restrict__ Ai, int n, const T* __restrict__ rc,
                                                    T* __restrict__ zc, const int* gate) {
  if (gate && *gate) return;
  const int row = blockIdx.x * (BS / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const double* a = Ai + (int64_t)row * n;
  double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int c = lane;
  for (; c + 7 * 64 < n; c += 8 * 64) {
    double av[8], rv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      av[u] = a[c + u * 64];
      rv[u] = (double)rc[c + u * 64];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) s[u] += av[u] * rv[u];
  }
  for (; c < n; c += 64) s[0] += a[c] * (double)rc[c];
  const double t = wave_sum(((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7])));
  if (lane == 0) zc[row] = T(t);
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
  k_pcg_update<T><<<vgrid(n), BS, 0, st>>>(z, r, p, q, rT, n, red, gate);
}
void vpcg_update_fin(hipStream_t st, int64_t n, const Red& red, const int* gate) {
  k_fin1<<<1, BS, 0, st>>>(red, vgrid(n), FIN_RN2, 0, gate);
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
void vcopy_positive(hipStream_t st, const double* src, double* dst, int64_t n, const Red& red) {
  k_copy_positive<<<vgrid(n), BS, 0, st>>>(src, dst, n, red);
}
void vset_omega(hipStream_t st, const Red& red, double* w, double* rho, int s_vav, int s_vdv, double omega,
                double product) {
  k_set_omega<<<1, 64, 0, st>>>(red, w, rho, s_vav, s_vdv, omega, product);
}
void vfill_small(hipStream_t st, double* w, int n, double value) { k_fill_value<<<1, 64, 0, st>>>(w, n, value); }
void dense_cholesky(hipStream_t st, double* A, int n, const Red& red) {
  for (int k0 = 0; k0 < n; k0 += CT) {
    const int kb = n - k0 < CT ? n - k0 : CT;
    const int m = (n - k0 - kb + CT - 1) / CT;          // tile rows below the diagonal tile
    k_chol_panel<<<1 + m, CTT, 0, st>>>(A, n, k0, red);
    if (m > 0) k_chol_update<<<m * (m + 1) / 2, CTT, 0, st>>>(A, n, k0);
  }
}
void dense_inverse(hipStream_t st, const double* L, double* Li, double* Ai, int n) {
  const int nt = (n + CT - 1) / CT;
  k_tri_inv_diag<<<nt, CTT, 0, st>>>(L, Li, n);
  if (nt > 1) k_zero_lower_tiles<<<nt * nt, CTT, 0, st>>>(Li, n);
  for (int K = 0; K < nt; ++K) {
    if (K > 0) k_trinv_row<<<K, CTT, 0, st>>>(Li, n, K);
    if (K + 1 < nt) k_trinv_update<<<dim3(nt - K - 1, K + 1), CTT, 0, st>>>(L, Li, n, K);
  }
  k_inv_product<<<nt * nt, CTT, 0, st>>>(Li, Ai, n);
}
template <typename T>
void dense_solve(hipStream_t st, const double* Ai, int n, const T* rc, T* zc, const int* gate) {
  k_dense_solve<T><<<(n + BS / 64 - 1) / (BS / 64), BS, 0, st>>>(Ai, n, rc, zc, gate);
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
template void dense_solve<float>(hipStream_t, const double*, int, const float*, float*, const int*);
template void dense_solve<double>(hipStream_t, const double*, int, const double*, double*, const int*);

}  // namespace ipmg

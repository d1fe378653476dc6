// Dense solve on the coarsest level (Algorithm MG, Sec. 5.1, exact solve with A_1):
// FP64 Cholesky factor A = L L', the inverse X = L^-1 and A^-1 = X' X, computed
// on DT x DT tiles of the packed lower block triangle (the layout is declared
// beside dense_tiles), and the product z = A^-1 r applied once per V-cycle (the
// FP32 V-cycle reads A^-1 rounded to FP32, written by the product kernel).
//
// One sweep over the block columns k does the factorization and the triangular
// inverse together, two launches per k:
//   panel:  L_ik = A_ik X_kk' (i > k), and X_kJ = X_kk B_kJ (J < k);
//   update: A_IJ -= L_Ik L_Jk' (I >= J > k), and B_IJ -= L_Ik X_kJ (I > k, J <= k),
// where B accumulates the right-looking block forward substitution L X = I; the
// block of the update that finishes A_{k+1,k+1} then forms L_{k+1,k+1} =
// chol(A_{k+1,k+1}) and X_{k+1,k+1} = L^-1 ("diag", a launch of its own for k = 0).  The
// working matrix W keeps every tile transposed (tile (I, J) holds A_IJ', then
// L_Ik' in the panel column, and X_kk' on the diagonal once factored), so every
// 64 x 64 x 64 tile product reads both operands from LDS with the summed index
// first and runs on the FP64 matrix cores (16 outputs per thread; the matrix-core
// and vector FP64 rates of gfx950 are the same, but the vector form needs 64 bytes
// of LDS per 16 FMAs and is bound by LDS bandwidth at about half of that rate).
// The padded order keeps every tile full.
#include "dense.h"

namespace ipmg {

namespace {

constexpr int DTT = 256;      // threads of the tile kernels

typedef double Tile[DT][DT];

__device__ inline void tri_index(int t, int& I, int& J) {   // t-th tile (I, J), J <= I, row order
  int i = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while (i * (i + 1) / 2 > t) --i;
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  I = i;
  J = t - i * (i + 1) / 2;
}

__device__ inline void stage(const double* __restrict__ g, Tile& s) {
  const double2* g2 = reinterpret_cast<const double2*>(g);
  double2* s2 = reinterpret_cast<double2*>(&s[0][0]);
#pragma unroll
  for (int u = 0; u < DT * DT / 2 / DTT; ++u) s2[threadIdx.x + u * DTT] = g2[threadIdx.x + u * DTT];
}

// A thread's 16 outputs of a 64 x 64 tile product, in the layout of the FP64
// matrix-core product v_mfma_f64_16x16x4f64 (checked with a probe of the builtin):
// wave w owns rows 16w..16w+15; accumulator (i, j) of lane l is row
// 16w + l/16 + 4i, column 16j + l%16.
__device__ inline int acc_row(int i) { return 16 * (int)(threadIdx.x >> 6) + (int)((threadIdx.x & 63) >> 4) + 4 * i; }
__device__ inline int acc_col(int j) { return 16 * j + (int)(threadIdx.x & 15); }

typedef double d4 __attribute__((ext_vector_type(4)));

// acc(row, col) += sum_m SA[m][row] SB[m][col] on the matrix cores: per step of
// four m, lane l supplies A[r][k] = SA[m0 + l/16][16w + l%16] and, for each column
// block j, B[k][c] = SB[m0 + l/16][16j + l%16]; four 16x16x4 products per step.
// The operands come from LDS once per product (one 8-byte read per operand), so
// the products run at the matrix cores' rate instead of the LDS bandwidth's.
__device__ inline void tile_mac(const Tile& SA, const Tile& SB, double (&acc)[4][4]) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, kr = l >> 4, lc = l & 15;
  d4 c[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) c[j] = d4{acc[0][j], acc[1][j], acc[2][j], acc[3][j]};
#pragma unroll 4
  for (int m0 = 0; m0 < DT; m0 += 4) {
    const double a = SA[m0 + kr][16 * w + lc];
    double b[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) b[j] = SB[m0 + kr][16 * j + lc];
#pragma unroll
    for (int j = 0; j < 4; ++j) c[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[j], c[j], 0, 0, 0);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i][j] = c[j][i];
}

// acc (the thread's outputs) from a global tile, or zero.
__device__ inline void acc_load(const double* __restrict__ g, double (&acc)[4][4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = g[acc_row(i) * DT + acc_col(j)];
}

__device__ inline void acc_zero(double (&acc)[4][4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
}

// g = base - acc (SUB) or g = acc; base is the tile's old content (acc_load).
template <bool SUB>
__device__ inline void acc_store(double* __restrict__ g, const double (&acc)[4][4], const double (&base)[4][4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) g[acc_row(i) * DT + acc_col(j)] = SUB ? base[i][j] - acc[i][j] : acc[i][j];
}

// Zero every tile; identity on the padded diagonal (rows >= n) when pad is set.
__global__ __launch_bounds__(DTT) void k_dense_init(double* __restrict__ A, int n, int pad) {
  int I, J;
  tri_index((int)blockIdx.x, I, J);
  double* g = A + (int64_t)blockIdx.x * DT * DT;
  for (int t = threadIdx.x; t < DT * DT; t += DTT) {
    const int r = t / DT, c = t % DT;
    g[t] = (pad && I == J && r == c && I * DT + r >= n) ? 1.0 : 0.0;
  }
}

// L_kk = chol(A_kk) and X_kk = L_kk^-1, right-looking in four panels of 16
// columns; X_kk goes to X, its transpose to W's diagonal tile (A_kk is symmetric
// there).  Lane r of wave w keeps entries 16w..16w+15 of row r of the tile and of
// column r of X (the forward substitution L x = e_r) in registers.  Panel W: the
// wave that holds it takes its 16 steps alone, with no barrier: step j takes the
// pivot from lane j, forms L_rj (lane r) and x_j = y_j / L_jj, and updates the
// panel's later columns (a_rc -= L_rj L_cj, y_c -= L_cj x_j) with L_cj read from
// lane c; then it puts the panel's L and x in LDS and, after one barrier, every
// later wave applies the 16 steps to its columns from broadcast reads.  Each
// entry sees the same fused multiply-adds in the same order as with one barrier
// per step.  A pivot that is not positive sets the breakdown flag and continues
// with 1.
__device__ inline double lane_value(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

constexpr int DW = DT / 4;   // tile columns per wave of the diagonal factor

template <int W>
__device__ inline void diag_panel(double (&row)[DW], double (&y)[DW], double (*Lc)[DT + 2], double (*Xc)[DT + 2],
                                  bool& bad) {
  const int r = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (w == W) {                             // this wave holds the panel: its 16 steps
#pragma unroll
    for (int jj = 0; jj < DW; ++jj) {
      const int j = W * DW + jj;
      double d = lane_value(row[jj], j);
      if (!(d > 0.0) || !isfinite(d)) {
        bad = true;
        d = 1.0;
      }
      double inv = __builtin_amdgcn_rsq(d);                 // 1/sqrt(d): two Newton steps
      inv = fma(0.5 * inv, fma(-d * inv, inv, 1.0), inv);
      inv = fma(0.5 * inv, fma(-d * inv, inv, 1.0), inv);
      const double sd = d * inv;
      const double lr = r > j ? row[jj] * inv : (r == j ? sd : 0.0);
      const double xj = y[jj] * inv;
      row[jj] = lr;                                          // column j of L
      y[jj] = xj;
#pragma unroll
      for (int c = jj + 1; c < DW; ++c) {
        const double l = lane_value(lr, W * DW + c);         // L_cj
        row[c] = fma(-lr, l, row[c]);
        y[c] = fma(-l, xj, y[c]);
      }
    }
#pragma unroll
    for (int jj = 0; jj < DW; ++jj) {
      Lc[W * DW + jj][r] = row[jj];
      Xc[W * DW + jj][r] = y[jj];
    }
  }
  __syncthreads();
  if (w > W) {
#pragma unroll
    for (int jj = 0; jj < DW; ++jj) {
      const int j = W * DW + jj;
      const double lr = Lc[j][r], xj = Xc[j][r];
#pragma unroll
      for (int c = 0; c < DW; ++c) {
        const double l = Lc[j][w * DW + c];
        row[c] = fma(-lr, l, row[c]);
        y[c] = fma(-l, xj, y[c]);
      }
    }
  }
}

typedef double DiagRows[DT + 2];
constexpr int DIAG_ROWS = DT * (DT + 2);   // doubles of each of the two LDS arrays of the factor

// Factor the symmetric tile A_kk held in Lc (row-major), writing X_kk to X and
// its transpose to W's diagonal tile.
__device__ __attribute__((always_inline)) inline void diag_factor(DiagRows* Lc, DiagRows* Xc, double* __restrict__ W, double* __restrict__ X,
                                   int k, const Red& red) {
  const int r = threadIdx.x & 63, w = threadIdx.x >> 6;
  double row[DW], y[DW];
#pragma unroll
  for (int c = 0; c < DW; ++c) {
    row[c] = Lc[r][w * DW + c];
    y[c] = w * DW + c == r ? 1.0 : 0.0;
  }
  __syncthreads();
  bool bad = false;
  diag_panel<0>(row, y, Lc, Xc, bad);
  diag_panel<1>(row, y, Lc, Xc, bad);
  diag_panel<2>(row, y, Lc, Xc, bad);
  diag_panel<3>(row, y, Lc, Xc, bad);
  if (bad && r == 0) red.flags[F_BAD] = 1;
  double* x = X + dense_tile_off(k, k);
  double* xt = W + dense_tile_off(k, k);
#pragma unroll
  for (int c = 0; c < DW; ++c) {
    x[(w * DW + c) * DT + r] = y[c];
    xt[r * DT + w * DW + c] = y[c];
  }
}

__global__ __launch_bounds__(DTT) void k_dense_diag(double* __restrict__ W, double* __restrict__ X, int k,
                                                    Red red) {
  __shared__ double smemA[DIAG_ROWS], smemB[DIAG_ROWS];   // separate arrays: the compiler sees no alias
  DiagRows* Lc = reinterpret_cast<DiagRows*>(smemA);
  DiagRows* Xc = reinterpret_cast<DiagRows*>(smemB);
  const double* a = W + dense_tile_off(k, k);
#pragma unroll   // all sixteen loads in flight (a rolled loop waited for each)
  for (int u = 0; u < DT * DT / DTT; ++u) {
    const int t = threadIdx.x + u * DTT;
    Lc[t / DT][t % DT] = a[t];
  }
  __syncthreads();
  diag_factor(Lc, Xc, W, X, k, red);
}

// Panel of block column k: blocks b < nt-k-1 form L_ik' = X_kk A_ik' for
// i = k+1+b (in place in W); the next k blocks form X_kJ = X_kk B_kJ (in place in X).
__global__ __launch_bounds__(DTT) void k_dense_panel(double* __restrict__ W, double* __restrict__ X, int k, int nt) {
  __shared__ Tile SA, SB;
  const int b = blockIdx.x, below = nt - k - 1;
  double* g = b < below ? W + dense_tile_off(k + 1 + b, k) : X + dense_tile_off(k, b - below);
  stage(W + dense_tile_off(k, k), SA);   // X_kk'
  stage(g, SB);                          // A_ik' or B_kJ
  __syncthreads();
  double acc[4][4];
  acc_zero(acc);
  tile_mac(SA, SB, acc);
  acc_store<false>(g, acc, acc);
}

// Trailing update after block column k: A_IJ' -= L_Jk L_Ik' for I >= J > k (first
// (nt-k-1)(nt-k)/2 blocks), then B_IJ -= L_Ik X_kJ for I > k, J <= k.
__global__ __launch_bounds__(DTT) void k_dense_update(double* __restrict__ W, double* __restrict__ X, int k,
                                                      int nt, Red red) {
  __shared__ double smemA[DIAG_ROWS], smemB[DIAG_ROWS];
  Tile& SA = *reinterpret_cast<Tile*>(smemA);
  Tile& SB = *reinterpret_cast<Tile*>(smemB);
  const int m = nt - k - 1, nchol = m * (m + 1) / 2;
  const int b = blockIdx.x;
  const double *ga, *gb;
  double* g;
  if (b < nchol) {
    int I, J;
    tri_index(b, I, J);
    I += k + 1;
    J += k + 1;
    ga = W + dense_tile_off(J, k);       // L_Jk'
    gb = W + dense_tile_off(I, k);       // L_Ik'
    g = W + dense_tile_off(I, J);
  } else {
    const int t = b - nchol;
    const int I = k + 1 + t / (k + 1), J = t % (k + 1);
    ga = W + dense_tile_off(I, k);       // L_Ik'
    gb = X + dense_tile_off(k, J);       // X_kJ
    g = X + dense_tile_off(I, J);
  }
  double old[4][4], acc[4][4];
  acc_load(g, old);
  stage(ga, SA);
  stage(gb, SB);
  __syncthreads();
  acc_zero(acc);
  tile_mac(SA, SB, acc);
  acc_store<true>(g, acc, old);
  if (b != 0 || nchol == 0) return;
  // Block 0 updated tile (k+1, k+1) for the last time: factor it here, from the
  // values in registers, instead of in a launch of its own.
  __syncthreads();                                  // SA, SB no longer read
  DiagRows* Lc = reinterpret_cast<DiagRows*>(smemA);
  DiagRows* Xc = reinterpret_cast<DiagRows*>(smemB);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) Lc[acc_row(i)][acc_col(j)] = old[i][j] - acc[i][j];
  __syncthreads();
  diag_factor(Lc, Xc, W, X, k + 1, red);
}

// A^-1 = X' X: tile (I, J), I >= J, is sum_{K >= I} X_KI' X_KJ.  Blocks run in
// row order, so the tiles with the longest sums start first.  With Af set, the
// tile is also stored rounded to FP32 (the inverse an FP32 V-cycle applies).
__global__ __launch_bounds__(DTT) void k_dense_product(const double* __restrict__ X, double* __restrict__ Ai,
                                                       float* __restrict__ Af, int nt) {
  __shared__ Tile SA, SB;
  int I, J;
  tri_index((int)blockIdx.x, I, J);
  double acc[4][4];
  acc_zero(acc);
  for (int K = I; K < nt; ++K) {
    __syncthreads();
    stage(X + dense_tile_off(K, I), SA);
    stage(X + dense_tile_off(K, J), SB);
    __syncthreads();
    tile_mac(SA, SB, acc);
  }
  acc_store<false>(Ai + dense_tile_off(I, J), acc, acc);
  if (Af) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) Af[dense_tile_off(I, J) + acc_row(i) * DT + acc_col(j)] = (float)acc[i][j];
  }
}

// z = A^-1 r, part 1 (inverse stored as M = double or float, sums in FP64):
// tile (I, J) of the packed inverse gives its row sums
// A_IJ r_J to part[I][J] and, off the diagonal, its column sums A_IJ' r_I to
// part[J][I] (64 values each), so every packed tile is read once.  Half-wave h of
// wave w reads rows w*16 + 2i + h (i < 8) as 16-byte column pairs; each row sum
// is a reduce-scatter over the 32 lanes of its half-wave (lane bits 4, 3, 2 pick
// the row, bits 1, 0 finish the sum).  The entries of r are loaded first and
// without branches (clamped index, then masked), so no wait on them stalls the
// tile loads.
template <typename T>
__device__ inline double masked_entry(const T* __restrict__ v, int i, int n) {
  const double x = (double)v[i < n ? i : n - 1];
  return i < n ? x : 0.0;
}

__device__ inline double2 pair_at(const double* __restrict__ a) { return *reinterpret_cast<const double2*>(a); }
__device__ inline double2 pair_at(const float* __restrict__ a) {
  const float2 v = *reinterpret_cast<const float2*>(a);
  return make_double2((double)v.x, (double)v.y);
}

template <typename T, typename M>
__global__ __launch_bounds__(DTT) void k_dense_apply(const M* __restrict__ Ai, int n, int nt,
                                                     const T* __restrict__ rc, double* __restrict__ part,
                                                     const int* gate) {
  if (gate && *gate) return;
  __shared__ double C[DTT / 64][DT];
  int I, J;
  tri_index((int)blockIdx.x, I, J);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int h = lane >> 5, c2 = 2 * (lane & 31);
  const int cj = J * DT + c2;
  const double rj0 = masked_entry(rc, cj, n), rj1 = masked_entry(rc, cj + 1, n);
  double ri[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) ri[i] = masked_entry(rc, I * DT + w * 16 + 2 * i + h, n);
  const M* a = Ai + (int64_t)blockIdx.x * DT * DT;
  double2 v[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = pair_at(a + (w * 16 + 2 * i + h) * DT + c2);
  double p[8], cs0 = 0.0, cs1 = 0.0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    p[i] = fma(v[i].x, rj0, v[i].y * rj1);
    cs0 = fma(v[i].x, ri[i], cs0);
    cs1 = fma(v[i].y, ri[i], cs1);
  }
  cs0 += __shfl_xor(cs0, 32);
  cs1 += __shfl_xor(cs1, 32);
  if (h == 0) {
    C[w][c2] = cs0;
    C[w][c2 + 1] = cs1;
  }
  const bool b4 = lane & 16, b3 = lane & 8, b2 = lane & 4;
  double q4[4], q2[2];
#pragma unroll
  for (int i = 0; i < 4; ++i) q4[i] = (b4 ? p[i + 4] : p[i]) + __shfl_xor(b4 ? p[i] : p[i + 4], 16);
#pragma unroll
  for (int i = 0; i < 2; ++i) q2[i] = (b3 ? q4[i + 2] : q4[i]) + __shfl_xor(b3 ? q4[i] : q4[i + 2], 8);
  double q = (b2 ? q2[1] : q2[0]) + __shfl_xor(b2 ? q2[0] : q2[1], 4);
  q += __shfl_xor(q, 2);
  q += __shfl_xor(q, 1);
  if ((lane & 3) == 0) {
    const int i = (b4 ? 4 : 0) + (b3 ? 2 : 0) + (b2 ? 1 : 0);
    part[((int64_t)I * nt + J) * DT + w * 16 + 2 * i + h] = q;
  }
  __syncthreads();
  if (I != J && threadIdx.x < DT)
    part[((int64_t)J * nt + I) * DT + threadIdx.x] =
        (C[0][threadIdx.x] + C[1][threadIdx.x]) + (C[2][threadIdx.x] + C[3][threadIdx.x]);
}

// z = A^-1 r, part 2: z_i = sum_K part[i / 64][K][i % 64] (one block per block
// row; wave w loads every fourth K at once).
constexpr int FIN_LOADS = (DENSE_MAX_TILES + DTT / 64 - 1) / (DTT / 64);

template <typename T>
__global__ __launch_bounds__(DTT) void k_dense_apply_fin(const double* __restrict__ part, int n, int nt,
                                                         T* __restrict__ zc, const int* gate) {
  if (gate && *gate) return;
  __shared__ double S[DTT / 64][DT];
  const int I = blockIdx.x, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double* p = part + (int64_t)I * nt * DT + lane;
  double v[FIN_LOADS];
#pragma unroll
  for (int u = 0; u < FIN_LOADS; ++u) {
    const int K = w + u * (DTT / 64);
    v[u] = K < nt ? p[(int64_t)K * DT] : 0.0;
  }
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < FIN_LOADS; ++u) s += v[u];
  S[w][lane] = s;
  __syncthreads();
  const int g = I * DT + threadIdx.x;
  if (threadIdx.x < DT && g < n)
    zc[g] = T((S[0][threadIdx.x] + S[1][threadIdx.x]) + (S[2][threadIdx.x] + S[3][threadIdx.x]));
}

}  // namespace

void dense_init(hipStream_t st, double* A, int n, int pad) {
  const int nt = dense_tiles(n);
  k_dense_init<<<nt * (nt + 1) / 2, DTT, 0, st>>>(A, n, pad);
}

void dense_factor_inverse(hipStream_t st, double* W, double* X, double* Ai, int n, const Red& red, float* Af) {
  const int nt = dense_tiles(n);
  k_dense_init<<<nt * (nt + 1) / 2, DTT, 0, st>>>(X, n, 0);
  k_dense_diag<<<1, DTT, 0, st>>>(W, X, 0, red);
  for (int k = 0; k < nt; ++k) {                  // the update of step k factors diagonal tile k+1
    const int m = nt - k - 1;
    if (nt > 1) k_dense_panel<<<nt - 1, DTT, 0, st>>>(W, X, k, nt);
    const int nu = m * (m + 1) / 2 + m * (k + 1);
    if (nu > 0) k_dense_update<<<nu, DTT, 0, st>>>(W, X, k, nt, red);
  }
  k_dense_product<<<nt * (nt + 1) / 2, DTT, 0, st>>>(X, Ai, Af, nt);
}

template <typename T, typename M>
void dense_apply(hipStream_t st, const M* Ai, double* part, int n, const T* rc, T* zc, const int* gate) {
  const int nt = dense_tiles(n);
  k_dense_apply<T, M><<<nt * (nt + 1) / 2, DTT, 0, st>>>(Ai, n, nt, rc, part, gate);
  k_dense_apply_fin<T><<<nt, DTT, 0, st>>>(part, n, nt, zc, gate);
}

template void dense_apply<float, double>(hipStream_t, const double*, double*, int, const float*, float*, const int*);
template void dense_apply<float, float>(hipStream_t, const float*, double*, int, const float*, float*, const int*);
template void dense_apply<double, double>(hipStream_t, const double*, double*, int, const double*, double*,
                                          const int*);

}  // namespace ipmg

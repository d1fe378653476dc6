// Coarse tail of the V-cycle: the smallest levels of Algorithm MG (pre-smoothing,
// restriction, coarsest solve, prolongation, post-smoothing) executed by a single
// workgroup in one launch.  Level vectors live in LDS; element matrices, border
// vectors and the coarsest inverse are read from global memory (L2-resident).
// On the small levels a kernel launch costs more than the work, so one launch
// replaces about seven per level.
#pragma once
#include "kernels.h"

namespace ipmg {

constexpr int TAIL_THREADS = 1024;
constexpr int MAX_TAIL = 12;

template <typename T>
struct TailLev {
  Dims d;
  const T* E;          // element matrices (nullptr: the finest level, top operator)
  const T* b;          // border of the augmented system (nullptr for K)
  const double* omg;   // damping weight (device)
  int off;             // offset of this level's three vectors in LDS (elements of T)
};

template <typename T>
struct TailArgs {
  TailLev<T> lv[MAX_TAIL];
  int nt;              // number of tail levels; lv[0] is the coarsest, lv[nt-1] the top
  const T* rin;        // right-hand side of the top level (global)
  T* zout;             // result of the top level (global)
  const double* Ainv;  // dense inverse of the coarsest operator (FP64, packed tiles)
  int n0;              // its size
  double c;            // corner of the augmented system
  int aug, nu1, nu2;
};

__device__ inline double block_sum_tail(double v, double* sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < TAIL_THREADS / 64; ++w) s += sh[w];
  return s;
}

// One level pass (mode as in k_level) by the whole workgroup.
template <int DIM, typename T, class Op, int MODE>
__device__ inline void tail_pass(const Op& op, const TailLev<T>& L, const T* v, const T* r, T* out, double c,
                                 double* sh) {
  const Dims& d = L.d;
  const T omega = L.omg ? T(*L.omg) : T(0);
  const T vl = (L.b && MODE != M_JACOBI0) ? v[d.nslots] : T(0);
  double bdot = 0.0, r0 = 0.0, r1 = 0.0;
  for (int64_t q = threadIdx.x; q < d.nnodes; q += TAIL_THREADS) {
    const int i = (int)(q % d.nx1), j = (int)((q / d.nx1) % d.ny1), k = (int)(q / ((int64_t)d.nx1 * d.ny1));
    level_node<DIM, T, Op, MODE>(op, d, i, j, k, v, r, out, omega, L.b, vl, 1.0, nullptr, bdot, r0, r1);
  }
  if (L.b) {
    if constexpr (MODE == M_JACOBI0) {
      if (threadIdx.x == 0) out[d.nslots] = T((double)omega * (double)r[d.nslots] / c);
    } else {
      const double tot = block_sum_tail(bdot, sh);
      if (threadIdx.x == 0) {
        const double rowl = tot + c * (double)vl;
        if constexpr (MODE == M_RESID) out[d.nslots] = T((double)r[d.nslots] - rowl);
        if constexpr (MODE == M_JACOBI) out[d.nslots] = T((double)vl + (double)omega * ((double)r[d.nslots] - rowl) / c);
      }
    }
  }
  __syncthreads();
}

template <int DIM, typename T>
__device__ inline void tail_restrict(const Dims& f, const Dims& cd, const T* rf, T* rc, int aug) {
  for (int64_t qc = threadIdx.x; qc < cd.nnodes; qc += TAIL_THREADS) {
    const int I = (int)(qc % cd.nx1), J = (int)((qc / cd.nx1) % cd.ny1), K = (int)(qc / ((int64_t)cd.nx1 * cd.ny1));
    T acc[DIM];
#pragma unroll
    for (int cc = 0; cc < DIM; ++cc) acc[cc] = T(0);
    if (I > 0) {
      for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            const int i = 2 * I + dx, j = 2 * J + dy, k = 2 * K + dz;
            if (i < 1 || i >= f.nx1 || j < 0 || j >= f.ny1 || k < 0 || k >= f.nz1) continue;
            const T w = T(w1(dx) * w1(dy) * (DIM == 3 ? w1(dz) : 1.0f));
            const int64_t qf = ((int64_t)k * f.ny1 + j) * f.nx1 + i;
#pragma unroll
            for (int cc = 0; cc < DIM; ++cc) acc[cc] += w * rf[qf * DIM + cc];
          }
    }
#pragma unroll
    for (int cc = 0; cc < DIM; ++cc) rc[qc * DIM + cc] = acc[cc];
  }
  if (aug && threadIdx.x == 0) rc[cd.nslots] = rf[f.nslots];
  __syncthreads();
}

template <int DIM, typename T>
__device__ inline void tail_prolong(const Dims& f, const Dims& cd, T* z, const T* zc, int aug) {
  for (int64_t q = threadIdx.x; q < f.nnodes; q += TAIL_THREADS) {
    const int i = (int)(q % f.nx1), j = (int)((q / f.nx1) % f.ny1), k = (int)(q / ((int64_t)f.nx1 * f.ny1));
    if (i == 0) continue;
    const int ni = (i & 1) ? 2 : 1, nj = (j & 1) ? 2 : 1, nk = (DIM == 3 && (k & 1)) ? 2 : 1;
    T acc[DIM];
#pragma unroll
    for (int cc = 0; cc < DIM; ++cc) acc[cc] = z[q * DIM + cc];
    for (int a = 0; a < nk; ++a)
      for (int b = 0; b < nj; ++b)
        for (int e = 0; e < ni; ++e) {
          const int I = (i >> 1) + e, J = (j >> 1) + b, K = DIM == 3 ? (k >> 1) + a : 0;
          const T w = T((ni == 2 ? 0.5f : 1.0f) * (nj == 2 ? 0.5f : 1.0f) * (nk == 2 ? 0.5f : 1.0f));
          const int64_t qc = ((int64_t)K * cd.ny1 + J) * cd.nx1 + I;
#pragma unroll
          for (int cc = 0; cc < DIM; ++cc) acc[cc] += w * zc[qc * DIM + cc];
        }
#pragma unroll
    for (int cc = 0; cc < DIM; ++cc) z[q * DIM + cc] = acc[cc];
  }
  if (aug && threadIdx.x == 0) z[f.nslots] += zc[cd.nslots];
  __syncthreads();
}

// Smoothing / residual pass on tail level k with the right operator.
template <int DIM, typename T, class TopOp, int MODE>
__device__ inline void tail_level_pass(const TopOp& top, bool top_is_fine, const TailArgs<T>& a, int k, const T* v,
                                       const T* r, T* out, double* sh) {
  const TailLev<T>& L = a.lv[k];
  if (k == a.nt - 1 && top_is_fine) tail_pass<DIM, T, TopOp, MODE>(top, L, v, r, out, a.c, sh);
  else tail_pass<DIM, T, OpCoarse<DIM, T>, MODE>(OpCoarse<DIM, T>{L.E, L.d.m}, L, v, r, out, a.c, sh);
}

template <int DIM, typename T, class TopOp>
__global__ __launch_bounds__(TAIL_THREADS) void k_tail(TopOp top, int top_is_fine, TailArgs<T> a, const int* gate) {
  if (gate && *gate) return;
  extern __shared__ __align__(16) unsigned char tail_smem[];
  T* sm = reinterpret_cast<T*>(tail_smem);
  __shared__ double sh[TAIL_THREADS / 64];
  const int nt = a.nt;
  T* cur[MAX_TAIL];
  T* nxt[MAX_TAIL];
  // top right-hand side into LDS
  {
    const TailLev<T>& L = a.lv[nt - 1];
    T* r = sm + L.off;
    const int64_t n = L.d.nslots + a.aug;
    for (int64_t t = threadIdx.x; t < n; t += TAIL_THREADS) r[t] = a.rin[t];
  }
  __syncthreads();
  for (int k = nt - 1; k >= 1; --k) {                      // down: pre-smooth, restrict
    const TailLev<T>& L = a.lv[k];
    const int64_t n1 = L.d.nslots + 1;
    T* r = sm + L.off;
    T* x0 = r + n1;
    T* x1 = x0 + n1;
    tail_level_pass<DIM, T, TopOp, M_JACOBI0>(top, top_is_fine, a, k, nullptr, r, x0, sh);
    for (int s = 1; s < a.nu1; ++s) {
      tail_level_pass<DIM, T, TopOp, M_JACOBI>(top, top_is_fine, a, k, x0, r, x1, sh);
      T* t = x0; x0 = x1; x1 = t;
    }
    tail_level_pass<DIM, T, TopOp, M_RESID>(top, top_is_fine, a, k, x0, r, x1, sh);
    tail_restrict<DIM, T>(L.d, a.lv[k - 1].d, x1, sm + a.lv[k - 1].off, a.aug);
    cur[k] = x0;
    nxt[k] = x1;
  }
  {                                                        // coarsest: dense solve
    const TailLev<T>& L = a.lv[0];
    const int64_t n1 = L.d.nslots + 1;
    T* r = sm + L.off;
    T* z = r + n1;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int row = wid; row < a.n0; row += TAIL_THREADS / 64) {
      double s = 0.0;
      for (int col = lane; col < a.n0; col += 64) s += a.Ainv[dense_sym_at(row, col)] * (double)r[col];
      s = wave_sum(s);
      if (lane == 0) z[row] = T(s);
    }
    cur[0] = z;
    __syncthreads();
  }
  for (int k = 1; k < nt; ++k) {                           // up: prolong, post-smooth
    const TailLev<T>& L = a.lv[k];
    T* r = sm + L.off;
    tail_prolong<DIM, T>(L.d, a.lv[k - 1].d, cur[k], cur[k - 1], a.aug);
    for (int s = 0; s < a.nu2; ++s) {
      tail_level_pass<DIM, T, TopOp, M_JACOBI>(top, top_is_fine, a, k, cur[k], r, nxt[k], sh);
      T* t = cur[k]; cur[k] = nxt[k]; nxt[k] = t;
    }
  }
  {
    const TailLev<T>& L = a.lv[nt - 1];
    const int64_t n = L.d.nslots + a.aug;
    T* z = nt > 1 ? cur[nt - 1] : cur[0];
    for (int64_t t = threadIdx.x; t < n; t += TAIL_THREADS) a.zout[t] = z[t];
  }
}

}  // namespace ipmg

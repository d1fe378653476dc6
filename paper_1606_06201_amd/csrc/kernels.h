// Device kernels of the ipmg library, generic in the dimension (2: bilinear
// quadrilaterals, 3: trilinear hexahedra) and in the V-cycle precision.
// Included by one translation unit per dimension (ops2d.hip, ops3d.hip).
#pragma once
#include <type_traits>

#include "common.h"

namespace ipmg {

// Element stiffness of the unit element, uploaded once per context
// (computed by k_element_stiffness below).  Row-major ND x ND.
static __constant__ double cK0d[576];
static __constant__ float cK0f[576];
// Galerkin images G_q = W_q' K0 W_q of the unit element on the next coarser grid,
// one 8x8 matrix per sub-element q of a coarse 2D element (row-major, q-major).
// With the square-element symmetry of K0 every entry is a signed copy of one of 18
// values: G[t] = sign * g[k] with kSqG2d[t] = sign * (k + 1).  The kernels keep the
// 18 values in scalar registers instead of loading 256 constants; the table follows
// from the structure of W_q and kSq2d and is checked against the computed images at
// set-up.
static __constant__ double cG18d[18];
static __constant__ float cG18f[18];
constexpr signed char kSqG2d[256] = {
      1,   2,   3,   4,   5,   6,   7,   8,   2,   1,   8,   7,   6,   5,   4,   3,
      3,   8,   9,   6,  10,  11,   5,  12,   4,   7,   6,  13,  14,  15,  16,   5,
      5,   6,  10,  14,  17,  18,  15,  11,   6,   5,  11,  15,  18,  17,  14,  10,
      7,   4,   5,  16,  15,  14,  13,   6,   8,   3,  12,   5,  11,  10,   6,   9,
      9,  -6,   3,  -8,   5, -12,  10, -11,  -6,  13,  -4,   7, -16,   5, -14,  15,
      3,  -4,   1,  -2,   7,  -8,   5,  -6,  -8,   7,  -2,   1,  -4,   3,  -6,   5,
      5, -16,   7,  -4,  13,  -6,  15, -14, -12,   5,  -8,   3,  -6,   9, -11,  10,
     10, -14,   5,  -6,  15, -11,  17, -18, -11,  15,  -6,   5, -14,  10, -18,  17,
     13,  -6,  15, -14,   5, -16,   7,  -4,  -6,   9, -11,  10, -12,   5,  -8,   3,
     15, -11,  17, -18,  10, -14,   5,  -6, -14,  10, -18,  17, -11,  15,  -6,   5,
      5, -12,  10, -11,   9,  -6,   3,  -8, -16,   5, -14,  15,  -6,  13,  -4,   7,
      7,  -8,   5,  -6,   3,  -4,   1,  -2,  -4,   3,  -6,   5,  -8,   7,  -2,   1,
     17,  18,  15,  11,   5,   6,  10,  14,  18,  17,  14,  10,   6,   5,  11,  15,
     15,  14,  13,   6,   7,   4,   5,  16,  11,  10,   6,   9,   8,   3,  12,   5,
      5,   6,   7,   8,   1,   2,   3,   4,   6,   5,   4,   3,   2,   1,   8,   7,
     10,  11,   5,  12,   3,   8,   9,   6,  14,  15,  16,   5,   4,   7,   6,  13};

template <typename T> __device__ inline T k0(int idx);
template <> __device__ inline double k0<double>(int idx) { return cK0d[idx]; }
template <> __device__ inline float k0<float>(int idx) { return cK0f[idx]; }
template <typename T> __device__ inline T g2(int idx);
// Square-element symmetry of the 2D Q1 element matrix (isotropic material, nodes
// counter-clockwise, DOFs x/y interleaved): every entry is a signed copy of an
// entry of the first row, K0[r][c] = sign * K0[0][t] with kSq2d[8r+c] = sign*(t+1).
// Only six distinct values occur, so the 2D kernels keep six constants live instead
// of 64.  Checked against the computed element matrix at set-up.
constexpr signed char kSq2d[64] = { 1,  2,  3,  4,  5, -2,  7, -4,
                                   2,  1, -4,  7, -2,  5,  4,  3,
                                   3, -4,  1, -2,  7,  4,  5,  2,
                                   4,  7, -2,  1, -4,  3,  2,  5,
                                   5, -2,  7, -4,  1,  2,  3,  4,
                                  -2,  5,  4,  3,  2,  1, -4,  7,
                                   7,  4,  5,  2,  3, -4,  1, -2,
                                  -4,  3,  2,  5,  4,  7, -2,  1};
template <typename T>
__device__ inline T k0sq(int r, int c) {
  const int t = kSq2d[r * 8 + c];
  return t > 0 ? k0<T>(t - 1) : -k0<T>(-t - 1);
}
// Cube symmetry of the 3D Q1 element matrix (isotropic material, unit cube): with
// s = position(b) - position(a) of the two nodes, the entry of rows (a, c) and
// columns (b, c') depends only on |s| component by component, and off the 3 x 3
// diagonal blocks on the sign (2 a_c - 1)(2 b_c' - 1) of the two shape-function
// slopes: 14 slots, slot 0..5 for c = c' (|s_c|, number of other nonzero s_k), slot
// 6..13 for c != c' (|s_c|, |s_c'|, |s_other|).  With the element loops unrolled the
// slot and sign of every entry are compile-time, so the 3D kernels keep 14
// constants in scalar registers instead of loading 576.  Checked against the
// computed element matrix at set-up.
__host__ __device__ constexpr int k0cube_slot(int r, int col) {
  const int a = r / 3, c = r % 3, b = col / 3, cp = col % 3;
  const int pa[3] = {loc_x(a), loc_y(a), loc_z(a)}, pb[3] = {loc_x(b), loc_y(b), loc_z(b)};
  int as[3] = {0, 0, 0};
  for (int k = 0; k < 3; ++k) as[k] = pb[k] != pa[k] ? 1 : 0;
  if (c == cp) {
    int others = 0;
    for (int k = 0; k < 3; ++k) others += (k != c) ? as[k] : 0;
    return 1 + as[c] * 3 + others;
  }
  const int o = 3 - c - cp;
  const int slot = 6 + as[c] * 4 + as[cp] * 2 + as[o];
  const int sg = (2 * pa[c] - 1) * (2 * pb[cp] - 1);
  return sg * (slot + 1);
}
static __constant__ double cK3d[14];
static __constant__ float cK3f[14];
template <typename T> __device__ inline T k3c(int slot);
template <> __device__ inline double k3c<double>(int slot) { return cK3d[slot]; }
template <> __device__ inline float k3c<float>(int slot) { return cK3f[slot]; }
template <typename T>
__device__ inline T k0cube(int r, int c) {
  const int t = k0cube_slot(r, c);
  return t > 0 ? k3c<T>(t - 1) : -k3c<T>(-t - 1);
}

// Entry (r, c) of the element matrix of the dimension (in 3D from the full table:
// the generic passes index it with a run-time row; node_apply_fine3 uses k0cube).
template <int DIM, typename T>
__device__ inline T k0rc(int r, int c) {
  if constexpr (DIM == 2) return k0sq<T>(r, c);
  else return k0<T>(r * Geo<DIM>::ND + c);
}

template <> __device__ inline double g2<double>(int idx) {
  const int t = kSqG2d[idx];
  return t > 0 ? cG18d[t - 1] : -cG18d[-t - 1];
}
template <> __device__ inline float g2<float>(int idx) {
  const int t = kSqG2d[idx];
  return t > 0 ? cG18f[t - 1] : -cG18f[-t - 1];
}

// ------------------------------------------------------------------ reductions --
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ inline double load_acquire(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// XCD-aware tile order.  The dispatcher deals workgroups round-robin over the
// GPU's 8 XCDs, each with its own L2.  Mapping linear block b (XCD b % 8, local
// index b / 8) to tile start(b % 8) + b / 8 gives every XCD a contiguous band of
// tiles, so the halo rows a tile shares with the tile above were fetched into the
// same L2 shortly before.  The map is a bijection on [0, nblocks).
constexpr unsigned NXCD = 8;
struct Tile { unsigned x, y, z; };
__device__ inline Tile xcd_tile() {
  const unsigned gx = gridDim.x, gy = gridDim.y;
  const unsigned nb = gx * gy * gridDim.z;
  const unsigned b = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const unsigned k = b % NXCD, l = b / NXCD;
  const unsigned q = nb / NXCD, rem = nb % NXCD;
  const unsigned t = k * q + (k < rem ? k : rem) + l;
  return Tile{t % gx, (t / gx) % gy, t / (gx * gy)};
}

// Deterministic two-stage reductions.  Stage 1 (inside a kernel): every block
// reduces its threads' values in a fixed order and writes one partial per value
// to red.partials[n * MAX_PARTIALS + block].  Stage 2 (a one-block finalize kernel
// launched next on the same stream): sum_partials adds the partials in block
// order.  Cross-block communication inside a kernel would need a device-scope
// release per block, which on a multi-XCD GPU writes back each XCD's L2 and
// serialises the blocks; the kernel boundary provides the visibility instead.
__device__ inline unsigned block_id() { return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z); }

template <int NV, bool IS_MIN = false, int NT = BS>
__device__ void block_partials(const double (&v)[NV], const Red& red) {
  __shared__ double sh[NV][NT / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int n = 0; n < NV; ++n) {
    const double s = IS_MIN ? wave_min(v[n]) : wave_sum(v[n]);
    if (lane == 0) sh[n][wid] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned bid = block_id();
#pragma unroll
    for (int n = 0; n < NV; ++n) {
      double s = sh[n][0];
      for (int w = 1; w < NT / 64; ++w) s = IS_MIN ? fmin(s, sh[n][w]) : s + sh[n][w];
      red.partials[(size_t)n * MAX_PARTIALS + bid] = s;
    }
  }
}

// Stage 2, called by all BS threads of a single block; totals valid in every thread.
// Four independent accumulators per thread keep several loads in flight (the
// partials come from other XCDs' L2s through memory, so latency dominates).
template <int NV, bool IS_MIN = false>
__device__ void sum_partials(const Red& red, unsigned nblocks, double (&tot)[NV]) {
  __shared__ double sh[NV][BS / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const double init = IS_MIN ? INFINITY : 0.0;
  double acc[NV][4];
#pragma unroll
  for (int n = 0; n < NV; ++n)
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[n][u] = init;
  unsigned b = threadIdx.x;
  for (; b + 3 * BS < nblocks; b += 4 * BS) {
    double p[NV][4];
#pragma unroll
    for (int n = 0; n < NV; ++n)
#pragma unroll
      for (int u = 0; u < 4; ++u) p[n][u] = red.partials[(size_t)n * MAX_PARTIALS + b + u * BS];
#pragma unroll
    for (int n = 0; n < NV; ++n)
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[n][u] = IS_MIN ? fmin(acc[n][u], p[n][u]) : acc[n][u] + p[n][u];
  }
  for (; b < nblocks; b += BS) {
#pragma unroll
    for (int n = 0; n < NV; ++n) {
      const double p = red.partials[(size_t)n * MAX_PARTIALS + b];
      acc[n][0] = IS_MIN ? fmin(acc[n][0], p) : acc[n][0] + p;
    }
  }
#pragma unroll
  for (int n = 0; n < NV; ++n) {
    double s = IS_MIN ? fmin(fmin(acc[n][0], acc[n][1]), fmin(acc[n][2], acc[n][3]))
                      : (acc[n][0] + acc[n][1]) + (acc[n][2] + acc[n][3]);
    s = IS_MIN ? wave_min(s) : wave_sum(s);
    if (lane == 0) sh[n][wid] = s;
  }
  __syncthreads();
#pragma unroll
  for (int n = 0; n < NV; ++n) {
    double s = sh[n][0];
    for (int w = 1; w < BS / 64; ++w) s = IS_MIN ? fmin(s, sh[n][w]) : s + sh[n][w];
    tot[n] = s;
  }
}

// Convergence test of a PCG step on ||r||^2 (Algorithm PCG, stopping rule):
// counts the step, sets the done flag when ||r||^2 <= tol^2 and the breakdown
// flag when it is not finite; zpend marks the step's z += alpha p as pending
// (done by the next direction kernel).  One thread.
__device__ inline void rn2_finish(double tot, const Red& red, bool zpend) {
  if (zpend) red.flags[F_ZPEND] = 1;
  red.scal[S_RN2] = tot;
  red.flags[F_ITERS] += 1;
  if (!isfinite(tot)) {
    red.flags[F_DONE] = 2;
    red.flags[F_STATUS] = IPMG_E_BREAKDOWN;
  } else if (tot <= red.scal[S_TOL2]) {
    red.flags[F_DONE] = 1;
  }
}

// --------------------------------------------------------------- operators ----
// Each operator gives, for element e and local node a, the contribution of the
// element matrix rows (a,c) times the local vector ve, and the diagonal entries.

// K(x) on the finest grid: A_e = x_e K0 (Sec. 1, problem (1)).
template <int DIM, typename T>
struct OpFineK {
  const T* x;
  int64_t m;
  const T* ye = nullptr;    // 3D: element products of the pass's vector (k_elem_fine3e)
  const T* dgn = nullptr;   // 3D: the diagonal per DOF slot, formed at set-up (k_fine_diag3)
  __device__ inline void rows(int64_t e, int, int, int, int a, const T* ve, T* acc) const {
    constexpr int ND = Geo<DIM>::ND;
    const T xe = x[e];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      const int r = a * DIM + c;
      T s = 0;
#pragma unroll
      for (int col = 0; col < ND; ++col) s += k0rc<DIM, T>(r, col) * ve[col];
      acc[c] += xe * s;
    }
  }
  __device__ inline void diag(int64_t e, int, int, int, int a, T* dg) const {
    constexpr int ND = Geo<DIM>::ND;
    const T xe = x[e];
#pragma unroll
    for (int c = 0; c < DIM; ++c) dg[c] += xe * k0rc<DIM, T>(a * DIM + c, a * DIM + c);
  }
  __device__ inline double entry(int64_t e, int r, int c) const {
    return (double)x[e] * (double)k0<T>(r * Geo<DIM>::ND + c);
  }
};

// Displacement block of the augmented Newton matrix on the finest grid:
// A_e = x_e K0 + h_e h_e', h_e = sqrt(1/D_e) K0 u_e (eq. (nwtr2Z)).  h is stored
// component-major: h[col * m + e].
template <int DIM, typename T>
struct OpFineZ {
  const T* x;
  const T* h;
  int64_t m;
  const T* hs = nullptr;   // h_e'v_e per element, formed beforehand by k_elem_hv (same sum)
  const T* ye = nullptr;   // 3D: element products of the pass's vector (k_elem_fine3e)
  const T* dgn = nullptr;  // 3D: the diagonal per DOF slot, formed at set-up (k_fine_diag3)
  // rows() sums h_e'v_e over ve itself: its callers may map an element outside the
  // grid to element 0 with a zero ve, where hs[0] would not be zero.
  __device__ inline void rows(int64_t e, int, int, int, int a, const T* ve, T* acc) const {
    rows_keep(e, a, ve, T(1), acc, false);
  }
  // keep = 0: an element outside the grid that the gather maps to element 0 (its
  // ve is zero, but hs[0] is element 0's value, so that term is scaled away).
  __device__ inline void rows_keep(int64_t e, int a, const T* ve, T keep, T* acc, bool use_hs = true) const {
    constexpr int ND = Geo<DIM>::ND;
    const T xe = x[e];
    T hv = 0;
    if (hs && use_hs) {
      hv = hs[e] * keep;
    } else {
#pragma unroll
      for (int col = 0; col < ND; ++col) hv += h[col * m + e] * ve[col];
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      const int r = a * DIM + c;
      T s = 0;
#pragma unroll
      for (int col = 0; col < ND; ++col) s += k0rc<DIM, T>(r, col) * ve[col];
      acc[c] += xe * s + h[r * m + e] * hv;
    }
  }
  __device__ inline void diag(int64_t e, int, int, int, int a, T* dg) const {
    constexpr int ND = Geo<DIM>::ND;
    const T xe = x[e];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      const int r = a * DIM + c;
      const T hr = h[r * m + e];
      dg[c] += xe * k0rc<DIM, T>(r, r) + hr * hr;
    }
  }
  __device__ inline double entry(int64_t e, int r, int c) const {
    return (double)x[e] * (double)k0<T>(r * Geo<DIM>::ND + c) +
           (double)h[r * m + e] * (double)h[c * m + e];
  }
};

// Coarse level: general symmetric element matrices from the Galerkin products,
// packed upper-triangular, stored E[sym(r,c) * m + e].
// ye (3D): the element products y_e = E_e v_e of the pass's vector, formed
// beforehand by k_elem_apply3 (component-major, ye[r * m + e]); the node passes
// then read three values per element instead of its 72 matrix entries and 24
// nodal values.
template <int DIM, typename T>
struct OpCoarse {
  const T* E;
  int64_t m;
  const T* ye = nullptr;
  // Entry k of every element starts at the uniform address E + k m, so a load is
  // that base plus the element's 32-bit offset (no per-load 64-bit arithmetic).
  __device__ inline void rows(int64_t e, int, int, int, int a, const T* ve, T* acc) const {
    constexpr int ND = Geo<DIM>::ND;
    const uint32_t e32 = (uint32_t)e;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      const int r = a * DIM + c;
      T s = 0;
#pragma unroll
      for (int col = 0; col < ND; ++col) s += (E + sym_index(r, col, ND) * m)[e32] * ve[col];
      acc[c] += s;
    }
  }
  __device__ inline void diag(int64_t e, int, int, int, int a, T* dg) const {
    constexpr int ND = Geo<DIM>::ND;
    const uint32_t e32 = (uint32_t)e;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      const int r = a * DIM + c;
      dg[c] += (E + sym_index(r, r, ND) * m)[e32];
    }
  }
  __device__ inline double entry(int64_t e, int r, int c) const {
    return (double)E[sym_index(r, c, Geo<DIM>::ND) * m + e];
  }
};

// First coarse level of K(x) in 2D, evaluated from the finest densities instead
// of stored element matrices: A_C = sum_q x_{e(C,q)} G_q over the four fine
// elements of C (the Galerkin product of the x-scaled unit element).  Reads one
// density per fine element instead of 36 matrix entries per coarse element.
template <int DIM, typename T>
struct OpCoarse2K {
  const T* x;      // finest-level densities, followed by a zero pad of fnx + 2 entries
  int fnx;         // finest-level elements along x
  int64_t fm;      // finest-level element count (start of the zero pad)
  __device__ inline void xs(int ei, int ej, T* xq) const { xs_at((int64_t)(2 * ej) * fnx + 2 * ei, xq); }
  // ok false: the four values come from the zero pad (an element outside the grid)
  __device__ inline void xs_or_zero(bool ok, int ei, int ej, T* xq) const {
    xs_at(ok ? (int64_t)(2 * ej) * fnx + 2 * ei : fm, xq);
  }
  __device__ inline void xs_at(int64_t b, T* xq) const {
    xq[0] = x[b];
    xq[1] = x[b + 1];
    xq[2] = x[b + fnx];
    xq[3] = x[b + fnx + 1];
  }
  // The four densities are loaded before the sub-element loop; the G_q entries are
  // signed copies of the 18 values held in scalar registers (kSqG2d).
  __device__ inline void rows(int64_t, int ei, int ej, int, int a, const T* ve, T* acc) const {
    T xv[4];
    xs(ei, ej, xv);
    T s0 = 0, s1 = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const T xq = q == 0 ? xv[0] : q == 1 ? xv[1] : q == 2 ? xv[2] : xv[3];
      const int r0 = q * 64 + (a * 2) * 8;
      T t0 = 0, t1 = 0;
#pragma unroll
      for (int col = 0; col < 8; ++col) {
        t0 += g2<T>(r0 + col) * ve[col];
        t1 += g2<T>(r0 + 8 + col) * ve[col];
      }
      s0 += xq * t0;
      s1 += xq * t1;
    }
    acc[0] += s0;
    acc[1] += s1;
  }
  __device__ inline void diag(int64_t, int ei, int ej, int, int a, T* dg) const {
    T xq[4];
    xs(ei, ej, xq);
    diag_x(xq, a, dg);
  }
  // The same with the four densities already loaded (node_apply loads those of
  // all elements around a node first, so their loads are in flight together).
  __device__ inline void rows_x(const T* xv, int a, const T* ve, T* acc) const {
    T s0 = 0, s1 = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const T xq = q == 0 ? xv[0] : q == 1 ? xv[1] : q == 2 ? xv[2] : xv[3];
      const int r0 = q * 64 + (a * 2) * 8;
      T t0 = 0, t1 = 0;
#pragma unroll
      for (int col = 0; col < 8; ++col) {
        t0 += g2<T>(r0 + col) * ve[col];
        t1 += g2<T>(r0 + 8 + col) * ve[col];
      }
      s0 += xq * t0;
      s1 += xq * t1;
    }
    acc[0] += s0;
    acc[1] += s1;
  }
  __device__ inline void diag_x(const T* xq, int a, T* dg) const {
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      const int r = a * DIM + c;
      T s = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) s += xq[q] * g2<T>(q * 64 + r * 8 + r);
      dg[c] += s;
    }
  }
};

// Operators whose per-element data node_apply loads for all elements first.
template <class Op>
struct preloads_x : std::false_type {};
template <typename T>
struct preloads_x<OpCoarse2K<2, T>> : std::true_type {};

// Border of the augmented matrix (lambda row/column): b (n_slots) and corner c.
template <typename T>
struct Aug {
  const T* b;     // nullptr: no border (plain K)
  double c;
  int64_t n;      // index of lambda in level vectors (= n_slots)
};

// ------------------------------------------------------------- node helpers --
template <int DIM, typename T>
__device__ inline void load_node(const T* __restrict__ v, int64_t q, T* out) {
  if constexpr (DIM == 2) {
    if constexpr (sizeof(T) == 8) {
      const double2 t = *reinterpret_cast<const double2*>(v + 2 * q);
      out[0] = t.x; out[1] = t.y;
    } else {
      const float2 t = *reinterpret_cast<const float2*>(v + 2 * q);
      out[0] = t.x; out[1] = t.y;
    }
  } else {
    out[0] = v[3 * q]; out[1] = v[3 * q + 1]; out[2] = v[3 * q + 2];
  }
}

template <int DIM, typename T>
__device__ inline void store_node(T* __restrict__ v, int64_t q, const T* in) {
  if constexpr (DIM == 2) {
    if constexpr (sizeof(T) == 8) {
      *reinterpret_cast<double2*>(v + 2 * q) = make_double2(in[0], in[1]);
    } else {
      *reinterpret_cast<float2*>(v + 2 * q) = make_float2(in[0], in[1]);
    }
  } else {
    v[3 * q] = in[0]; v[3 * q + 1] = in[1]; v[3 * q + 2] = in[2];
  }
}

// Gather v on the 3^dim neighbourhood of node (i,j,k); nodes outside the grid and
// clamped nodes (i == 0) read as zero.
template <int DIM, typename T>
__device__ inline void load_neighbourhood(const T* __restrict__ v, const Dims& d, int i, int j, int k,
                                          T (&vn)[Geo<DIM>::NB][DIM]) {
#pragma unroll
  for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int nb = nb_index<DIM>(dx, dy, dz);
        const int ii = i + dx, jj = j + dy, kk = k + dz;
        const bool in = ii >= 1 && ii < d.nx1 && jj >= 0 && jj < d.ny1 && kk >= 0 && kk < d.nz1;
        if (in) {
          load_node<DIM, T>(v, ((int64_t)kk * d.ny1 + jj) * d.nx1 + ii, vn[nb]);
        } else {
#pragma unroll
          for (int c = 0; c < DIM; ++c) vn[nb][c] = T(0);
        }
      }
}

// acc += (A v) at node (i,j,k) and dg += diag(A) there, summing over the 2^dim
// elements that share the node (gather form: no atomics, fixed order).
template <int DIM, typename T, class Op, bool ROWS, bool DIAG, bool INTERIOR = false>
__device__ inline void node_apply(const Op& op, const Dims& d, int i, int j, int k,
                                  const T (&vn)[Geo<DIM>::NB][DIM], T* acc, T* dg) {
  constexpr int NN = Geo<DIM>::NN, ND = Geo<DIM>::ND;
  constexpr bool PRE = preloads_x<Op>::value;
  T xpre[PRE ? NN : 1][4];
  if constexpr (PRE) {
#pragma unroll
    for (int q = 0; q < NN; ++q) {
      const int ex = q & 1, ey = (q >> 1) & 1;
      const int ei = i - 1 + ex, ej = j - 1 + ey;
      op.xs_or_zero(INTERIOR || (ei >= 0 && ei < d.nx && ej >= 0 && ej < d.ny), ei, ej, xpre[q]);
    }
  }
#pragma unroll
  for (int q = 0; q < NN; ++q) {
    const int ex = q & 1, ey = (q >> 1) & 1, ez = (q >> 2) & 1;
    int ei = i - 1 + ex, ej = j - 1 + ey, ek = k - 1 + ez;
    // Elements outside the grid contribute nothing.  Off the interior they are
    // replaced by element 0 with zero vertex values and a masked diagonal, so the
    // loads of all elements are issued without branches.
    bool ok = true;
    if constexpr (!INTERIOR) {
      ok = ei >= 0 && ei < d.nx && ej >= 0 && ej < d.ny && (DIM == 2 || (ek >= 0 && ek < d.nz));
      ei = ok ? ei : 0;
      ej = ok ? ej : 0;
      ek = ok ? ek : 0;
    }
    const int64_t e = ((int64_t)(DIM == 3 ? ek : 0) * d.ny + ej) * d.nx + ei;
    const int a = loc_index(1 - ex, 1 - ey, DIM == 3 ? 1 - ez : 0);
    if constexpr (ROWS) {
      T ve[ND];
#pragma unroll
      for (int b = 0; b < NN; ++b) {
        const int nb = nb_index<DIM>(ex + loc_x(b) - 1, ey + loc_y(b) - 1,
                                     DIM == 3 ? ez + loc_z(b) - 1 : 0);
#pragma unroll
        for (int c = 0; c < DIM; ++c) ve[b * DIM + c] = ok ? vn[nb][c] : T(0);
      }
      if constexpr (PRE) op.rows_x(xpre[q], a, ve, acc);
      else op.rows(e, ei, ej, ek, a, ve, acc);
    }
    if constexpr (DIAG) {
      if constexpr (INTERIOR) {
        if constexpr (PRE) op.diag_x(xpre[q], a, dg);
        else op.diag(e, ei, ej, ek, a, dg);
      } else {
        T dt[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) dt[c] = T(0);
        if constexpr (PRE) op.diag_x(xpre[q], a, dt);
        else op.diag(e, ei, ej, ek, a, dt);
#pragma unroll
        for (int c = 0; c < DIM; ++c) dg[c] += ok ? dt[c] : T(0);
      }
    }
  }
}

// ------------------------------------------------------------ level kernels --
enum LevelMode {
  M_APPLY = 0, M_RESID = 1, M_JACOBI = 2, M_JACOBI0 = 3, M_POWER = 4, M_RAYLEIGH = 5, M_JACOBI_BETA = 6,
  M_PJACOBI = 7,  // 2D tiled passes only: Jacobi sweep from z2 + P zc (prolongation folded in)
  M_JACOBI2 = 8   // 2D tiled finest-level K only: the first two sweeps from a zero iterate in one pass
};

// Post-processing of the PCG ratio by the thread that owns the final sum
// tot = r~'y~: beta = r~'y~ / r'y (Algorithm PCG) or, with scal[S_FLEX] set, the
// Polak-Ribiere form r~'(y~ - y) / r'y, which stays effective when the
// preconditioner varies slightly between steps (an FP32 V-cycle).  r~'y follows
// from r~ = r + alpha q: r~'y = r'y + alpha q'y.
__device__ inline void finish_beta(double tot, const Red& red) {
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

// Reciprocal of a Jacobi diagonal: the hardware reciprocal (about 1 ulp) in the
// FP32 V-cycle, exact division in FP64.
__device__ inline float recip(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ inline double recip(double v) { return 1.0 / v; }

// Output of one node of a pass over a level (see k_level), given its row sums
// acc = (A v)_node (without the border term), the diagonal dg and the centre
// value vc (unused for M_JACOBI0).  Adds the border term b*v_lambda and
// accumulates the border dot b.v (augmented system) in bdot and the mode's
// reduction terms in red0/red1.
template <int MODE>
constexpr bool mode_reads_r() {
  return MODE == M_RESID || MODE == M_JACOBI || MODE == M_JACOBI0 || MODE == M_JACOBI_BETA || MODE == M_PJACOBI ||
         MODE == M_JACOBI2;
}

// As level_node_finish with the node's entries of r (rr), of dot64 (d64, M_JACOBI_BETA)
// and of the border (bb, when augb) already loaded.
template <int DIM, typename T, int MODE>
__device__ inline void level_node_finish_vals(int64_t q, T* acc, const T* dg, const T* vc, const T* rr, T* out,
                                              T omega, bool augb, const T* bb, T vl, double pin, const double* d64,
                                              double& bdot, double& red0, double& red1) {
  constexpr bool NEED_ROWS = MODE != M_JACOBI0;
  T o[DIM];
  if constexpr (NEED_ROWS) {
    if (augb) {
#pragma unroll
      for (int c = 0; c < DIM; ++c) {
        acc[c] += bb[c] * vl;
        bdot += (double)bb[c] * (double)vc[c];
      }
    }
  }
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    if constexpr (MODE == M_APPLY) o[c] = acc[c];
    if constexpr (MODE == M_RESID) o[c] = rr[c] - acc[c];
    if constexpr (MODE == M_JACOBI || MODE == M_JACOBI_BETA || MODE == M_PJACOBI || MODE == M_JACOBI2)
      o[c] = vc[c] + omega * (rr[c] - acc[c]) * recip(dg[c]);
    if constexpr (MODE == M_JACOBI0) o[c] = omega * rr[c] * recip(dg[c]);
    if constexpr (MODE == M_POWER) {
      o[c] = T(pin * (double)(acc[c] / dg[c]));
      red0 += (double)o[c] * (double)o[c];
    }
    if constexpr (MODE == M_RAYLEIGH) {
      red0 += (double)vc[c] * (double)acc[c];
      red1 += (double)vc[c] * (double)dg[c] * (double)vc[c];
    }
    if constexpr (MODE == M_JACOBI_BETA) red0 += d64[c] * (double)o[c];
  }
  if constexpr (MODE != M_RAYLEIGH) store_node<DIM, T>(out, q, o);
}

template <int DIM, typename T, int MODE>
__device__ inline void level_node_finish(int64_t q, T* acc, const T* dg, const T* vc, const T* r, T* out,
                                         T omega, const T* augb, T vl, double pin, const double* dot64,
                                         double& bdot, double& red0, double& red1) {
  constexpr bool NEED_ROWS = MODE != M_JACOBI0;
  T o[DIM];
  if constexpr (NEED_ROWS) {
    if (augb) {
#pragma unroll
      for (int c = 0; c < DIM; ++c) {
        const T bc = augb[q * DIM + c];
        acc[c] += bc * vl;
        bdot += (double)bc * (double)vc[c];
      }
    }
  }
  T rr[DIM];
  if constexpr (mode_reads_r<MODE>())
    load_node<DIM, T>(r, q, rr);
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    if constexpr (MODE == M_APPLY) o[c] = acc[c];
    if constexpr (MODE == M_RESID) o[c] = rr[c] - acc[c];
    if constexpr (MODE == M_JACOBI || MODE == M_JACOBI_BETA) o[c] = vc[c] + omega * (rr[c] - acc[c]) * recip(dg[c]);
    if constexpr (MODE == M_JACOBI0) o[c] = omega * rr[c] * recip(dg[c]);
    if constexpr (MODE == M_POWER) {
      o[c] = T(pin * (double)(acc[c] / dg[c]));
      red0 += (double)o[c] * (double)o[c];
    }
    if constexpr (MODE == M_RAYLEIGH) {
      red0 += (double)vc[c] * (double)acc[c];
      red1 += (double)vc[c] * (double)dg[c] * (double)vc[c];
    }
    if constexpr (MODE == M_JACOBI_BETA) red0 += dot64[q * DIM + c] * (double)o[c];
  }
  if constexpr (MODE != M_RAYLEIGH) store_node<DIM, T>(out, q, o);
}

// Per-node part of one pass over a level (see k_level), given the neighbourhood
// vn of v (ignored for M_JACOBI0).
template <int DIM, typename T, class Op, int MODE, bool INTERIOR = false>
__device__ inline void level_node_core(const Op& op, const Dims& d, int i, int j, int k,
                                       const T (&vn)[Geo<DIM>::NB][DIM], const T* r, T* out, T omega,
                                       const T* augb, T vl, double pin, const double* dot64, double& bdot,
                                       double& red0, double& red1) {
  constexpr bool NEED_ROWS = MODE != M_JACOBI0;
  const int64_t q = ((int64_t)k * d.ny1 + j) * d.nx1 + i;
  if (i == 0) {
    T o[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) o[c] = T(0);
    if constexpr (MODE != M_RAYLEIGH) store_node<DIM, T>(out, q, o);
    return;
  }
  T acc[DIM], dg[DIM], vc[DIM];
#pragma unroll
  for (int c = 0; c < DIM; ++c) { acc[c] = T(0); dg[c] = T(0); vc[c] = T(0); }
  node_apply<DIM, T, Op, NEED_ROWS, true, INTERIOR>(op, d, i, j, k, vn, acc, dg);
  if constexpr (NEED_ROWS) {
#pragma unroll
    for (int c = 0; c < DIM; ++c) vc[c] = vn[nb_index<DIM>(0, 0, 0)][c];
  }
  level_node_finish<DIM, T, MODE>(q, acc, dg, vc, r, out, omega, augb, vl, pin, dot64, bdot, red0, red1);
}

// 3D row sums and diagonal of node (i, j, k): the loop over the 8 elements stays
// rolled and each element's 24 nodal values are gathered from v (L1/L2) when it is
// processed, so the 81 neighbourhood values are never live in registers
// at once (they were: over 256 VGPRs, one wave per SIMD).  Elements outside the
// grid contribute nothing; clamped nodes (i == 0), and every node of an element
// outside the grid, are read at node 0, which is clamped and holds zero in every
// level vector, so the loads carry no branch.
template <class Op> struct fine3_op : std::false_type {};
template <typename T> struct fine3_op<OpFineK<3, T>> : std::true_type {};
template <typename T> struct fine3_op<OpFineZ<3, T>> : std::true_type {};

// Finest 3D level (A_e = x_e K0, plus h_e h_e' for Z): every element around node
// (i, j, k) is mapped onto the element that has the node at its local node 0 by
// reflecting the axes along which the element lies below the node (d_k = -1).  The
// cube's element matrix is invariant under these reflections with the matching
// component signs, so row c of node a of element e is
//   d_c * sum_{b', c'} K0[c][3 b' + c'] d_c' v(node + (b'_x d_x, b'_y d_y, b'_z d_z), c'),
// and only the three rows of local node 0 occur: their 72 entries are signed copies
// of the 14 cube constants at compile time, while the loop over the 8 elements stays
// rolled (registers) and loads no matrix entries.  Same operator as the generic
// form; the sum runs in the reflected column order.
template <typename T, class Op, bool ROWS, bool DIAG>
__device__ inline void node_apply_fine3(const Op& op, const Dims& d, int i, int j, int k, const T* __restrict__ v,
                                        T* acc, T* dg) {
#pragma unroll 1
  for (int q = 0; q < 8; ++q) {
    const int ex = q & 1, ey = (q >> 1) & 1, ez = q >> 2;
    int ei = i - 1 + ex, ej = j - 1 + ey, ek = k - 1 + ez;
    const bool ok = ei >= 0 && ei < d.nx && ej >= 0 && ej < d.ny && ek >= 0 && ek < d.nz;
    ei = ok ? ei : 0;
    ej = ok ? ej : 0;
    ek = ok ? ek : 0;
    const int64_t e = ((int64_t)ek * d.ny + ej) * d.nx + ei;
    const int a = loc_index(1 - ex, 1 - ey, 1 - ez);
    const int dx = 2 * ex - 1, dy = 2 * ey - 1, dz = 2 * ez - 1;
    const T xe = op.x[e];
    if constexpr (ROWS) {
      const T sg[3] = {T(dx), T(dy), T(dz)};
      T ve[24];
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const int ni = i + loc_x(b) * dx, nj = j + loc_y(b) * dy, nk = k + loc_z(b) * dz;
        const bool nok = ok && ni >= 1;
        const int64_t qn = nok ? ((int64_t)nk * d.ny1 + nj) * d.nx1 + ni : 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) ve[b * 3 + c] = sg[c] * v[3 * qn + c];
      }
      T hv = 0;
      if constexpr (std::is_same<Op, OpFineZ<3, T>>::value) {
        hv = op.hs[e] * (ok ? T(1) : T(0));     // an element outside the grid reads element 0
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        T s = 0;
#pragma unroll
        for (int col = 0; col < 24; ++col) s += k0cube<T>(c, col) * ve[col];
        acc[c] += xe * sg[c] * s;
        if constexpr (std::is_same<Op, OpFineZ<3, T>>::value) acc[c] += op.h[(a * 3 + c) * op.m + e] * hv;
      }
    }
    if constexpr (DIAG) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        T dt = xe * k0cube<T>(c, c);
        if constexpr (std::is_same<Op, OpFineZ<3, T>>::value) {
          const T hr = op.h[(a * 3 + c) * op.m + e];
          dt += hr * hr;
        }
        dg[c] += ok ? dt : T(0);
      }
    }
  }
}

// Element products of a stored 3D level, y_e = E_e v_e.  A block of 8 waves takes
// 64 consecutive elements; wave a forms the three rows of local node a for all of
// them (every matrix load coalesced over 64 elements, 72 entries and the 24 nodal
// values per thread).  Nodal values of clamped nodes are read at node 0 (zero).
constexpr int EA3_THREADS = 512;
template <typename T>
__global__ __launch_bounds__(EA3_THREADS) void k_elem_apply3(Dims d, const T* __restrict__ E,
                                                             const T* __restrict__ v, T* __restrict__ ye,
                                                             const int* gate) {
  if (gate && *gate) return;
  const int64_t e = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  const int a = threadIdx.x >> 6;
  if (e >= d.m) return;
  const int ei = (int)(e % d.nx), ej = (int)((e / d.nx) % d.ny), ek = (int)(e / ((int64_t)d.nx * d.ny));
  T ve[24];
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const int ni = ei + loc_x(b), nj = ej + loc_y(b), nk = ek + loc_z(b);
    const int64_t qn = ni >= 1 ? ((int64_t)nk * d.ny1 + nj) * d.nx1 + ni : 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) ve[b * 3 + c] = v[3 * qn + c];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int r = a * 3 + c;
    T y = T(0);
#pragma unroll
    for (int col = 0; col < 24; ++col) y += E[sym_index(r, col, 24) * d.m + e] * ve[col];
    ye[r * d.m + e] = y;
  }
}

// Node rows and diagonal of a stored 3D level from the element products ye.
template <typename T, bool ROWS, bool DIAG>
__device__ inline void node_apply_ye3(const OpCoarse<3, T>& op, const Dims& d, int i, int j, int k, T* acc, T* dg) {
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int ex = q & 1, ey = (q >> 1) & 1, ez = q >> 2;
    int ei = i - 1 + ex, ej = j - 1 + ey, ek = k - 1 + ez;
    const bool ok = ei >= 0 && ei < d.nx && ej >= 0 && ej < d.ny && ek >= 0 && ek < d.nz;
    const int64_t e = ok ? ((int64_t)ek * d.ny + ej) * d.nx + ei : 0;
    const int a = loc_index(1 - ex, 1 - ey, 1 - ez);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int r = a * 3 + c;
      if constexpr (ROWS) acc[c] += ok ? op.ye[r * op.m + e] : T(0);
      if constexpr (DIAG) dg[c] += ok ? op.E[sym_index(r, r, 24) * op.m + e] : T(0);
    }
  }
}

// Element products of the finest 3D level, y_e = x_e K0 v_e (+ h_e (h_e'v_e) for the
// augmented system), one thread per element: all 24 rows, every matrix entry a
// signed copy of one of the 14 cube constants at compile time (no matrix loads),
// h_e'v_e summed in column order; 32-bit index arithmetic (the grid has < 2^31
// slots).  Measured faster than 8 waves per 64 elements (one row group each, h_e'v_e
// combined in LDS) and than the node passes gathering the element rows themselves.
template <typename T, bool Z>
__global__ __launch_bounds__(BS) void k_elem_fine3e(Dims d, const T* __restrict__ x, const T* __restrict__ h,
                                                    const T* __restrict__ v, T* __restrict__ ye, const int* gate) {
  if (gate && *gate) return;
  const int e = (int)(blockIdx.x * BS + threadIdx.x);
  if (e >= (int)d.m) return;
  const int ei = e % d.nx, t = e / d.nx, ej = t % d.ny, ek = t / d.ny;
  T ve[24];
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const int ni = ei + loc_x(b), nj = ej + loc_y(b), nk = ek + loc_z(b);
    const int qn = ni >= 1 ? (nk * d.ny1 + nj) * d.nx1 + ni : 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) ve[b * 3 + c] = v[3 * qn + c];
  }
  const int m = (int)d.m;
  T hh[Z ? 24 : 1];
  T hv = 0;
  if constexpr (Z) {
#pragma unroll
    for (int col = 0; col < 24; ++col) hh[col] = h[col * m + e];
#pragma unroll
    for (int col = 0; col < 24; ++col) hv += hh[col] * ve[col];
  }
  const T xe = x[e];
#pragma unroll
  for (int r = 0; r < 24; ++r) {
    T y = 0;
#pragma unroll
    for (int col = 0; col < 24; ++col) y += k0cube<T>(r, col) * ve[col];
    y *= xe;
    if constexpr (Z) y += hh[r] * hv;
    ye[r * m + e] = y;
  }
}

// Rows (from the element products ye) and diagonal (per slot, dgn) of a node of the
// finest 3D level.
template <typename T, bool ROWS, bool DIAG>
__device__ inline void node_apply_fine_ye3(const T* __restrict__ ye, const T* __restrict__ dgn, int64_t m,
                                           const Dims& d, int i, int j, int k, T* acc, T* dg) {
  if constexpr (ROWS) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int ex = q & 1, ey = (q >> 1) & 1, ez = q >> 2;
      const int ei = i - 1 + ex, ej = j - 1 + ey, ek = k - 1 + ez;
      const bool ok = ei >= 0 && ei < d.nx && ej >= 0 && ej < d.ny && ek >= 0 && ek < d.nz;
      const int64_t e = ok ? ((int64_t)ek * d.ny + ej) * d.nx + ei : 0;
      const int a = loc_index(1 - ex, 1 - ey, 1 - ez);
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[c] += ok ? ye[(a * 3 + c) * m + e] : T(0);
    }
  }
  if constexpr (DIAG) {
    const int64_t q = ((int64_t)k * d.ny1 + j) * d.nx1 + i;
#pragma unroll
    for (int c = 0; c < 3; ++c) dg[c] += dgn[3 * q + c];
  }
}

template <typename T, class Op, bool ROWS, bool DIAG>
__device__ inline void node_apply_gather3(const Op& op, const Dims& d, int i, int j, int k, const T* __restrict__ v,
                                          T* acc, T* dg) {
  if constexpr (fine3_op<Op>::value) {
    if ((!ROWS || op.ye) && (!DIAG || op.dgn))
      return node_apply_fine_ye3<T, ROWS, DIAG>(op.ye, op.dgn, op.m, d, i, j, k, acc, dg);
  }
  if constexpr (std::is_same<Op, OpCoarse<3, T>>::value) {
    if (!ROWS || op.ye) return node_apply_ye3<T, ROWS, DIAG>(op, d, i, j, k, acc, dg);
  }
  if constexpr (std::is_same<Op, OpFineK<3, T>>::value) {
    return node_apply_fine3<T, Op, ROWS, DIAG>(op, d, i, j, k, v, acc, dg);
  } else if constexpr (std::is_same<Op, OpFineZ<3, T>>::value) {
    // the reflected form reads h_e'v_e per element (hs) for the rank-one term
    if (!ROWS || op.hs != nullptr) return node_apply_fine3<T, Op, ROWS, DIAG>(op, d, i, j, k, v, acc, dg);
  }
#pragma unroll 1
  for (int q = 0; q < 8; ++q) {
    const int ex = q & 1, ey = (q >> 1) & 1, ez = q >> 2;
    int ei = i - 1 + ex, ej = j - 1 + ey, ek = k - 1 + ez;
    const bool ok = ei >= 0 && ei < d.nx && ej >= 0 && ej < d.ny && ek >= 0 && ek < d.nz;
    ei = ok ? ei : 0;
    ej = ok ? ej : 0;
    ek = ok ? ek : 0;
    const int64_t e = ((int64_t)ek * d.ny + ej) * d.nx + ei;
    const int a = loc_index(1 - ex, 1 - ey, 1 - ez);
    if constexpr (ROWS) {
      T ve[24];
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const int ni = ei + loc_x(b), nj = ej + loc_y(b), nk = ek + loc_z(b);
        const bool nok = ok && ni >= 1;
        const int64_t qn = nok ? ((int64_t)nk * d.ny1 + nj) * d.nx1 + ni : 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) ve[b * 3 + c] = v[3 * qn + c];
      }
      if constexpr (std::is_same<Op, OpFineZ<3, T>>::value) op.rows_keep(e, a, ve, ok ? T(1) : T(0), acc);
      else op.rows(e, ei, ej, ek, a, ve, acc);
    }
    if constexpr (DIAG) {
      T dt[3] = {T(0), T(0), T(0)};
      op.diag(e, ei, ej, ek, a, dt);
#pragma unroll
      for (int c = 0; c < 3; ++c) dg[c] += ok ? dt[c] : T(0);
    }
  }
}

// Diagonal of the finest 3D level per DOF slot (0 on clamped slots), formed once per
// hierarchy set-up: the level passes then read three values per node.
template <typename T, class Op>
__global__ __launch_bounds__(BS) void k_fine_diag3(Op op, Dims d, T* __restrict__ dgn) {
  const int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (t >= d.nnodes) return;
  const int i = (int)(t % d.nx1), j = (int)((t / d.nx1) % d.ny1), k = (int)(t / ((int64_t)d.nx1 * d.ny1));
  T acc[3] = {T(0), T(0), T(0)}, dg[3] = {T(0), T(0), T(0)};
  op.ye = nullptr;
  op.dgn = nullptr;
  if (i > 0) node_apply_fine3<T, Op, false, true>(op, d, i, j, k, nullptr, acc, dg);
#pragma unroll
  for (int c = 0; c < 3; ++c) dgn[3 * t + c] = dg[c];
}

// Generic form: gathers the neighbourhood with bounds checks first (2D); in 3D,
// element by element (node_apply_gather3).
template <int DIM, typename T, class Op, int MODE>
__device__ inline void level_node(const Op& op, const Dims& d, int i, int j, int k, const T* v, const T* r, T* out,
                                  T omega, const T* augb, T vl, double pin, const double* dot64, double& bdot,
                                  double& red0, double& red1) {
  if constexpr (DIM == 3) {
    const int64_t q = ((int64_t)k * d.ny1 + j) * d.nx1 + i;
    if (i == 0) {
      const T z[3] = {T(0), T(0), T(0)};
      if constexpr (MODE != M_RAYLEIGH) store_node<3, T>(out, q, z);
      return;
    }
    T acc[3] = {T(0), T(0), T(0)}, dg[3] = {T(0), T(0), T(0)}, vc[3] = {T(0), T(0), T(0)};
    if constexpr (MODE != M_JACOBI0) load_node<3, T>(v, q, vc);
    node_apply_gather3<T, Op, MODE != M_JACOBI0, true>(op, d, i, j, k, v, acc, dg);
    level_node_finish<3, T, MODE>(q, acc, dg, vc, r, out, omega, augb, vl, pin, dot64, bdot, red0, red1);
  } else {
    T vn[Geo<DIM>::NB][DIM];
    if constexpr (MODE != M_JACOBI0) load_neighbourhood<DIM, T>(v, d, i, j, k, vn);
    level_node_core<DIM, T, Op, MODE>(op, d, i, j, k, vn, r, out, omega, augb, vl, pin, dot64, bdot, red0, red1);
  }
}

// Lambda entry of a pass over an augmented level, given the border dot tot0 =
// b.v_u and the node reductions tot1, tot2 (done by one thread).
template <typename T, int MODE>
__device__ inline void level_lambda(const T* v, const T* r, T* out, double omega, double c, int64_t n, double pin,
                                    const double* dot64, double tot0, double tot1, double tot2, const Red& red,
                                    int sidx) {
  const double vl = (double)v[n];
  const double rowl = tot0 + c * vl;   // (Z v)_lambda
  if constexpr (MODE == M_APPLY) out[n] = T(rowl);
  if constexpr (MODE == M_RESID) out[n] = T((double)r[n] - rowl);
  if constexpr (MODE == M_JACOBI || MODE == M_JACOBI_BETA) {
    const T ol = T(vl + omega * ((double)r[n] - rowl) / c);
    out[n] = ol;
    if constexpr (MODE == M_JACOBI_BETA) finish_beta(tot1 + dot64[n] * (double)ol, red);
  }
  if constexpr (MODE == M_POWER) {
    const double ol = pin * rowl / c;
    out[n] = T(ol);
    red.scal[sidx] = tot1 + ol * ol;
  }
  if constexpr (MODE == M_RAYLEIGH) {
    red.scal[sidx] = tot1 + vl * rowl;
    red.scal[sidx + 1] = tot2 + vl * c * vl;
  }
}

// One pass over the nodes of a level.
//   M_APPLY       out = A v
//   M_RESID       out = r - A v
//   M_JACOBI      out = v + omega D^-1 (r - A v)       (damped Jacobi sweep)
//   M_JACOBI0     out = omega D^-1 r                   (first sweep from v = 0)
//   M_JACOBI_BETA M_JACOBI, then beta = dot64'out / rho (the PCG ratio) on the device
//   M_POWER       out = D^-1 A v / ||v||, scal[sidx] = ||out||^2 (||v||^2 read from
//                 scal[sidx_in] when sidx_in >= 0, else taken as 1)
//   M_RAYLEIGH    scal[sidx] = v'Av, scal[sidx+1] = v'Dv
// Clamped slots of out are written as 0.  With a border (aug.b != nullptr) the
// lambda entry (index aug.n) is handled by the last block of a reduction.
template <int DIM, typename T, class Op, int MODE>
__global__ __launch_bounds__(BS) void k_level(Op op, Dims d, const T* __restrict__ v,
                                              const T* __restrict__ r, T* __restrict__ out,
                                              const double* __restrict__ omg, Aug<T> aug, Red red, int sidx,
                                              int sidx_in, const double* __restrict__ dot64, const int* gate) {
  if (gate && *gate) return;
  const T omega = omg ? T(*omg) : T(0);
  double pin = 1.0;
  if constexpr (MODE == M_POWER) {
    if (sidx_in >= 0) {
      const double s = red.scal[sidx_in];
      pin = s > 0.0 ? 1.0 / sqrt(s) : 1.0;
    }
  }
  const Tile tl = xcd_tile();
  const int i = tl.x * 64 + (threadIdx.x & 63);
  const int j = tl.y * (BS / 64) + (threadIdx.x >> 6);
  const int k = tl.z;
  constexpr bool NEED_RED = MODE == M_POWER || MODE == M_RAYLEIGH || MODE == M_JACOBI_BETA;
  double red0 = 0.0, red1 = 0.0, bdot = 0.0;
  const T vl = (aug.b && MODE != M_JACOBI0) ? v[aug.n] : T(0);
  if (i < d.nx1 && j < d.ny1)
    level_node<DIM, T, Op, MODE>(op, d, i, j, k, v, r, out, omega, aug.b, vl, pin, dot64, bdot, red0, red1);
  if (aug.b) {
    if constexpr (MODE == M_JACOBI0) {
      if (blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x == 0)
        out[aug.n] = T((double)omega * (double)r[aug.n] / aug.c);
    } else {
      const double vals[3] = {bdot, red0, red1};
      block_partials<3>(vals, red);
    }
  } else if constexpr (NEED_RED) {
    const double vals[3] = {red0, red1, 0.0};
    block_partials<3>(vals, red);
  }
}

// Finalize of a level pass that reduces (augmented border, M_POWER, M_RAYLEIGH,
// M_JACOBI_BETA): one block of BS threads, launched right after k_level.
// The device flags into pinned host memory (thread 0): the last kernel of a PCG
// iteration hands the host its stop test this way instead of a separate copy.
__device__ inline void flags_to_host(const Red& red, int* __restrict__ h) {
#pragma unroll
  for (int f = 0; f < F_COUNT; ++f) h[f] = red.flags[f];
  __threadfence_system();
}

// hflags (M_JACOBI_BETA, may be null): pinned host slot that receives the flags.
template <typename T, int MODE>
__global__ __launch_bounds__(BS) void k_level_fin(const T* __restrict__ v, const T* __restrict__ r,
                                                  T* __restrict__ out, const double* __restrict__ omg, int aug,
                                                  double c, int64_t n, const double* __restrict__ dot64, Red red,
                                                  unsigned nblocks, int sidx, int sidx_in, const int* gate,
                                                  int* hflags) {
  if (gate && *gate) {
    if (hflags && threadIdx.x == 0) flags_to_host(red, hflags);
    return;
  }
  double tot[3];
  sum_partials<3>(red, nblocks, tot);
  if (threadIdx.x != 0) return;
  double pin = 1.0;
  if constexpr (MODE == M_POWER) {
    if (sidx_in >= 0) {
      const double s = red.scal[sidx_in];
      pin = s > 0.0 ? 1.0 / sqrt(s) : 1.0;
    }
  }
  if (aug) {
    level_lambda<T, MODE>(v, r, out, omg ? *omg : 0.0, c, n, pin, dot64, tot[0], tot[1], tot[2], red, sidx);
  } else {
    if constexpr (MODE == M_JACOBI_BETA) {
      finish_beta(tot[0], red);
    } else {
      red.scal[sidx] = tot[0];
      if constexpr (MODE == M_RAYLEIGH) red.scal[sidx + 1] = tot[1];
    }
  }
  if (hflags) flags_to_host(red, hflags);
}

// Lane-shared register tiles.  The 64 lanes of a wave hold 64 consecutive node
// columns; lane l forms its own column's values once and reads column i-1 from lane
// l-1 and column i+1 from lane l+1 (wave-wide DPP shifts, no memory traffic).  The
// first and last lanes of a tile have no neighbour on one side: they keep their own
// value there and serve only as halo columns for lanes 1 and 62 (62 output columns
// per tile).  Every lane of the wave must be active at a shift.
__device__ inline float lane_from_left(float v) {     // value of lane l-1 (wave_shr:1)
  const int b = __builtin_bit_cast(int, v);
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(b, b, 0x138, 0xf, 0xf, false));
}
__device__ inline float lane_from_right(float v) {    // value of lane l+1 (wave_shl:1)
  const int b = __builtin_bit_cast(int, v);
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(b, b, 0x130, 0xf, 0xf, false));
}
__device__ inline double lane_from_left(double v) {
  const int2 b = __builtin_bit_cast(int2, v);
  return __builtin_bit_cast(double, make_int2(__builtin_amdgcn_update_dpp(b.x, b.x, 0x138, 0xf, 0xf, false),
                                              __builtin_amdgcn_update_dpp(b.y, b.y, 0x138, 0xf, 0xf, false)));
}
__device__ inline double lane_from_right(double v) {
  const int2 b = __builtin_bit_cast(int2, v);
  return __builtin_bit_cast(double, make_int2(__builtin_amdgcn_update_dpp(b.x, b.x, 0x130, 0xf, 0xf, false),
                                              __builtin_amdgcn_update_dpp(b.y, b.y, 0x130, 0xf, 0xf, false)));
}
constexpr int LS_COLS = 62;    // output columns of a lane-shared tile

// Columns i-1 and i+1 of the neighbourhood from the neighbouring lanes.
template <typename T, int NJ>
__device__ inline void share_columns(T (&w)[NJ + 2][3][2]) {
#pragma unroll
  for (int rr = 0; rr < NJ + 2; ++rr)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      w[rr][0][c] = lane_from_left(w[rr][1][c]);
      w[rr][2][c] = lane_from_right(w[rr][1][c]);
    }
}

// Row sums (A v) and diagonals of the NJ nodes (i, j0..j0+NJ-1) of one thread of
// the tiled 2D pass.  w holds v on the nodes (i-1..i+1, j0-1..j0+NJ), zero outside
// the grid and on clamped nodes: w[rr][cc] is node (i-1+cc, j0-1+rr).  The thread's
// nodes touch the elements (i-1+ec, j0-1+er), er = 0..NJ, ec = 0..1; node n is
// corner loc_index(1-ex, 1-ey) of element (ec, er) = (ex, n+ey).  EDGE: some of
// these nodes or elements may lie outside the grid (elements outside contribute
// nothing); otherwise all of them are inside.
template <typename T, class Op, bool ROWS, int NJ>
struct TileApply {
  template <bool EDGE>
  __device__ static inline void run(const Op& op, const Dims& d, int i, int j0, const T (&w)[NJ + 2][3][2],
                                    T (&acc)[NJ][2], T (&dg)[NJ][2]) {
#pragma unroll
    for (int n = 0; n < NJ; ++n) {
      T vn[9][2];
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          vn[nb_index<2>(dx, dy, 0)][0] = ROWS ? w[n + 1 + dy][dx + 1][0] : T(0);
          vn[nb_index<2>(dx, dy, 0)][1] = ROWS ? w[n + 1 + dy][dx + 1][1] : T(0);
        }
      acc[n][0] = acc[n][1] = dg[n][0] = dg[n][1] = T(0);
      node_apply<2, T, Op, ROWS, true, !EDGE>(op, d, i, j0 + n, 0, vn, acc[n], dg[n]);
    }
  }
};

// Element (ei, ej) of a 2D level lies inside the grid.
__device__ inline bool elem_in(const Dims& d, int ei, int ej) { return ei >= 0 && ei < d.nx && ej >= 0 && ej < d.ny; }

// Finest level: A_e = x_e K0.  The densities of the 2(NJ+1) elements are loaded up
// front (zero outside the grid).
template <typename T, bool ROWS, int NJ>
struct TileApply<T, OpFineK<2, T>, ROWS, NJ> {
  template <bool EDGE>
  __device__ static inline void run(const OpFineK<2, T>& op, const Dims& d, int i, int j0,
                                    const T (&w)[NJ + 2][3][2], T (&acc)[NJ][2], T (&dg)[NJ][2]) {
    T xe[NJ + 1][2];
    load_x<EDGE>(op, d, i, j0, xe);
    run_x(xe, w, acc, dg);
  }
  // Elements outside the grid read the zero pad after the densities (index m), so
  // the loads need no branch and no select.
  template <bool EDGE>
  __device__ static inline void load_x(const OpFineK<2, T>& op, const Dims& d, int i, int j0, T (&xe)[NJ + 1][2]) {
#pragma unroll
    for (int er = 0; er <= NJ; ++er)
#pragma unroll
      for (int ec = 0; ec < 2; ++ec) {
        const int ei = i - 1 + ec, ej = j0 - 1 + er;
        const int64_t e = (int64_t)ej * d.nx + ei;
        xe[er][ec] = op.x[(!EDGE || elem_in(d, ei, ej)) ? e : op.m];
      }
  }
  // Lane-shared tiles: the thread loads element column i-1 only and takes column i
  // from the lane to its right (on the tile's last lane, a halo lane whose result is
  // not used, that value is its own).
  template <bool EDGE>
  __device__ static inline void run_ls(const OpFineK<2, T>& op, const Dims& d, int i, int j0,
                                       const T (&w)[NJ + 2][3][2], T (&acc)[NJ][2], T (&dg)[NJ][2]) {
    T xe[NJ + 1][2];
#pragma unroll
    for (int er = 0; er <= NJ; ++er) {
      const int ei = i - 1, ej = j0 - 1 + er;
      xe[er][0] = op.x[(!EDGE || elem_in(d, ei, ej)) ? (int64_t)ej * d.nx + ei : op.m];
    }
#pragma unroll
    for (int er = 0; er <= NJ; ++er) xe[er][1] = lane_from_right(xe[er][0]);
    run_x(xe, w, acc, dg);
  }
  __device__ static inline void run_x(const T (&xe)[NJ + 1][2], const T (&w)[NJ + 2][3][2], T (&acc)[NJ][2],
                                      T (&dg)[NJ][2]) {
#pragma unroll
    for (int n = 0; n < NJ; ++n) {
      acc[n][0] = acc[n][1] = dg[n][0] = dg[n][1] = T(0);
#pragma unroll
      for (int ey = 0; ey < 2; ++ey)
#pragma unroll
        for (int ex = 0; ex < 2; ++ex) {
          const int er = n + ey, ec = ex;
          const int a = loc_index(1 - ex, 1 - ey, 0);
          const T x = xe[er][ec];
          if constexpr (ROWS) {
            const T ve[8] = {w[er][ec][0],         w[er][ec][1],         w[er][ec + 1][0], w[er][ec + 1][1],
                             w[er + 1][ec + 1][0], w[er + 1][ec + 1][1], w[er + 1][ec][0], w[er + 1][ec][1]};
            T t0 = 0, t1 = 0;
#pragma unroll
            for (int col = 0; col < 8; ++col) {
              t0 += k0sq<T>(2 * a, col) * ve[col];
              t1 += k0sq<T>(2 * a + 1, col) * ve[col];
            }
            acc[n][0] += x * t0;
            acc[n][1] += x * t1;
          }
          dg[n][0] += x * k0sq<T>(2 * a, 2 * a);
          dg[n][1] += x * k0sq<T>(2 * a + 1, 2 * a + 1);
        }
    }
  }
};

// First coarse level formed on the fly: the element matrix of a coarse element is
// sum_q x_q G_q over its four fine sub-elements q.  The densities of every element
// the thread touches are loaded up front; the G_q entries are signed copies of 18
// values held in scalar registers (kSqG2d), so no load waits inside the loops.
template <typename T, bool ROWS, int NJ>
struct TileApply<T, OpCoarse2K<2, T>, ROWS, NJ> {
  template <bool EDGE>
  __device__ static inline void run(const OpCoarse2K<2, T>& op, const Dims& d, int i, int j0,
                                    const T (&w)[NJ + 2][3][2], T (&acc)[NJ][2], T (&dg)[NJ][2]) {
    T xs[NJ + 1][2][4];
#pragma unroll
    for (int er = 0; er <= NJ; ++er)
#pragma unroll
      for (int ec = 0; ec < 2; ++ec) {
        const int ei = i - 1 + ec, ej = j0 - 1 + er;
        op.xs_or_zero(!EDGE || elem_in(d, ei, ej), ei, ej, xs[er][ec]);   // zero pad outside: no branch
      }
#pragma unroll
    for (int n = 0; n < NJ; ++n) acc[n][0] = acc[n][1] = dg[n][0] = dg[n][1] = T(0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      T xq[NJ + 1][2];
#pragma unroll
      for (int er = 0; er <= NJ; ++er)
#pragma unroll
        for (int ec = 0; ec < 2; ++ec)
          xq[er][ec] = q == 0 ? xs[er][ec][0] : q == 1 ? xs[er][ec][1] : q == 2 ? xs[er][ec][2] : xs[er][ec][3];
      const int gq = q * 64;
#pragma unroll
      for (int n = 0; n < NJ; ++n)
#pragma unroll
        for (int ey = 0; ey < 2; ++ey)
#pragma unroll
          for (int ex = 0; ex < 2; ++ex) {
            const int er = n + ey, ec = ex;
            const int a = loc_index(1 - ex, 1 - ey, 0);
            const T xe = xq[er][ec];
            if constexpr (ROWS) {
              const T ve[8] = {w[er][ec][0],         w[er][ec][1],         w[er][ec + 1][0], w[er][ec + 1][1],
                               w[er + 1][ec + 1][0], w[er + 1][ec + 1][1], w[er + 1][ec][0], w[er + 1][ec][1]};
              T t0 = 0, t1 = 0;
#pragma unroll
              for (int col = 0; col < 8; ++col) {
                t0 += g2<T>(gq + (2 * a) * 8 + col) * ve[col];
                t1 += g2<T>(gq + (2 * a + 1) * 8 + col) * ve[col];
              }
              acc[n][0] += xe * t0;
              acc[n][1] += xe * t1;
            }
            dg[n][0] += xe * g2<T>(gq + (2 * a) * 9);
            dg[n][1] += xe * g2<T>(gq + (2 * a + 1) * 9);
          }
    }
  }
};

// v on the (NJ+2) x 3 node neighbourhood of a thread's column (see TileApply);
// EDGE: nodes outside the grid and clamped nodes (i == 0) read as zero.
template <typename T, int NJ, bool EDGE>
__device__ inline void load_tile(const T* __restrict__ v, const Dims& d, int i, int j0, T (&w)[NJ + 2][3][2]) {
#pragma unroll
  for (int rr = 0; rr < NJ + 2; ++rr)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      const int ii = i - 1 + cc, jj = j0 - 1 + rr;
      if (!EDGE) {
        const unsigned o = 2u * ((unsigned)jj * (unsigned)d.nx1 + (unsigned)ii);
        w[rr][cc][0] = v[o];
        w[rr][cc][1] = v[o + 1];
      } else {                                     // clamped index, selected value: no branch
        const bool ok = ii >= 1 && ii < d.nx1 && jj >= 0 && jj < d.ny1;
        const unsigned o = 2u * ((unsigned)min(max(jj, 0), d.ny1 - 1) * (unsigned)d.nx1 +
                                 (unsigned)min(max(ii, 0), d.nx1 - 1));
        const T a = v[o], b = v[o + 1];
        w[rr][cc][0] = ok ? a : T(0);
        w[rr][cc][1] = ok ? b : T(0);
      }
    }
}

// As load_tile, of z2 + P zc: the fine values z2 plus the bilinear prolongation of
// the coarse correction zc (Sec. 5.1 solution update, summed in the order of
// k_prolong), zero outside the grid and on clamped nodes.  NJ is even, so j0 is
// even and the coarse rows of every fine row are fixed; the thread loads the
// (NJ/2+2) x 3 coarse nodes from row j0/2-1 and column (i-1)>>1 once, and the
// parity of i picks, per fine column, which of them a node interpolates from.
template <typename T, int NJ, bool EDGE>
__device__ inline void load_tile_prolong(const T* __restrict__ z2, const T* __restrict__ zc, const Dims& d,
                                         const Dims& dc, int i, int j0, T (&w)[NJ + 2][3][2]) {
  static_assert(NJ % 2 == 0, "the folded prolongation needs an even node count per thread");
  constexpr int CR = NJ / 2 + 2;
  const int c0 = (i - 1) >> 1, jb = (j0 >> 1) - 1;
  T cv[CR][3][2];
#pragma unroll
  for (int cr = 0; cr < CR; ++cr)
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const int J = min(max(jb + cr, 0), dc.ny1 - 1), I = min(max(c0 + t, 0), dc.nx1 - 1);
      load_node<2, T>(zc, (int64_t)J * dc.nx1 + I, cv[cr][t]);
    }
  const bool ieven = ((i - 1) & 1) != 0;
  // per fine column cc: first and second coarse column (relative to c0) and count,
  // for odd i and for even i
  constexpr int I0o[3] = {0, 0, 1}, I1o[3] = {0, 1, 1}, Nio[3] = {1, 2, 1};
  constexpr int I0e[3] = {0, 1, 1}, I1e[3] = {1, 1, 2}, Nie[3] = {2, 1, 2};
#pragma unroll
  for (int rr = 0; rr < NJ + 2; ++rr) {
    const int jj = j0 - 1 + rr;
    const int nj = (rr & 1) == 0 ? 2 : 1;             // fine row j0-1+rr is odd when rr is even
    const int J0 = (rr + 1) >> 1;
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      const int ii = i - 1 + cc;
      const bool ok = !EDGE || (ii >= 1 && ii < d.nx1 && jj >= 0 && jj < d.ny1);
      const unsigned o = 2u * ((unsigned)min(max(jj, 0), d.ny1 - 1) * (unsigned)d.nx1 + (unsigned)(ok ? ii : 0));
      T acc[2] = {z2[o], z2[o + 1]};
      const int ni = ieven ? Nie[cc] : Nio[cc];
      const T wgt = T((ni == 2 ? 0.5f : 1.0f) * (nj == 2 ? 0.5f : 1.0f));
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const bool use = e < ni && b < nj;
          const int Jr = J0 + (b < nj ? b : 0);
          const int Io = e == 0 ? I0o[cc] : I1o[cc], Ie = e == 0 ? I0e[cc] : I1e[cc];
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            const T vv = ieven ? cv[Jr][Ie][c] : cv[Jr][Io][c];
            acc[c] += use ? wgt * vv : T(0);
          }
        }
      w[rr][cc][0] = ok ? acc[0] : T(0);
      w[rr][cc][1] = ok ? acc[1] : T(0);
    }
  }
}

// First two damped-Jacobi sweeps from a zero iterate on the finest level: w gets
// z1 = omega D^-1 r on the thread's (NJ+2) x 3 neighbourhood (zero outside the grid
// and on clamped nodes), then acc = A z1 and dg = D on its NJ nodes.  D at each
// neighbourhood node is summed over its four elements in the order of TileApply.
template <typename T, int NJ, bool EDGE>
__device__ inline void jacobi2_tile(const OpFineK<2, T>& op, const Dims& d, int i, int j0, const T* __restrict__ r,
                                    T omega, T (&w)[NJ + 2][3][2], T (&acc)[NJ][2], T (&dg)[NJ][2]) {
  // Element (i-2+ec, j0-2+er), the zero pad outside the grid.  The outer ring can
  // lie outside the grid even on interior tiles (a node on the last row or column
  // has no element beyond it), so every index is checked.
  T xb[NJ + 3][4];
#pragma unroll
  for (int er = 0; er < NJ + 3; ++er)
#pragma unroll
    for (int ec = 0; ec < 4; ++ec) {
      const int ei = i - 2 + ec, ej = j0 - 2 + er;
      xb[er][ec] = op.x[elem_in(d, ei, ej) ? (int64_t)ej * d.nx + ei : op.m];
    }
  load_tile<T, NJ, EDGE>(r, d, i, j0, w);   // r on the neighbourhood, then z1 in place
#pragma unroll
  for (int rr = 0; rr < NJ + 2; ++rr)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      const int ii = i - 1 + cc, jj = j0 - 1 + rr;
      const bool ok = !EDGE || (ii >= 1 && ii < d.nx1 && jj >= 0 && jj < d.ny1);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        T dd = T(0);
#pragma unroll
        for (int ey = 0; ey < 2; ++ey)
#pragma unroll
          for (int ex = 0; ex < 2; ++ex) {
            const int a = loc_index(1 - ex, 1 - ey, 0);
            dd += xb[rr + ey][cc + ex] * k0sq<T>(2 * a + c, 2 * a + c);
          }
        w[rr][cc][c] = ok ? omega * w[rr][cc][c] * recip(dd) : T(0);
      }
    }
  T xe[NJ + 1][2];
#pragma unroll
  for (int er = 0; er <= NJ; ++er)
#pragma unroll
    for (int ec = 0; ec < 2; ++ec) xe[er][ec] = xb[er + 1][ec + 1];
  TileApply<T, OpFineK<2, T>, true, NJ>::run_x(xe, w, acc, dg);
}

// Lane-shared forms of load_tile, load_tile_prolong and jacobi2_tile: the thread
// forms column i of the neighbourhood (the same values, in the same order, as the
// per-thread forms) and takes columns i-1 and i+1 from its neighbouring lanes.
template <typename T, int NJ, bool EDGE>
__device__ inline void load_col(const T* __restrict__ v, const Dims& d, int i, int j0, T (&w)[NJ + 2][3][2]) {
#pragma unroll
  for (int rr = 0; rr < NJ + 2; ++rr) {
    const int jj = j0 - 1 + rr;
    if (!EDGE) {
      const unsigned o = 2u * ((unsigned)jj * (unsigned)d.nx1 + (unsigned)i);
      w[rr][1][0] = v[o];
      w[rr][1][1] = v[o + 1];
    } else {
      const bool ok = i >= 1 && i < d.nx1 && jj >= 0 && jj < d.ny1;
      const unsigned o = 2u * ((unsigned)min(max(jj, 0), d.ny1 - 1) * (unsigned)d.nx1 +
                               (unsigned)min(max(i, 0), d.nx1 - 1));
      const T a = v[o], b = v[o + 1];
      w[rr][1][0] = ok ? a : T(0);
      w[rr][1][1] = ok ? b : T(0);
    }
  }
  share_columns<T, NJ>(w);
}

template <typename T, int NJ, bool EDGE>
__device__ inline void load_col_prolong(const T* __restrict__ z2, const T* __restrict__ zc, const Dims& d,
                                        const Dims& dc, int i, int j0, T (&w)[NJ + 2][3][2]) {
  static_assert(NJ % 2 == 0, "the folded prolongation needs an even node count per thread");
  constexpr int CR = NJ / 2 + 2;
  const int jb = (j0 >> 1) - 1;
  const bool odd = (i & 1) != 0;                 // odd column: two coarse columns, weight 1/2
  const int I0 = min(max(i >> 1, 0), dc.nx1 - 1), I1 = min(max((i + 1) >> 1, 0), dc.nx1 - 1);
  T cv[CR][2][2];
#pragma unroll
  for (int cr = 0; cr < CR; ++cr) {
    const int J = min(max(jb + cr, 0), dc.ny1 - 1);
    load_node<2, T>(zc, (int64_t)J * dc.nx1 + I0, cv[cr][0]);
    load_node<2, T>(zc, (int64_t)J * dc.nx1 + I1, cv[cr][1]);
  }
#pragma unroll
  for (int rr = 0; rr < NJ + 2; ++rr) {
    const int jj = j0 - 1 + rr;
    const int nj = (rr & 1) == 0 ? 2 : 1;
    const int J0 = (rr + 1) >> 1;
    const bool ok = !EDGE || (i >= 1 && i < d.nx1 && jj >= 0 && jj < d.ny1);
    const unsigned o = 2u * ((unsigned)min(max(jj, 0), d.ny1 - 1) * (unsigned)d.nx1 + (unsigned)(ok ? i : 0));
    T acc[2] = {z2[o], z2[o + 1]};
    const int ni = odd ? 2 : 1;
    const T wgt = T((ni == 2 ? 0.5f : 1.0f) * (nj == 2 ? 0.5f : 1.0f));
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const bool use = e < ni && b < nj;
        const int Jr = J0 + (b < nj ? b : 0);
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[c] += use ? wgt * cv[Jr][e][c] : T(0);
      }
    w[rr][1][0] = ok ? acc[0] : T(0);
    w[rr][1][1] = ok ? acc[1] : T(0);
  }
  share_columns<T, NJ>(w);
}

// EDGE false: the caller has checked that the elements (i-1..i, j0-2..j0+NJ) of every
// lane lie inside the grid.
template <typename T, int NJ, bool EDGE>
__device__ inline void jacobi2_col(const OpFineK<2, T>& op, const Dims& d, int i, int j0, const T* __restrict__ r,
                                   T omega, T (&w)[NJ + 2][3][2], T (&acc)[NJ][2], T (&dg)[NJ][2]) {
  // elements (i-1+ec, j0-2+er), the zero pad outside the grid
  T xb[NJ + 3][2];
#pragma unroll
  for (int er = 0; er < NJ + 3; ++er)
#pragma unroll
    for (int ec = 0; ec < 2; ++ec) {
      const int ei = i - 1 + ec, ej = j0 - 2 + er;
      xb[er][ec] = op.x[(!EDGE || elem_in(d, ei, ej)) ? (int64_t)ej * d.nx + ei : op.m];
    }
#pragma unroll
  for (int rr = 0; rr < NJ + 2; ++rr) {
    const int jj = j0 - 1 + rr;
    const bool ok = !EDGE || (i >= 1 && i < d.nx1 && jj >= 0 && jj < d.ny1);
    T rv[2];
    if (!EDGE) {
      const unsigned o = 2u * ((unsigned)jj * (unsigned)d.nx1 + (unsigned)i);
      rv[0] = r[o];
      rv[1] = r[o + 1];
    } else {
      const unsigned o = 2u * ((unsigned)min(max(jj, 0), d.ny1 - 1) * (unsigned)d.nx1 +
                               (unsigned)min(max(i, 0), d.nx1 - 1));
      const T a = r[o], b = r[o + 1];
      rv[0] = ok ? a : T(0);
      rv[1] = ok ? b : T(0);
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      T dd = T(0);
#pragma unroll
      for (int ey = 0; ey < 2; ++ey)
#pragma unroll
        for (int ex = 0; ex < 2; ++ex) {
          const int a = loc_index(1 - ex, 1 - ey, 0);
          dd += xb[rr + ey][ex] * k0sq<T>(2 * a + c, 2 * a + c);
        }
      w[rr][1][c] = ok ? omega * rv[c] * recip(dd) : T(0);
    }
  }
  share_columns<T, NJ>(w);
  T xe[NJ + 1][2];
#pragma unroll
  for (int er = 0; er <= NJ; ++er)
#pragma unroll
    for (int ec = 0; ec < 2; ++ec) xe[er][ec] = xb[er + 1][ec];
  TileApply<T, OpFineK<2, T>, true, NJ>::run_x(xe, w, acc, dg);
}

// The two pre-smoothing sweeps from zero and the residual of their result, in one
// lane-shared pass (finest level of K): z1 = omega D^-1 r on the lane's column over
// NJ+4 rows, z2 = z1 + omega D^-1 (r - A z1) over NJ+2 rows, t = r - A z2 on its NJ
// rows, with columns i-1 and i+1 of z1 and of z2 read from the neighbouring lanes.
// Every value is formed as in the separate passes (z2 as M_JACOBI2 stores it, zero on
// nodes outside the grid and on clamped ones, as M_RESID reads it back), so z2 and
// t equal theirs bit for bit.  Lanes 0, 1, 62 and 63 are halo columns (z2 on lanes
// 0 and 63 lacks a neighbour); LS2_COLS output columns per tile.
// EDGE false: every load of every lane lies inside the grid, off the clamped column.
constexpr int LS2_COLS = 60;
template <typename T, int NJ, bool EDGE>
__device__ inline void jacobi2_resid_col(const OpFineK<2, T>& op, const Dims& d, int i, int j0,
                                         const T* __restrict__ r, T omega, T (&z2o)[NJ][2], T (&acc)[NJ][2],
                                         T (&ro)[NJ][2]) {
  constexpr int R1 = NJ + 4, R2 = NJ + 2;
  // elements (i-1+ec, j0-3+er), the zero pad outside the grid
  T xb[NJ + 5][2];
#pragma unroll
  for (int er = 0; er < NJ + 5; ++er)
#pragma unroll
    for (int ec = 0; ec < 2; ++ec) {
      const int ei = i - 1 + ec, ej = j0 - 3 + er;
      xb[er][ec] = op.x[(!EDGE || elem_in(d, ei, ej)) ? (int64_t)ej * d.nx + ei : op.m];
    }
  // r on rows j0-2 .. j0+NJ+1 of the lane's column (zero outside the grid, clamped)
  T rv[R1][2];
  bool ok[R1];
#pragma unroll
  for (int rr = 0; rr < R1; ++rr) {
    const int jj = j0 - 2 + rr;
    ok[rr] = !EDGE || (i >= 1 && i < d.nx1 && jj >= 0 && jj < d.ny1);
    const unsigned o = EDGE ? 2u * ((unsigned)min(max(jj, 0), d.ny1 - 1) * (unsigned)d.nx1 +
                                    (unsigned)min(max(i, 0), d.nx1 - 1))
                            : 2u * ((unsigned)jj * (unsigned)d.nx1 + (unsigned)i);
    const T a = r[o], b = r[o + 1];
    rv[rr][0] = ok[rr] ? a : T(0);
    rv[rr][1] = ok[rr] ? b : T(0);
  }
  // z1 on the R1 rows (diagonal summed as in jacobi2_tile)
  T w1[R1][3][2];
#pragma unroll
  for (int rr = 0; rr < R1; ++rr)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      T dd = T(0);
#pragma unroll
      for (int ey = 0; ey < 2; ++ey)
#pragma unroll
        for (int ex = 0; ex < 2; ++ex) {
          const int a = loc_index(1 - ex, 1 - ey, 0);
          dd += xb[rr + ey][ex] * k0sq<T>(2 * a + c, 2 * a + c);
        }
      w1[rr][1][c] = ok[rr] ? omega * rv[rr][c] * recip(dd) : T(0);
    }
  share_columns<T, NJ + 2>(w1);
  // A z1 and D on rows j0-1 .. j0+NJ, then z2 there
  T a1[R2][2], d1[R2][2];
  {
    T xe[R2 + 1][2];
#pragma unroll
    for (int er = 0; er <= R2; ++er)
#pragma unroll
      for (int ec = 0; ec < 2; ++ec) xe[er][ec] = xb[er + 1][ec];
    TileApply<T, OpFineK<2, T>, true, R2>::run_x(xe, w1, a1, d1);
  }
  T w2[R2][3][2];
#pragma unroll
  for (int n = 0; n < R2; ++n)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const T o = w1[n + 1][1][c] + omega * (rv[n + 1][c] - a1[n][c]) * recip(d1[n][c]);
      w2[n][1][c] = ok[n + 1] ? o : T(0);
    }
  share_columns<T, NJ>(w2);
  // A z2 on the lane's NJ rows
  T xe2[NJ + 1][2], dg[NJ][2];
#pragma unroll
  for (int er = 0; er <= NJ; ++er)
#pragma unroll
    for (int ec = 0; ec < 2; ++ec) xe2[er][ec] = xb[er + 2][ec];
  TileApply<T, OpFineK<2, T>, true, NJ>::run_x(xe2, w2, acc, dg);
#pragma unroll
  for (int n = 0; n < NJ; ++n)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      z2o[n][c] = w2[n + 1][1][c];
      ro[n][c] = rv[n + 2][c];
    }
}

// Pass of jacobi2_resid_col: z2 into z2out, t = r - A z2 into tout.  fin_blocks != 0:
// the first block also finalizes the preceding residual update's ||r||^2 (as the
// M_JACOBI2 pass does).
template <typename T, int NJ>
__global__ __launch_bounds__(BS) void k_jacobi2r2d(OpFineK<2, T> op, Dims d, const T* __restrict__ r,
                                                   T* __restrict__ z2out, T* __restrict__ tout,
                                                   const double* __restrict__ omg, Red red, const int* gate,
                                                   unsigned fin_blocks, int fin_zpend) {
  if (gate && *gate) return;
  const T omega = T(*omg);
  const Tile tl = xcd_tile();
  constexpr int RJ = (BS / 64) * NJ;
  const int lane = threadIdx.x & 63;
  const int ti0 = (int)tl.x * LS2_COLS - 2, tj0 = tl.y * RJ;
  const int i = ti0 + lane;
  const int j0 = tj0 + (threadIdx.x >> 6) * NJ;
  const bool interior = ti0 >= 1 && ti0 + 65 <= d.nx1 && tj0 >= 3 && tj0 + RJ + 3 <= d.ny1;
  T z2[NJ][2], acc[NJ][2], rr[NJ][2];
  if (interior) jacobi2_resid_col<T, NJ, false>(op, d, i, j0, r, omega, z2, acc, rr);
  else jacobi2_resid_col<T, NJ, true>(op, d, i, j0, r, omega, z2, acc, rr);
  if (lane >= 2 && lane < 2 + LS2_COLS) {
#pragma unroll
    for (int n = 0; n < NJ; ++n) {
      const int j = j0 + n;
      if (!interior && (i >= d.nx1 || j >= d.ny1)) continue;
      const int64_t q = (int64_t)j * d.nx1 + i;
      T t[2];
#pragma unroll
      for (int c = 0; c < 2; ++c) t[c] = rr[n][c] - acc[n][c];
      if (!interior && i == 0) {
        const T z[2] = {T(0), T(0)};
        store_node<2, T>(z2out, q, z);
        store_node<2, T>(tout, q, z);
        continue;
      }
      store_node<2, T>(z2out, q, z2[n]);
      store_node<2, T>(tout, q, t);
    }
  }
  if (fin_blocks && block_id() == 0) {
    double tot[1];
    sum_partials<1>(red, fin_blocks, tot);
    if (threadIdx.x == 0) rn2_finish(tot[0], red, fin_zpend != 0);
  }
}

// The solution update z2 + P zc and the two post-smoothing sweeps in one lane-shared
// pass (finest level of K): v = z2 + P zc on NJ+4 rows of the lane's column (summed
// as load_col_prolong does), z3 = v + omega D^-1 (r - A v) on NJ+2 rows, and
// z4 = z3 + omega D^-1 (r - A z3) on its NJ rows, the neighbouring columns of v and
// of z3 read from the neighbouring lanes; zero on nodes outside the grid and on
// clamped ones, as the separate passes store and read them.  BETA: the last sweep's
// partial sum r~'z4 for the PCG ratio (dot64 = r~ in FP64), as M_JACOBI_BETA.
// LS2_COLS output columns per tile, lanes 0, 1, 62 and 63 halo columns.
template <typename T, int NJ, bool EDGE>
__device__ inline void pjacobi2_col(const OpFineK<2, T>& op, const Dims& d, const Dims& dc, int i, int j0,
                                    const T* __restrict__ z2, const T* __restrict__ zc, const T* __restrict__ r,
                                    T omega, T (&z4)[NJ][2]) {
  static_assert(NJ % 2 == 0, "the folded prolongation needs an even node count per thread");
  constexpr int R1 = NJ + 4, R2 = NJ + 2, CR = NJ / 2 + 3;
  T xb[NJ + 5][2];                                    // elements (i-1+ec, j0-3+er)
#pragma unroll
  for (int er = 0; er < NJ + 5; ++er)
#pragma unroll
    for (int ec = 0; ec < 2; ++ec) {
      const int ei = i - 1 + ec, ej = j0 - 3 + er;
      xb[er][ec] = op.x[(!EDGE || elem_in(d, ei, ej)) ? (int64_t)ej * d.nx + ei : op.m];
    }
  // coarse rows j0/2-1 .. j0/2+NJ/2+1, columns i>>1 and (i+1)>>1
  const int jb = (j0 >> 1) - 1;
  const bool odd = (i & 1) != 0;
  const int I0 = min(max(i >> 1, 0), dc.nx1 - 1), I1 = min(max((i + 1) >> 1, 0), dc.nx1 - 1);
  T cv[CR][2][2];
#pragma unroll
  for (int cr = 0; cr < CR; ++cr) {
    const int J = min(max(jb + cr, 0), dc.ny1 - 1);
    load_node<2, T>(zc, (int64_t)J * dc.nx1 + I0, cv[cr][0]);
    load_node<2, T>(zc, (int64_t)J * dc.nx1 + I1, cv[cr][1]);
  }
  // r on rows j0-1 .. j0+NJ (clamped index; results on other nodes are masked)
  T rv[R2][2];
#pragma unroll
  for (int n = 0; n < R2; ++n) {
    const int jj = min(max(j0 - 1 + n, 0), d.ny1 - 1), ic = min(max(i, 0), d.nx1 - 1);
    load_node<2, T>(r, (int64_t)jj * d.nx1 + ic, rv[n]);
  }
  // v = z2 + P zc on rows j0-2 .. j0+NJ+1 (row j0-2+rr is odd when rr is odd)
  T w1[R1][3][2];
  bool ok[R1];
#pragma unroll
  for (int rr = 0; rr < R1; ++rr) {
    const int jj = j0 - 2 + rr;
    const int nj = (rr & 1) ? 2 : 1;
    const int J0 = rr >> 1;
    ok[rr] = !EDGE || (i >= 1 && i < d.nx1 && jj >= 0 && jj < d.ny1);
    const unsigned o = 2u * ((unsigned)min(max(jj, 0), d.ny1 - 1) * (unsigned)d.nx1 + (unsigned)(ok[rr] ? i : 0));
    T acc[2] = {z2[o], z2[o + 1]};
    const int ni = odd ? 2 : 1;
    const T wgt = T((ni == 2 ? 0.5f : 1.0f) * (nj == 2 ? 0.5f : 1.0f));
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const bool use = e < ni && b < nj;
        const int Jr = J0 + (b < nj ? b : 0);
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[c] += use ? wgt * cv[Jr][e][c] : T(0);
      }
    w1[rr][1][0] = ok[rr] ? acc[0] : T(0);
    w1[rr][1][1] = ok[rr] ? acc[1] : T(0);
  }
  share_columns<T, NJ + 2>(w1);
  // z3 on rows j0-1 .. j0+NJ
  T a1[R2][2], d1[R2][2];
  {
    T xe[R2 + 1][2];
#pragma unroll
    for (int er = 0; er <= R2; ++er)
#pragma unroll
      for (int ec = 0; ec < 2; ++ec) xe[er][ec] = xb[er + 1][ec];
    TileApply<T, OpFineK<2, T>, true, R2>::run_x(xe, w1, a1, d1);
  }
  T w2[R2][3][2];
#pragma unroll
  for (int n = 0; n < R2; ++n)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const T o = w1[n + 1][1][c] + omega * (rv[n][c] - a1[n][c]) * recip(d1[n][c]);
      w2[n][1][c] = ok[n + 1] ? o : T(0);
    }
  share_columns<T, NJ>(w2);
  // z4 on the lane's rows
  T xe2[NJ + 1][2], acc[NJ][2], dg[NJ][2];
#pragma unroll
  for (int er = 0; er <= NJ; ++er)
#pragma unroll
    for (int ec = 0; ec < 2; ++ec) xe2[er][ec] = xb[er + 2][ec];
  TileApply<T, OpFineK<2, T>, true, NJ>::run_x(xe2, w2, acc, dg);
#pragma unroll
  for (int n = 0; n < NJ; ++n)
#pragma unroll
    for (int c = 0; c < 2; ++c)
      z4[n][c] = w2[n + 1][1][c] + omega * (rv[n + 1][c] - acc[n][c]) * recip(dg[n][c]);
}

template <typename T, int NJ, bool BETA>
__global__ __launch_bounds__(BS) void k_pjacobi2d(OpFineK<2, T> op, Dims d, Dims dc, const T* __restrict__ z2,
                                                  const T* __restrict__ zc, const T* __restrict__ r,
                                                  T* __restrict__ out, const double* __restrict__ omg,
                                                  const double* __restrict__ dot64, Red red, const int* gate) {
  if (gate && *gate) return;
  const T omega = T(*omg);
  const Tile tl = xcd_tile();
  constexpr int RJ = (BS / 64) * NJ;
  const int lane = threadIdx.x & 63;
  const int ti0 = (int)tl.x * LS2_COLS - 2, tj0 = tl.y * RJ;
  const int i = ti0 + lane;
  const int j0 = tj0 + (threadIdx.x >> 6) * NJ;
  const bool interior = ti0 >= 1 && ti0 + 65 <= d.nx1 && tj0 >= 3 && tj0 + RJ + 3 <= d.ny1;
  double dpre[NJ][2];
  if constexpr (BETA) {
#pragma unroll
    for (int n = 0; n < NJ; ++n) {
      const int j = min(j0 + n, d.ny1 - 1), ic = min(max(i, 0), d.nx1 - 1);
      const double2 t = *reinterpret_cast<const double2*>(dot64 + 2 * ((int64_t)j * d.nx1 + ic));
      dpre[n][0] = t.x;
      dpre[n][1] = t.y;
    }
  }
  T z4[NJ][2];
  if (interior) pjacobi2_col<T, NJ, false>(op, d, dc, i, j0, z2, zc, r, omega, z4);
  else pjacobi2_col<T, NJ, true>(op, d, dc, i, j0, z2, zc, r, omega, z4);
  double red0 = 0.0;
  if (lane >= 2 && lane < 2 + LS2_COLS) {
#pragma unroll
    for (int n = 0; n < NJ; ++n) {
      const int j = j0 + n;
      if (!interior && (i >= d.nx1 || j >= d.ny1)) continue;
      const int64_t q = (int64_t)j * d.nx1 + i;
      if (!interior && i == 0) {
        const T z[2] = {T(0), T(0)};
        store_node<2, T>(out, q, z);
        continue;
      }
      if constexpr (BETA) {
#pragma unroll
        for (int c = 0; c < 2; ++c) red0 += dpre[n][c] * (double)z4[n][c];
      }
      store_node<2, T>(out, q, z4[n]);
    }
  }
  if constexpr (BETA) {
    const double vals[3] = {red0, 0.0, 0.0};
    block_partials<3>(vals, red);
  }
}

// 2D level pass with register blocking: each thread owns NJ consecutive nodes
// along y of one column and loads the (NJ+2) x 3 window of neighbours once.  Tiles
// whose nodes are all at least one node away from every boundary (and off the
// clamped column) skip every bounds check; the others run the same code with
// masked loads, so that no block waits on a chain of per-node loads.
// Modes as in k_level except M_POWER and M_RAYLEIGH.
// M_PJACOBI: v is z2 on this level and zc the coarse correction on level dc; the
// sweep starts from z2 + P zc (the prolongation of the V-cycle's up path folded in).
// M_JACOBI2 (finest level, A_e = x_e K0): the first two pre-smoothing sweeps from a
// zero iterate in one pass; the first sweep's z1 = omega D^-1 r is formed on the
// thread's neighbourhood from r and the densities of the (NJ+3) x 4 elements around
// it (same arithmetic and order as the M_JACOBI0 pass), so z1 is never stored.
// LS (finest level of K): lane-shared tiles of LS_COLS output columns, lanes 0 and
// 63 the halo columns (see lane_from_left); the same values in the same order.
template <typename T, class Op, int MODE, int NJ, bool LS = false>
__global__ __launch_bounds__(BS) void k_level2d(Op op, Dims d, const T* __restrict__ v,
                                                const T* __restrict__ r, T* __restrict__ out,
                                                const double* __restrict__ omg, Aug<T> aug, Red red,
                                                const double* __restrict__ dot64, const int* gate,
                                                const T* __restrict__ zc, Dims dc, unsigned fin_blocks,
                                                int fin_zpend) {
  if (gate && *gate) return;
  const T omega = omg ? T(*omg) : T(0);
  static_assert(!LS || std::is_same<Op, OpFineK<2, T>>::value, "lane-shared tiles: finest level of K");
  const Tile tl = xcd_tile();
  constexpr int RJ = (BS / 64) * NJ;               // node rows per tile
  const int lane = threadIdx.x & 63;
  const int ti0 = LS ? (int)tl.x * LS_COLS - 1 : (int)tl.x * 64, tj0 = tl.y * RJ;
  const int i = ti0 + lane;
  const int j0 = tj0 + (threadIdx.x >> 6) * NJ;
  const T vl = (aug.b && MODE != M_JACOBI0) ? v[aug.n] : T(0);
  double bdot = 0.0, red0 = 0.0, red1 = 0.0;
  // interior: every load of the tile is inside the grid and off the clamped column
  // (lane-shared M_JACOBI2: also the ring of elements around the neighbourhood)
  const bool interior = LS ? (MODE == M_JACOBI2 ? (ti0 >= 1 && ti0 + 65 <= d.nx1 && tj0 >= 2 && tj0 + RJ + 2 <= d.ny1)
                                                : (ti0 >= 1 && ti0 + 64 <= d.nx1 && tj0 >= 1 && tj0 + RJ + 1 <= d.ny1))
                           : (ti0 >= 2 && ti0 + 65 <= d.nx1 && tj0 >= 1 && tj0 + RJ + 1 <= d.ny1);
  constexpr bool ROWS = MODE != M_JACOBI0;
  // The thread's entries of r, of the FP64 dot vector and of the border are loaded
  // first, without branches (index clamped into the grid), so they are in flight
  // with the tile's loads instead of waiting one by one after the arithmetic.
  T rpre[NJ][2], bpre[NJ][2];
  double dpre[NJ][2];
#pragma unroll
  for (int n = 0; n < NJ; ++n) {
    const int j = min(j0 + n, d.ny1 - 1), ic = min(max(i, 0), d.nx1 - 1);
    const int64_t q = (int64_t)j * d.nx1 + ic;
    if constexpr (mode_reads_r<MODE>()) load_node<2, T>(r, q, rpre[n]);
    if constexpr (MODE == M_JACOBI_BETA) {
      const double2 t = *reinterpret_cast<const double2*>(dot64 + 2 * q);
      dpre[n][0] = t.x;
      dpre[n][1] = t.y;
    }
    if (ROWS && aug.b) load_node<2, T>(aug.b, q, bpre[n]);
  }
  T w[NJ + 2][3][2];
  T acc[NJ][2], dg[NJ][2];
  if constexpr (MODE == M_JACOBI2) {
    static_assert(std::is_same<Op, OpFineK<2, T>>::value, "two fused sweeps from zero: finest level only");
    if constexpr (LS) {
      if (interior) jacobi2_col<T, NJ, false>(op, d, i, j0, r, omega, w, acc, dg);
      else jacobi2_col<T, NJ, true>(op, d, i, j0, r, omega, w, acc, dg);
    } else {
      if (interior) jacobi2_tile<T, NJ, false>(op, d, i, j0, r, omega, w, acc, dg);
      else jacobi2_tile<T, NJ, true>(op, d, i, j0, r, omega, w, acc, dg);
    }
  } else if constexpr (LS) {
    if (interior) {
      if constexpr (MODE == M_PJACOBI) load_col_prolong<T, NJ, false>(v, zc, d, dc, i, j0, w);
      else if constexpr (ROWS) load_col<T, NJ, false>(v, d, i, j0, w);
      TileApply<T, Op, ROWS, NJ>::template run_ls<false>(op, d, i, j0, w, acc, dg);
    } else {
      if constexpr (MODE == M_PJACOBI) load_col_prolong<T, NJ, true>(v, zc, d, dc, i, j0, w);
      else if constexpr (ROWS) load_col<T, NJ, true>(v, d, i, j0, w);
      TileApply<T, Op, ROWS, NJ>::template run_ls<true>(op, d, i, j0, w, acc, dg);
    }
  } else if (interior) {
    if constexpr (MODE == M_PJACOBI) load_tile_prolong<T, NJ, false>(v, zc, d, dc, i, j0, w);
    else if constexpr (ROWS) load_tile<T, NJ, false>(v, d, i, j0, w);
    TileApply<T, Op, ROWS, NJ>::template run<false>(op, d, i, j0, w, acc, dg);
  } else {
    if constexpr (MODE == M_PJACOBI) load_tile_prolong<T, NJ, true>(v, zc, d, dc, i, j0, w);
    else if constexpr (ROWS) load_tile<T, NJ, true>(v, d, i, j0, w);
    TileApply<T, Op, ROWS, NJ>::template run<true>(op, d, i, j0, w, acc, dg);
  }
#pragma unroll
  for (int n = 0; n < NJ; ++n) {
    const int j = j0 + n;
    if (LS && (lane == 0 || lane > LS_COLS)) continue;     // halo lanes
    if (!interior && (i >= d.nx1 || j >= d.ny1)) continue;
    const int64_t q = (int64_t)j * d.nx1 + i;
    if (!interior && i == 0) {
      const T z[2] = {T(0), T(0)};
      store_node<2, T>(out, q, z);
      continue;
    }
    const T vc[2] = {ROWS ? w[n + 1][1][0] : T(0), ROWS ? w[n + 1][1][1] : T(0)};
    level_node_finish_vals<2, T, MODE>(q, acc[n], dg[n], vc, rpre[n], out, omega, aug.b != nullptr, bpre[n], vl,
                                       1.0, dpre[n], bdot, red0, red1);
  }
  if (aug.b) {
    if constexpr (MODE == M_JACOBI0) {
      if (blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x == 0)
        out[aug.n] = T((double)omega * (double)r[aug.n] / aug.c);
    } else {
      const double vals[3] = {bdot, red0, red1};
      block_partials<3>(vals, red);
    }
  } else if constexpr (MODE == M_JACOBI_BETA) {
    const double vals[3] = {red0, red1, 0.0};
    block_partials<3>(vals, red);
  }
  if constexpr (MODE == M_JACOBI2) {
    // fin_blocks != 0: this pass follows the PCG residual update (same gate) and
    // its first block also finalizes that update's ||r||^2, in place of a
    // one-block kernel between the two; the later passes are gated on the result.
    if (fin_blocks && block_id() == 0) {
      double tot[1];
      sum_partials<1>(red, fin_blocks, tot);
      if (threadIdx.x == 0) rn2_finish(tot[0], red, fin_zpend != 0);
    }
  }
}

// First step of a PCG iteration, fused: p = -y + beta p_old (p_old, p in separate
// buffers), q = A p with the FP64 finest-level operator, and alpha = r'y / p'q
// (Algorithm PCG; the search direction uses the new preconditioned residual).
// first != 0: beta = 0 (p = -y).
template <int DIM, typename TY, class Op>
__global__ __launch_bounds__(BS) void k_dir_apply(Op op, Dims d, const TY* __restrict__ y,
                                                  const double* __restrict__ pold, double* __restrict__ p,
                                                  double* __restrict__ q, Aug<double> aug, Red red, int first,
                                                  const int* gate) {
  if (gate && *gate) return;
  const double beta = first ? 0.0 : red.scal[S_BETA];
  const Tile tl = xcd_tile();
  const int i = tl.x * 64 + (threadIdx.x & 63);
  const int j = tl.y * (BS / 64) + (threadIdx.x >> 6);
  const int k = tl.z;
  double pq = 0.0, bdot = 0.0, qy = 0.0;
  const double pl = aug.b ? (-(double)y[aug.n] + beta * (first ? 0.0 : pold[aug.n])) : 0.0;
  if (i < d.nx1 && j < d.ny1) {
    const int64_t qn = ((int64_t)k * d.ny1 + j) * d.nx1 + i;
    double o[DIM], pc[DIM];
    if (i == 0) {
#pragma unroll
      for (int c = 0; c < DIM; ++c) { o[c] = 0.0; pc[c] = 0.0; }
    } else {
      double vn[Geo<DIM>::NB][DIM];
#pragma unroll
      for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
          for (int dx = -1; dx <= 1; ++dx) {
            const int nb = nb_index<DIM>(dx, dy, dz);
            const int ii = i + dx, jj = j + dy, kk = k + dz;
            if (ii >= 1 && ii < d.nx1 && jj >= 0 && jj < d.ny1 && kk >= 0 && kk < d.nz1) {
              const int64_t qq = ((int64_t)kk * d.ny1 + jj) * d.nx1 + ii;
              TY yy[DIM];
              load_node<DIM, TY>(y, qq, yy);
              if (first) {
#pragma unroll
                for (int c = 0; c < DIM; ++c) vn[nb][c] = -(double)yy[c];
              } else {
                double po[DIM];
                load_node<DIM, double>(pold, qq, po);
#pragma unroll
                for (int c = 0; c < DIM; ++c) vn[nb][c] = -(double)yy[c] + beta * po[c];
              }
            } else {
#pragma unroll
              for (int c = 0; c < DIM; ++c) vn[nb][c] = 0.0;
            }
          }
      double acc[DIM], dg[DIM];
#pragma unroll
      for (int c = 0; c < DIM; ++c) { acc[c] = 0.0; dg[c] = 0.0; pc[c] = vn[nb_index<DIM>(0, 0, 0)][c]; }
      node_apply<DIM, double, Op, true, false>(op, d, i, j, k, vn, acc, dg);
      if (aug.b) {
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
          const double bc = aug.b[qn * DIM + c];
          acc[c] += bc * pl;
          bdot += bc * pc[c];
        }
      }
      TY yc[DIM];
      load_node<DIM, TY>(y, qn, yc);
#pragma unroll
      for (int c = 0; c < DIM; ++c) {
        o[c] = acc[c];
        pq += pc[c] * acc[c];
        qy += acc[c] * (double)yc[c];
      }
    }
    store_node<DIM, double>(p, qn, pc);
    store_node<DIM, double>(q, qn, o);
  }
  const double vals[3] = {pq, bdot, qy};
  block_partials<3>(vals, red);
}

// 2D form of k_dir_apply with register-blocked tiles (as k_level2d): each thread
// owns NJ nodes of one column, forms p = -y + beta p_old on the (NJ+2) x 3
// neighbourhood once and reuses it for the NJ rows of q = A p.
// ZF: the previous step's solution update zs += alpha p_old (alpha still in
// scal[S_ALPHA]) is done here on the thread's own nodes, where p_old is loaded
// anyway, when flags[F_ZPEND] is set; with the gate set only that update runs,
// so the last step's update is not lost when the stop test passed.  The zs
// loads follow the neighbourhood loads, so the operator's work hides them.
template <typename TY, class Op, int NJ, bool ZF>
__global__ __launch_bounds__(BS) void k_dir_apply2d(Op op, Dims d, const TY* __restrict__ y,
                                                    const double* __restrict__ pold, double* __restrict__ p,
                                                    double* __restrict__ q, Aug<double> aug, Red red, int first,
                                                    const int* gate, double* __restrict__ zs) {
  const bool zup = ZF && red.flags[F_ZPEND] != 0;
  const double alpha_prev = ZF ? red.scal[S_ALPHA] : 0.0;
  const Tile tl = xcd_tile();
  constexpr int RJ = (BS / 64) * NJ;
  const int ti0 = tl.x * 64, tj0 = tl.y * RJ;
  const int i = ti0 + (threadIdx.x & 63);
  const int j0 = tj0 + (threadIdx.x >> 6) * NJ;
  if (gate && *gate) {
    if (zup && i < d.nx1) {
#pragma unroll
      for (int n = 0; n < NJ; ++n) {
        const int j = j0 + n;
        if (j >= d.ny1) break;
        const int64_t qn = (int64_t)j * d.nx1 + i;
        double po[2], zz[2];
        load_node<2, double>(pold, qn, po);
        load_node<2, double>(zs, qn, zz);
#pragma unroll
        for (int c = 0; c < 2; ++c) zz[c] += alpha_prev * po[c];
        store_node<2, double>(zs, qn, zz);
      }
    }
    return;
  }
  const double beta = first ? 0.0 : red.scal[S_BETA];
  double pq = 0.0, bdot = 0.0, qy = 0.0;
  const double pl = aug.b ? (-(double)y[aug.n] + beta * (first ? 0.0 : pold[aug.n])) : 0.0;
  const bool interior = ti0 >= 2 && ti0 + 65 <= d.nx1 && tj0 >= 1 && tj0 + RJ + 1 <= d.ny1;
  // p = -y + beta p_old on the neighbourhood; yc keeps y on the thread's own nodes
  // (for q'y).  A neighbour outside the grid or clamped is read at the clamped node
  // (0, j) of its row, where y and p_old are zero, so no load sits under a branch
  // or feeds a select and all of them are in flight together.  (p_old is finite
  // on the first iteration too: both direction buffers start zeroed.)
  const double bf = first ? 0.0 : beta;
  TY yc[NJ][2];
  double w[NJ + 2][3][2], acc[NJ][2], dg[NJ][2];
  double zc[ZF ? NJ : 1][2];   // own nodes: p_old, then zs + alpha_prev p_old
#pragma unroll
  for (int rr = 0; rr < NJ + 2; ++rr)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      const int ii = i - 1 + cc, jj = j0 - 1 + rr;
      const bool ok = interior || (ii >= 1 && ii < d.nx1 && jj >= 0 && jj < d.ny1);
      const int64_t qq = (int64_t)min(max(jj, 0), d.ny1 - 1) * d.nx1 + (ok ? ii : 0);
      TY yy[2];
      double po[2];
      load_node<2, TY>(y, qq, yy);
      load_node<2, double>(pold, qq, po);
#pragma unroll
      for (int c = 0; c < 2; ++c) w[rr][cc][c] = -(double)yy[c] + bf * po[c];
      if (cc == 1 && rr >= 1 && rr <= NJ) {
        yc[rr - 1][0] = yy[0];
        yc[rr - 1][1] = yy[1];
        if constexpr (ZF) {
          zc[rr - 1][0] = po[0];
          zc[rr - 1][1] = po[1];
        }
      }
    }
  if constexpr (ZF) {
    if (zup) {
#pragma unroll
      for (int n = 0; n < NJ; ++n) {   // clamped into the grid like the neighbourhood
        const int jj = min(j0 + n, d.ny1 - 1);
        const int64_t qq = (int64_t)jj * d.nx1 + (interior || i < d.nx1 ? i : 0);
        double zz[2];
        load_node<2, double>(zs, qq, zz);
#pragma unroll
        for (int c = 0; c < 2; ++c) zc[n][c] = zz[c] + alpha_prev * zc[n][c];
      }
    }
  }
  if (interior) TileApply<double, Op, true, NJ>::template run<false>(op, d, i, j0, w, acc, dg);
  else TileApply<double, Op, true, NJ>::template run<true>(op, d, i, j0, w, acc, dg);
#pragma unroll
  for (int n = 0; n < NJ; ++n) {
    const int j = j0 + n;
    if (!interior && (i >= d.nx1 || j >= d.ny1)) continue;
    const int64_t qn = (int64_t)j * d.nx1 + i;
    double o[2] = {acc[n][0], acc[n][1]};
    double pc[2] = {w[n + 1][1][0], w[n + 1][1][1]};
    if (!interior && i == 0) {
      o[0] = o[1] = pc[0] = pc[1] = 0.0;
    } else {
      if (aug.b) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const double bc = aug.b[qn * 2 + c];
          o[c] += bc * pl;
          bdot += bc * pc[c];
        }
      }
      pq += pc[0] * o[0] + pc[1] * o[1];
      qy += o[0] * (double)yc[n][0] + o[1] * (double)yc[n][1];
    }
    store_node<2, double>(p, qn, pc);
    store_node<2, double>(q, qn, o);
    if constexpr (ZF) {
      if (zup) store_node<2, double>(zs, qn, zc[n]);
    }
  }
  const double vals[3] = {pq, bdot, qy};
  block_partials<3>(vals, red);
}

// 3D form of the first step of a PCG iteration, in two kernels: k_pdir3 writes
// p = -y + beta p_old (zero on clamped nodes), k_dir_apply3 gathers q = A p element
// by element (node_apply_gather3) with the border term b p_lambda and the partials
// of p'q, b'p and q'y.  Finalized by k_dir_fin like k_dir_apply.
template <typename TY>
__global__ __launch_bounds__(BS) void k_pdir3(Dims d, const TY* __restrict__ y, const double* __restrict__ pold,
                                              double* __restrict__ p, Red red, int first, const int* gate) {
  if (gate && *gate) return;
  const double beta = first ? 0.0 : red.scal[S_BETA];
  const int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (t >= d.nslots) return;
  const int64_t q = t / 3;
  const int i = (int)(q % d.nx1);
  p[t] = i == 0 ? 0.0 : -(double)y[t] + (first ? 0.0 : beta * pold[t]);
}

template <typename TY, class Op>
__global__ __launch_bounds__(BS) void k_dir_apply3(Op op, Dims d, const TY* __restrict__ y,
                                                   const double* __restrict__ pold, const double* __restrict__ p,
                                                   double* __restrict__ q, Aug<double> aug, Red red, int first,
                                                   const int* gate) {
  if (gate && *gate) return;
  const double beta = first ? 0.0 : red.scal[S_BETA];
  const Tile tl = xcd_tile();
  const int i = tl.x * 64 + (threadIdx.x & 63);
  const int j = tl.y * (BS / 64) + (threadIdx.x >> 6);
  const int k = tl.z;
  double pq = 0.0, bdot = 0.0, qy = 0.0;
  const double pl = aug.b ? (-(double)y[aug.n] + beta * (first ? 0.0 : pold[aug.n])) : 0.0;
  if (i < d.nx1 && j < d.ny1) {
    const int64_t qn = ((int64_t)k * d.ny1 + j) * d.nx1 + i;
    double o[3] = {0.0, 0.0, 0.0};
    if (i > 0) {
      double dg[3];
      node_apply_gather3<double, Op, true, false>(op, d, i, j, k, p, o, dg);
      double pc[3];
      load_node<3, double>(p, qn, pc);
      TY yc[3];
      load_node<3, TY>(y, qn, yc);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (aug.b) {
          const double bc = aug.b[qn * 3 + c];
          o[c] += bc * pl;
          bdot += bc * pc[c];
        }
        pq += pc[c] * o[c];
        qy += o[c] * (double)yc[c];
      }
    }
    store_node<3, double>(q, qn, o);
  }
  const double vals[3] = {pq, bdot, qy};
  block_partials<3>(vals, red);
}

// Finalize of k_dir_apply: lambda entries of p and q (augmented system) and
// alpha = rho / p'q, with the breakdown test p'q > 0.  With zs (solution update
// folded into the direction kernel) it also updates the lambda entry of zs and
// clears the pending flag, gate or not.
template <typename TY>
__global__ __launch_bounds__(BS) void k_dir_fin(const TY* __restrict__ y, const double* __restrict__ pold,
                                                double* __restrict__ p, double* __restrict__ q, int aug, double c,
                                                int64_t n, int first, Red red, unsigned nblocks, const int* gate,
                                                double* __restrict__ zs) {
  if (zs && threadIdx.x == 0 && red.flags[F_ZPEND]) {
    if (aug) zs[n] += red.scal[S_ALPHA] * pold[n];
    red.flags[F_ZPEND] = 0;
  }
  if (gate && *gate) return;
  double tot[3];
  sum_partials<3>(red, nblocks, tot);
  if (threadIdx.x != 0) return;
  double ptq = tot[0], qy = tot[2];
  if (aug) {
    const double beta = first ? 0.0 : red.scal[S_BETA];
    const double pl = -(double)y[n] + (first ? 0.0 : beta * pold[n]);
    const double ql = tot[1] + c * pl;
    p[n] = pl;
    q[n] = ql;
    ptq += pl * ql;
    qy += ql * (double)y[n];
  }
  red.scal[S_PQ] = ptq;
  red.scal[S_QY] = qy;
  if (!(ptq > 0.0) || !isfinite(ptq)) {
    red.flags[F_DONE] = 2;
    red.flags[F_STATUS] = IPMG_E_BREAKDOWN;
  } else {
    red.scal[S_ALPHA] = red.scal[S_RHO] / ptq;
  }
}

// ---------------------------------------------------------------- transfers --
// 1D linear interpolation weight between a fine offset and its coarse node.
__device__ inline float w1(int off) { return off == 0 ? 1.0f : 0.5f; }

// Restriction rc = P' rf (transpose of the bilinear / trilinear prolongation,
// Sec. 7), one thread per coarse node; clamped coarse nodes get 0.
template <int DIM, typename T, typename TS = T>
__global__ __launch_bounds__(BS) void k_restrict(Dims f, Dims c, const TS* __restrict__ rf,
                                                 T* __restrict__ rc, int aug, const int* gate) {
  if (gate && *gate) return;
  const Tile tl = xcd_tile();
  const int I = tl.x * 64 + (threadIdx.x & 63);
  const int J = tl.y * (BS / 64) + (threadIdx.x >> 6);
  const int K = tl.z;
  if (aug && I == 0 && J == 0 && K == 0) rc[c.nslots] = T(rf[f.nslots]);
  if (I >= c.nx1 || J >= c.ny1) return;
  const int64_t qc = ((int64_t)K * c.ny1 + J) * c.nx1 + I;
  T acc[DIM];
#pragma unroll
  for (int cc = 0; cc < DIM; ++cc) acc[cc] = T(0);
  // Branch-free: every neighbour is loaded (index clamped into the grid) and the
  // ones outside the grid, or of a clamped coarse node, are dropped by a select,
  // so all loads are in flight together.
#pragma unroll
  for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int i = 2 * I + dx, j = 2 * J + dy, k = 2 * K + dz;
        const bool ok = I > 0 && i >= 1 && i < f.nx1 && j >= 0 && j < f.ny1 && k >= 0 && k < f.nz1;
        const int ic = min(max(i, 0), f.nx1 - 1), jc = min(max(j, 0), f.ny1 - 1), kc = min(max(k, 0), f.nz1 - 1);
        const T w = T(w1(dx) * w1(dy) * (DIM == 3 ? w1(dz) : 1.0f));
        TS vv[DIM];
        load_node<DIM, TS>(rf, ((int64_t)kc * f.ny1 + jc) * f.nx1 + ic, vv);
#pragma unroll
        for (int cc = 0; cc < DIM; ++cc) acc[cc] += ok ? w * T(vv[cc]) : T(0);
      }
  store_node<DIM, T>(rc, qc, acc);
}

// Prolongation and correction z += P zc (Sec. 5.1 solution update), one thread
// per fine node.
template <int DIM, typename T>
__global__ __launch_bounds__(BS) void k_prolong(Dims f, Dims c, T* __restrict__ z,
                                                const T* __restrict__ zc, int aug, const int* gate) {
  if (gate && *gate) return;
  const Tile tl = xcd_tile();
  const int i = tl.x * 64 + (threadIdx.x & 63);
  const int j = tl.y * (BS / 64) + (threadIdx.x >> 6);
  const int k = tl.z;
  if (aug && i == 0 && j == 0 && k == 0) z[f.nslots] += zc[c.nslots];
  if (i >= f.nx1 || j >= f.ny1 || i == 0) return;
  const int64_t q = ((int64_t)k * f.ny1 + j) * f.nx1 + i;
  T acc[DIM];
  load_node<DIM, T>(z, q, acc);
  // The 2^dim coarse corners around the node are all loaded (a second corner
  // along an axis where the node is even repeats the first) and the unused ones
  // dropped by a select, so all loads are in flight together.
  const int ni = (i & 1) ? 2 : 1, nj = (j & 1) ? 2 : 1, nk = (DIM == 3 && (k & 1)) ? 2 : 1;
  const T w = T((ni == 2 ? 0.5f : 1.0f) * (nj == 2 ? 0.5f : 1.0f) * (nk == 2 ? 0.5f : 1.0f));
#pragma unroll
  for (int a = 0; a < (DIM == 3 ? 2 : 1); ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const bool use = e < ni && b < nj && a < nk;
        const int I = (i >> 1) + (e < ni ? e : 0), J = (j >> 1) + (b < nj ? b : 0);
        const int K = DIM == 3 ? (k >> 1) + (a < nk ? a : 0) : 0;
        T vv[DIM];
        load_node<DIM, T>(zc, ((int64_t)K * c.ny1 + J) * c.nx1 + I, vv);
#pragma unroll
        for (int cc = 0; cc < DIM; ++cc) acc[cc] += use ? w * vv[cc] : T(0);
      }
  store_node<DIM, T>(z, q, acc);
}

// ------------------------------------------------------------------ Galerkin --
// Coarse element matrices A_C = sum_{fine e in C} W_e' A_e W_e (Sec. 5.1), where
// W_e interpolates the 2^dim coarse corner values of C to the nodes of fine
// element e (each fine node interpolates only from the corners of the coarse
// element containing it, so the sum equals the Galerkin product P' A P).
// One wave per (64 coarse elements, coarse local row R = (A, comp)): the lane is
// the coarse element, R is the same on every lane, so the interpolation weights
// that select the fine rows are uniform and the zero ones are skipped without
// divergence.  For each fine sub-element q of C:
//   t = sum_a W_q[a][A] A_q[(a, comp), :]                (row combination, per Op)
//   row[(B, cb)] += sum_b W_q[b][B] t[(b, cb)]           (weights known at compile time)
// and the packed entries (R, col >= R) are stored, lane-contiguous.  Accumulation
// in FP64, stored as T.  Four waves per block; blocks of one group of coarse
// elements are dealt to one XCD (its L2 holds the group's fine element data).

// 1D hat value of the coarse corner at offset L (0, 1) at fine position p (0, 1, 2).
__host__ __device__ constexpr double hat2(int p, int L) { return p == 2 * L ? 1.0 : (p == 1 ? 0.5 : 0.0); }
template <int DIM>
__host__ __device__ constexpr double sub_weight(int q, int a, int B) {
  return hat2((q & 1) + loc_x(a), loc_x(B)) * hat2(((q >> 1) & 1) + loc_y(a), loc_y(B)) *
         (DIM == 3 ? hat2(((q >> 2) & 1) + loc_z(a), loc_z(B)) : 1.0);
}

// Weight of coarse corner A at local node a of sub-element q (wave-uniform).
template <int DIM>
__device__ inline double row_weight(int q, int a, int A) {
  return hat2((q & 1) + loc_x(a), loc_x(A)) * hat2(((q >> 1) & 1) + loc_y(a), loc_y(A)) *
         (DIM == 3 ? hat2(((q >> 2) & 1) + loc_z(a), loc_z(A)) : 1.0);
}

// t[col] = sum_a W_q[a][A] A_e[(a, comp), col], from the element matrix entries
// (one fine row at a time, its 24 or 8 loads in flight together).
template <int DIM, class Op>
__device__ inline void galerkin_rows(const Op& op, int64_t e, int q, int A, int comp, double* t) {
  constexpr int NN = Geo<DIM>::NN, ND = Geo<DIM>::ND;
#pragma unroll
  for (int col = 0; col < ND; ++col) t[col] = 0.0;
#pragma unroll 1
  for (int a = 0; a < NN; ++a) {
    const double wa = row_weight<DIM>(q, a, A);
    if (wa == 0.0) continue;
    double v[ND];
#pragma unroll
    for (int col = 0; col < ND; ++col) v[col] = op.entry(e, a * DIM + comp, col);
#pragma unroll
    for (int col = 0; col < ND; ++col) t[col] = fma(wa, v[col], t[col]);
  }
}
// A_e = x_e K0: t = x_e (sum_a W_q[a][A] K0[(a, comp), :]).
template <int DIM>
__device__ inline void galerkin_rows(const OpFineK<DIM, double>& op, int64_t e, int q, int A, int comp,
                                     double* t) {
  constexpr int NN = Geo<DIM>::NN, ND = Geo<DIM>::ND;
  const double xe = op.x[e];
  double w[NN];
#pragma unroll
  for (int a = 0; a < NN; ++a) w[a] = row_weight<DIM>(q, a, A);
#pragma unroll
  for (int col = 0; col < ND; ++col) {
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < NN; ++a) s = fma(w[a], k0<double>((a * DIM + comp) * ND + col), s);
    t[col] = xe * s;
  }
}
// A_e = x_e K0 + h_e h_e': t = x_e (sum_a W_q[a][A] K0[(a, comp), :]) + (sum_a W_q[a][A] h_(a, comp)) h_e.
template <int DIM>
__device__ inline void galerkin_rows(const OpFineZ<DIM, double>& op, int64_t e, int q, int A, int comp,
                                     double* t) {
  constexpr int NN = Geo<DIM>::NN, ND = Geo<DIM>::ND;
  const double xe = op.x[e];
  double w[NN], hv[ND];
#pragma unroll
  for (int col = 0; col < ND; ++col) hv[col] = op.h[col * op.m + e];
  double hw = 0.0;
#pragma unroll
  for (int a = 0; a < NN; ++a) {
    w[a] = row_weight<DIM>(q, a, A);
    hw = fma(w[a], op.h[(a * DIM + comp) * op.m + e], hw);
  }
#pragma unroll
  for (int col = 0; col < ND; ++col) {
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < NN; ++a) s = fma(w[a], k0<double>((a * DIM + comp) * ND + col), s);
    t[col] = fma(xe, s, hw * hv[col]);
  }
}

// row[(B, cb)] += sum_b W_Q[b][B] t[(b, cb)], the weights constant after unrolling.
template <int DIM, int Q>
__device__ inline void galerkin_scatter(const double* t, double* row) {
  constexpr int NN = Geo<DIM>::NN;
#pragma unroll
  for (int bb = 0; bb < NN; ++bb)
#pragma unroll
    for (int B = 0; B < NN; ++B) {
      const double wb = sub_weight<DIM>(Q, bb, B);
      if (wb == 0.0) continue;
#pragma unroll
      for (int cb = 0; cb < DIM; ++cb) row[B * DIM + cb] = fma(wb, t[bb * DIM + cb], row[B * DIM + cb]);
    }
}
template <int DIM>
__device__ inline void galerkin_scatter_q(int q, const double* t, double* row) {
  switch (q) {
    case 0: galerkin_scatter<DIM, 0>(t, row); break;
    case 1: galerkin_scatter<DIM, 1>(t, row); break;
    case 2: galerkin_scatter<DIM, 2>(t, row); break;
    case 3: galerkin_scatter<DIM, 3>(t, row); break;
    default:
      if constexpr (DIM == 3) {
        switch (q) {
          case 4: galerkin_scatter<DIM, 4>(t, row); break;
          case 5: galerkin_scatter<DIM, 5>(t, row); break;
          case 6: galerkin_scatter<DIM, 6>(t, row); break;
          default: galerkin_scatter<DIM, 7>(t, row); break;
        }
      }
  }
}

constexpr int GAL_WAVES = 4;
template <int DIM, typename T, class Op>
__global__ __launch_bounds__(64 * GAL_WAVES) void k_galerkin(Op op, Dims f, Dims c, T* __restrict__ Ec) {
  constexpr int NN = Geo<DIM>::NN, ND = Geo<DIM>::ND;
  constexpr int RB = ND / GAL_WAVES;                // blocks per group of 64 coarse elements
  static_assert(ND % GAL_WAVES == 0, "rows split evenly over the waves");
  const unsigned b = xcd_tile().x;
  // the row is the same on every lane of the wave: kept in scalar registers
  const int R = __builtin_amdgcn_readfirstlane((int)(b % RB) * GAL_WAVES + (int)(threadIdx.x >> 6));
  const int64_t C = (int64_t)(b / RB) * 64 + (threadIdx.x & 63);
  if (C >= c.m) return;
  const int CI = (int)(C % c.nx), CJ = (int)((C / c.nx) % c.ny), CK = DIM == 3 ? (int)(C / ((int64_t)c.nx * c.ny)) : 0;
  const int A = R / DIM, comp = R % DIM;
  double row[ND];
#pragma unroll
  for (int col = 0; col < ND; ++col) row[col] = 0.0;
#pragma unroll 1
  for (int q = 0; q < NN; ++q) {
    const int qx = q & 1, qy = (q >> 1) & 1, qz = (q >> 2) & 1;
    const int64_t e = ((int64_t)(2 * CK + qz) * f.ny + (2 * CJ + qy)) * f.nx + (2 * CI + qx);
    double t[ND];
    galerkin_rows<DIM>(op, e, q, A, comp, t);
    galerkin_scatter_q<DIM>(q, t, row);
  }
#pragma unroll
  for (int col = 0; col < ND; ++col)
    if (col >= R) Ec[(int64_t)sym_index(R, col, ND) * c.m + C] = T(row[col]);
}

// G_q = W_q' K0 W_q for the four sub-elements q of a coarse 2D element (one
// thread per entry), W_q the bilinear interpolation from the coarse corners to the
// nodes of sub-element q.
static __global__ void k_galerkin_images2d(const double* __restrict__ K0, double* __restrict__ G) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 256) return;
  const int q = t / 64, r = (t / 8) % 8, cc = t % 8;
  const int qx = q & 1, qy = q >> 1;
  const int A = r / 2, ci = r % 2, B = cc / 2, cj = cc % 2;
  double s = 0.0;
  for (int a = 0; a < 4; ++a) {
    const double wa = (1.0 - fabs(0.5 * (qx + loc_x(a)) - loc_x(A))) * (1.0 - fabs(0.5 * (qy + loc_y(a)) - loc_y(A)));
    if (wa == 0.0) continue;
    for (int b = 0; b < 4; ++b) {
      const double wb = (1.0 - fabs(0.5 * (qx + loc_x(b)) - loc_x(B))) * (1.0 - fabs(0.5 * (qy + loc_y(b)) - loc_y(B)));
      s += wa * K0[(a * 2 + ci) * 8 + b * 2 + cj] * wb;
    }
  }
  G[t] = s;
}

// ---------------------------------------------------------- coarsest solve --
// Dense operator of the coarsest level over all slots (+ lambda) into the packed
// tiles (zeroed, padded), each tile transposed (dense_lowerT_at) and the diagonal
// tiles in full: rows gathered from the element matrices; clamped rows/columns
// replaced by identity.  Thread `row` writes the entries (row, col <= row), their
// mirror images inside a diagonal tile, and for the augmented system entry
// (n-1, row) of the border row; no two threads write one entry.
template <int DIM, class Op, typename TB>
__global__ __launch_bounds__(BS) void k_dense_assemble(Op op, Dims d, const TB* border, double corner,
                                                       int aug, double* __restrict__ A, int n) {
  constexpr int NN = Geo<DIM>::NN;
  const int row = blockIdx.x * BS + threadIdx.x;
  if (row >= n) return;
  if (aug && row == n - 1) {
    A[dense_lowerT_at(row, row)] = corner;
    return;
  }
  const int q = row / DIM, comp = row % DIM;
  const int i = q % d.nx1, j = (q / d.nx1) % d.ny1, k = DIM == 3 ? q / (d.nx1 * d.ny1) : 0;
  if (aug) {
    const double v = i == 0 ? 0.0 : (double)border[row];
    A[dense_lowerT_at(n - 1, row)] = v;
    if ((n - 1) / DT == row / DT) A[dense_lower_at(n - 1, row)] = v;
  }
  if (i == 0) {
    A[dense_lowerT_at(row, row)] = 1.0;
    return;
  }
  for (int qq = 0; qq < NN; ++qq) {
    const int ex = qq & 1, ey = (qq >> 1) & 1, ez = (qq >> 2) & 1;
    const int ei = i - 1 + ex, ej = j - 1 + ey, ek = k - 1 + ez;
    if (ei < 0 || ei >= d.nx || ej < 0 || ej >= d.ny || (DIM == 3 && (ek < 0 || ek >= d.nz))) continue;
    const int64_t e = ((int64_t)(DIM == 3 ? ek : 0) * d.ny + ej) * d.nx + ei;
    const int a = loc_index(1 - ex, 1 - ey, DIM == 3 ? 1 - ez : 0);
    for (int b = 0; b < NN; ++b) {
      const int bi = ei + loc_x(b), bj = ej + loc_y(b), bk = DIM == 3 ? ek + loc_z(b) : 0;
      if (bi == 0) continue;
      const int qb = (bk * d.ny1 + bj) * d.nx1 + bi;
      for (int cb = 0; cb < DIM; ++cb) {
        const int col = qb * DIM + cb;
        if (col > row) continue;
        const double v = op.entry(e, a * DIM + comp, b * DIM + cb);
        A[dense_lowerT_at(row, col)] += v;
        if (col != row && col / DT == row / DT) A[dense_lower_at(row, col)] += v;
      }
    }
  }
}

}  // namespace ipmg

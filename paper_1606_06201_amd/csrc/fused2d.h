// Fused passes of the 2D V-cycle on a coarse level k (stored operators, or the
// first coarse level formed from the densities), for Algorithm MG with two pre-
// and two post-smoothing sweeps of damped Jacobi (Sec. 5.1, Sec. 7):
//   down: z1 = w D^-1 r, z2 = z1 + w D^-1 (r - A z1), t = r - A z2, rc = P' t
//   up:   z = z2 + P zc, z3 = z + w D^-1 (r - A z), out = z3 + w D^-1 (r - A z3)
// Each workgroup computes one tile of the level in LDS together with the halo
// each later step needs (recomputed by neighbouring tiles), so the two launches
// replace seven on levels where a launch costs more than the work.  Arithmetic per
// node is that of k_level (same operator rows, diagonal and reciprocal).
//   k_down2d / k_up2d: stored operators read from global memory (16x8 or 16x9
//     coarse-node and 32x16 or 32x18 fine-node tiles, 1024 threads: every phase is
//     one pass);
//   k_down2d_x / k_up2d_x: the first coarse level formed from the densities, the
//     four densities of every element of the tile staged in LDS first;
//   k_down2d_staged / k_up2d_staged: the FP32 element matrices of the tile's
//     elements copied into LDS first, so the phases wait on LDS only (small stored
//     levels; 8x4 and 16x8 tiles, 512 threads).
#pragma once
#include "kernels.h"

namespace ipmg {

constexpr int FBS = 1024;           // every phase of a tile is one pass of the workgroup
constexpr int SCX = 8, SCY = 4;     // coarse nodes per k_down2d_staged tile
constexpr int STX = 16, STY = 8;    // fine nodes per k_up2d_staged tile
constexpr int SBS_STORED = 512;     // threads of the staged passes: every phase one pass

__device__ inline bool node_free(const Dims& d, int i, int j) { return i >= 1 && i < d.nx1 && j >= 0 && j < d.ny1; }

// Neighbourhood of node (li, lj) of an LDS array of row width W (2 values per node).
template <typename T>
__device__ inline void lds_neighbourhood(const T* s, int W, int li, int lj, T (&vn)[9][2]) {
#pragma unroll
  for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx) {
      const int o = 2 * ((lj + dy) * W + li + dx);
      vn[nb_index<2>(dx, dy, 0)][0] = s[o];
      vn[nb_index<2>(dx, dy, 0)][1] = s[o + 1];
    }
}

// Stored element matrices of a block of elements held in LDS: E[sym * ne + le],
// le = (ej - ey0) * lw + (ei - ex0).  Elements outside the block (which the masked
// element loop of node_apply only produces for elements outside the grid) read a
// clamped local index; their contribution is masked there.
template <typename T>
struct OpCoarseLDS {
  const T* E;
  int ex0, ey0, lw, ne;
  __device__ inline int local(int ei, int ej) const {
    const int le = (ej - ey0) * lw + (ei - ex0);
    return le < 0 ? 0 : (le >= ne ? ne - 1 : le);
  }
  __device__ inline void rows(int64_t, int ei, int ej, int, int a, const T* ve, T* acc) const {
    const int le = local(ei, ej);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int r = a * 2 + c;
      T s = 0;
#pragma unroll
      for (int col = 0; col < 8; ++col) s += E[sym_index(r, col, 8) * ne + le] * ve[col];
      acc[c] += s;
    }
  }
  __device__ inline void diag(int64_t, int ei, int ej, int, int a, T* dg) const {
    const int le = local(ei, ej);
#pragma unroll
    for (int c = 0; c < 2; ++c) dg[c] += E[sym_index(a * 2 + c, a * 2 + c, 8) * ne + le];
  }
};

// Copies the stored matrices of elements [ex0, ex0+LW) x [ey0, ey0+LH) of a level
// into LDS (zero outside the grid), entry k of local element le at k NE + le.
// Thread t takes the elements t, t + NT, ...: their offsets are formed once, and
// entry k of each sits k m further on (a uniform step), so a load needs no index
// arithmetic of its own.  Every thread issues all of its loads before its first
// LDS store, so the copy costs one memory latency: indices are clamped into the
// grid and the (finite) value is multiplied by 0 or 1, since a select on the
// loaded value would be compiled back into a branch around each load.
template <typename T, int NT, int LW, int LH>
__device__ inline void stage_elements(const T* __restrict__ Eg, const Dims& d, int ex0, int ey0, T* El) {
  constexpr int NE = LW * LH, PE = (NE + NT - 1) / NT;
  uint32_t off[PE];
  T keep[PE];
#pragma unroll
  for (int j = 0; j < PE; ++j) {
    const int le = min((int)threadIdx.x + j * NT, NE - 1);
    const int ei = ex0 + le % LW, ej = ey0 + le / LW;
    const bool in = ei >= 0 && ei < d.nx && ej >= 0 && ej < d.ny;
    off[j] = (uint32_t)(min(max(ej, 0), d.ny - 1) * d.nx + min(max(ei, 0), d.nx - 1));
    keep[j] = T(in ? 1 : 0);
  }
  T v[PE][36];
#pragma unroll
  for (int k = 0; k < 36; ++k)
#pragma unroll
    for (int j = 0; j < PE; ++j) v[j][k] = (Eg + k * d.m)[off[j]];
#pragma unroll
  for (int j = 0; j < PE; ++j) {
    const int le = (int)threadIdx.x + j * NT;
    if (le < NE) {
#pragma unroll
      for (int k = 0; k < 36; ++k) El[k * NE + le] = v[j][k] * keep[j];
    }
  }
}

// First coarse level formed from the finest densities, with the four densities of
// each element of a block held in LDS (xl[q * ne + le], le as in OpCoarseLDS; zero
// outside the grid), so the passes read no global memory for the operator.  The
// element matrix sum_q x_q G_q is formed inside each node evaluation, as in
// OpCoarse2K.
template <typename T>
struct OpCoarse2KLDS : OpCoarse2K<2, T> {
  const T* xl;
  int ex0, ey0, lw, ne;
  __device__ inline int local(int ei, int ej) const {
    const int le = (ej - ey0) * lw + (ei - ex0);
    return le < 0 ? 0 : (le >= ne ? ne - 1 : le);
  }
  __device__ inline void xs_or_zero(bool, int ei, int ej, T* xq) const {
    const int le = local(ei, ej);
#pragma unroll
    for (int q = 0; q < 4; ++q) xq[q] = xl[q * ne + le];
  }
};
template <typename T>
struct preloads_x<OpCoarse2KLDS<T>> : std::true_type {};

// The four finest densities of the coarse elements [ex0, ex0+LW) x [ey0, ey0+LH)
// into LDS as OpCoarse2KLDS reads them (outside the grid: the zero pad after the
// densities, fine m = fnx * 2 ny).  One element per thread and pass, all loads
// issued before the first LDS store.
template <typename T, int NT, int LW, int LH>
__device__ inline void stage_x4(const T* __restrict__ x, int fnx, const Dims& d, int ex0, int ey0, T* xl) {
  constexpr int NE = LW * LH, PE = (NE + NT - 1) / NT;
  T v[PE][4];
#pragma unroll
  for (int j = 0; j < PE; ++j) {
    const int le = min((int)threadIdx.x + j * NT, NE - 1);
    const int ei = ex0 + le % LW, ej = ey0 + le / LW;
    const bool in = ei >= 0 && ei < d.nx && ej >= 0 && ej < d.ny;
    const uint32_t b = in ? (uint32_t)(2 * ej) * (uint32_t)fnx + (uint32_t)(2 * ei) : (uint32_t)fnx * 2u * (uint32_t)d.ny;
    v[j][0] = x[b];
    v[j][1] = x[b + 1];
    v[j][2] = x[b + fnx];
    v[j][3] = x[b + fnx + 1];
  }
#pragma unroll
  for (int j = 0; j < PE; ++j) {
    const int le = (int)threadIdx.x + j * NT;
    if (le < NE) {
#pragma unroll
      for (int q = 0; q < 4; ++q) xl[q * NE + le] = v[j][q];
    }
  }
}

// Global operands of the first phase of a down tile (r on region 1) and of the
// first two phases of an up tile (z2 and the coarse corners on region 0, r on
// region 1).  Kernels load them before they stage element data, so all of a
// thread's global loads are in flight together.  A node that is not free reads the
// clamped node (0, j) of its row, where every level vector is zero, so no load sits
// under a branch.
template <typename T, int CX, int CY, int NT>
struct DownLoads {
  static constexpr int W1 = 2 * CX + 5, H1 = 2 * CY + 5, P1 = (W1 * H1 + NT - 1) / NT;
  T r[P1][2];
  __device__ inline void load(const Dims& d, int CI0, int CJ0, const T* __restrict__ rg) {
    const int ox = 2 * CI0 - 3, oy = 2 * CJ0 - 3;
#pragma unroll
    for (int u = 0; u < P1; ++u) {
      const int t = threadIdx.x + u * NT;
      const int gi = ox + t % W1, gj = oy + t / W1;
      const bool fr = t < W1 * H1 && node_free(d, gi, gj);
      load_node<2, T>(rg, (int64_t)min(max(gj, 0), d.ny1 - 1) * d.nx1 + (fr ? gi : 0), r[u]);
    }
  }
  // The first coarse level under the finest: r = P' t formed here from the finest
  // residual t (df its grid) with the weights, masks and summation order of
  // k_restrict, and stored (rout) on the nodes the tile owns, for the up pass.
  __device__ inline void load_restrict(const Dims& d, const Dims& df, int CI0, int CJ0, const T* __restrict__ tf,
                                       T* __restrict__ rout) {
    const int ox = 2 * CI0 - 3, oy = 2 * CJ0 - 3;
#pragma unroll
    for (int u = 0; u < P1; ++u) {
      const int t = threadIdx.x + u * NT;
      const int gi = ox + t % W1, gj = oy + t / W1;
      T vv[9][2];
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const int i = 2 * gi + dx, j = 2 * gj + dy;
          const int ic = min(max(i, 0), df.nx1 - 1), jc = min(max(j, 0), df.ny1 - 1);
          load_node<2, T>(tf, (int64_t)jc * df.nx1 + ic, vv[3 * (dy + 1) + dx + 1]);
        }
      T acc[2] = {T(0), T(0)};
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const int i = 2 * gi + dx, j = 2 * gj + dy;
          const bool ok = gi > 0 && i >= 1 && i < df.nx1 && j >= 0 && j < df.ny1;
          const T w = T(w1(dx) * w1(dy));
#pragma unroll
          for (int c = 0; c < 2; ++c) acc[c] += ok ? w * vv[3 * (dy + 1) + dx + 1][c] : T(0);
        }
      r[u][0] = acc[0];
      r[u][1] = acc[1];
      const bool own = t < W1 * H1 && gi >= 2 * CI0 && gi < 2 * CI0 + 2 * CX && gi < d.nx1 && gj >= 2 * CJ0 &&
                       gj < 2 * CJ0 + 2 * CY && gj < d.ny1;
      if (own) store_node<2, T>(rout, (int64_t)gj * d.nx1 + gi, acc);
    }
  }
};

template <typename T, int TX, int TY, int NT>
struct UpLoads {
  static constexpr int W0 = TX + 4, H0 = TY + 4, W1 = TX + 2, H1 = TY + 2;
  static constexpr int P0 = (W0 * H0 + NT - 1) / NT, P1 = (W1 * H1 + NT - 1) / NT;
  T z[P0][2], c[P0][4][2], r[P1][2];
  // Region 0: z2 at the node and the four coarse corners around it (indices
  // clamped into the grid; a second corner along an axis where the node is even
  // repeats the first).  Region 1: r.
  __device__ inline void load(const Dims& d, const Dims& dc, int I0, int J0, const T* __restrict__ rg,
                              const T* __restrict__ z2, const T* __restrict__ zc) {
#pragma unroll
    for (int u = 0; u < P0; ++u) {
      const int t = threadIdx.x + u * NT;
      const int gi = I0 - 2 + t % W0, gj = J0 - 2 + t / W0;
      const int ci = min(max(gi, 1), d.nx1 - 1), cj = min(max(gj, 0), d.ny1 - 1);
      load_node<2, T>(z2, (int64_t)cj * d.nx1 + ci, z[u]);
      const int i1 = (ci & 1) ? 1 : 0, j1 = (cj & 1) ? 1 : 0;
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int e = 0; e < 2; ++e)
          load_node<2, T>(zc, (int64_t)((cj >> 1) + b * j1) * dc.nx1 + (ci >> 1) + e * i1, c[u][2 * b + e]);
    }
#pragma unroll
    for (int u = 0; u < P1; ++u) {
      const int t = threadIdx.x + u * NT;
      const int gi = I0 - 1 + t % W1, gj = J0 - 1 + t / W1;
      const bool fr = t < W1 * H1 && node_free(d, gi, gj);
      load_node<2, T>(rg, (int64_t)min(max(gj, 0), d.ny1 - 1) * d.nx1 + (fr ? gi : 0), r[u]);
    }
  }
};

// Last phase of a down tile: rc = P' t on the tile's coarse nodes (t in s3, over
// region 3) and z2 (in s2, over region 2) on the fine nodes the tile owns.
template <typename T, int CX, int CY, int NT>
__device__ inline void down_tile_out(const Dims& d, const Dims& dc, int CI0, int CJ0, T* z2out, T* rc, const T* s2,
                                     const T* s3) {
  constexpr int W1 = 2 * CX + 5, W2 = W1 - 2, W3 = W1 - 4;
  const int ox = 2 * CI0 - 3, oy = 2 * CJ0 - 3;
  for (int t = threadIdx.x; t < CX * CY; t += NT) {     // rc = P' t on the tile's coarse nodes
    const int I = CI0 + t % CX, J = CJ0 + t / CX;
    if (I >= dc.nx1 || J >= dc.ny1) continue;
    T acc[2] = {T(0), T(0)};
    if (I > 0) {
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const int li = 2 * (I - CI0) + 1 + dx, lj = 2 * (J - CJ0) + 1 + dy;   // position in region 3
          const T w = T(w1(dx) * w1(dy));
          acc[0] += w * s3[2 * (lj * W3 + li)];
          acc[1] += w * s3[2 * (lj * W3 + li) + 1];
        }
    }
    store_node<2, T>(rc, (int64_t)J * dc.nx1 + I, acc);
  }
  for (int t = threadIdx.x; t < 4 * CX * CY; t += NT) {   // z2 on the fine nodes the tile owns
    const int gi = 2 * CI0 + t % (2 * CX), gj = 2 * CJ0 + t / (2 * CX);
    if (gi >= d.nx1 || gj >= d.ny1) continue;
    const int q = 2 * ((gj - oy - 1) * W2 + gi - ox - 1);
    const T o[2] = {s2[q], s2[q + 1]};
    store_node<2, T>(z2out, (int64_t)gj * d.nx1 + gi, o);
  }
}

// Down pass of one tile of CX x CY coarse nodes with corner (CI0, CJ0).  LDS:
// sr, sd, s1 over region 1 ((2CX+5) x (2CY+5) fine nodes from (2CI0-3, 2CJ0-3)),
// s2 over region 2 (one node inside), s3 over region 3 (two nodes inside).
template <typename T, class Op, int CX, int CY, int NT>
__device__ inline void down_tile(const Op& op, const Dims& d, const Dims& dc, int CI0, int CJ0,
                                 const DownLoads<T, CX, CY, NT>& pre, T* z2out, T* rc, T omega, T* sr, T* sd,
                                 T* s1, T* s2, T* s3) {
  constexpr int W1 = 2 * CX + 5, H1 = 2 * CY + 5;
  constexpr int W2 = W1 - 2, H2 = H1 - 2;
  constexpr int W3 = W1 - 4, H3 = H1 - 4;
  const int ox = 2 * CI0 - 3, oy = 2 * CJ0 - 3;
#pragma unroll
  for (int u = 0; u < DownLoads<T, CX, CY, NT>::P1; ++u) {
    const int t = threadIdx.x + u * NT;
    if (t >= W1 * H1) break;
    const int gi = ox + t % W1, gj = oy + t / W1;
    T rr[2] = {T(0), T(0)}, dg[2] = {T(0), T(0)}, o[2] = {T(0), T(0)};
    if (node_free(d, gi, gj)) {
      rr[0] = pre.r[u][0];
      rr[1] = pre.r[u][1];
      T vn[9][2], acc[2] = {T(0), T(0)};
      node_apply<2, T, Op, false, true, false>(op, d, gi, gj, 0, vn, acc, dg);
#pragma unroll
      for (int c = 0; c < 2; ++c) o[c] = omega * rr[c] * recip(dg[c]);
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) { sr[2 * t + c] = rr[c]; sd[2 * t + c] = dg[c]; s1[2 * t + c] = o[c]; }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < W2 * H2; t += NT) {
    const int li = t % W2 + 1, lj = t / W2 + 1;        // position in region 1
    const int gi = ox + li, gj = oy + lj;
    T o[2] = {T(0), T(0)};
    if (node_free(d, gi, gj)) {
      T vn[9][2], acc[2] = {T(0), T(0)}, dg[2];
      lds_neighbourhood<T>(s1, W1, li, lj, vn);
      node_apply<2, T, Op, true, false, false>(op, d, gi, gj, 0, vn, acc, dg);
      const int q = 2 * (lj * W1 + li);
#pragma unroll
      for (int c = 0; c < 2; ++c) o[c] = s1[q + c] + omega * (sr[q + c] - acc[c]) * recip(sd[q + c]);
    }
    s2[2 * t] = o[0];
    s2[2 * t + 1] = o[1];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < W3 * H3; t += NT) {
    const int li = t % W3 + 1, lj = t / W3 + 1;        // position in region 2
    const int gi = ox + 1 + li, gj = oy + 1 + lj;
    T o[2] = {T(0), T(0)};
    if (node_free(d, gi, gj)) {
      T vn[9][2], acc[2] = {T(0), T(0)}, dg[2];
      lds_neighbourhood<T>(s2, W2, li, lj, vn);
      node_apply<2, T, Op, true, false, false>(op, d, gi, gj, 0, vn, acc, dg);
      const int q = 2 * ((lj + 1) * W1 + li + 1);
#pragma unroll
      for (int c = 0; c < 2; ++c) o[c] = sr[q + c] - acc[c];
    }
    s3[2 * t] = o[0];
    s3[2 * t + 1] = o[1];
  }
  __syncthreads();
  down_tile_out<T, CX, CY, NT>(d, dc, CI0, CJ0, z2out, rc, s2, s3);
}

// Up pass of one tile of TX x TY fine nodes with corner (I0, J0).  LDS: s0 over
// region 0 ((TX+4) x (TY+4) nodes from (I0-2, J0-2)); sr, sd, s1 over region 1
// (one node inside).
// First phase of an up tile: s0 = z2 + P zc over region 0 (zero on nodes that are
// not free).
template <typename T, int TX, int TY, int NT>
__device__ inline void up_tile_prolong(const Dims& d, int I0, int J0, const UpLoads<T, TX, TY, NT>& pre, T* s0) {
  constexpr int W0 = TX + 4, H0 = TY + 4;
#pragma unroll
  for (int u = 0; u < UpLoads<T, TX, TY, NT>::P0; ++u) {
    const int t = threadIdx.x + u * NT;
    if (t >= W0 * H0) break;
    const int gi = I0 - 2 + t % W0, gj = J0 - 2 + t / W0;
    // z2 + P zc at free nodes (operands from UpLoads; the select drops the corners
    // an even coordinate does not use)
    const bool fr = node_free(d, gi, gj);
    const int ci = min(max(gi, 1), d.nx1 - 1), cj = min(max(gj, 0), d.ny1 - 1);
    T o[2] = {pre.z[u][0], pre.z[u][1]};
    const int ni = (ci & 1) ? 2 : 1, nj = (cj & 1) ? 2 : 1;
    const T w = T((ni == 2 ? 0.5f : 1.0f) * (nj == 2 ? 0.5f : 1.0f));
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const bool use = e < ni && b < nj;
        o[0] += use ? w * pre.c[u][2 * b + e][0] : T(0);
        o[1] += use ? w * pre.c[u][2 * b + e][1] : T(0);
      }
    s0[2 * t] = fr ? o[0] : T(0);
    s0[2 * t + 1] = fr ? o[1] : T(0);
  }
}

template <typename T, class Op, int TX, int TY, int NT>
__device__ inline void up_tile(const Op& op, const Dims& d, const Dims& dc, int I0, int J0,
                               const UpLoads<T, TX, TY, NT>& pre, T* out, T omega, T* s0, T* sr, T* sd, T* s1) {
  constexpr int W0 = TX + 4;
  constexpr int W1 = TX + 2, H1 = TY + 2;
  up_tile_prolong<T, TX, TY, NT>(d, I0, J0, pre, s0);
  __syncthreads();
#pragma unroll
  for (int u = 0; u < UpLoads<T, TX, TY, NT>::P1; ++u) {
    const int t = threadIdx.x + u * NT;
    if (t >= W1 * H1) break;
    const int li = t % W1, lj = t / W1;                 // position in region 1
    const int gi = I0 - 1 + li, gj = J0 - 1 + lj;
    T rr[2] = {T(0), T(0)}, dg[2] = {T(0), T(0)}, o[2] = {T(0), T(0)};
    if (node_free(d, gi, gj)) {
      rr[0] = pre.r[u][0];
      rr[1] = pre.r[u][1];
      T vn[9][2], acc[2] = {T(0), T(0)};
      lds_neighbourhood<T>(s0, W0, li + 1, lj + 1, vn);
      node_apply<2, T, Op, true, true, false>(op, d, gi, gj, 0, vn, acc, dg);
      const int q = 2 * ((lj + 1) * W0 + li + 1);
#pragma unroll
      for (int c = 0; c < 2; ++c) o[c] = s0[q + c] + omega * (rr[c] - acc[c]) * recip(dg[c]);
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) { sr[2 * t + c] = rr[c]; sd[2 * t + c] = dg[c]; s1[2 * t + c] = o[c]; }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < TX * TY; t += NT) {
    const int gi = I0 + t % TX, gj = J0 + t / TX;
    if (gi >= d.nx1 || gj >= d.ny1) continue;
    T o[2] = {T(0), T(0)};
    if (gi >= 1) {
      const int li = gi - I0 + 1, lj = gj - J0 + 1;     // position in region 1
      T vn[9][2], acc[2] = {T(0), T(0)}, dg[2];
      lds_neighbourhood<T>(s1, W1, li, lj, vn);
      node_apply<2, T, Op, true, false, false>(op, d, gi, gj, 0, vn, acc, dg);
      const int q = 2 * (lj * W1 + li);
#pragma unroll
      for (int c = 0; c < 2; ++c) o[c] = s1[q + c] + omega * (sr[q + c] - acc[c]) * recip(sd[q + c]);
    }
    store_node<2, T>(out, (int64_t)gj * d.nx1 + gi, o);
  }
}

// Grid: (ceil(dc.nx1 / CX), ceil(dc.ny1 / CY)); d is level k, dc level k-1.
template <typename T, class Op, int CX, int CY>
__global__ __launch_bounds__(FBS) void k_down2d(Op op, Dims d, Dims dc, const T* __restrict__ r,
                                                T* __restrict__ z2out, T* __restrict__ rc,
                                                const double* __restrict__ omg, const int* gate) {
  if (gate && *gate) return;
  constexpr int W1 = 2 * CX + 5, H1 = 2 * CY + 5, W2 = W1 - 2, H2 = H1 - 2, W3 = W1 - 4, H3 = H1 - 4;
  __shared__ T sr[H1 * W1 * 2], sd[H1 * W1 * 2], s1[H1 * W1 * 2], s2[H2 * W2 * 2], s3[H3 * W3 * 2];
  const Tile tl = xcd_tile();
  DownLoads<T, CX, CY, FBS> pre;
  pre.load(d, (int)tl.x * CX, (int)tl.y * CY, r);
  down_tile<T, Op, CX, CY, FBS>(op, d, dc, (int)tl.x * CX, (int)tl.y * CY, pre, z2out, rc, T(*omg), sr, sd, s1,
                                s2, s3);
}

// Grid: (ceil(d.nx1 / TX), ceil(d.ny1 / TY)).
template <typename T, class Op, int TX, int TY>
__global__ __launch_bounds__(FBS) void k_up2d(Op op, Dims d, Dims dc, const T* __restrict__ r,
                                              const T* __restrict__ z2, const T* __restrict__ zc,
                                              T* __restrict__ out, const double* __restrict__ omg,
                                              const int* gate) {
  if (gate && *gate) return;
  constexpr int W0 = TX + 4, H0 = TY + 4, W1 = TX + 2, H1 = TY + 2;
  __shared__ T s0[H0 * W0 * 2], sr[H1 * W1 * 2], sd[H1 * W1 * 2], s1[H1 * W1 * 2];
  const Tile tl = xcd_tile();
  UpLoads<T, TX, TY, FBS> pre;
  pre.load(d, dc, (int)tl.x * TX, (int)tl.y * TY, r, z2, zc);
  up_tile<T, Op, TX, TY, FBS>(op, d, dc, (int)tl.x * TX, (int)tl.y * TY, pre, out, T(*omg), s0, sr, sd, s1);
}

// k_down2d / k_up2d on the first coarse level formed from the densities, with the
// tile's densities staged in LDS first (OpCoarse2KLDS).  x: finest densities with
// their zero pad, fnx finest elements along x.
template <typename T, bool FROM_T, int CX, int CY>
__global__ __launch_bounds__(FBS) void k_down2d_x(const T* __restrict__ x, int fnx, Dims d, Dims dc,
                                                  const T* __restrict__ r, T* __restrict__ z2out, T* __restrict__ rc,
                                                  const double* __restrict__ omg, const int* gate, Dims df,
                                                  const T* __restrict__ tf, T* __restrict__ rw) {
  if (gate && *gate) return;
  constexpr int W1 = 2 * CX + 5, H1 = 2 * CY + 5, W2 = W1 - 2, H2 = H1 - 2, W3 = W1 - 4, H3 = H1 - 4;
  constexpr int LW = W1 + 1, LH = H1 + 1;
  __shared__ T xl[4 * LW * LH];
  __shared__ T sr[H1 * W1 * 2], sd[H1 * W1 * 2], s1[H1 * W1 * 2], s2[H2 * W2 * 2], s3[H3 * W3 * 2];
  const Tile tl = xcd_tile();
  const int CI0 = (int)tl.x * CX, CJ0 = (int)tl.y * CY;
  const int ex0 = 2 * CI0 - 4, ey0 = 2 * CJ0 - 4;
  DownLoads<T, CX, CY, FBS> pre;
  if constexpr (FROM_T) pre.load_restrict(d, df, CI0, CJ0, tf, rw);
  else pre.load(d, CI0, CJ0, r);
  stage_x4<T, FBS, LW, LH>(x, fnx, d, ex0, ey0, xl);
  __syncthreads();
  OpCoarse2KLDS<T> op;
  op.xl = xl;
  op.ex0 = ex0;
  op.ey0 = ey0;
  op.lw = LW;
  op.ne = LW * LH;
  down_tile<T, OpCoarse2KLDS<T>, CX, CY, FBS>(op, d, dc, CI0, CJ0, pre, z2out, rc, T(*omg), sr, sd, s1, s2, s3);
}

template <typename T, int TX, int TY>
__global__ __launch_bounds__(FBS) void k_up2d_x(const T* __restrict__ x, int fnx, Dims d, Dims dc,
                                                const T* __restrict__ r, const T* __restrict__ z2,
                                                const T* __restrict__ zc, T* __restrict__ out,
                                                const double* __restrict__ omg, const int* gate) {
  if (gate && *gate) return;
  constexpr int W0 = TX + 4, H0 = TY + 4, W1 = TX + 2, H1 = TY + 2;
  constexpr int LW = W1 + 1, LH = H1 + 1;
  __shared__ T xl[4 * LW * LH];
  __shared__ T s0[H0 * W0 * 2], sr[H1 * W1 * 2], sd[H1 * W1 * 2], s1[H1 * W1 * 2];
  const Tile tl = xcd_tile();
  const int I0 = (int)tl.x * TX, J0 = (int)tl.y * TY;
  const int ex0 = I0 - 2, ey0 = J0 - 2;
  UpLoads<T, TX, TY, FBS> pre;
  pre.load(d, dc, I0, J0, r, z2, zc);
  stage_x4<T, FBS, LW, LH>(x, fnx, d, ex0, ey0, xl);
  __syncthreads();
  OpCoarse2KLDS<T> op;
  op.xl = xl;
  op.ex0 = ex0;
  op.ey0 = ey0;
  op.lw = LW;
  op.ne = LW * LH;
  up_tile<T, OpCoarse2KLDS<T>, TX, TY, FBS>(op, d, dc, I0, J0, pre, out, T(*omg), s0, sr, sd, s1);
}

// ------------------------------------------------------------ matrix cores --
// The first coarse level's element products on the matrix cores.  For a group of
// 32 elements, U = [G_0; G_1; G_2; G_3] V (32 x 8 times 8 x 32, four
// v_mfma_f32_32x32x2f32 steps of K = 2), V the elements' vertex values as columns;
// then y_e = sum_q x_q U_q[:, e] (the x-weighted sum of each element's four 8-row
// blocks), and the node passes gather y_e of the four elements around each node.
// Lane layout of the 32x32x2 product: lane l supplies A[l % 32][2s + l / 32] and
// B[2s + l / 32][l % 32] at step s and receives D[8 (v / 4) + 4 (l / 32) + v % 4]
// [l % 32] in result register v, so each lane holds rows 4 h .. 4 h + 3 (h = l / 32)
// of all four blocks of its element.
static __constant__ float cG256f[256];   // G_q[r][k] at 64 q + 8 r + k (q-major stack)
typedef float mfma_f32x16 __attribute__((ext_vector_type(16)));

// This lane's A operands of the four K steps (row l % 32 of the stack).
__device__ inline void gstack_operands(float (&aG)[4]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < 4; ++s) aG[s] = cG256f[(lane & 31) * 8 + 2 * s + (lane >> 5)];
}

// Element products in LDS as four vertex planes: plane a holds rows 2a and 2a + 1
// of every element's product as a float pair at 2 t (t the element's index in its
// block), so a node's gather and a half-wave's store both touch consecutive pairs.
// The plane pitch is a multiple of 32 floats plus 16, which puts the planes the two
// half-waves store to on different banks.
__host__ __device__ constexpr int ye_pitch(int ne) { return ((2 * ne + 31) / 32) * 32 + 16; }

// y_e for the NEX x NEY elements of a block: element (ex, ey) has vertex b at node
// (ex + loc_x(b), ey + loc_y(b)) of sv (row width WV, two values per node) and the
// four densities of staged element (ex + ELX, ey + ELY) of xl (row width LW, LH
// rows, as OpCoarse2KLDS).  Writes the vertex planes of ye (pitch ye_pitch(NE)),
// t = ey NEX + ex.  The waves of the workgroup take the groups of 32 elements in
// turn.
template <int NEX, int NEY, int WV, int LW, int LH, int ELX, int ELY, int NT>
__device__ inline void elem_products_mfma(const float* sv, const float* xl, const float (&aG)[4], float* ye) {
  constexpr int NE = NEX * NEY, NG = (NE + 31) / 32, NW = NT / 64, NEL = LW * LH, YP = ye_pitch(NE);
  const int lane = threadIdx.x & 63, h = lane >> 5;
  for (int g = (int)threadIdx.x >> 6; g < NG; g += NW) {
    const int t0 = g * 32 + (lane & 31), t = min(t0, NE - 1);
    const int ex = t % NEX, ey = t / NEX;
    float b[4], xq[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) b[s] = sv[2 * ((ey + loc_y(s)) * WV + ex + loc_x(s)) + h];
    const int le = (ey + ELY) * LW + ex + ELX;
#pragma unroll
    for (int q = 0; q < 4; ++q) xq[q] = xl[q * NEL + le];
    mfma_f32x16 acc = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f,
                       0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(aG[s], b[s], acc, 0, 0, 0);
    float2 y0, y1;                                   // rows 4h, 4h+1 (vertex 2h) and 4h+2, 4h+3
    y0.x = xq[0] * acc[0] + xq[1] * acc[4] + xq[2] * acc[8] + xq[3] * acc[12];
    y0.y = xq[0] * acc[1] + xq[1] * acc[5] + xq[2] * acc[9] + xq[3] * acc[13];
    y1.x = xq[0] * acc[2] + xq[1] * acc[6] + xq[2] * acc[10] + xq[3] * acc[14];
    y1.y = xq[0] * acc[3] + xq[1] * acc[7] + xq[2] * acc[11] + xq[3] * acc[15];
    if (t0 < NE) {
      *reinterpret_cast<float2*>(ye + 2 * h * YP + 2 * t) = y0;
      *reinterpret_cast<float2*>(ye + (2 * h + 1) * YP + 2 * t) = y1;
    }
  }
}

// Row sums of node (li, lj) from the products of the four elements around it:
// element (li - 1 + ex + OX, lj - 1 + ey + OY) of a block of NEX x NEY elements, the
// node its vertex loc_index(1 - ex, 1 - ey).
template <int NEX, int NEY, int OX, int OY>
__device__ inline void gather_rows(const float* ye, int li, int lj, float (&acc)[2]) {
  constexpr int YP = ye_pitch(NEX * NEY);
  acc[0] = acc[1] = 0.0f;
#pragma unroll
  for (int ey = 0; ey < 2; ++ey)
#pragma unroll
    for (int ex = 0; ex < 2; ++ex) {
      const int t = (lj - 1 + ey + OY) * NEX + li - 1 + ex + OX;
      const int a = loc_index(1 - ex, 1 - ey, 0);
      const float2 v = *reinterpret_cast<const float2*>(ye + a * YP + 2 * t);
      acc[0] += v.x;
      acc[1] += v.y;
    }
}

// k_down2d_x with the operator applications of its second and third phases on the
// matrix cores (FP32).  Regions and outputs as in down_tile.
template <bool FROM_T, int CX, int CY>
__global__ __launch_bounds__(FBS) void k_down2d_m(const float* __restrict__ x, int fnx, Dims d, Dims dc,
                                                  const float* __restrict__ r, float* __restrict__ z2out,
                                                  float* __restrict__ rc, const double* __restrict__ omg,
                                                  const int* gate, Dims df, const float* __restrict__ tf,
                                                  float* __restrict__ rw) {
  if (gate && *gate) return;
  constexpr int W1 = 2 * CX + 5, H1 = 2 * CY + 5, W2 = W1 - 2, H2 = H1 - 2, W3 = W1 - 4, H3 = H1 - 4;
  constexpr int LW = W1 + 1, LH = H1 + 1;
  constexpr int NEX2 = W1 - 1, NEY2 = H1 - 1, NEX3 = W1 - 3, NEY3 = H1 - 3;   // element blocks of phases 2, 3
  __shared__ float xl[4 * LW * LH];
  __shared__ float sr[H1 * W1 * 2], sd[H1 * W1 * 2], s1[H1 * W1 * 2], s2[H2 * W2 * 2], s3[H3 * W3 * 2];
  __shared__ __align__(16) float ye[4 * ye_pitch(NEX2 * NEY2)];
  const Tile tl = xcd_tile();
  const int CI0 = (int)tl.x * CX, CJ0 = (int)tl.y * CY;
  const int ox = 2 * CI0 - 3, oy = 2 * CJ0 - 3;
  const int ex0 = ox - 1, ey0 = oy - 1;
  DownLoads<float, CX, CY, FBS> pre;
  if constexpr (FROM_T) pre.load_restrict(d, df, CI0, CJ0, tf, rw);
  else pre.load(d, CI0, CJ0, r);
  stage_x4<float, FBS, LW, LH>(x, fnx, d, ex0, ey0, xl);
  float aG[4];
  gstack_operands(aG);
  __syncthreads();
  OpCoarse2KLDS<float> op;
  op.xl = xl;
  op.ex0 = ex0;
  op.ey0 = ey0;
  op.lw = LW;
  op.ne = LW * LH;
  const float omega = (float)*omg;
  // phase 1: z1 = w D^-1 r on region 1
#pragma unroll
  for (int u = 0; u < DownLoads<float, CX, CY, FBS>::P1; ++u) {
    const int t = threadIdx.x + u * FBS;
    if (t >= W1 * H1) break;
    const int gi = ox + t % W1, gj = oy + t / W1;
    float rr[2] = {0.0f, 0.0f}, dg[2] = {0.0f, 0.0f}, o[2] = {0.0f, 0.0f};
    if (node_free(d, gi, gj)) {
      rr[0] = pre.r[u][0];
      rr[1] = pre.r[u][1];
      float vn[9][2], acc[2] = {0.0f, 0.0f};
      node_apply<2, float, OpCoarse2KLDS<float>, false, true, false>(op, d, gi, gj, 0, vn, acc, dg);
#pragma unroll
      for (int c = 0; c < 2; ++c) o[c] = omega * rr[c] * recip(dg[c]);
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) { sr[2 * t + c] = rr[c]; sd[2 * t + c] = dg[c]; s1[2 * t + c] = o[c]; }
  }
  __syncthreads();
  // phase 2: z2 = z1 + w D^-1 (r - A z1) on region 2
  elem_products_mfma<NEX2, NEY2, W1, LW, LH, 1, 1, FBS>(s1, xl, aG, ye);
  __syncthreads();
  for (int t = threadIdx.x; t < W2 * H2; t += FBS) {
    const int li = t % W2 + 1, lj = t / W2 + 1;        // position in region 1
    const int gi = ox + li, gj = oy + lj;
    float o[2] = {0.0f, 0.0f};
    if (node_free(d, gi, gj)) {
      float acc[2];
      gather_rows<NEX2, NEY2, 0, 0>(ye, li, lj, acc);
      const int q = 2 * (lj * W1 + li);
#pragma unroll
      for (int c = 0; c < 2; ++c) o[c] = s1[q + c] + omega * (sr[q + c] - acc[c]) * recip(sd[q + c]);
    }
    s2[2 * t] = o[0];
    s2[2 * t + 1] = o[1];
  }
  __syncthreads();
  // phase 3: t = r - A z2 on region 3 (elements with lower-left node 1 .. W1-3 of region 1)
  elem_products_mfma<NEX3, NEY3, W2, LW, LH, 2, 2, FBS>(s2, xl, aG, ye);
  __syncthreads();
  for (int t = threadIdx.x; t < W3 * H3; t += FBS) {
    const int li = t % W3 + 2, lj = t / W3 + 2;        // position in region 1
    const int gi = ox + li, gj = oy + lj;
    float o[2] = {0.0f, 0.0f};
    if (node_free(d, gi, gj)) {
      float acc[2];
      gather_rows<NEX3, NEY3, -1, -1>(ye, li, lj, acc);
      const int q = 2 * (lj * W1 + li);
#pragma unroll
      for (int c = 0; c < 2; ++c) o[c] = sr[q + c] - acc[c];
    }
    s3[2 * t] = o[0];
    s3[2 * t + 1] = o[1];
  }
  __syncthreads();
  down_tile_out<float, CX, CY, FBS>(d, dc, CI0, CJ0, z2out, rc, s2, s3);
}

// k_up2d_x with the operator applications of its two sweeps on the matrix cores
// (FP32).  Regions and output as in up_tile.
template <int TX, int TY>
__global__ __launch_bounds__(FBS) void k_up2d_m(const float* __restrict__ x, int fnx, Dims d, Dims dc,
                                                const float* __restrict__ r, const float* __restrict__ z2,
                                                const float* __restrict__ zc, float* __restrict__ out,
                                                const double* __restrict__ omg, const int* gate) {
  if (gate && *gate) return;
  constexpr int W0 = TX + 4, H0 = TY + 4, W1 = TX + 2, H1 = TY + 2;
  constexpr int LW = W1 + 1, LH = H1 + 1;
  constexpr int NEXA = W1 + 1, NEYA = H1 + 1, NEXB = W1 - 1, NEYB = H1 - 1;   // element blocks of the sweeps
  __shared__ float xl[4 * LW * LH];
  __shared__ float s0[H0 * W0 * 2], sr[H1 * W1 * 2], sd[H1 * W1 * 2], s1[H1 * W1 * 2];
  __shared__ __align__(16) float ye[4 * ye_pitch(NEXA * NEYA)];
  const Tile tl = xcd_tile();
  const int I0 = (int)tl.x * TX, J0 = (int)tl.y * TY;
  const int ex0 = I0 - 2, ey0 = J0 - 2;
  UpLoads<float, TX, TY, FBS> pre;
  pre.load(d, dc, I0, J0, r, z2, zc);
  stage_x4<float, FBS, LW, LH>(x, fnx, d, ex0, ey0, xl);
  float aG[4];
  gstack_operands(aG);
  OpCoarse2KLDS<float> op;
  op.xl = xl;
  op.ex0 = ex0;
  op.ey0 = ey0;
  op.lw = LW;
  op.ne = LW * LH;
  const float omega = (float)*omg;
  up_tile_prolong<float, TX, TY, FBS>(d, I0, J0, pre, s0);
  __syncthreads();
  // first sweep on region 1: elements with lower-left node 0 .. W1 of region 0
  elem_products_mfma<NEXA, NEYA, W0, LW, LH, 0, 0, FBS>(s0, xl, aG, ye);
  __syncthreads();
#pragma unroll
  for (int u = 0; u < UpLoads<float, TX, TY, FBS>::P1; ++u) {
    const int t = threadIdx.x + u * FBS;
    if (t >= W1 * H1) break;
    const int li = t % W1, lj = t / W1;                 // position in region 1
    const int gi = I0 - 1 + li, gj = J0 - 1 + lj;
    float rr[2] = {0.0f, 0.0f}, dg[2] = {0.0f, 0.0f}, o[2] = {0.0f, 0.0f};
    if (node_free(d, gi, gj)) {
      rr[0] = pre.r[u][0];
      rr[1] = pre.r[u][1];
      float vn[9][2], acc[2];
      node_apply<2, float, OpCoarse2KLDS<float>, false, true, false>(op, d, gi, gj, 0, vn, acc, dg);
      gather_rows<NEXA, NEYA, 1, 1>(ye, li, lj, acc);
      const int q = 2 * ((lj + 1) * W0 + li + 1);
#pragma unroll
      for (int c = 0; c < 2; ++c) o[c] = s0[q + c] + omega * (rr[c] - acc[c]) * recip(dg[c]);
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) { sr[2 * t + c] = rr[c]; sd[2 * t + c] = dg[c]; s1[2 * t + c] = o[c]; }
  }
  __syncthreads();
  // second sweep on the tile: elements with lower-left node 0 .. TX of region 1
  elem_products_mfma<NEXB, NEYB, W1, LW, LH, 1, 1, FBS>(s1, xl, aG, ye);
  __syncthreads();
  for (int t = threadIdx.x; t < TX * TY; t += FBS) {
    const int gi = I0 + t % TX, gj = J0 + t / TX;
    if (gi >= d.nx1 || gj >= d.ny1) continue;
    float o[2] = {0.0f, 0.0f};
    if (gi >= 1) {
      const int li = gi - I0 + 1, lj = gj - J0 + 1;     // position in region 1
      float acc[2];
      gather_rows<NEXB, NEYB, 0, 0>(ye, li, lj, acc);
      const int q = 2 * (lj * W1 + li);
#pragma unroll
      for (int c = 0; c < 2; ++c) o[c] = s1[q + c] + omega * (sr[q + c] - acc[c]) * recip(sd[q + c]);
    }
    store_node<2, float>(out, (int64_t)gj * d.nx1 + gi, o);
  }
}

// Stored FP32 element matrices staged in LDS, tiles of CX x CY coarse nodes and NT
// threads.  Grid: (ceil(dc.nx1 / CX), ceil(dc.ny1 / CY)).  Region 1 of a tile has
// nodes (2CI0-3 .. 2CI0+2CX+1); the elements around them are
// (2CI0-4 .. 2CI0+2CX+1) x (2CJ0-4 .. 2CJ0+2CY+1).
template <int CX, int CY, int NT>
__global__ __launch_bounds__(NT) void k_down2d_staged(const float* __restrict__ Eg, Dims d, Dims dc,
                                                      const float* __restrict__ r, float* __restrict__ z2out,
                                                      float* __restrict__ rc, const double* __restrict__ omg,
                                                      const int* gate) {
  if (gate && *gate) return;
  constexpr int W1 = 2 * CX + 5, H1 = 2 * CY + 5, W2 = W1 - 2, H2 = H1 - 2, W3 = W1 - 4, H3 = H1 - 4;
  constexpr int LW = W1 + 1, LH = H1 + 1;
  __shared__ float El[36 * LW * LH];
  __shared__ float sr[H1 * W1 * 2], sd[H1 * W1 * 2], s1[H1 * W1 * 2], s2[H2 * W2 * 2], s3[H3 * W3 * 2];
  const Tile tl = xcd_tile();
  const int CI0 = (int)tl.x * CX, CJ0 = (int)tl.y * CY;
  const int ex0 = 2 * CI0 - 4, ey0 = 2 * CJ0 - 4;
  DownLoads<float, CX, CY, NT> pre;
  pre.load(d, CI0, CJ0, r);
  stage_elements<float, NT, LW, LH>(Eg, d, ex0, ey0, El);
  __syncthreads();
  const OpCoarseLDS<float> op{El, ex0, ey0, LW, LW * LH};
  down_tile<float, OpCoarseLDS<float>, CX, CY, NT>(op, d, dc, CI0, CJ0, pre, z2out, rc, float(*omg), sr, sd, s1, s2,
                                                   s3);
}

// Tiles of TX x TY fine nodes and NT threads.  Grid: (ceil(d.nx1 / TX),
// ceil(d.ny1 / TY)).  Region 1 has nodes (I0-1 .. I0+TX); the elements around them
// are (I0-2 .. I0+TX) x (J0-2 .. J0+TY).
template <int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void k_up2d_staged(const float* __restrict__ Eg, Dims d, Dims dc,
                                                    const float* __restrict__ r, const float* __restrict__ z2,
                                                    const float* __restrict__ zc, float* __restrict__ out,
                                                    const double* __restrict__ omg, const int* gate) {
  if (gate && *gate) return;
  constexpr int W0 = TX + 4, H0 = TY + 4, W1 = TX + 2, H1 = TY + 2;
  constexpr int LW = W1 + 1, LH = H1 + 1;
  __shared__ float El[36 * LW * LH];
  __shared__ float s0[H0 * W0 * 2], sr[H1 * W1 * 2], sd[H1 * W1 * 2], s1[H1 * W1 * 2];
  const Tile tl = xcd_tile();
  const int I0 = (int)tl.x * TX, J0 = (int)tl.y * TY;
  const int ex0 = I0 - 2, ey0 = J0 - 2;
  UpLoads<float, TX, TY, NT> pre;
  pre.load(d, dc, I0, J0, r, z2, zc);
  stage_elements<float, NT, LW, LH>(Eg, d, ex0, ey0, El);
  __syncthreads();
  const OpCoarseLDS<float> op{El, ex0, ey0, LW, LW * LH};
  up_tile<float, OpCoarseLDS<float>, TX, TY, NT>(op, d, dc, I0, J0, pre, out, float(*omg), s0, sr, sd, s1);
}

}  // namespace ipmg

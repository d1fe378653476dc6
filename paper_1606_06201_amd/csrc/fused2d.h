// Fused passes of the 2D V-cycle on a coarse level k (stored operators, or the
// first coarse level formed from the densities), for
// Algorithm MG with two pre- and two post-smoothing sweeps of damped Jacobi
// (Sec. 5.1, Sec. 7):
//   k_down2d: z1 = w D^-1 r, z2 = z1 + w D^-1 (r - A z1), t = r - A z2, rc = P' t
//   k_up2d:   z = z2 + P zc, z3 = z + w D^-1 (r - A z), out = z3 + w D^-1 (r - A z3)
// Each workgroup computes one tile of the level in LDS together with the halo
// each later step needs (recomputed by neighbouring tiles), so the two launches
// replace seven on levels where a launch costs more than the work.  Arithmetic per
// node is that of k_level (same operator rows, diagonal and reciprocal).
#pragma once
#include "kernels.h"

namespace ipmg {

constexpr int FCX = 16, FCY = 8;    // coarse nodes per k_down2d tile
constexpr int FTX = 32, FTY = 16;   // fine nodes per k_up2d tile
constexpr int FBS = 1024;   // every phase of a tile is one pass of the workgroup

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

// Grid: (ceil(dc.nx1 / FCX), ceil(dc.ny1 / FCY)); d is level k, dc level k-1.
template <typename T, class Op>
__global__ __launch_bounds__(FBS) void k_down2d(Op op, Dims d, Dims dc, const T* __restrict__ r,
                                                T* __restrict__ z2out, T* __restrict__ rc,
                                                const double* __restrict__ omg, const int* gate) {
  if (gate && *gate) return;
  constexpr int W1 = 2 * FCX + 5, H1 = 2 * FCY + 5;   // region of r, D and z1
  constexpr int W2 = W1 - 2, H2 = H1 - 2;             // region of z2
  constexpr int W3 = W1 - 4, H3 = H1 - 4;             // region of t
  __shared__ T sr[H1 * W1 * 2], sd[H1 * W1 * 2], s1[H1 * W1 * 2], s2[H2 * W2 * 2], s3[H3 * W3 * 2];
  const T omega = T(*omg);
  const Tile tl = xcd_tile();
  const int CI0 = (int)tl.x * FCX, CJ0 = (int)tl.y * FCY;
  const int ox = 2 * CI0 - 3, oy = 2 * CJ0 - 3;      // origin of region 1 (fine node indices)
  for (int t = threadIdx.x; t < W1 * H1; t += FBS) {
    const int gi = ox + t % W1, gj = oy + t / W1;
    T rr[2] = {T(0), T(0)}, dg[2] = {T(0), T(0)}, o[2] = {T(0), T(0)};
    if (node_free(d, gi, gj)) {
      load_node<2, T>(r, (int64_t)gj * d.nx1 + gi, rr);
      T vn[9][2], acc[2] = {T(0), T(0)};
      node_apply<2, T, Op, false, true, false>(op, d, gi, gj, 0, vn, acc, dg);
#pragma unroll
      for (int c = 0; c < 2; ++c) o[c] = omega * rr[c] * recip(dg[c]);
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) { sr[2 * t + c] = rr[c]; sd[2 * t + c] = dg[c]; s1[2 * t + c] = o[c]; }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < W2 * H2; t += FBS) {
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
  for (int t = threadIdx.x; t < W3 * H3; t += FBS) {
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
  for (int t = threadIdx.x; t < FCX * FCY; t += FBS) {  // rc = P' t on the tile's coarse nodes
    const int I = CI0 + t % FCX, J = CJ0 + t / FCX;
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
  for (int t = threadIdx.x; t < 4 * FCX * FCY; t += FBS) {   // z2 on the fine nodes the tile owns
    const int gi = 2 * CI0 + t % (2 * FCX), gj = 2 * CJ0 + t / (2 * FCX);
    if (gi >= d.nx1 || gj >= d.ny1) continue;
    const int q = 2 * ((gj - oy - 1) * W2 + gi - ox - 1);
    const T o[2] = {s2[q], s2[q + 1]};
    store_node<2, T>(z2out, (int64_t)gj * d.nx1 + gi, o);
  }
}

// Grid: (ceil(d.nx1 / FTX), ceil(d.ny1 / FTY)).
template <typename T, class Op>
__global__ __launch_bounds__(FBS) void k_up2d(Op op, Dims d, Dims dc, const T* __restrict__ r,
                                              const T* __restrict__ z2, const T* __restrict__ zc,
                                              T* __restrict__ out, const double* __restrict__ omg,
                                              const int* gate) {
  if (gate && *gate) return;
  constexpr int W0 = FTX + 4, H0 = FTY + 4;           // region of z2 + P zc
  constexpr int W1 = FTX + 2, H1 = FTY + 2;           // region of r, D and z3
  __shared__ T s0[H0 * W0 * 2], sr[H1 * W1 * 2], sd[H1 * W1 * 2], s1[H1 * W1 * 2];
  const T omega = T(*omg);
  const Tile tl = xcd_tile();
  const int I0 = (int)tl.x * FTX, J0 = (int)tl.y * FTY;
  for (int t = threadIdx.x; t < W0 * H0; t += FBS) {
    const int gi = I0 - 2 + t % W0, gj = J0 - 2 + t / W0;
    T o[2] = {T(0), T(0)};
    if (node_free(d, gi, gj)) {
      load_node<2, T>(z2, (int64_t)gj * d.nx1 + gi, o);
      const int ni = (gi & 1) ? 2 : 1, nj = (gj & 1) ? 2 : 1;
      for (int b = 0; b < nj; ++b)
        for (int e = 0; e < ni; ++e) {
          const int I = (gi >> 1) + e, J = (gj >> 1) + b;
          const T w = T((ni == 2 ? 0.5f : 1.0f) * (nj == 2 ? 0.5f : 1.0f));
          T vv[2];
          load_node<2, T>(zc, (int64_t)J * dc.nx1 + I, vv);
          o[0] += w * vv[0];
          o[1] += w * vv[1];
        }
    }
    s0[2 * t] = o[0];
    s0[2 * t + 1] = o[1];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < W1 * H1; t += FBS) {
    const int li = t % W1, lj = t / W1;                 // position in region 1
    const int gi = I0 - 1 + li, gj = J0 - 1 + lj;
    T rr[2] = {T(0), T(0)}, dg[2] = {T(0), T(0)}, o[2] = {T(0), T(0)};
    if (node_free(d, gi, gj)) {
      load_node<2, T>(r, (int64_t)gj * d.nx1 + gi, rr);
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
  for (int t = threadIdx.x; t < FTX * FTY; t += FBS) {
    const int gi = I0 + t % FTX, gj = J0 + t / FTX;
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

}  // namespace ipmg

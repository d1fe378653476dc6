// Per-dimension kernel set: element stiffness, sensitivities, interior-point
// element/node kernels and the dispatch of the level kernels (kernels.h).
#pragma once
#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>
#include <unordered_map>
#include "ctx.h"
#include "kernels.h"
#include "fused2d.h"

namespace ipmg {

// ---------------------------------------------------------- element matrix --
// K0 = integral over the unit element of the isotropic elasticity bilinear form
//   K[(a,i),(b,j)] = int lam dN_a/dx_i dN_b/dx_j + mu (delta_ij grad N_a . grad N_b
//                                                     + dN_a/dx_j dN_b/dx_i)
// (plane stress in 2D: lam = E nu / (1 - nu^2)), 2-point Gauss rule per axis.
template <int DIM>
__global__ void k_element_stiffness(double E, double nu, double* __restrict__ K) {
  constexpr int NN = Geo<DIM>::NN, ND = Geo<DIM>::ND;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ND * ND) return;
  const int r = t / ND, c = t % ND;
  const int a = r / DIM, i = r % DIM, b = c / DIM, j = c % DIM;
  const double mu = E / (2.0 * (1.0 + nu));
  const double lam = DIM == 2 ? E * nu / (1.0 - nu * nu) : E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  const double g = 0.5 / sqrt(3.0);
  const double pts[2] = {0.5 - g, 0.5 + g};
  const double w = DIM == 2 ? 0.25 : 0.125;
  int oa[3] = {loc_x(a), loc_y(a), loc_z(a)}, ob[3] = {loc_x(b), loc_y(b), loc_z(b)};
  double s = 0.0;
  for (int gp = 0; gp < NN; ++gp) {
    double xi[3] = {pts[gp & 1], pts[(gp >> 1) & 1], pts[(gp >> 2) & 1]};
    double da[3], db[3];
    for (int d = 0; d < DIM; ++d) {
      double pa = oa[d] ? 1.0 : -1.0, pb = ob[d] ? 1.0 : -1.0;
      for (int e = 0; e < DIM; ++e) {
        if (e == d) continue;
        pa *= oa[e] ? xi[e] : 1.0 - xi[e];
        pb *= ob[e] ? xi[e] : 1.0 - xi[e];
      }
      da[d] = pa; db[d] = pb;
    }
    double dot = 0.0;
    for (int d = 0; d < DIM; ++d) dot += da[d] * db[d];
    s += w * (lam * da[i] * db[j] + mu * ((i == j ? dot : 0.0) + da[j] * db[i]));
  }
  K[t] = s;
}

// Element coordinates of element e.
template <int DIM>
__device__ inline void elem_coords(const Dims& d, int64_t e, int& ei, int& ej, int& ek) {
  ei = (int)(e % d.nx);
  ej = (int)((e / d.nx) % d.ny);
  ek = DIM == 3 ? (int)(e / ((int64_t)d.nx * d.ny)) : 0;
}

// Gather the local vector of element e from a slot vector (clamped slots read 0).
template <int DIM>
__device__ inline void gather_elem(const double* __restrict__ v, const Dims& d, int ei, int ej, int ek,
                                   double* ve) {
  constexpr int NN = Geo<DIM>::NN;
#pragma unroll
  for (int b = 0; b < NN; ++b) {
    const int i = ei + loc_x(b), j = ej + loc_y(b), k = DIM == 3 ? ek + loc_z(b) : 0;
    const int64_t q = ((int64_t)k * d.ny1 + j) * d.nx1 + i;
#pragma unroll
    for (int c = 0; c < DIM; ++c) ve[b * DIM + c] = (i == 0) ? 0.0 : v[q * DIM + c];
  }
}

// s_e = h_e' v_e for every element, summed as OpFineZ::rows sums it, so that the
// node passes of the augmented operator read one value per element instead of
// all of h_e (each element is visited by all of its nodes).
template <int DIM, typename T>
__global__ __launch_bounds__(BS) void k_elem_hv(Dims d, const T* __restrict__ h, const T* __restrict__ v,
                                                T* __restrict__ s) {
  constexpr int NN = Geo<DIM>::NN;
  const int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (e >= d.m) return;
  int ei, ej, ek;
  elem_coords<DIM>(d, e, ei, ej, ek);
  T ve[NN * DIM];
#pragma unroll
  for (int b = 0; b < NN; ++b) {
    const int i = ei + loc_x(b), j = ej + loc_y(b), k = DIM == 3 ? ek + loc_z(b) : 0;
    const int64_t q = ((int64_t)k * d.ny1 + j) * d.nx1 + i;
#pragma unroll
    for (int c = 0; c < DIM; ++c) ve[b * DIM + c] = (i == 0) ? T(0) : v[q * DIM + c];
  }
  T hv = 0;
#pragma unroll
  for (int col = 0; col < NN * DIM; ++col) hv += h[col * d.m + e] * ve[col];
  s[e] = hv;
}

// g_e = scale * w_e' K0 u_e  (B(u)' w scaled).
template <int DIM>
__global__ __launch_bounds__(BS) void k_elem_sens(Dims d, const double* __restrict__ w, const double* __restrict__ u,
                                                  double scale, double* __restrict__ g) {
  constexpr int ND = Geo<DIM>::ND;
  const int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (e >= d.m) return;
  int ei, ej, ek;
  elem_coords<DIM>(d, e, ei, ej, ek);
  double we[ND], ue[ND];
  gather_elem<DIM>(w, d, ei, ej, ek, we);
  gather_elem<DIM>(u, d, ei, ej, ek, ue);
  double s = 0.0;
#pragma unroll
  for (int r = 0; r < ND; ++r) {
    double t = 0.0;
#pragma unroll
    for (int c = 0; c < ND; ++c) t += cK0d[r * ND + c] * ue[c];
    s += we[r] * t;
  }
  g[e] = scale * s;
}

// OC update (Sec. 4): t_e = x_e * E_e^q with the element energy E_e = u_e'K0u_e
// (negative rounding residue of a zero energy taken as 0).
template <int DIM>
__global__ __launch_bounds__(BS) void k_oc_energy(Dims d, const double* __restrict__ u, const double* __restrict__ x,
                                                  double q, double* __restrict__ t) {
  constexpr int ND = Geo<DIM>::ND;
  const int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (e >= d.m) return;
  int ei, ej, ek;
  elem_coords<DIM>(d, e, ei, ej, ek);
  double ue[ND];
  gather_elem<DIM>(u, d, ei, ej, ek, ue);
  double s = 0.0;
#pragma unroll
  for (int r = 0; r < ND; ++r) {
    double tr = 0.0;
#pragma unroll
    for (int c = 0; c < ND; ++c) tr += cK0d[r * ND + c] * ue[c];
    s += ue[r] * tr;
  }
  s = fmax(s, 0.0);
  t[e] = x[e] * (q == 1.0 ? s : (q == 0.5 ? sqrt(s) : pow(s, q)));
}

// Density filter of the SIMP model (Sec. 9): W^_ij = max(0, rmin - dist(i, j)) with
// the Manhattan distance of element centres, W_ji = W^_ji / s_i, s_i = sum_k W^_ki
// (every column of W sums to one).  transpose = 0: out = W in, i.e.
// out_j = sum_i W^_ji in_i / s_i; transpose = 1: out = W' in, out_i = sum_j W^_ji in_j / s_i.
// The column sums are formed on the fly from the grid geometry; neighbours in a
// fixed order, so the result is deterministic.
template <int DIM>
__device__ inline double filter_colsum(const Dims& d, int ei, int ej, int ek, double rmin, int R) {
  double s = 0.0;
  for (int dz = (DIM == 3 ? -R : 0); dz <= (DIM == 3 ? R : 0); ++dz)
    for (int dy = -R; dy <= R; ++dy)
      for (int dx = -R; dx <= R; ++dx) {
        const int i = ei + dx, j = ej + dy, k = ek + dz;
        if (i < 0 || i >= d.nx || j < 0 || j >= d.ny || (DIM == 3 && (k < 0 || k >= d.nz))) continue;
        s += fmax(0.0, rmin - (double)(abs(dx) + abs(dy) + abs(dz)));
      }
  return s;
}

// mode 0: out = W in; 1: out = W' in; 2: out = W2 in with (W2)_ji = W_ji^2.
template <int DIM>
__global__ __launch_bounds__(BS) void k_filter(Dims d, double rmin, int R, const double* __restrict__ in,
                                               double* __restrict__ out, int mode) {
  const int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (e >= d.m) return;
  int ei, ej, ek;
  elem_coords<DIM>(d, e, ei, ej, ek);
  double acc = 0.0;
  for (int dz = (DIM == 3 ? -R : 0); dz <= (DIM == 3 ? R : 0); ++dz)
    for (int dy = -R; dy <= R; ++dy)
      for (int dx = -R; dx <= R; ++dx) {
        const int i = ei + dx, j = ej + dy, k = ek + dz;
        if (i < 0 || i >= d.nx || j < 0 || j >= d.ny || (DIM == 3 && (k < 0 || k >= d.nz))) continue;
        const double w = rmin - (double)(abs(dx) + abs(dy) + abs(dz));
        if (!(w > 0.0)) continue;
        const int64_t o = ((int64_t)(DIM == 3 ? k : 0) * d.ny + j) * d.nx + i;
        if (mode == 1) {
          acc += w * in[o];
        } else {
          const double wc = w / filter_colsum<DIM>(d, i, j, k, rmin, R);
          acc += mode == 2 ? wc * wc * in[o] : wc * in[o];
        }
      }
  out[e] = mode == 1 ? acc / filter_colsum<DIM>(d, ei, ej, ek, rmin, R) : acc;
}

// Workgroups of a kernel (threads per group, static LDS) resident on one CU, from
// HIP's occupancy calculator; cached per kernel.
inline int resident_per_cu(const void* fn, int threads) {
  static std::mutex mu;
  static std::unordered_map<const void*, int> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(fn);
  if (it != cache.end()) return it->second;
  int n = 0;
  IPMG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, threads, 0));
  n = std::max(n, 1);
  cache[fn] = n;
  return n;
}

// Of two tilings of one fused pass (kernels fa, fb of FBS threads on grids ga, gb,
// tiles of aa, ab nodes with their halos), true when the second is cheaper.  Tiles
// are dealt out in rounds of (CUs x resident groups) and a round lasts about as long
// as one tile, so the cost is rounds x tile size: a tile count just above a multiple
// of the resident capacity would run a nearly empty last round.
inline bool pick_tiles(const Ctx& c, const void* fa, dim3 ga, int aa, const void* fb, dim3 gb, int ab) {
  auto cost = [&](const void* fn, dim3 g, int area) {
    const int64_t slots = (int64_t)c.cus * resident_per_cu(fn, FBS);
    const int64_t tiles = (int64_t)g.x * g.y;
    return ((tiles + slots - 1) / slots) * (int64_t)area;
  };
  return cost(fb, gb, ab) < cost(fa, ga, aa);
}

// SIMP penalisation: xp = x~^p, and the chain-rule factor q_e = p x~_e^(p-1) E_e of
// the compliance gradient (E_e = u_e'K0u_e in q on entry).
static __global__ __launch_bounds__(BS) void k_simp_pow(int64_t m, const double* __restrict__ xt, double p,
                                                 double* __restrict__ xp, double* __restrict__ q) {
  const int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (e >= m) return;
  if (xp) xp[e] = pow(xt[e], p);
  if (q) q[e] = p * pow(xt[e], p - 1.0) * q[e];
}

// Start vector of the spectral-radius estimate: (-1)^(i+j+k) (1 + c), 0 on clamped
// slots, 1 on lambda.
template <int DIM, typename T>
__global__ __launch_bounds__(BS) void k_power_start(Dims d, int aug, T* __restrict__ v) {
  const int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (t == d.nslots && aug) v[t] = T(1);
  if (t >= d.nslots) return;
  const int64_t q = t / DIM;
  const int c = (int)(t % DIM);
  const int i = (int)(q % d.nx1), j = (int)((q / d.nx1) % d.ny1), k = (int)(q / ((int64_t)d.nx1 * d.ny1));
  const double sg = ((i + j + k) & 1) ? -1.0 : 1.0;
  v[t] = i == 0 ? T(0) : T(sg * (1.0 + c));
}

// ---------------------------------------------------------- interior point --
// Per element at the current iterate (Sec. 2): g = K0 u_e, F3, F4, F5,
// D = phi/x + psi/(xbar-x), G3 = F3 + F4/x - F5/(xbar-x), w = 1/D,
// h = sqrt(w) g (rank-one factor of Z), and the sums
//   scal[S_TMP0..6] = sum w, sum G3 w, sum x, ||G3||^2, ||phi||^2, ||psi||^2,
//                     phi'x + psi'(xbar - x).
template <int DIM, typename T>
__global__ __launch_bounds__(BS) void k_ip_elements(Dims d, const double* __restrict__ u, const double* __restrict__ x,
                                                    const double* __restrict__ phi, const double* __restrict__ psi,
                                                    double lam, double s, double r, double xbar,
                                                    double* __restrict__ G3o, double* __restrict__ Wo,
                                                    double* __restrict__ SWo, double* __restrict__ h64,
                                                    T* __restrict__ hT, Red red) {
  constexpr int ND = Geo<DIM>::ND;
  const int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x;
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  if (e < d.m) {
    int ei, ej, ek;
    elem_coords<DIM>(d, e, ei, ej, ek);
    double ue[ND], g[ND];
    gather_elem<DIM>(u, d, ei, ej, ek, ue);
    double en = 0.0;
#pragma unroll
    for (int rr = 0; rr < ND; ++rr) {
      double t = 0.0;
#pragma unroll
      for (int c = 0; c < ND; ++c) t += cK0d[rr * ND + c] * ue[c];
      g[rr] = t;
      en += ue[rr] * t;
    }
    const double xe = x[e], ph = phi[e], ps = psi[e], xt = xbar - xe;
    if (!(xe > 0.0) || !(xt > 0.0) || !isfinite(xe) || !isfinite(ph) || !isfinite(ps) || !isfinite(en))
      red.flags[F_BAD] = 1;
    const double F3 = -0.5 * en - lam - ph + ps;
    const double F4 = ph * xe - s;
    const double F5 = ps * xt - r;
    const double D = ph / xe + ps / xt;
    const double G3 = F3 + F4 / xe - F5 / xt;
    const double w = 1.0 / D, sw = sqrt(w);
    G3o[e] = G3;
    Wo[e] = w;
    SWo[e] = sw;
#pragma unroll
    for (int rr = 0; rr < ND; ++rr) {
      const double hv = sw * g[rr];
      h64[rr * d.m + e] = hv;
      if (hT) hT[rr * d.m + e] = T(hv);
    }
    acc[0] = w; acc[1] = G3 * w; acc[2] = xe; acc[3] = G3 * G3;
    acc[4] = ph * ph; acc[5] = ps * ps; acc[6] = ph * xe + ps * xt;
  }
  block_partials<7>(acc, red);
}

// Sums of k_ip_elements into scal[S_TMP0..6].
static __global__ __launch_bounds__(BS) void k_ip_elements_fin(Red red, unsigned nblocks) {
  double tot[7];
  sum_partials<7>(red, nblocks, tot);
  if (threadIdx.x == 0)
    for (int n = 0; n < 7; ++n) red.scal[S_TMP0 + n] = tot[n];
}

// Per node: F1 = K u - f, border b = sum_e sqrt(w_e) h_e (= B D^-1 e), right-hand
// side rhs_u = -F1 + sum_e G3_e sqrt(w_e) h_e (= -F1 + B D^-1 G3, eq. (nwtr2rhs)),
// and rhs_lambda = -(sum x - V) + sum G3 w.  Sums: scal[S_MIN0..2] = ||F1||^2,
// ||f||^2, f'u.
template <int DIM>
__global__ __launch_bounds__(BS) void k_ip_nodes(Dims d, const double* __restrict__ Ku, const double* __restrict__ f,
                                                 const double* __restrict__ u, const double* __restrict__ G3,
                                                 const double* __restrict__ SW, const double* __restrict__ h64,
                                                 double V, double* __restrict__ rhs, double* __restrict__ bZ,
                                                 Red red) {
  constexpr int NN = Geo<DIM>::NN;
  const Tile tl = xcd_tile();
  const int i = tl.x * 64 + (threadIdx.x & 63);
  const int j = tl.y * (BS / 64) + (threadIdx.x >> 6);
  const int k = tl.z;
  double acc[3] = {0, 0, 0};
  if (i < d.nx1 && j < d.ny1) {
    const int64_t q = ((int64_t)k * d.ny1 + j) * d.nx1 + i;
    double bb[DIM], tt[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) { bb[c] = 0.0; tt[c] = 0.0; }
    if (i > 0) {
#pragma unroll
      for (int qq = 0; qq < NN; ++qq) {
        const int ex = qq & 1, ey = (qq >> 1) & 1, ez = (qq >> 2) & 1;
        const int ei = i - 1 + ex, ej = j - 1 + ey, ek = k - 1 + ez;
        if (ei < 0 || ei >= d.nx || ej < 0 || ej >= d.ny || (DIM == 3 && (ek < 0 || ek >= d.nz))) continue;
        const int64_t e = ((int64_t)(DIM == 3 ? ek : 0) * d.ny + ej) * d.nx + ei;
        const int a = loc_index(1 - ex, 1 - ey, DIM == 3 ? 1 - ez : 0);
        const double sw = SW[e], gw = G3[e] * sw;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
          const double hv = h64[(a * DIM + c) * d.m + e];
          bb[c] += sw * hv;
          tt[c] += gw * hv;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      const int64_t sl = q * DIM + c;
      const double fc = i > 0 ? f[sl] : 0.0;
      const double F1 = i > 0 ? Ku[sl] - fc : 0.0;
      rhs[sl] = i > 0 ? -F1 + tt[c] : 0.0;
      bZ[sl] = bb[c];
      acc[0] += F1 * F1;
      acc[1] += fc * fc;
      acc[2] += fc * (i > 0 ? u[sl] : 0.0);
    }
  }
  block_partials<3>(acc, red);
}

// Sums of k_ip_nodes into scal[S_MIN0..2] and the lambda entry of the right-hand side.
static __global__ __launch_bounds__(BS) void k_ip_nodes_fin(Red red, unsigned nblocks, double V, double* rhs, int64_t n) {
  double tot[3];
  sum_partials<3>(red, nblocks, tot);
  if (threadIdx.x == 0) {
    red.scal[S_MIN0] = tot[0];
    red.scal[S_MIN1] = tot[1];
    red.scal[S_MIN2] = tot[2];
    rhs[n] = -(red.scal[S_TMP2] - V) + red.scal[S_TMP1];
  }
}

// Recovery of d_x, d_phi, d_psi from (d_u, d_lambda) and the fraction-to-boundary
// step length (Sec. 3.3): scal[S_ALPHA] = min(1, frac * distance ratios).
template <int DIM>
__global__ __launch_bounds__(BS) void k_ip_recover(Dims d, const double* __restrict__ du, const double* __restrict__ x,
                                                   const double* __restrict__ phi, const double* __restrict__ psi,
                                                   const double* __restrict__ G3, const double* __restrict__ W,
                                                   const double* __restrict__ SW, const double* __restrict__ h64,
                                                   double s, double r, double xbar, double frac, int all_blocks,
                                                   double* __restrict__ dx, double* __restrict__ dphi,
                                                   double* __restrict__ dpsi, Red red) {
  constexpr int ND = Geo<DIM>::ND;
  const int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x;
  double mins[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
  if (e < d.m) {
    int ei, ej, ek;
    elem_coords<DIM>(d, e, ei, ej, ek);
    double de[ND];
    gather_elem<DIM>(du, d, ei, ej, ek, de);
    double hd = 0.0;
#pragma unroll
    for (int rr = 0; rr < ND; ++rr) hd += h64[rr * d.m + e] * de[rr];
    const double dl = du[d.nslots];
    const double xe = x[e], ph = phi[e], ps = psi[e], xt = xbar - xe;
    // d_x = D^-1 (B' d_u + d_lambda - G3), B' d_u = g . d_u = (h . d_u) / sqrt(w)
    const double ddx = SW[e] * hd + W[e] * (dl - G3[e]);
    const double F4 = ph * xe - s, F5 = ps * xt - r;
    const double ddphi = (-F4 - ph * ddx) / xe;
    const double ddpsi = (-F5 + ps * ddx) / xt;
    dx[e] = ddx; dphi[e] = ddphi; dpsi[e] = ddpsi;
    if (!isfinite(ddx) || !isfinite(ddphi) || !isfinite(ddpsi) || !isfinite(dl)) red.flags[F_BAD] = 1;
    if (ddx < 0.0) mins[0] = -xe / ddx;
    if (ddx > 0.0) mins[1] = xt / ddx;
    if (ddphi < 0.0) mins[2] = -ph / ddphi;
    if (ddpsi < 0.0) mins[3] = -ps / ddpsi;
  }
  block_partials<4, true>(mins, red);
}

// Step length from the minima of k_ip_recover.
static __global__ __launch_bounds__(BS) void k_ip_recover_fin(Red red, unsigned nblocks, double frac, int all_blocks) {
  double tot[4];
  sum_partials<4, true>(red, nblocks, tot);
  if (threadIdx.x == 0) {
    double a = fmin(1.0, fmin(frac * tot[0], frac * tot[1]));
    if (all_blocks) a = fmin(a, fmin(frac * tot[2], frac * tot[3]));
    red.scal[S_ALPHA] = a;
    for (int n = 0; n < 4; ++n) red.scal[S_MIN0 + n] = tot[n];
  }
}

// z += alpha d for (u, x, phi, psi).
template <int DIM>
__global__ __launch_bounds__(BS) void k_ip_update(Dims d, double* __restrict__ u, const double* __restrict__ du,
                                                  double* __restrict__ x, double* __restrict__ phi,
                                                  double* __restrict__ psi, const double* __restrict__ dx,
                                                  const double* __restrict__ dphi, const double* __restrict__ dpsi,
                                                  Red red) {
  const double a = red.scal[S_ALPHA];
  const int64_t n = d.nslots > d.m ? d.nslots : d.m;
  for (int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x; t < n; t += (int64_t)gridDim.x * BS) {
    if (t < d.nslots) u[t] += a * du[t];
    if (t < d.m) {
      x[t] += a * dx[t];
      phi[t] += a * dphi[t];
      psi[t] += a * dpsi[t];
    }
  }
}

// ------------------------------------------------------ SIMP interior point --
// The interior-point method on the SIMP model (Sec. 9): K^ = sum x~^p K_e with the
// filtered densities x~ = W x, and B^(u) = B(u) C W in place of B(u) in the Newton
// system, C = diag(c), c = p x~^(p-1), B(u) = (K_1 u, ..., K_m u) with the unit
// element matrices.  The exact Newton matrix Z^ is applied matrix-free; the
// multigrid hierarchy is built from an element-local SPD approximation (the
// couplings between the elements of a filter patch dropped).

// g_e = K0 u_e (entry r at r m + e) and E_e = u_e'g_e.
template <int DIM>
__global__ __launch_bounds__(BS) void k_simp_elem(Dims d, const double* __restrict__ u, double* __restrict__ g,
                                                  double* __restrict__ E) {
  constexpr int ND = Geo<DIM>::ND;
  const int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (e >= d.m) return;
  int ei, ej, ek;
  elem_coords<DIM>(d, e, ei, ej, ek);
  double ue[ND];
  gather_elem<DIM>(u, d, ei, ej, ek, ue);
  double en = 0.0;
#pragma unroll
  for (int rr = 0; rr < ND; ++rr) {
    double t = 0.0;
#pragma unroll
    for (int c = 0; c < ND; ++c) t += cK0d[rr * ND + c] * ue[c];
    g[rr * d.m + e] = t;
    en += ue[rr] * t;
  }
  E[e] = en;
}

// Per design variable, with t = W'(c o E) (the filtered energy term of the modified
// KKT3): F3 = -t/2 - lambda - phi + psi, F4, F5, D, G3, w = 1/D, and the sums of
// k_ip_elements (finalized by k_ip_elements_fin into scal[S_TMP0..6]).
static __global__ __launch_bounds__(BS) void k_simp_design(int64_t m, const double* __restrict__ t,
                                                           const double* __restrict__ x,
                                                           const double* __restrict__ phi,
                                                           const double* __restrict__ psi, double lam, double s,
                                                           double r, double xbar, double* __restrict__ G3o,
                                                           double* __restrict__ Wo, Red red) {
  const int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x;
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  if (e < m) {
    const double xe = x[e], ph = phi[e], ps = psi[e], xt = xbar - xe;
    if (!(xe > 0.0) || !(xt > 0.0) || !isfinite(xe) || !isfinite(ph) || !isfinite(ps) || !isfinite(t[e]))
      red.flags[F_BAD] = 1;
    const double F3 = -0.5 * t[e] - lam - ph + ps;
    const double F4 = ph * xe - s;
    const double F5 = ps * xt - r;
    const double D = ph / xe + ps / xt;
    const double G3 = F3 + F4 / xe - F5 / xt;
    const double w = 1.0 / D;
    G3o[e] = G3;
    Wo[e] = w;
    acc[0] = w; acc[1] = G3 * w; acc[2] = xe; acc[3] = G3 * G3;
    acc[4] = ph * ph; acc[5] = ps * ps; acc[6] = ph * xe + ps * xt;
  }
  block_partials<7>(acc, red);
}

// Per element: bcoef = c (W w), rcoef = c (W (G3 w)) (coefficients of K0 u_e in the
// border B^ D^-1 e and in B^ D^-1 G3), the lumped rank-one weight wt = c^2 (W2 w)
// ((W2)_ji = W_ji^2), the preconditioner's factor h_e = sqrt(wt) g_e (h64, and the
// V-cycle copy hT), and the partials of its corner sum bcoef^2 / wt.
template <int DIM, typename T>
__global__ __launch_bounds__(BS) void k_simp_coef(Dims d, const double* __restrict__ cf,
                                                  const double* __restrict__ Ww, const double* __restrict__ WGw,
                                                  const double* __restrict__ W2w, const double* __restrict__ g,
                                                  double* __restrict__ bcoef, double* __restrict__ rcoef,
                                                  double* __restrict__ h64, T* __restrict__ hT, Red red) {
  constexpr int ND = Geo<DIM>::ND;
  const int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x;
  double acc[1] = {0.0};
  if (e < d.m) {
    const double c = cf[e], bc = c * Ww[e], wt = c * c * W2w[e], sw = sqrt(wt);
    bcoef[e] = bc;
    rcoef[e] = c * WGw[e];
#pragma unroll
    for (int rr = 0; rr < ND; ++rr) {
      const double hv = sw * g[rr * d.m + e];
      h64[rr * d.m + e] = hv;
      if (hT) hT[rr * d.m + e] = T(hv);
    }
    acc[0] = bc * bc / wt;
    if (!(wt > 0.0) || !isfinite(wt)) red.flags[F_BAD] = 1;
  }
  block_partials<1>(acc, red);
}

static __global__ __launch_bounds__(BS) void k_simp_coef_fin(Red red, unsigned nblocks) {
  double tot[1];
  sum_partials<1>(red, nblocks, tot);
  if (threadIdx.x == 0) red.scal[S_TMP7] = tot[0];
}

// Per node: F1 = K^ u - f, the border b = sum_e bcoef_e g_e (= B^ D^-1 e) and
// rhs_u = -F1 + sum_e rcoef_e g_e (= -F1 + B^ D^-1 G3); sums as k_ip_nodes
// (finalized by k_ip_nodes_fin).
template <int DIM>
__global__ __launch_bounds__(BS) void k_simp_nodes(Dims d, const double* __restrict__ Ku,
                                                   const double* __restrict__ f, const double* __restrict__ u,
                                                   const double* __restrict__ g, const double* __restrict__ bcoef,
                                                   const double* __restrict__ rcoef, double* __restrict__ rhs,
                                                   double* __restrict__ bZ, Red red) {
  constexpr int NN = Geo<DIM>::NN;
  const Tile tl = xcd_tile();
  const int i = tl.x * 64 + (threadIdx.x & 63);
  const int j = tl.y * (BS / 64) + (threadIdx.x >> 6);
  const int k = tl.z;
  double acc[3] = {0, 0, 0};
  if (i < d.nx1 && j < d.ny1) {
    const int64_t q = ((int64_t)k * d.ny1 + j) * d.nx1 + i;
    double bb[DIM], tt[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) { bb[c] = 0.0; tt[c] = 0.0; }
    if (i > 0) {
#pragma unroll
      for (int qq = 0; qq < NN; ++qq) {
        const int ex = qq & 1, ey = (qq >> 1) & 1, ez = (qq >> 2) & 1;
        const int ei = i - 1 + ex, ej = j - 1 + ey, ek = k - 1 + ez;
        if (ei < 0 || ei >= d.nx || ej < 0 || ej >= d.ny || (DIM == 3 && (ek < 0 || ek >= d.nz))) continue;
        const int64_t e = ((int64_t)(DIM == 3 ? ek : 0) * d.ny + ej) * d.nx + ei;
        const int a = loc_index(1 - ex, 1 - ey, DIM == 3 ? 1 - ez : 0);
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
          const double gv = g[(a * DIM + c) * d.m + e];
          bb[c] += bcoef[e] * gv;
          tt[c] += rcoef[e] * gv;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      const int64_t sl = q * DIM + c;
      const double fc = i > 0 ? f[sl] : 0.0;
      const double F1 = i > 0 ? Ku[sl] - fc : 0.0;
      rhs[sl] = i > 0 ? -F1 + tt[c] : 0.0;
      bZ[sl] = bb[c];
      acc[0] += F1 * F1;
      acc[1] += fc * fc;
      acc[2] += fc * (i > 0 ? u[sl] : 0.0);
    }
  }
  block_partials<3>(acc, red);
}

// y_u += sum_e coef_e g_e + b v_lambda on the free slots: the rank-one and border
// part of Z^ v (coef = c o W (w o W'(c o s)), s_e = g_e . v_e).
template <int DIM>
__global__ __launch_bounds__(BS) void k_simp_gather(Dims d, const double* __restrict__ g,
                                                    const double* __restrict__ coef, const double* __restrict__ bZ,
                                                    const double* __restrict__ v, double* __restrict__ y) {
  constexpr int NN = Geo<DIM>::NN;
  const Tile tl = xcd_tile();
  const int i = tl.x * 64 + (threadIdx.x & 63);
  const int j = tl.y * (BS / 64) + (threadIdx.x >> 6);
  const int k = tl.z;
  if (i < 1 || i >= d.nx1 || j >= d.ny1) return;
  const int64_t q = ((int64_t)k * d.ny1 + j) * d.nx1 + i;
  double tt[DIM];
#pragma unroll
  for (int c = 0; c < DIM; ++c) tt[c] = 0.0;
#pragma unroll
  for (int qq = 0; qq < NN; ++qq) {
    const int ex = qq & 1, ey = (qq >> 1) & 1, ez = (qq >> 2) & 1;
    const int ei = i - 1 + ex, ej = j - 1 + ey, ek = k - 1 + ez;
    if (ei < 0 || ei >= d.nx || ej < 0 || ej >= d.ny || (DIM == 3 && (ek < 0 || ek >= d.nz))) continue;
    const int64_t e = ((int64_t)(DIM == 3 ? ek : 0) * d.ny + ej) * d.nx + ei;
    const int a = loc_index(1 - ex, 1 - ey, DIM == 3 ? 1 - ez : 0);
#pragma unroll
    for (int c = 0; c < DIM; ++c) tt[c] += coef[e] * g[(a * DIM + c) * d.m + e];
  }
  const double vl = v[d.nslots];
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    const int64_t sl = q * DIM + c;
    y[sl] += tt[c] + bZ[sl] * vl;
  }
}

// Recovery of the SIMP direction: d_x = w (B^'d_u + d_lambda - G3) with btdu =
// B^'d_u = W'(c o (g . d_u)), d_phi, d_psi and the step-length minima (finalized by
// k_ip_recover_fin).
static __global__ __launch_bounds__(BS) void k_simp_recover(int64_t m, int64_t nslots,
                                                            const double* __restrict__ btdu,
                                                            const double* __restrict__ du,
                                                            const double* __restrict__ x,
                                                            const double* __restrict__ phi,
                                                            const double* __restrict__ psi,
                                                            const double* __restrict__ G3,
                                                            const double* __restrict__ W, double s, double r,
                                                            double xbar, double* __restrict__ dx,
                                                            double* __restrict__ dphi, double* __restrict__ dpsi,
                                                            Red red) {
  const int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x;
  double mins[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
  if (e < m) {
    const double dl = du[nslots];
    const double xe = x[e], ph = phi[e], ps = psi[e], xt = xbar - xe;
    const double ddx = W[e] * (btdu[e] + dl - G3[e]);
    const double F4 = ph * xe - s, F5 = ps * xt - r;
    const double ddphi = (-F4 - ph * ddx) / xe;
    const double ddpsi = (-F5 + ps * ddx) / xt;
    dx[e] = ddx; dphi[e] = ddphi; dpsi[e] = ddpsi;
    if (!isfinite(ddx) || !isfinite(ddphi) || !isfinite(ddpsi) || !isfinite(dl)) red.flags[F_BAD] = 1;
    if (ddx < 0.0) mins[0] = -xe / ddx;
    if (ddx > 0.0) mins[1] = xt / ddx;
    if (ddphi < 0.0) mins[2] = -ph / ddphi;
    if (ddpsi < 0.0) mins[3] = -ps / ddpsi;
  }
  block_partials<4, true>(mins, red);
}

// ------------------------------------------------------------------- dispatch --
template <int DIM>
struct OpsImpl : Ops {
  static dim3 node_grid(const Dims& d) {
    return dim3((unsigned)((d.nx1 + 63) / 64), (unsigned)((d.ny1 + BS / 64 - 1) / (BS / 64)), (unsigned)d.nz1);
  }
  static unsigned lin_grid(int64_t n) { return (unsigned)((n + BS - 1) / BS); }

  void element_stiffness(Ctx& c, double* dK0) override {
    constexpr int ND = Geo<DIM>::ND;
    k_element_stiffness<DIM><<<(ND * ND + 63) / 64, 64, 0, c.stream>>>(c.desc.E, c.desc.nu, dK0);
  }
  void upload_k0(const double* K0) override {
    constexpr int ND = Geo<DIM>::ND;
    if constexpr (DIM == 2) {
      double kmax = 0.0;
      for (int t = 0; t < 64; ++t) kmax = std::max(kmax, std::fabs(K0[t]));
      for (int t = 0; t < 64; ++t) {
        const int e = kSq2d[t];
        const double want = e > 0 ? K0[e - 1] : -K0[-e - 1];
        IPMG_REQUIRE(std::fabs(K0[t] - want) <= 1e-12 * kmax, IPMG_E_INVALID,
                     "element matrix lacks the square-element symmetry");
      }
    }
    if constexpr (DIM == 3) {
      double kmax = 0.0, k14[14] = {0.0};
      bool have[14] = {false};
      for (int t = 0; t < 576; ++t) kmax = std::max(kmax, std::fabs(K0[t]));
      for (int r = 0; r < 24; ++r)
        for (int col = 0; col < 24; ++col) {
          const int e = k0cube_slot(r, col), sl = (e > 0 ? e : -e) - 1;
          const double v = e > 0 ? K0[r * 24 + col] : -K0[r * 24 + col];
          if (!have[sl]) { k14[sl] = v; have[sl] = true; }
          IPMG_REQUIRE(std::fabs(v - k14[sl]) <= 1e-12 * kmax, IPMG_E_INVALID,
                       "element matrix lacks the cube symmetry");
        }
      float k14f[14];
      for (int t = 0; t < 14; ++t) k14f[t] = (float)k14[t];
      IPMG_HIP(hipMemcpyToSymbol(HIP_SYMBOL(cK3d), k14, sizeof(double) * 14));
      IPMG_HIP(hipMemcpyToSymbol(HIP_SYMBOL(cK3f), k14f, sizeof(float) * 14));
    }
    float kf[576];
    for (int t = 0; t < ND * ND; ++t) kf[t] = (float)K0[t];
    IPMG_HIP(hipMemcpyToSymbol(HIP_SYMBOL(cK0d), K0, sizeof(double) * ND * ND));
    IPMG_HIP(hipMemcpyToSymbol(HIP_SYMBOL(cK0f), kf, sizeof(float) * ND * ND));
    if constexpr (DIM == 2) {
      double *dK = nullptr, *dG = nullptr;
      IPMG_HIP(hipMalloc((void**)&dK, sizeof(double) * 64));
      IPMG_HIP(hipMalloc((void**)&dG, sizeof(double) * 256));
      IPMG_HIP(hipMemcpy(dK, K0, sizeof(double) * 64, hipMemcpyHostToDevice));
      k_galerkin_images2d<<<4, 64>>>(dK, dG);
      double G[256];
      IPMG_HIP(hipMemcpy(G, dG, sizeof(double) * 256, hipMemcpyDeviceToHost));
      (void)hipFree(dK);
      (void)hipFree(dG);
      // the 18 distinct values, and every entry checked against its signed copy
      double g18[18] = {0.0};
      bool have[18] = {false};
      double gmax = 0.0;
      for (int t = 0; t < 256; ++t) gmax = std::max(gmax, std::fabs(G[t]));
      for (int t = 0; t < 256; ++t) {
        const int e = kSqG2d[t], k = (e > 0 ? e : -e) - 1;
        if (!have[k]) { g18[k] = e > 0 ? G[t] : -G[t]; have[k] = true; }
        const double want = e > 0 ? g18[k] : -g18[k];
        IPMG_REQUIRE(std::fabs(G[t] - want) <= 1e-12 * gmax, IPMG_E_INVALID,
                     "Galerkin images lack the square-element symmetry");
      }
      float g18f[18];
      for (int k = 0; k < 18; ++k) g18f[k] = (float)g18[k];
      IPMG_HIP(hipMemcpyToSymbol(HIP_SYMBOL(cG18d), g18, sizeof(double) * 18));
      IPMG_HIP(hipMemcpyToSymbol(HIP_SYMBOL(cG18f), g18f, sizeof(float) * 18));
      float g256f[256];
      for (int t = 0; t < 256; ++t) {
        const int e = kSqG2d[t], k = (e > 0 ? e : -e) - 1;
        g256f[t] = e > 0 ? g18f[k] : -g18f[k];
      }
      IPMG_HIP(hipMemcpyToSymbol(HIP_SYMBOL(cG256f), g256f, sizeof(float) * 256));
    }
  }

  // 2D level pass on register-blocked tiles of 64 x 4*NJ nodes.  On the finest level
  // of K, the two passes that form their neighbourhood from other vectors (the two
  // sweeps from zero, the folded prolongation) run on lane-shared tiles of LS_COLS x
  // 4*NJ output nodes (c.lane_share); the passes that only load it are bound by
  // their traffic and read fewer cache lines on tiles that start on 64-node
  // boundaries.
  template <typename T, class Op, int NJ>
  void launch_l2d(Ctx& c, const Dims& d, const Op& op, int mode, const T* v, const T* r, T* out, const double* omg,
                  Aug<T> aug, int sidx, int sidx_in, const int* gate, const double* dot64, bool fin,
                  const T* zc = nullptr, const Dims* dcp = nullptr) {
    if constexpr (std::is_same<Op, OpFineK<2, T>>::value) {
      if (c.lane_share && (mode == M_JACOBI2 || mode == M_PJACOBI)) {
        launch_l2d_t<T, Op, NJ, true>(c, d, op, mode, v, r, out, omg, aug, sidx, sidx_in, gate, dot64, fin, zc, dcp);
        return;
      }
    }
    launch_l2d_t<T, Op, NJ, false>(c, d, op, mode, v, r, out, omg, aug, sidx, sidx_in, gate, dot64, fin, zc, dcp);
  }
  template <typename T, class Op, int NJ, bool LS>
  void launch_l2d_t(Ctx& c, const Dims& d, const Op& op, int mode, const T* v, const T* r, T* out,
                    const double* omg, Aug<T> aug, int sidx, int sidx_in, const int* gate, const double* dot64,
                    bool fin, const T* zc, const Dims* dcp) {
    const Dims dc = dcp ? *dcp : d;
    const int cols = LS ? LS_COLS : 64;
    const dim3 g2((unsigned)((d.nx1 + cols - 1) / cols), (unsigned)((d.ny1 + 4 * NJ - 1) / (4 * NJ)), 1);
    const unsigned nb2 = g2.x * g2.y;
    IPMG_REQUIRE((int64_t)nb2 <= MAX_PARTIALS, IPMG_E_INVALID, "grid too large for one reduction");
#define IPMG_L2D_CASE(M)                                                                                     \
  case M:                                                                                                    \
    {                                                                                                        \
      ProfScope ps_(c, c.prof_tag);                                                                          \
      k_level2d<T, Op, M, NJ, LS><<<g2, BS, 0, c.stream>>>(op, d, v, r, out, omg, aug, c.red, dot64, gate, zc, \
                                                           dc, 0u, 0);                                       \
    }                                                                                                        \
    if (fin)                                                                                                 \
      k_level_fin<T, M><<<1, BS, 0, c.stream>>>(v, r, out, omg, aug.b != nullptr, aug.c, aug.n, dot64, c.red, nb2, \
                                                 sidx, sidx_in, gate,                                       \
                                                 M == M_JACOBI_BETA ? c.take_flag_dst() : nullptr);         \
    return;
    switch (mode) {
      IPMG_L2D_CASE(M_APPLY)
      IPMG_L2D_CASE(M_RESID)
      IPMG_L2D_CASE(M_JACOBI)
      IPMG_L2D_CASE(M_JACOBI0)
      IPMG_L2D_CASE(M_JACOBI_BETA)
      default: break;
    }
#undef IPMG_L2D_CASE
    if constexpr (std::is_same<Op, OpFineK<2, T>>::value) {
      if (mode == M_JACOBI2) {
        ProfScope ps_(c, c.prof_tag);
        k_level2d<T, Op, M_JACOBI2, NJ, LS><<<g2, BS, 0, c.stream>>>(op, d, v, r, out, omg, aug, c.red, dot64, gate,
                                                                     zc, dc, c.rn2_fin_blocks,
                                                                     c.rn2_fin_zpend ? 1 : 0);
        c.rn2_fin_blocks = 0;
      }
    }
    if constexpr (NJ % 2 == 0) {
      if (mode == M_PJACOBI) {
        ProfScope ps_(c, c.prof_tag);
        k_level2d<T, Op, M_PJACOBI, NJ, LS><<<g2, BS, 0, c.stream>>>(op, d, v, r, out, omg, aug, c.red, dot64, gate,
                                                                     zc, dc, 0u, 0);
      }
    }
  }

  // z2 + P zc, then one Jacobi sweep, in one tiled pass (2D, operator K, even
  // register-block width); false when it does not apply (the caller prolongs and
  // sweeps separately).
  template <typename T, class Op>
  bool pjacobi_t(Ctx& c, const Dims& d, const Dims& dc, const Op& op, const T* z2, const T* zc, const T* r, T* out,
                 const double* omg, const int* gate) {
    const int nj = sizeof(T) == 4 ? c.nj32 : c.nj64;
    if (!c.tiled2d || d.nnodes < c.tiled_min_nodes || nj % 2 != 0) return false;
    const Aug<T> aug{nullptr, 0.0, d.nslots};
    if (nj == 2) launch_l2d<T, Op, 2>(c, d, op, M_PJACOBI, z2, r, out, omg, aug, 0, -1, gate, nullptr, false, zc, &dc);
    else if (nj == 8) launch_l2d<T, Op, 8>(c, d, op, M_PJACOBI, z2, r, out, omg, aug, 0, -1, gate, nullptr, false, zc, &dc);
    else launch_l2d<T, Op, 4>(c, d, op, M_PJACOBI, z2, r, out, omg, aug, 0, -1, gate, nullptr, false, zc, &dc);
    return true;
  }
  // The first two pre-smoothing sweeps (zero start) in one tiled pass on the finest
  // level of K; false when that pass does not apply.
  template <typename T>
  bool jacobi2_t(Ctx& c, const Dims& d, const T* r, T* out, const double* omg, const int* gate) {
    const int nj = sizeof(T) == 4 ? c.nj32 : c.nj64;
    if (!c.tiled2d || d.nnodes < c.tiled_min_nodes) return false;
    const OpFineK<2, T> op{(const T*)c.xT, d.m};
    const Aug<T> aug{nullptr, 0.0, d.nslots};
    if (nj == 1) launch_l2d<T, OpFineK<2, T>, 1>(c, d, op, M_JACOBI2, nullptr, r, out, omg, aug, 0, -1, gate, nullptr, false);
    else if (nj == 2) launch_l2d<T, OpFineK<2, T>, 2>(c, d, op, M_JACOBI2, nullptr, r, out, omg, aug, 0, -1, gate, nullptr, false);
    else if (nj == 8) launch_l2d<T, OpFineK<2, T>, 8>(c, d, op, M_JACOBI2, nullptr, r, out, omg, aug, 0, -1, gate, nullptr, false);
    else launch_l2d<T, OpFineK<2, T>, 4>(c, d, op, M_JACOBI2, nullptr, r, out, omg, aug, 0, -1, gate, nullptr, false);
    return true;
  }
  template <typename T, int NJ>
  void launch_jacobi2r(Ctx& c, const Dims& d, const T* r, T* out, T* t, const double* omg, const int* gate) {
    constexpr int RJ = 4 * NJ;
    const dim3 g((unsigned)((d.nx1 + LS2_COLS - 1) / LS2_COLS), (unsigned)((d.ny1 + RJ - 1) / RJ), 1);
    const OpFineK<2, T> op{(const T*)c.xT, d.m};
    ProfScope ps(c, c.prof_tag);
    k_jacobi2r2d<T, NJ><<<g, BS, 0, c.stream>>>(op, d, r, out, t, omg, c.red, gate, c.rn2_fin_blocks,
                                                c.rn2_fin_zpend ? 1 : 0);
    c.rn2_fin_blocks = 0;
  }
  bool jacobi2_resid(Ctx& c, int lev, int op, const void* r, void* out, void* t, const double* omg,
                     const int* gate) override {
    if constexpr (DIM != 2) {
      return false;
    } else {
      if (op != IPMG_OP_K || !c.fold_prolong || !c.lane_share || !c.fuse_resid || lev != c.L - 1) return false;
      const Dims& d = c.lev[lev].d;
      if (!c.tiled2d || d.nnodes < c.tiled_min_nodes) return false;
      const int nj = c.fp32 ? c.nj32 : c.nj64;
      if (nj != 2 && nj != 4) return false;
      if (c.fp32) {
        if (nj == 4) launch_jacobi2r<float, 4>(c, d, (const float*)r, (float*)out, (float*)t, omg, gate);
        else launch_jacobi2r<float, 2>(c, d, (const float*)r, (float*)out, (float*)t, omg, gate);
      } else {
        if (nj == 4) launch_jacobi2r<double, 4>(c, d, (const double*)r, (double*)out, (double*)t, omg, gate);
        else launch_jacobi2r<double, 2>(c, d, (const double*)r, (double*)out, (double*)t, omg, gate);
      }
      return true;
    }
  }
  template <typename T, int NJ>
  void launch_pjacobi2(Ctx& c, const Dims& d, const Dims& dc, const T* z2, const T* zc, const T* r, T* out,
                       const double* omg, const int* gate, const double* dot64) {
    constexpr int RJ = 4 * NJ;
    const dim3 g((unsigned)((d.nx1 + LS2_COLS - 1) / LS2_COLS), (unsigned)((d.ny1 + RJ - 1) / RJ), 1);
    const unsigned nb = g.x * g.y;
    IPMG_REQUIRE((int64_t)nb <= MAX_PARTIALS, IPMG_E_INVALID, "grid too large for one reduction");
    const OpFineK<2, T> op{(const T*)c.xT, d.m};
    {
      ProfScope ps(c, c.prof_tag);
      if (dot64) k_pjacobi2d<T, NJ, true><<<g, BS, 0, c.stream>>>(op, d, dc, z2, zc, r, out, omg, dot64, c.red, gate);
      else k_pjacobi2d<T, NJ, false><<<g, BS, 0, c.stream>>>(op, d, dc, z2, zc, r, out, omg, dot64, c.red, gate);
    }
    if (dot64)
      k_level_fin<T, M_JACOBI_BETA><<<1, BS, 0, c.stream>>>(z2, r, out, omg, 0, c.cZ, d.nslots, dot64, c.red, nb, 0,
                                                           -1, gate, c.take_flag_dst());
  }
  bool prolong_jacobi2(Ctx& c, int lev, int op, const void* z2, const void* zc, const void* r, void* out,
                       const double* omg, const int* gate, const double* dot64) override {
    if constexpr (DIM != 2) {
      return false;
    } else {
      if (op != IPMG_OP_K || !c.fold_prolong || !c.lane_share || !c.fuse_post || lev != c.L - 1) return false;
      const Dims& d = c.lev[lev].d;
      const Dims& dc = c.lev[lev - 1].d;
      if (!c.tiled2d || d.nnodes < c.tiled_min_nodes) return false;
      const int nj = c.fp32 ? c.nj32 : c.nj64;
      if (nj != 2 && nj != 4) return false;
      using F = float;
      using D = double;
      if (c.fp32 && nj == 4) launch_pjacobi2<F, 4>(c, d, dc, (const F*)z2, (const F*)zc, (const F*)r, (F*)out, omg, gate, dot64);
      else if (c.fp32) launch_pjacobi2<F, 2>(c, d, dc, (const F*)z2, (const F*)zc, (const F*)r, (F*)out, omg, gate, dot64);
      else if (nj == 4) launch_pjacobi2<D, 4>(c, d, dc, (const D*)z2, (const D*)zc, (const D*)r, (D*)out, omg, gate, dot64);
      else launch_pjacobi2<D, 2>(c, d, dc, (const D*)z2, (const D*)zc, (const D*)r, (D*)out, omg, gate, dot64);
      return true;
    }
  }
  bool jacobi2(Ctx& c, int lev, int op, const void* r, void* out, const double* omg, const int* gate) override {
    if constexpr (DIM != 2) {
      return false;
    } else {
      if (op != IPMG_OP_K || !c.fold_prolong || lev != c.L - 1) return false;
      const Dims& d = c.lev[lev].d;
      if (c.fp32) return jacobi2_t<float>(c, d, (const float*)r, (float*)out, omg, gate);
      return jacobi2_t<double>(c, d, (const double*)r, (double*)out, omg, gate);
    }
  }
  bool prolong_jacobi(Ctx& c, int lev, int op, const void* z2, const void* zc, const void* r, void* out,
                      const double* omg, const int* gate) override {
    if constexpr (DIM != 2) {
      return false;
    } else {
      if (op != IPMG_OP_K || !c.fold_prolong) return false;
      const Dims& d = c.lev[lev].d;
      const Dims& dc = c.lev[lev - 1].d;
      if (c.fp32) {
        using T = float;
        if (lev == c.L - 1)
          return pjacobi_t<T>(c, d, dc, OpFineK<2, T>{(const T*)c.xT, d.m}, (const T*)z2, (const T*)zc, (const T*)r,
                              (T*)out, omg, gate);
        if (lev == c.L - 2 && c.coarse_from_x)
          return pjacobi_t<T>(c, d, dc, OpCoarse2K<2, T>{(const T*)c.xT, c.fine().nx, c.fine().m}, (const T*)z2,
                              (const T*)zc, (const T*)r, (T*)out, omg, gate);
        return pjacobi_t<T>(c, d, dc, OpCoarse<2, T>{(const T*)c.lev[lev].E, d.m}, (const T*)z2, (const T*)zc,
                            (const T*)r, (T*)out, omg, gate);
      } else {
        using T = double;
        if (lev == c.L - 1)
          return pjacobi_t<T>(c, d, dc, OpFineK<2, T>{(const T*)c.xT, d.m}, (const T*)z2, (const T*)zc, (const T*)r,
                              (T*)out, omg, gate);
        if (lev == c.L - 2 && c.coarse_from_x)
          return pjacobi_t<T>(c, d, dc, OpCoarse2K<2, T>{(const T*)c.xT, c.fine().nx, c.fine().m}, (const T*)z2,
                              (const T*)zc, (const T*)r, (T*)out, omg, gate);
        return pjacobi_t<T>(c, d, dc, OpCoarse<2, T>{(const T*)c.lev[lev].E, d.m}, (const T*)z2, (const T*)zc,
                            (const T*)r, (T*)out, omg, gate);
      }
    }
  }

  template <typename T, class Op>
  void launch_level(Ctx& c, const Dims& d, const Op& op, int mode, const T* v, const T* r, T* out,
                    const double* omg, Aug<T> aug, int sidx, int sidx_in, const int* gate,
                    const double* dot64 = nullptr) {
    const dim3 g = node_grid(d);
    const unsigned nb = g.x * g.y * g.z;
    IPMG_REQUIRE((int64_t)nb <= MAX_PARTIALS, IPMG_E_INVALID, "grid too large for one reduction");
    const bool fin = (aug.b && mode != M_JACOBI0) || mode == M_POWER || mode == M_RAYLEIGH || mode == M_JACOBI_BETA;
    if constexpr (DIM == 2) {
      // register-blocked tiles pay on large levels; small levels are latency-bound
      // and need one node per thread
      if (mode != M_POWER && mode != M_RAYLEIGH && c.tiled2d && d.nnodes >= c.tiled_min_nodes) {
        const int nj = sizeof(T) == 4 ? c.nj32 : c.nj64;
        if (nj == 1) return launch_l2d<T, Op, 1>(c, d, op, mode, v, r, out, omg, aug, sidx, sidx_in, gate, dot64, fin);
        if (nj == 2) return launch_l2d<T, Op, 2>(c, d, op, mode, v, r, out, omg, aug, sidx, sidx_in, gate, dot64, fin);
        if (nj == 8) return launch_l2d<T, Op, 8>(c, d, op, mode, v, r, out, omg, aug, sidx, sidx_in, gate, dot64, fin);
        return launch_l2d<T, Op, 4>(c, d, op, mode, v, r, out, omg, aug, sidx, sidx_in, gate, dot64, fin);
      }
    }
#define IPMG_LEVEL_CASE(M)                                                                                   \
  case M:                                                                                                    \
    {                                                                                                        \
      ProfScope ps_(c, c.prof_tag);                                                                          \
      k_level<DIM, T, Op, M><<<g, BS, 0, c.stream>>>(op, d, v, r, out, omg, aug, c.red, sidx, sidx_in, dot64, gate); \
    }                                                                                                        \
    if (fin)                                                                                                 \
      k_level_fin<T, M><<<1, BS, 0, c.stream>>>(v, r, out, omg, aug.b != nullptr, aug.c, aug.n, dot64, c.red, nb, \
                                                 sidx, sidx_in, gate,                                       \
                                                 M == M_JACOBI_BETA ? c.take_flag_dst() : nullptr);         \
    break;
    switch (mode) {
      IPMG_LEVEL_CASE(M_APPLY)
      IPMG_LEVEL_CASE(M_RESID)
      IPMG_LEVEL_CASE(M_JACOBI)
      IPMG_LEVEL_CASE(M_JACOBI0)
      IPMG_LEVEL_CASE(M_POWER)
      IPMG_LEVEL_CASE(M_RAYLEIGH)
      IPMG_LEVEL_CASE(M_JACOBI_BETA)
      default: throw Error(IPMG_E_INVALID, "bad level mode");
    }
#undef IPMG_LEVEL_CASE
  }

  // 3D finest level: element products of v into ye (the operator's rows for the
  // node pass) and the set-up diagonal; false when the element passes are off.
  template <typename T, class Op>
  bool fine_elem3(Ctx& c, Op& o, const T* v, T* ye, const T* dgn, const int* gate, int cls) {
    if constexpr (DIM != 3) {
      return false;
    } else {
      if (!ye) return false;
      const Dims& d = c.fine();
      if (v) {
        constexpr bool Z = std::is_same<Op, OpFineZ<3, T>>::value;
        const T* h = nullptr;
        if constexpr (Z) h = o.h;
        ProfScope ps(c, cls);
        k_elem_fine3e<T, Z><<<lin_grid(d.m), BS, 0, c.stream>>>(d, o.x, h, v, ye, gate);
        o.ye = ye;
      }
      o.dgn = dgn;
      return true;
    }
  }

  // The finest-level augmented operator for a pass over v (null: the pass reads
  // no v).  In 3D, h_e'v_e is formed per element first (k_elem_hv) and the pass
  // reads it, instead of every node of an element summing all of h_e again.
  template <typename T>
  OpFineZ<DIM, T> fine_z(Ctx& c, const T* h, const T* v) {
    const Dims& d = c.fine();
    OpFineZ<DIM, T> o{(const T*)(sizeof(T) == 8 ? (const void*)c.x64 : c.xT), h, d.m};
    if (DIM == 3 && c.elem_hv && v) {
      k_elem_hv<DIM, T><<<lin_grid(d.m), BS, 0, c.stream>>>(d, h, v, (T*)c.hsbuf);
      o.hs = (const T*)c.hsbuf;
    }
    return o;
  }

  template <typename T>
  void level_t(Ctx& c, int lev, int op, int mode, const void* v, const void* r, void* out, const double* omg,
               int sidx, int sidx_in, const int* gate, const double* dot64) {
    const Dims& d = c.lev[lev].d;
    Aug<T> aug{op == IPMG_OP_Z ? (const T*)c.lev[lev].bZ : nullptr, c.cZ, d.nslots};
    if (lev == c.L - 1) {
      // 3D: element products first, the diagonal from set-up (formed before the
      // damping estimates)
      const T* vv = mode != M_JACOBI0 ? (const T*)v : nullptr;
      const bool elem = DIM == 3 && c.fine_ye && c.fine_dg;
      if (op == IPMG_OP_K) {
        OpFineK<DIM, T> o{(const T*)c.xT, d.m};
        if (elem) fine_elem3<T>(c, o, vv, (T*)c.fine_ye, (const T*)c.fine_dg, gate, PC_ELEM3);
        launch_level<T>(c, d, o, mode, (const T*)v, (const T*)r, (T*)out, omg, aug, sidx, sidx_in, gate, dot64);
      } else if (elem) {
        OpFineZ<DIM, T> o{(const T*)(sizeof(T) == 8 ? (const void*)c.x64 : c.xT), (const T*)c.hT, d.m};
        fine_elem3<T>(c, o, vv, (T*)c.fine_ye, (const T*)c.fine_dg, gate, PC_ELEM3);
        launch_level<T>(c, d, o, mode, (const T*)v, (const T*)r, (T*)out, omg, aug, sidx, sidx_in, gate, dot64);
      } else {
        launch_level<T>(c, d, fine_z<T>(c, (const T*)c.hT, vv), mode,
                        (const T*)v, (const T*)r, (T*)out, omg, aug, sidx, sidx_in, gate, dot64);
      }
    } else if (DIM == 2 && op == IPMG_OP_K && lev == c.L - 2 && c.coarse_from_x) {
      launch_level<T>(c, d, OpCoarse2K<DIM, T>{(const T*)c.xT, c.fine().nx, c.fine().m}, mode, (const T*)v, (const T*)r,
                      (T*)out, omg, aug, sidx, sidx_in, gate, dot64);
    } else {
      OpCoarse<DIM, T> o{(const T*)c.lev[lev].E, d.m};
      // element products first (levels of 8192 elements and more: below, the
      // extra launch costs more than the gathers it saves)
      if (DIM == 3 && c.ye && mode != M_JACOBI0 && v && d.m >= c.elem_apply3_min) {
        k_elem_apply3<T><<<(unsigned)((d.m + 63) / 64), EA3_THREADS, 0, c.stream>>>(d, o.E, (const T*)v,
                                                                                     (T*)c.ye, gate);
        o.ye = (const T*)c.ye;
      }
      launch_level<T>(c, d, o, mode, (const T*)v, (const T*)r, (T*)out, omg, aug, sidx, sidx_in, gate, dot64);
    }
  }

  void level(Ctx& c, int lev, int op, int mode, const void* v, const void* r, void* out, const double* omg,
             int sidx, int sidx_in, const int* gate, const double* dot64) override {
    if (c.fp32) level_t<float>(c, lev, op, mode, v, r, out, omg, sidx, sidx_in, gate, dot64);
    else level_t<double>(c, lev, op, mode, v, r, out, omg, sidx, sidx_in, gate, dot64);
  }

  template <typename TY, class Op, int NJ>
  void launch_dir2d(Ctx& c, const Op& op, const TY* y, const double* pold, double* p, double* q, Aug<double> aug,
                    int first, const int* gate, double* zs) {
    const Dims& d = c.fine();
    const dim3 g((unsigned)((d.nx1 + 63) / 64), (unsigned)((d.ny1 + 4 * NJ - 1) / (4 * NJ)), 1);
    IPMG_REQUIRE((int64_t)g.x * g.y <= MAX_PARTIALS, IPMG_E_INVALID, "grid too large for one reduction");
    {
      const ProfLaunch pl(c, PC_DIR_APPLY);
      if (zs)
        hipExtLaunchKernelGGL(k_dir_apply2d<TY, Op, NJ, true>, g, dim3(BS), 0, c.stream, pl.t0, pl.t1, 0, op, d, y,
                              pold, p, q, aug, c.red, first, gate, zs);
      else
        hipExtLaunchKernelGGL(k_dir_apply2d<TY, Op, NJ, false>, g, dim3(BS), 0, c.stream, pl.t0, pl.t1, 0, op, d, y,
                              pold, p, q, aug, c.red, first, gate, zs);
    }
    k_dir_fin<TY><<<1, BS, 0, c.stream>>>(y, pold, p, q, aug.b != nullptr, aug.c, d.nslots, first, c.red,
                                          g.x * g.y, gate, zs);
  }
  template <typename TY, class Op>
  void launch_dir_apply(Ctx& c, const Op& op, const TY* y, const double* pold, double* p, double* q,
                        Aug<double> aug, int first, const int* gate, double* zs) {
    const Dims& d = c.fine();
    dim3 g = node_grid(d);
    if constexpr (DIM == 2) {
      if (dir_tiled(c)) {
        if (c.nj_dir == 1) return launch_dir2d<TY, Op, 1>(c, op, y, pold, p, q, aug, first, gate, zs);
        if (c.nj_dir == 4) return launch_dir2d<TY, Op, 4>(c, op, y, pold, p, q, aug, first, gate, zs);
        if (c.nj_dir == 3) return launch_dir2d<TY, Op, 3>(c, op, y, pold, p, q, aug, first, gate, zs);
        return launch_dir2d<TY, Op, 2>(c, op, y, pold, p, q, aug, first, gate, zs);
      }
    }
    IPMG_REQUIRE(!zs, IPMG_E_STATE, "solution update folded into an untiled direction kernel");
    if constexpr (DIM == 3) {
      k_pdir3<TY><<<lin_grid(d.nslots), BS, 0, c.stream>>>(d, y, pold, p, c.red, first, gate);
      Op o = op;
      if (!fine_elem3<double>(c, o, p, c.fine_ye64, nullptr, gate, PC_ELEM3_DIR)) {
        if constexpr (std::is_same<Op, OpFineZ<DIM, double>>::value) o = fine_z<double>(c, c.h64, p);   // h_e'p_e
      }
      ProfScope ps(c, PC_DIR_APPLY);
      k_dir_apply3<TY, Op><<<g, BS, 0, c.stream>>>(o, d, y, pold, p, q, aug, c.red, first, gate);
    } else {
      ProfScope ps(c, PC_DIR_APPLY);
      k_dir_apply<DIM, TY, Op><<<g, BS, 0, c.stream>>>(op, d, y, pold, p, q, aug, c.red, first, gate);
    }
    k_dir_fin<TY><<<1, BS, 0, c.stream>>>(y, pold, p, q, aug.b != nullptr, aug.c, d.nslots, first, c.red,
                                          g.x * g.y * g.z, gate, nullptr);
  }
  bool dir_tiled(const Ctx& c) const { return DIM == 2 && c.tiled2d && c.fine().nnodes >= c.tiled_min_nodes; }
  bool dir_folds_solution(const Ctx& c) const override { return c.fold_solution && dir_tiled(c); }
  void dir_apply(Ctx& c, int op, const void* y, const double* pold, double* p, double* q, int first,
                 const int* gate, double* zs) override {
    const Dims& d = c.fine();
    if (op == IPMG_OP_K) {
      OpFineK<DIM, double> o{c.x64, d.m};
      Aug<double> a{nullptr, 0.0, d.nslots};
      if (c.fp32) launch_dir_apply<float>(c, o, (const float*)y, pold, p, q, a, first, gate, zs);
      else launch_dir_apply<double>(c, o, (const double*)y, pold, p, q, a, first, gate, zs);
    } else {
      OpFineZ<DIM, double> o{c.x64, c.h64, d.m};
      Aug<double> a{c.bZ64, c.cZ, d.nslots};
      if (c.fp32) launch_dir_apply<float>(c, o, (const float*)y, pold, p, q, a, first, gate, zs);
      else launch_dir_apply<double>(c, o, (const double*)y, pold, p, q, a, first, gate, zs);
    }
  }

  void fine_apply64(Ctx& c, int op, const double* v, double* y, const int* gate) override {
    const Dims& d = c.fine();
    if (op == IPMG_OP_K) {
      OpFineK<DIM, double> o{c.x64, d.m};
      fine_elem3<double>(c, o, v, c.fine_ye64, nullptr, gate, -1);
      launch_level<double>(c, d, o, M_APPLY, v, nullptr, y, nullptr, Aug<double>{nullptr, 0.0, d.nslots}, 0, -1,
                           gate);
    } else {
      OpFineZ<DIM, double> o{c.x64, c.h64, d.m};
      if (!fine_elem3<double>(c, o, v, c.fine_ye64, nullptr, gate, -1)) o = fine_z<double>(c, c.h64, v);
      launch_level<double>(c, d, o, M_APPLY, v, nullptr, y, nullptr, Aug<double>{c.bZ64, c.cZ, d.nslots}, 0, -1,
                           gate);
    }
  }

  void fine_diag(Ctx& c, int op) override {
    if constexpr (DIM == 3) {
      if (!c.fine_dg) return;
      const Dims& d = c.fine();
      if (c.fp32) fine_diag_t<float>(c, op, d);
      else fine_diag_t<double>(c, op, d);
    }
  }
  template <typename T>
  void fine_diag_t(Ctx& c, int op, const Dims& d) {
    const unsigned g = lin_grid(d.nnodes);
    if (op == IPMG_OP_K)
      k_fine_diag3<T, OpFineK<DIM, T>><<<g, BS, 0, c.stream>>>(OpFineK<DIM, T>{(const T*)c.xT, d.m}, d, (T*)c.fine_dg);
    else
      k_fine_diag3<T, OpFineZ<DIM, T>><<<g, BS, 0, c.stream>>>(
          OpFineZ<DIM, T>{(const T*)(sizeof(T) == 8 ? (const void*)c.x64 : c.xT), (const T*)c.hT, d.m}, d,
          (T*)c.fine_dg);
  }

  void restrict_to(Ctx& c, int lev_f, const void* rf, void* rc, int aug, const int* gate) override {
    const Dims& f = c.lev[lev_f].d;
    const Dims& cd = c.lev[lev_f - 1].d;
    if (c.fp32)
      k_restrict<DIM, float><<<node_grid(cd), BS, 0, c.stream>>>(f, cd, (const float*)rf, (float*)rc, aug, gate);
    else
      k_restrict<DIM, double><<<node_grid(cd), BS, 0, c.stream>>>(f, cd, (const double*)rf, (double*)rc, aug, gate);
  }
  void restrict64(Ctx& c, int lev_f, const double* rf, double* rc) override {
    const Dims& f = c.lev[lev_f].d;
    const Dims& cd = c.lev[lev_f - 1].d;
    k_restrict<DIM, double, double><<<node_grid(cd), BS, 0, c.stream>>>(f, cd, rf, rc, 0, nullptr);
  }
  void prolong_from(Ctx& c, int lev_f, void* z, const void* zc, int aug, const int* gate) override {
    const Dims& f = c.lev[lev_f].d;
    const Dims& cd = c.lev[lev_f - 1].d;
    if (c.fp32)
      k_prolong<DIM, float><<<node_grid(f), BS, 0, c.stream>>>(f, cd, (float*)z, (const float*)zc, aug, gate);
    else
      k_prolong<DIM, double><<<node_grid(f), BS, 0, c.stream>>>(f, cd, (double*)z, (const double*)zc, aug, gate);
  }

  bool fused_applies(const Ctx& c, int lev, int op) const override {
    if constexpr (DIM != 2) {
      return false;
    } else {
      // Coarse levels only (the finest level's separate register-blocked passes are
      // faster).  The first coarse level formed from the densities is VALU-bound:
      // fused (with its recomputed halos) it pays in FP32 only.
      const bool from_x = lev == c.L - 2 && c.coarse_from_x;
      return c.fused2d && op == IPMG_OP_K && c.desc.nu_pre == 2 && c.desc.nu_post == 2 && lev >= 1 &&
             lev < c.L - 1 && (!from_x || c.fp32);
    }
  }
  // Down pass of a fused coarse level: the first coarse level formed from the
  // densities (k_down2d_x, densities staged in LDS); stored levels below 2^16 nodes
  // with their FP32 element matrices staged in LDS (k_down2d_staged); larger stored
  // levels reading the matrices from global memory (k_down2d).
  template <typename T>
  void fused_down_t(Ctx& c, int lev, const int* gate) {
    const Dims& d = c.lev[lev].d;
    const Dims& dc = c.lev[lev - 1].d;
    const Dims& df = c.fine();
    ProfScope ps(c, lev == c.L - 2 ? PC_SUB_DOWN : -1);
    if constexpr (std::is_same<T, float>::value) {   // (fused_applies: from x in FP32 only)
      if (lev == c.L - 2 && c.coarse_from_x) {
        if (c.down_from_t) {   // restriction of the finest residual done in the tile
          down_x<true>(c, lev, nullptr, df, (const float*)c.down_from_t, (float*)c.lev[lev].r, gate);
          c.down_from_t = nullptr;
        } else {
          down_x<false>(c, lev, (const float*)c.lev[lev].r, df, nullptr, nullptr, gate);
        }
        return;
      }
      if (c.fused_staged && d.nnodes < c.staged_max_nodes) {
        const dim3 gs((unsigned)((dc.nx1 + SCX - 1) / SCX), (unsigned)((dc.ny1 + SCY - 1) / SCY), 1);
        k_down2d_staged<SCX, SCY, SBS_STORED><<<gs, SBS_STORED, 0, c.stream>>>(
            (const float*)c.lev[lev].E, d, dc, (const float*)c.lev[lev].r, (float*)c.lev[lev].z,
            (float*)c.lev[lev - 1].r, c.omega_dev + lev, gate);
        return;
      }
    }
    down_global<T>(c, OpCoarse<2, T>{(const T*)c.lev[lev].E, d.m}, lev, gate);
  }
  // k_down2d on 16x8 or 16x9 coarse-node tiles, whichever runs fewer rounds x area
  // (see pick_tiles).
  template <typename T, class Op>
  void down_global(Ctx& c, const Op& op, int lev, const int* gate) {
    const Dims& d = c.lev[lev].d;
    const Dims& dc = c.lev[lev - 1].d;
    const dim3 g8((unsigned)((dc.nx1 + 15) / 16), (unsigned)((dc.ny1 + 7) / 8), 1);
    const dim3 g9((unsigned)((dc.nx1 + 15) / 16), (unsigned)((dc.ny1 + 8) / 9), 1);
    const bool nine = pick_tiles(c, (const void*)k_down2d<T, Op, 16, 8>, g8, 37 * 21,
                                 (const void*)k_down2d<T, Op, 16, 9>, g9, 37 * 23);
    const T* r = (const T*)c.lev[lev].r;
    T* z = (T*)c.lev[lev].z;
    T* rc = (T*)c.lev[lev - 1].r;
    if (nine) k_down2d<T, Op, 16, 9><<<g9, FBS, 0, c.stream>>>(op, d, dc, r, z, rc, c.omega_dev + lev, gate);
    else k_down2d<T, Op, 16, 8><<<g8, FBS, 0, c.stream>>>(op, d, dc, r, z, rc, c.omega_dev + lev, gate);
  }
  // First coarse level formed from the densities (FP32): k_down2d_m (element
  // products on the matrix cores) or k_down2d_x, on 16x8 or 16x9 coarse-node tiles
  // (see pick_tiles).
  template <bool FROM_T>
  void down_x(Ctx& c, int lev, const float* r, const Dims& df, const float* tf, float* rw, const int* gate) {
    const Dims& d = c.lev[lev].d;
    const Dims& dc = c.lev[lev - 1].d;
    const dim3 g8((unsigned)((dc.nx1 + 15) / 16), (unsigned)((dc.ny1 + 7) / 8), 1);
    const dim3 g9((unsigned)((dc.nx1 + 15) / 16), (unsigned)((dc.ny1 + 8) / 9), 1);
    const float* x = (const float*)c.xT;
    const int fnx = c.fine().nx;
    float* z = (float*)c.lev[lev].z;
    float* rc = (float*)c.lev[lev - 1].r;
    const double* w = c.omega_dev + lev;
    if (c.mfma) {
      if (pick_tiles(c, (const void*)k_down2d_m<FROM_T, 16, 8>, g8, 37 * 21, (const void*)k_down2d_m<FROM_T, 16, 9>,
                     g9, 37 * 23))
        k_down2d_m<FROM_T, 16, 9><<<g9, FBS, 0, c.stream>>>(x, fnx, d, dc, r, z, rc, w, gate, df, tf, rw);
      else
        k_down2d_m<FROM_T, 16, 8><<<g8, FBS, 0, c.stream>>>(x, fnx, d, dc, r, z, rc, w, gate, df, tf, rw);
    } else {
      if (pick_tiles(c, (const void*)k_down2d_x<float, FROM_T, 16, 8>, g8, 37 * 21,
                     (const void*)k_down2d_x<float, FROM_T, 16, 9>, g9, 37 * 23))
        k_down2d_x<float, FROM_T, 16, 9><<<g9, FBS, 0, c.stream>>>(x, fnx, d, dc, r, z, rc, w, gate, df, tf, rw);
      else
        k_down2d_x<float, FROM_T, 16, 8><<<g8, FBS, 0, c.stream>>>(x, fnx, d, dc, r, z, rc, w, gate, df, tf, rw);
    }
  }
  // The down pass of level lev (the first coarse level formed from the densities,
  // FP32) restricts the finest residual itself.
  bool down_restricts(const Ctx& c, int lev, int op) const override {
    if constexpr (DIM != 2) {
      return false;
    } else {
      return c.fold_restrict && c.fp32 && op == IPMG_OP_K && lev == c.L - 2 && c.coarse_from_x &&
             fused_applies(c, lev, op);
    }
  }
  // Up pass of a fused coarse level (the kernels as in fused_down_t).
  template <typename T>
  void fused_up_t(Ctx& c, int lev, const void* zc, void* out, const int* gate) {
    const Dims& d = c.lev[lev].d;
    const Dims& dc = c.lev[lev - 1].d;
    ProfScope ps(c, lev == c.L - 2 ? PC_SUB_UP : -1);
    if constexpr (std::is_same<T, float>::value) {
      if (lev == c.L - 2 && c.coarse_from_x) {
        up_x(c, lev, zc, out, gate);
        return;
      }
      if (c.fused_staged && d.nnodes < c.staged_max_nodes) {
        const dim3 gs((unsigned)((d.nx1 + STX - 1) / STX), (unsigned)((d.ny1 + STY - 1) / STY), 1);
        k_up2d_staged<STX, STY, SBS_STORED><<<gs, SBS_STORED, 0, c.stream>>>(
            (const float*)c.lev[lev].E, d, dc, (const float*)c.lev[lev].r, (const float*)c.lev[lev].z,
            (const float*)zc, (float*)out, c.omega_dev + lev, gate);
        return;
      }
    }
    up_global<T>(c, OpCoarse<2, T>{(const T*)c.lev[lev].E, d.m}, lev, zc, out, gate);
  }
  // k_up2d on 32x16 or 32x18 fine-node tiles (see pick_tiles).
  template <typename T, class Op>
  void up_global(Ctx& c, const Op& op, int lev, const void* zc, void* out, const int* gate) {
    const Dims& d = c.lev[lev].d;
    const Dims& dc = c.lev[lev - 1].d;
    const dim3 g16((unsigned)((d.nx1 + 31) / 32), (unsigned)((d.ny1 + 15) / 16), 1);
    const dim3 g18((unsigned)((d.nx1 + 31) / 32), (unsigned)((d.ny1 + 17) / 18), 1);
    const bool tall = pick_tiles(c, (const void*)k_up2d<T, Op, 32, 16>, g16, 36 * 20,
                                 (const void*)k_up2d<T, Op, 32, 18>, g18, 36 * 22);
    const T* r = (const T*)c.lev[lev].r;
    const T* z2 = (const T*)c.lev[lev].z;
    if (tall)
      k_up2d<T, Op, 32, 18><<<g18, FBS, 0, c.stream>>>(op, d, dc, r, z2, (const T*)zc, (T*)out, c.omega_dev + lev, gate);
    else
      k_up2d<T, Op, 32, 16><<<g16, FBS, 0, c.stream>>>(op, d, dc, r, z2, (const T*)zc, (T*)out, c.omega_dev + lev, gate);
  }
  // First coarse level formed from the densities (FP32): k_up2d_m or k_up2d_x, on
  // 32x16 or 32x18 fine-node tiles (see pick_tiles).
  void up_x(Ctx& c, int lev, const void* zc, void* out, const int* gate) {
    const Dims& d = c.lev[lev].d;
    const Dims& dc = c.lev[lev - 1].d;
    const dim3 g16((unsigned)((d.nx1 + 31) / 32), (unsigned)((d.ny1 + 15) / 16), 1);
    const dim3 g18((unsigned)((d.nx1 + 31) / 32), (unsigned)((d.ny1 + 17) / 18), 1);
    const float* x = (const float*)c.xT;
    const int fnx = c.fine().nx;
    const float* r = (const float*)c.lev[lev].r;
    const float* z2 = (const float*)c.lev[lev].z;
    const float* zf = (const float*)zc;
    float* o = (float*)out;
    const double* w = c.omega_dev + lev;
    if (c.mfma) {
      if (pick_tiles(c, (const void*)k_up2d_m<32, 16>, g16, 36 * 20, (const void*)k_up2d_m<32, 18>, g18, 36 * 22))
        k_up2d_m<32, 18><<<g18, FBS, 0, c.stream>>>(x, fnx, d, dc, r, z2, zf, o, w, gate);
      else
        k_up2d_m<32, 16><<<g16, FBS, 0, c.stream>>>(x, fnx, d, dc, r, z2, zf, o, w, gate);
    } else {
      if (pick_tiles(c, (const void*)k_up2d_x<float, 32, 16>, g16, 36 * 20, (const void*)k_up2d_x<float, 32, 18>, g18,
                     36 * 22))
        k_up2d_x<float, 32, 18><<<g18, FBS, 0, c.stream>>>(x, fnx, d, dc, r, z2, zf, o, w, gate);
      else
        k_up2d_x<float, 32, 16><<<g16, FBS, 0, c.stream>>>(x, fnx, d, dc, r, z2, zf, o, w, gate);
    }
  }
  void fused_down(Ctx& c, int lev, const int* gate) override {
    if constexpr (DIM == 2) {
      if (c.fp32) fused_down_t<float>(c, lev, gate);
      else fused_down_t<double>(c, lev, gate);
    }
  }
  void fused_up(Ctx& c, int lev, const void* zc, void* out, const int* gate) override {
    if constexpr (DIM == 2) {
      if (c.fp32) fused_up_t<float>(c, lev, zc, out, gate);
      else fused_up_t<double>(c, lev, zc, out, gate);
    }
  }

  template <class Op>
  void launch_galerkin(Ctx& c, const Op& op, const Dims& f, const Dims& cd, double* Ec) {
    constexpr int ND = Geo<DIM>::ND;
    const unsigned groups = (unsigned)((cd.m + 63) / 64);
    k_galerkin<DIM, double, Op><<<groups * (ND / GAL_WAVES), 64 * GAL_WAVES, 0, c.stream>>>(op, f, cd, Ec);
  }
  // E64 of level lev_f-1 from level lev_f, accumulated and stored in FP64.
  void galerkin(Ctx& c, int lev_f, int op) override {
    const Dims& f = c.lev[lev_f].d;
    const Dims& cd = c.lev[lev_f - 1].d;
    double* Ec = c.lev[lev_f - 1].E64;
    if (lev_f == c.L - 1) {
      if (op == IPMG_OP_K) launch_galerkin(c, OpFineK<DIM, double>{c.x64, f.m}, f, cd, Ec);
      else launch_galerkin(c, OpFineZ<DIM, double>{c.x64, c.h64, f.m}, f, cd, Ec);
    } else {
      launch_galerkin(c, OpCoarse<DIM, double>{c.lev[lev_f].E64, f.m}, f, cd, Ec);
    }
  }

  void dense_assemble(Ctx& c, int op, double* A, int n) override {
    const Dims& d = c.lev[0].d;
    const int aug = op == IPMG_OP_Z;
    const unsigned g = lin_grid(n);
    if (c.L == 1) {
      if (op == IPMG_OP_K)
        k_dense_assemble<DIM, OpFineK<DIM, double>, double><<<g, BS, 0, c.stream>>>(
            OpFineK<DIM, double>{c.x64, d.m}, d, c.bZ64, c.cZ, aug, A, n);
      else
        k_dense_assemble<DIM, OpFineZ<DIM, double>, double><<<g, BS, 0, c.stream>>>(
            OpFineZ<DIM, double>{c.x64, c.h64, d.m}, d, c.bZ64, c.cZ, aug, A, n);
    } else {
      k_dense_assemble<DIM, OpCoarse<DIM, double>, double><<<g, BS, 0, c.stream>>>(
          OpCoarse<DIM, double>{c.lev[0].E64, d.m}, d, c.lev[0].bZ64, c.cZ, aug, A, n);
    }
  }

  void power_start(Ctx& c, int lev, int aug, void* v) override {
    const Dims& d = c.lev[lev].d;
    if (c.fp32) k_power_start<DIM, float><<<lin_grid(d.nslots + 1), BS, 0, c.stream>>>(d, aug, (float*)v);
    else k_power_start<DIM, double><<<lin_grid(d.nslots + 1), BS, 0, c.stream>>>(d, aug, (double*)v);
  }

  void filter(Ctx& c, double rmin, const double* in, double* out, int mode) override {
    const Dims& d = c.fine();
    const int R = (int)std::ceil(rmin) - 1;
    k_filter<DIM><<<lin_grid(d.m), BS, 0, c.stream>>>(d, rmin, R, in, out, mode);
  }
  void simp_pow(Ctx& c, const double* xt, double p, double* xp, double* q) override {
    k_simp_pow<<<lin_grid(c.fine().m), BS, 0, c.stream>>>(c.fine().m, xt, p, xp, q);
  }

  void oc_energy(Ctx& c, const double* u, const double* x, double q, double* t) override {
    const Dims& d = c.fine();
    k_oc_energy<DIM><<<lin_grid(d.m), BS, 0, c.stream>>>(d, u, x, q, t);
  }

  void element_sens(Ctx& c, const double* w, const double* u, double scale, double* g) override {
    const Dims& d = c.fine();
    k_elem_sens<DIM><<<lin_grid(d.m), BS, 0, c.stream>>>(d, w, u, scale, g);
  }

  void ip_elements(Ctx& c, const double* u, const double* x, const double* phi, const double* psi, double lam,
                   double s, double r, double xbar) override {
    const Dims& d = c.fine();
    IPMG_REQUIRE(lin_grid(d.m) <= (unsigned)MAX_PARTIALS, IPMG_E_INVALID, "grid too large for one reduction");
    if (c.fp32)
      k_ip_elements<DIM, float><<<lin_grid(d.m), BS, 0, c.stream>>>(d, u, x, phi, psi, lam, s, r, xbar, c.ipG3,
                                                                     c.ipW, c.ipSW, c.h64, (float*)c.hT, c.red);
    else
      k_ip_elements<DIM, double><<<lin_grid(d.m), BS, 0, c.stream>>>(d, u, x, phi, psi, lam, s, r, xbar, c.ipG3,
                                                                      c.ipW, c.ipSW, c.h64, nullptr, c.red);
    k_ip_elements_fin<<<1, BS, 0, c.stream>>>(c.red, lin_grid(d.m));
  }
  void ip_nodes(Ctx& c, const double* Ku, const double* f, const double* u, double* rhs) override {
    const Dims& d = c.fine();
    const dim3 g = node_grid(d);
    k_ip_nodes<DIM><<<g, BS, 0, c.stream>>>(d, Ku, f, u, c.ipG3, c.ipSW, c.h64, c.ipV, rhs, c.bZ64, c.red);
    k_ip_nodes_fin<<<1, BS, 0, c.stream>>>(c.red, g.x * g.y * g.z, c.ipV, rhs, d.nslots);
  }
  void ip_recover(Ctx& c, const double* du, const double* x, const double* phi, const double* psi, double s,
                  double r, double xbar, double frac, int all_blocks) override {
    const Dims& d = c.fine();
    k_ip_recover<DIM><<<lin_grid(d.m), BS, 0, c.stream>>>(d, du, x, phi, psi, c.ipG3, c.ipW, c.ipSW, c.h64, s, r,
                                                           xbar, frac, all_blocks, c.ipDx, c.ipDphi, c.ipDpsi, c.red);
    k_ip_recover_fin<<<1, BS, 0, c.stream>>>(c.red, lin_grid(d.m), frac, all_blocks);
  }
  void ip_update(Ctx& c, double* u, const double* du, double* x, double* phi, double* psi) override {
    const Dims& d = c.fine();
    const int64_t n = d.nslots > d.m ? d.nslots : d.m;
    const unsigned g = lin_grid(n) < 2048 ? lin_grid(n) : 2048;
    k_ip_update<DIM><<<g, BS, 0, c.stream>>>(d, u, du, x, phi, psi, c.ipDx, c.ipDphi, c.ipDpsi, c.red);
  }

  void simp_elem(Ctx& c, const double* u, double* g, double* E) override {
    const Dims& d = c.fine();
    k_simp_elem<DIM><<<lin_grid(d.m), BS, 0, c.stream>>>(d, u, g, E);
  }
  void simp_design(Ctx& c, const double* t, const double* x, const double* phi, const double* psi, double lam,
                   double s, double r, double xbar) override {
    const Dims& d = c.fine();
    IPMG_REQUIRE(lin_grid(d.m) <= (unsigned)MAX_PARTIALS, IPMG_E_INVALID, "grid too large for one reduction");
    k_simp_design<<<lin_grid(d.m), BS, 0, c.stream>>>(d.m, t, x, phi, psi, lam, s, r, xbar, c.ipG3, c.ipW, c.red);
    k_ip_elements_fin<<<1, BS, 0, c.stream>>>(c.red, lin_grid(d.m));
  }
  void simp_coef(Ctx& c, const double* cf, const double* Ww, const double* WGw, const double* W2w, const double* g,
                 double* bcoef, double* rcoef) override {
    const Dims& d = c.fine();
    if (c.fp32)
      k_simp_coef<DIM, float><<<lin_grid(d.m), BS, 0, c.stream>>>(d, cf, Ww, WGw, W2w, g, bcoef, rcoef, c.h64,
                                                                  (float*)c.hT, c.red);
    else
      k_simp_coef<DIM, double><<<lin_grid(d.m), BS, 0, c.stream>>>(d, cf, Ww, WGw, W2w, g, bcoef, rcoef, c.h64,
                                                                   nullptr, c.red);
    k_simp_coef_fin<<<1, BS, 0, c.stream>>>(c.red, lin_grid(d.m));
  }
  void simp_nodes(Ctx& c, const double* Ku, const double* f, const double* u, const double* g, const double* bcoef,
                  const double* rcoef, double* rhs) override {
    const Dims& d = c.fine();
    const dim3 gr = node_grid(d);
    k_simp_nodes<DIM><<<gr, BS, 0, c.stream>>>(d, Ku, f, u, g, bcoef, rcoef, rhs, c.bZ64, c.red);
    k_ip_nodes_fin<<<1, BS, 0, c.stream>>>(c.red, gr.x * gr.y * gr.z, c.ipV, rhs, d.nslots);
  }
  void simp_gather(Ctx& c, const double* g, const double* coef, const double* v, double* y) override {
    const Dims& d = c.fine();
    k_simp_gather<DIM><<<node_grid(d), BS, 0, c.stream>>>(d, g, coef, c.bZ64, v, y);
  }
  void simp_recover(Ctx& c, const double* btdu, const double* du, const double* x, const double* phi,
                    const double* psi, double s, double r, double xbar, double frac, int all_blocks) override {
    const Dims& d = c.fine();
    k_simp_recover<<<lin_grid(d.m), BS, 0, c.stream>>>(d.m, d.nslots, btdu, du, x, phi, psi, c.ipG3, c.ipW, s, r,
                                                       xbar, c.ipDx, c.ipDphi, c.ipDpsi, c.red);
    k_ip_recover_fin<<<1, BS, 0, c.stream>>>(c.red, lin_grid(d.m), frac, all_blocks);
  }
};

}  // namespace ipmg

// Internal declarations of the ipmg library (gfx950 / HIP).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <cstdint>
#include <string>
#include <vector>
#include <stdexcept>

#include "../../include/ipmg.h"

namespace ipmg {

// ---------------------------------------------------------------- errors ----
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define IPMG_HIP(call)                                                                 \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      throw ::ipmg::Error(IPMG_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_) + \
                                          " (" __FILE__ ":" + std::to_string(__LINE__) + ")"); \
  } while (0)

#define IPMG_REQUIRE(cond, code, msg) \
  do { if (!(cond)) throw ::ipmg::Error((code), (msg)); } while (0)

// ------------------------------------------------------------ geometry ----
// Element local node a (0..2^dim-1): counter-clockwise on face z, then face z+1.
__host__ __device__ constexpr int loc_x(int a) { return ((a & 3) == 1 || (a & 3) == 2) ? 1 : 0; }
__host__ __device__ constexpr int loc_y(int a) { return (a & 3) >= 2 ? 1 : 0; }
__host__ __device__ constexpr int loc_z(int a) { return a >> 2; }
__host__ __device__ constexpr int loc_index(int ox, int oy, int oz) {
  return 4 * oz + (oy ? (ox ? 2 : 3) : (ox ? 1 : 0));
}

template <int DIM>
struct Geo {
  static constexpr int NN = 1 << DIM;             // nodes per element
  static constexpr int ND = DIM * NN;             // DOFs per element
  static constexpr int NSYM = ND * (ND + 1) / 2;  // packed symmetric element matrix
  static constexpr int NB = DIM == 2 ? 9 : 27;    // node neighbourhood
};

// Packed upper-triangular index of (r, c) in an n x n symmetric matrix.
__host__ __device__ constexpr int sym_index(int r, int c, int n) {
  return r <= c ? r * n - (r * (r - 1)) / 2 + (c - r) : c * n - (c * (c - 1)) / 2 + (r - c);
}

// Neighbourhood index of node offset (dx,dy,dz) in {-1,0,1}^dim.
template <int DIM>
__host__ __device__ constexpr int nb_index(int dx, int dy, int dz) {
  return (DIM == 3 ? (dz + 1) * 9 : 0) + (dy + 1) * 3 + (dx + 1);
}

// Grid of one level: elements per axis and nodes per axis (nz = 0 -> 2D).
struct Dims {
  int nx, ny, nz;      // elements (nz = 1 in 2D for element counts)
  int nx1, ny1, nz1;   // nodes (nz1 = 1 in 2D)
  int64_t nnodes, nslots, m;
};

inline Dims make_dims(int dim, int nx, int ny, int nz) {
  Dims d;
  d.nx = nx; d.ny = ny; d.nz = dim == 3 ? nz : 1;
  d.nx1 = nx + 1; d.ny1 = ny + 1; d.nz1 = dim == 3 ? nz + 1 : 1;
  d.nnodes = (int64_t)d.nx1 * d.ny1 * d.nz1;
  d.nslots = d.nnodes * dim;
  d.m = (int64_t)d.nx * d.ny * d.nz;
  return d;
}

// ----------------------------------------------------------- scratch ----
// Indices into the FP64 device scalar array.
enum Scal {
  S_RHO = 0, S_PQ, S_ALPHA, S_BETA, S_RN2, S_BN2, S_TOL2, S_RHONEW, S_TMP0, S_TMP1, S_TMP2,
  S_TMP3, S_TMP4, S_TMP5, S_TMP6, S_TMP7, S_MIN0, S_MIN1, S_MIN2, S_MIN3,
  S_QY,    // q'y of the current PCG step (q = A p, y the preconditioned residual)
  S_FLEX,  // 1: Polak-Ribiere ratio in PCG, 0: the ratio of Algorithm PCG
  // bisection of the OC update: bracket, last trial, trial count, sum of x_new
  S_OCLO, S_OCHI, S_OCLAM, S_OCSTEPS, S_OCSUM,
  S_COUNT = 32
};
// Indices into the int device flag array.
// F_ZPEND: the solution update z += alpha p of the last PCG step is pending (it
// is folded into the next step's direction kernel).
// F_OCDONE: the bisection of the OC update has narrowed its bracket to tau.
enum Flag { F_DONE = 0, F_ITERS, F_STATUS, F_BAD, F_ZPEND, F_OCDONE, F_COUNT = 8 };
// Trial multipliers of one bisection pass: the midpoints of the next OC_LEVELS
// levels of the bisection tree.
constexpr int OC_LEVELS = 5;
constexpr int OC_CAND = (1 << OC_LEVELS) - 1;
// Reduction counters (one per concurrently pending reduction kind).
enum { C_MAIN = 0, C_AUX, C_COUNT = 8 };

constexpr int BS = 256;           // threads per block for level and vector kernels
constexpr int MAX_PARTIALS = 1 << 16;

struct Red {
  double* partials;   // MAX_PARTIALS * 8 doubles (eight value slots)
  unsigned* counter;  // C_COUNT
  double* scal;       // S_COUNT
  int* flags;         // F_COUNT
};

// Scalar type of the V-cycle.
enum Prec { P64 = 0, P32 = 1 };

// Symmetric matrices of the coarsest-level solve are stored as the tiles (I, J),
// I >= J, of their lower block triangle on DT x DT tiles: every tile row-major and
// contiguous, tiles in row order (tile (I, J) at I(I+1)/2 + J).  The order is
// padded to a multiple of DT with identity rows and columns.
constexpr int DT = 64;
constexpr int DENSE_MAX_N = 6000;                            // largest coarsest-level order
constexpr int DENSE_MAX_TILES = (DENSE_MAX_N + DT - 1) / DT;
__host__ __device__ inline int dense_tiles(int n) { return (n + DT - 1) / DT; }
__host__ __device__ inline int64_t dense_tile_off(int I, int J) {
  return ((int64_t)I * (I + 1) / 2 + J) * (DT * DT);
}
__host__ __device__ inline int64_t dense_packed_size(int n) {
  const int nt = dense_tiles(n);
  return (int64_t)nt * (nt + 1) / 2 * DT * DT;
}
// Offset of entry (r, c), r >= c or both in one diagonal tile (stored in full).
__host__ __device__ inline int64_t dense_lower_at(int r, int c) {
  return dense_tile_off(r / DT, c / DT) + (int64_t)(r % DT) * DT + c % DT;
}
// Offset of entry (r, c), r >= c, when tile (I, J) holds the transpose A_IJ' (the
// working layout of the factorization: its tile products then read every operand
// with the summed index first).
__host__ __device__ inline int64_t dense_lowerT_at(int r, int c) {
  return dense_tile_off(r / DT, c / DT) + (int64_t)(c % DT) * DT + r % DT;
}
// Offset of entry (r, c) of a symmetric matrix whose diagonal tiles are stored in full.
__host__ __device__ inline int64_t dense_sym_at(int r, int c) {
  return r / DT >= c / DT ? dense_lower_at(r, c) : dense_lower_at(c, r);
}

}  // namespace ipmg

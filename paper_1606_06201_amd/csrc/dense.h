// Dense coarsest-level solve (dense.hip): packed lower block-triangular FP64
// matrices on DT x DT tiles (layout beside dense_tiles in common.h).
#pragma once
#include "common.h"

namespace ipmg {

// Every tile of the packed matrix to zero; with pad, identity on the padded rows.
void dense_init(hipStream_t st, double* A, int n, int pad);
// W: the assembled matrix (lower triangle, padded), overwritten by the factor's
// panels; X: L^-1 (packed lower); Ai: A^-1 (packed, diagonal tiles in full);
// Af (optional): A^-1 rounded to FP32, same layout.  A pivot that is not
// positive sets red.flags[F_BAD].
void dense_factor_inverse(hipStream_t st, double* W, double* X, double* Ai, int n, const Red& red,
                          float* Af = nullptr);
// zc = Ai rc (Ai in FP64 or FP32, sums in FP64); part holds
// dense_tiles(n)^2 * DT doubles of per-tile partial sums.
template <typename T, typename M>
void dense_apply(hipStream_t st, const M* Ai, double* part, int n, const T* rc, T* zc, const int* gate);

}  // namespace ipmg

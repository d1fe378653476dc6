// Launchers of the dimension-independent kernels (vec.hip).
#pragma once
#include "common.h"

namespace ipmg {

void vdot(hipStream_t st, const double* a, const double* b, int64_t n, const Red& red, int sidx, const int* gate);
void vdot_alpha(hipStream_t st, const double* p, const double* q, int64_t n, const Red& red, const int* gate);
template <typename T>
void vdot_beta(hipStream_t st, const double* r, const T* y, int64_t n, const Red& red, const int* gate);
template <typename T>
void vdot_store(hipStream_t st, const double* r, const T* y, int64_t n, const Red& red, int sidx, const int* gate);
template <typename T>
void vpcg_update(hipStream_t st, double* z, double* r, const double* p, const double* q, T* rT, int64_t n,
                 const Red& red, const int* gate);   // z may be null; block partials of ||r||^2 ...
// ... summed, done flag; zpend: z was left out (flags[F_ZPEND] set for the next step)
void vpcg_update_fin(hipStream_t st, int64_t n, const Red& red, const int* gate, bool zpend = false);
unsigned vpcg_update_blocks(int64_t n);   // partials vpcg_update writes
void vpcg_update_fin_nb(hipStream_t st, unsigned nblocks, const Red& red, const int* gate, bool zpend);
// z += alpha p if flags[F_ZPEND], then the flag cleared (after the PCG step loop).
void vzflush(hipStream_t st, double* z, const double* p, int64_t n, const Red& red);
template <typename T>
void vpcg_dir(hipStream_t st, double* p, const T* y, int64_t n, const Red& red, int first, const int* gate);
void vsub_norm(hipStream_t st, const double* a, const double* b, double* out, int64_t n, const Red& red, int sidx);
void vmask_copy(hipStream_t st, const double* src, double* dst, int64_t n, int64_t nslots, int dim, int nx1,
                const Red& red, int sidx);
template <typename TD, typename TS>
void vconvert(hipStream_t st, const TS* src, TD* dst, int64_t n, const int* gate);
void vset_tol(hipStream_t st, const Red& red, double rtol);
void vset_rho(hipStream_t st, const Red& red, int sidx);
template <typename T>
void vnormalize(hipStream_t st, T* x, int64_t n, const Red& red, int sidx);
void vfill(hipStream_t st, double* dst, double value, int64_t n);
void vscale(hipStream_t st, double* v, double a, int64_t n);   // v *= a
void vmul(hipStream_t st, const double* a, const double* b, double* out, int64_t n);   // out = a o b
void vlincomb(hipStream_t st, double* out, double a, const double* x, double b, const double* y,
              int64_t n);   // out = a x + b y (out may alias x or y)
void vlam_row(hipStream_t st, double* y, const double* v, const Red& red, int sidx, double c,
              int64_t n);   // y[n] = scal[sidx] + c v[n]
void vcopy_positive(hipStream_t st, const double* src, double* dst, int64_t n, const Red& red);
void vset_omega(hipStream_t st, const Red& red, double* w, double* rho, int s_vav, int s_vdv, double omega,
                double product);
void vfill_small(hipStream_t st, double* w, int n, double value);   // n <= 64
// Bisection of the OC update (Sec. 4): x_new(lambda) = min(t / lambda, xbar) with
// sum x_new = V.  voc_init sets the bracket [0, lam_hi] and the first pass's trial
// tree; each voc_pass evaluates the sums at the OC_CAND trials of the next
// OC_LEVELS bisection levels and walks them in the order of sequential bisection
// (gated once the bracket is narrower than tau); voc_apply writes x_new at the last
// trial (blend: x_new = (blend + x_new) / 2) and its sum into scal[S_OCSUM].
void voc_init(hipStream_t st, const Red& red, double* cand, double lam_hi);
void voc_pass(hipStream_t st, const double* t, int64_t m, double xbar, double V, double tau, double* cand,
              const Red& red);
void voc_apply(hipStream_t st, const double* t, int64_t m, double xbar, const double* blend, double* x_new,
               const Red& red);

}  // namespace ipmg

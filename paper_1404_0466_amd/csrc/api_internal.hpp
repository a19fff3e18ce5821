// Host-side helpers shared by the C-ABI sources (api.hip, batch.hip):
// argument checks, fold split, the fit's pseudo-inverse, hold-out counts.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "kernels.hpp"
#include "pichol.h"

namespace pichol {

pichol_status hip_status(hipError_t e);
size_t align256(size_t b);
bool profiling_on();
bool fold_split(int64_t n, int k, int normalize, FoldSplit* fs);
bool precision_ok(int32_t precision);
bool problem_ok(const pichol_problem* p);
bool samples_ok(const double* lam, int g);
double basis_var(double lam, double lam_ref, int basis);
bool basis_ok(int basis, const double* lam, int n);
bool fit_coef(int g, int r, const double* lam_s, double lam_ref, int basis,
              FitCoef* fc);
void holdout_norm(const pichol_problem* p, HoldoutNorm* hn);
hipError_t upload_tau(const double* lam, int nlam, double lam_ref, int basis,
                      double* dst, hipStream_t stream);

}  // namespace pichol

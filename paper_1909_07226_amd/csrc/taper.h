// Host-side optimal window of image domain gridding (§4.3, Appendix A) and the
// rms window the master-grid image is divided by.
#pragma once

#include <vector>

#include "idg.h"

namespace idg {

// eps^2 below this fraction of the largest eigenvalue is not resolved in float64
constexpr double kTaperMinEps2 = 1e-13;

// Rbar = Qbar o Sbar, L x L row-major, for sample shifts |s| <= max_shift uv pixels.
std::vector<double> taper_error_matrix(int L, double max_shift);

// The eigenvector of Rbar's smallest eigenvalue, scaled to taper[L/2] = 1, and
// eps = sqrt(that eigenvalue).  IDG_OK, or IDG_ERANGE when eps^2 is below
// float64 resolution (the outputs are still written).
int optimal_taper(int L, double max_shift, double *taper, double *epsilon);

// corr[X] = L sqrt(mean_s |f(L X / N, s)|^2), X = 0 .. N-1.
void taper_correction(int L, double max_shift, const double *taper, int N, float *corr);

}  // namespace idg

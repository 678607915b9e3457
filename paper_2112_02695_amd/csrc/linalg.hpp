// FP64 tall-skinny QR and small SVD used by the low-rank step.
#pragma once

#include "internal.hpp"

namespace blr {

// A: column-major rows x r (leading dim lda).  Q (may be null): column-major,
// leading dim ldq, rows x r with orthonormal columns; R_rowmajor (may be
// null): r x r upper triangular with diag >= 0; A = Q R.  Async on ctx stream.
// in_scale multiplies A on load, out_scale multiplies Q on store (A is not
// modified): QR of (in_scale A) with Q scaled by out_scale.
void tsqr(blr_ctx ctx, const double* A, long lda, long rows, int r, double* Q, long ldq,
          double* R_rowmajor, const std::string& tag, double in_scale = 1.0,
          double out_scale = 1.0);

// A = U diag(sig) W^T for an r x r row-major A (U, W row-major; sig descending).
void svd_small(blr_ctx ctx, const double* A, int r, double* U, double* sig, double* W);

}  // namespace blr

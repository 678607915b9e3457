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

// Shifted Cholesky QR in three passes (r <= 16): the first Cholesky
// factorisation is of A^T A + s I with s = 11 (rows r + r (r + 1)) u
// ||A||_F^2, which keeps it defined for any A, and two plain passes on the
// result restore orthogonality to rounding; Gram matrices on the FP64
// matrix cores.  Same contract as tsqr (Q and R_rowmajor required), except
// for numerically rank-deficient A: then flag[0] is set to 1 (never cleared
// here) and Q, R are not valid.
void cholqr(blr_ctx ctx, const double* A, long lda, long rows, int r, double* Q, long ldq,
            double* R_rowmajor, const std::string& tag, double in_scale, double out_scale,
            int* flag);

// A = U diag(sig) W^T for an r x r row-major A (U, W row-major; sig descending).
// trans: factor A^T (A is read transposed).  complete: U's columns of
// underflowing sigma are completed to an orthonormal U (else left zero).
// W0 (used for r > 16; nullptr: the identity): an orthogonal r x r start for
// the right singular vectors, row-major like W.
void svd_small(blr_ctx ctx, const double* A, int r, double* U, double* sig, double* W,
               bool trans = false, bool complete = true, const double* W0 = nullptr);

}  // namespace blr

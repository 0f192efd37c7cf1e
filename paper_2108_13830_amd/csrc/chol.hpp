// chol.hpp -- blocked FP64 Cholesky factorisation and triangular solves.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "common.hpp"

namespace vqmc {

// Device bytes of scratch chol_factor_solve needs for an n x n matrix.
size_t chol_workspace_bytes(int64_t n);

// Factor the SPD matrix M (n x n, row-major with even row stride ld >= n,
// 16-byte aligned; lower triangle read and overwritten by L) and solve
// M x = r, where row n of the same buffer (n + 1 rows in all) holds r on
// entry and is consumed.  x (n) receives the solution; ws holds
// chol_workspace_bytes(n) bytes (16-byte aligned).  *status (device) is set
// to 1 if a pivot is not positive (the factorisation then continues with a
// unit pivot so that every kernel still completes).  Enqueued on st.
vqmc_status chol_factor_solve(double *M, int64_t n, int64_t ld, double *x, void *ws, int *status, hipStream_t st);

}  // namespace vqmc

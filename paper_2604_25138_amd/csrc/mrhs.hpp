// Multi right-hand-side kernel product of the preconditioner fit (mrhs.hip).
#pragma once

#include "internal.hpp"

namespace lk {

// Bytes of the float32 / bfloat16 copy of Z the product reads (n x nr).
size_t mrhs_z_bytes(int64_t n, int nr);

// U = lambda Z + G Z in float32 or bfloat16 arithmetic (prec), from the prepared
// embeddings Eh (n x dp, pre-scaled for exp2, precision prec) and Z (n x nr
// float64, row-major); Zr is scratch of mrhs_z_bytes(n, nr) bytes; U is float64.
hipError_t mrhs_mfma(int prec, int dp, const void* Eh, int64_t n, const double* Z, void* Zr, int nr, double lam,
                     double* U, hipStream_t st);

}  // namespace lk

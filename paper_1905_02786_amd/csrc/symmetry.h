// Device helpers of spatial-symmetry targeting (Abelian irrep labels).
#pragma once
#include "device.h"

namespace mbefci {

// Irrep label of a one-spin string of tuple t (bits: active positions): the
// XOR of its occupied orbitals' labels.  Level shift of determinant (ma, mb)
// away from the target irrep (zero on the target irrep).
__device__ inline int string_irrep(const Batch &b, int t, uint32_t m) {
    int g = 0;
    for (; m; m &= m - 1) g ^= b.orb_irrep[b.act[(int64_t)t * b.nA + __ffs(m) - 1]];
    return g;
}
__device__ inline double sym_pen(const Batch &b, int t, uint32_t ma, uint32_t mb) {
    return (string_irrep(b, t, ma) ^ string_irrep(b, t, mb)) != b.irrep ? b.sym_shift : 0.0;
}

}  // namespace mbefci

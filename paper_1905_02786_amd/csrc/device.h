// Device helpers shared by the kernel sources.
#pragma once
#include "internal.h"

namespace mbefci {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef double dbl2v __attribute__((ext_vector_type(2)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

#define ERI_AT(eri, n, p, q, r, s) (eri)[((((int64_t)(p) * (n) + (q)) * (n) + (r)) * (n) + (s))]

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the block (blockDim.x a multiple of 64, at most 1024); result valid
// in every thread.  `sh` holds >= 16 doubles.
__device__ inline double block_sum(double v, double *sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = blockDim.x >> 6;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    for (int i = 0; i < nw; ++i) r += sh[i];
    return r;
}

__device__ __forceinline__ void pair_of(int P, int &p, int &q) {
    p = 0;
    while ((p + 1) * (p + 2) / 2 <= P) ++p;
    q = P - p * (p + 1) / 2;
}

// First entry i of the new projected-matrix column (V_i . S_m, i <= m) that
// the GEMM's epilogue forms: m when k_ritz supplied the others as S_i . V_m
// (subspace bound <= kSdMax, V_m the correction as k_ritz stored it, i.e. no
// explicit Gram-Schmidt pass changed it afterwards), else 0.
__device__ __forceinline__ int gemm_dot_first(const Batch &b, int t, int m) {
    return (b.max_space <= kSdMax && m > 0 && !b.cgs2[t]) ? m : 0;
}

__device__ __forceinline__ const double *vref(const VecRef &r, int t, int64_t dim) {
    const int32_t k = r.idx ? r.idx[t] : r.idx_const;
    return r.base + (int64_t)t * r.tstride + (int64_t)k * dim;
}

__device__ __forceinline__ void link_decode(uint32_t L, int &J, int &Q, double &sg) {
    J = (int)(L & 0xFFFFFu);
    Q = (int)((L >> 20) & 0x3FFu);
    sg = (L >> 31) ? -1.0 : 1.0;
}

// Block partials of tuple t: [B][nblk + 1][kParts] (the extra block holds the
// P-space corrections of the Davidson reductions).
__device__ __forceinline__ double *parts(const Batch &b, int t, int blk) {
    return b.part + ((int64_t)t * (b.nblk + 1) + blk) * kParts;
}

// (S_- S_+ c)(I_a, I_b) over the active orbitals, with S_- S_+ = N_b -
// sum_pq E^a_qp E^b_pq (the doubly occupied core adds nothing): the diagonal
// (n_b - orbitals holding both spins) c(I), and for each alpha link
// J_a = E_pq I_a (q in I_a, p not) with p in I_b and q not, the beta string
// J_b = E_qp I_b from the dense pair table: - s_a s_b c(J_a, J_b).
__device__ __forceinline__ double spin_ss(const Batch &b, const double *c, int64_t Ia, int64_t Ib) {
    const uint32_t ma = b.strA[Ia], mb = b.strB[Ib];
    const int nA = b.nA, P = b.pl.P;
    double acc = (double)(b.nb - __popc(ma & mb)) * c[Ia * b.Nb + Ib];
    const uint32_t *la = b.linkA + Ia * b.nentA;
    for (int e = 0; e < b.nentA; ++e) {
        const uint32_t L = la[e];
        const int Q = (int)((L >> 20) & 0x3FFu);
        int hi, lo;
        pair_of(Q, hi, lo);
        if (hi == lo) continue;
        const int q = ((ma >> hi) & 1u) ? hi : lo, p = q == hi ? lo : hi;   // q annihilated, p created
        if (!((mb >> p) & 1u) || ((mb >> q) & 1u)) continue;
        const uint32_t eb = b.pairB[Ib * P + nA + Q - hi];   // E_qp on I_b (p in I_b, q not)
        const double x = c[(int64_t)(L & 0xFFFFFu) * b.Nb + (eb & kPairJ)];
        acc += ((L ^ eb) >> 31) ? x : -x;
    }
    return acc;
}

static inline int grid_for(int64_t work, int per_block, int cap) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace mbefci

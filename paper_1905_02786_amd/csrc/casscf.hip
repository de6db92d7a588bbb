// Kernels of the CASSCF expansion reference (Sec. 2: the orbitals of the
// reference space chosen to minimise its CASCI energy): the integrals in
// rotated orbitals phi'_j = sum_i phi_i U_ij, and the Fock matrices that give
// the orbital gradient and the canonical orbitals.
#include "device.h"

namespace mbefci {

// h' = U^T h U; one thread per entry (n <= 64).
__global__ __launch_bounds__(256) void k_rot_h(const double *h, const double *U, double *out, int n) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= n * n) return;
    const int i = idx / n, j = idx % n;
    double s = 0.0;
    for (int p = 0; p < n; ++p) {
        double t = 0.0;
        for (int q = 0; q < n; ++q) t += h[p * n + q] * U[q * n + j];
        s += U[p * n + i] * t;
    }
    out[idx] = s;
}

// One quarter of the four-index transformation: out[j][a] = sum_s in[a][s]
// U[s][j] for the n^3 leading indices a, i.e. the last index is contracted
// with U and the new index moves to the front.  Four passes turn (pq|rs) into
// (ij|kl)'.  A block takes 32 consecutive a and every j: the 32 x n tile of
// `in` and U sit in LDS, each half-wave owns an eighth of the j (U reads are
// broadcasts), each lane one a (writes coalesced along a).
constexpr int kQuarterRows = 32;

__global__ __launch_bounds__(256) void k_quarter(const double *in, const double *U, double *out, int n) {
    __shared__ double X[kQuarterRows][kMaxOrb + 1];
    __shared__ double Us[kMaxOrb][kMaxOrb + 1];
    const int64_t n3 = (int64_t)n * n * n;
    const int64_t a0 = (int64_t)blockIdx.x * kQuarterRows;
    const int tid = threadIdx.x;
    for (int i = tid; i < n * n; i += 256) Us[i / n][i % n] = U[i];
    for (int i = tid; i < kQuarterRows * n; i += 256) {
        const int r = i / n, s = i % n;
        X[r][s] = (a0 + r < n3) ? in[(a0 + r) * n + s] : 0.0;
    }
    __syncthreads();
    const int a = tid & (kQuarterRows - 1), jg = tid / kQuarterRows;   // 8 groups of j
    constexpr int JW = kMaxOrb / 8;
    double acc[JW];
#pragma unroll
    for (int k = 0; k < JW; ++k) acc[k] = 0.0;
    for (int s = 0; s < n; ++s) {
        const double x = X[a][s];
#pragma unroll
        for (int k = 0; k < JW; ++k) {
            const int j = jg + 8 * k;
            if (j < n) acc[k] += x * Us[s][j];
        }
    }
    if (a0 + a < n3) {
#pragma unroll
        for (int k = 0; k < JW; ++k) {
            const int j = jg + 8 * k;
            if (j < n) out[(int64_t)j * n3 + a0 + a] = acc[k];
        }
    }
}

hipError_t launch_rotate_integrals(const double *h0, const double *eri0, const double *U, double *h, double *eri,
                                   double *tmp, int n, hipStream_t s) {
    if (n < 1 || n > kMaxOrb) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_rot_h, dim3((n * n + 255) / 256), dim3(256), 0, s, h0, U, h, n);
    const int64_t n3 = (int64_t)n * n * n;
    const dim3 grid((unsigned)((n3 + kQuarterRows - 1) / kQuarterRows));
    hipLaunchKernelGGL(k_quarter, grid, dim3(256), 0, s, eri0, U, tmp, n);
    hipLaunchKernelGGL(k_quarter, grid, dim3(256), 0, s, (const double *)tmp, U, eri, n);
    hipLaunchKernelGGL(k_quarter, grid, dim3(256), 0, s, (const double *)eri, U, tmp, n);
    hipLaunchKernelGGL(k_quarter, grid, dim3(256), 0, s, (const double *)tmp, U, eri, n);
    return hipGetLastError();
}

// Generalised Fock matrix F_pq = sum_r gamma_pr h_qr + sum_rst Gamma_prst
// (qr|st) (rows p with density only: the frozen, core and active orbitals,
// `occ`; Gamma vanishes unless all its indices are among them) and the Fock
// matrix f_pq = h_pq + sum_rs gamma_rs [(pq|rs) - 1/2 (pr|sq)].  g2h holds
// Gamma / 2 (the gradient accumulators' convention).
__global__ __launch_bounds__(256) void k_fock(const double *h, const double *eri, const double *g1, const double *g2h,
                                              const int32_t *occ, int no, int n, double *F, double *f) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= n * n) return;
    const int p = idx / n, q = idx % n;
    const int64_t n2 = (int64_t)n * n, n3 = n2 * n;
    // Fock matrix (every p)
    double fv = h[idx];
    for (int ri = 0; ri < no; ++ri)
        for (int si = 0; si < no; ++si) {
            const int r = occ[ri], s = occ[si];
            const double g = g1[r * n + s];
            if (g != 0.0) fv += g * (eri[p * n3 + q * n2 + r * n + s] - 0.5 * eri[p * n3 + r * n2 + s * n + q]);
        }
    f[idx] = fv;
    if (!g2h) return;   // the Fock matrix alone
    // generalised Fock matrix (zero rows without density)
    bool has = false;
    for (int i = 0; i < no; ++i) has |= occ[i] == p;
    double Fv = 0.0;
    if (has) {
        for (int ri = 0; ri < no; ++ri) {
            const int r = occ[ri];
            Fv += g1[p * n + r] * h[q * n + r];
            for (int si = 0; si < no; ++si)
                for (int ti = 0; ti < no; ++ti) {
                    const int s = occ[si], t = occ[ti];
                    Fv += 2.0 * g2h[p * n3 + r * n2 + s * n + t] * eri[q * n3 + r * n2 + s * n + t];
                }
        }
    }
    F[idx] = Fv;
}

hipError_t launch_fock(const double *h, const double *eri, const double *g1, const double *g2h, const int32_t *occ,
                       int no, int n, double *F, double *f, hipStream_t s) {
    hipLaunchKernelGGL(k_fock, dim3((n * n + 255) / 256), dim3(256), 0, s, h, eri, g1, g2h, occ, no, n, F, f);
    return hipGetLastError();
}

}  // namespace mbefci

// Base-model energies of tuples: the expansion of eps(S) - eps_base(S) of
// MBE-FCI-b (Sec. 4.2.1, Table 3; the paper's base is CCSD(T), here the
// base is second-order perturbation theory on the tuple's reference
// determinant).  For the determinant Phi of the tuple's CAS with the core
// doubly occupied and the active orbitals of index below n_alpha (n_beta)
// occupied by alpha (beta) electrons, and H0 = sum_p f_p n_p with f the
// diagonal of Phi's spin-orbital Fock operator,
//   eps_base = <Phi|H|Phi>
//            - sum_{sigma, i occ, a virt} f_sigma(a,i)^2 / (f_a - f_i)
//            - sum_{sigma, i<j occ, a<b virt} ((ai|bj) - (aj|bi))^2 / (f_a + f_b - f_i - f_j)
//            - sum_{i occ a, j occ b, a virt a, b virt b} (ai|bj)^2 / (f_a + f_b - f_i - f_j)
// (occupied and virtual within the active orbitals; Slater-Condon couplings
// of single and double excitations).  One workgroup per tuple, on the
// resident full-space integrals.
#include "device.h"

namespace mbefci {

constexpr int kBaseThreads = 256;

__global__ __launch_bounds__(kBaseThreads) void k_base(const double *h, const double *eri, int n, const int32_t *act,
                                                       const int32_t *nact, int sa, const int32_t *core,
                                                       const int32_t *ncore, int sc, int nalpha, int nbeta,
                                                       double e_const, double *out) {
    const int t = blockIdx.x, tid = threadIdx.x;
    const int nA = nact[t], nC = ncore[t];
    const int32_t *A = act + (int64_t)t * sa, *C = core + (int64_t)t * sc;
    const int64_t n2 = (int64_t)n * n, n3 = n2 * n;
    auto E = [&](int p, int q, int r, int s) { return eri[p * n3 + q * n2 + r * n + s]; };
    __shared__ int la[kMaxOrb], lc[kMaxOrb];
    __shared__ double fd[2][kMaxOrb];   // diagonal of the Fock operator (alpha, beta) on the active orbitals
    __shared__ double red[kBaseThreads / 64][2];
    __shared__ int bad[kBaseThreads / 64];
    for (int i = tid; i < nA; i += kBaseThreads) la[i] = A[i];
    for (int i = tid; i < nC; i += kBaseThreads) lc[i] = C[i];
    __syncthreads();
    auto occ = [&](int p, int s) { return p < (s ? nbeta : nalpha); };
    // Fock matrix element f_sigma(p, q) of Phi
    auto fock = [&](int p, int q, int s) {
        double v = h[p * n + q];
        for (int k = 0; k < nC; ++k) {
            const int c = lc[k];
            v += 2.0 * E(p, q, c, c) - E(p, c, c, q);
        }
        for (int k = 0; k < nA; ++k) {
            const int j = la[k];
            const int nj = (j < nalpha) + (j < nbeta);
            if (nj) v += nj * E(p, q, j, j);
            if (occ(j, s)) v -= E(p, j, j, q);
        }
        return v;
    };
    for (int i = tid; i < 2 * nA; i += kBaseThreads) fd[i / nA][i % nA] = fock(la[i % nA], la[i % nA], i / nA);
    __syncthreads();
    double e = 0.0;   // this thread's share of eps_base - e_const
    int nonpos = 0;
    // <Phi|H|Phi>: occupied spin-orbitals of the core and of the active space
    {
        const int no = 2 * nC + 2 * nA;   // (orbital, spin) candidates: core both spins, active both spins
        auto orb = [&](int k, int &p, int &s) -> bool {
            if (k < 2 * nC) {
                p = lc[k >> 1];
                s = k & 1;
                return true;
            }
            k -= 2 * nC;
            p = la[k >> 1];
            s = k & 1;
            return occ(p, s);
        };
        for (int k = tid; k < no; k += kBaseThreads) {
            int p, s;
            if (orb(k, p, s)) e += h[p * n + p];
        }
        for (int kk = tid; kk < no * no; kk += kBaseThreads) {
            const int k1 = kk / no, k2 = kk % no;
            int p, s, q, s2;
            if (!orb(k1, p, s) || !orb(k2, q, s2)) continue;
            e += 0.5 * (E(p, p, q, q) - (s == s2 ? E(p, q, q, p) : 0.0));
        }
    }
    // single excitations i -> a, each spin
    for (int k = tid; k < 2 * nA * nA; k += kBaseThreads) {
        const int s = k / (nA * nA), ia = k % (nA * nA), ii = ia / nA, ai = ia % nA;
        const int i = la[ii], a = la[ai];
        if (!occ(i, s) || occ(a, s)) continue;
        const double den = fd[s][ai] - fd[s][ii];
        if (!(den > 0.0)) {
            nonpos = 1;
            continue;
        }
        const double f = fock(a, i, s);
        e -= f * f / den;
    }
    // double excitations: index quadruples (i, j, a, b) of active orbitals
    const int64_t n4 = (int64_t)nA * nA * nA * nA;
    for (int64_t k = tid; k < 3 * n4; k += kBaseThreads) {
        const int kind = (int)(k / n4);   // 0: alpha alpha, 1: beta beta, 2: alpha beta
        int64_t r = k % n4;
        const int bi = (int)(r % nA);
        r /= nA;
        const int ai = (int)(r % nA);
        r /= nA;
        const int ji = (int)(r % nA);
        const int ii = (int)(r / nA);
        const int i = la[ii], j = la[ji], a = la[ai], b = la[bi];
        double num, den;
        if (kind < 2) {
            const int s = kind;
            if (!(ii < ji && ai < bi) || !occ(i, s) || !occ(j, s) || occ(a, s) || occ(b, s)) continue;
            num = E(a, i, b, j) - E(a, j, b, i);
            den = fd[s][ai] + fd[s][bi] - fd[s][ii] - fd[s][ji];
        } else {
            if (!occ(i, 0) || !occ(j, 1) || occ(a, 0) || occ(b, 1)) continue;
            num = E(a, i, b, j);
            den = fd[0][ai] + fd[1][bi] - fd[0][ii] - fd[1][ji];
        }
        if (!(den > 0.0)) {
            nonpos = 1;
            continue;
        }
        e -= num * num / den;
    }
    // (fixed-order block sum: wave sums, then the waves in order)
    const double we = wave_sum(e);
    const int wnon = __any(nonpos) ? 1 : 0;
    if ((tid & 63) == 0) {
        red[tid >> 6][0] = we;
        bad[tid >> 6] = wnon;
    }
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        int b2 = 0;
        for (int w = 0; w < kBaseThreads / 64; ++w) {
            s += red[w][0];
            b2 |= bad[w];
        }
        out[t] = b2 ? __builtin_nan("") : e_const + s;
    }
}

hipError_t launch_base(const double *h, const double *eri, int n, const int32_t *act, const int32_t *nact, int sa,
                       const int32_t *core, const int32_t *ncore, int sc, int nalpha, int nbeta, double e_const,
                       int ntup, double *out, hipStream_t s) {
    if (ntup <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_base, dim3(ntup), dim3(kBaseThreads), 0, s, h, eri, n, act, nact, sa, core, ncore, sc, nalpha,
                       nbeta, e_const, out);
    return hipGetLastError();
}

}  // namespace mbefci

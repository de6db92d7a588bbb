// HIP kernels (gfx950 / CDNA4, FP64) of the batched CASCI solver.
//
// Every kernel works on a batch of tuples of one shape class (same active
// orbital count and active electron counts, hence the same determinant space
// and string tables); blockIdx.y (or blockIdx.x for per-tuple kernels) selects
// the tuple.  Reductions are block partial sums followed by a fixed-order sum,
// so results do not depend on scheduling.
//
// The active-space Hamiltonian (CASCI of Sec. 2 with a frozen core) is
//   H = E_core + sum_pq k_pq E_pq + 1/2 sum_pqrs (pq|rs) E_pq E_rs,
//   k_pq = h^eff_pq - 1/2 sum_r (pr|rq),  h^eff_pq = h_pq + sum_c [2(pq|cc) - (pc|cq)],
//   E_core = E_const + sum_c 2 h_cc + sum_cd [2(cc|dd) - (cd|dc)],
// over p, q, r, s in A and c in the core C.
#include "device.h"
#include "symmetry.h"

namespace mbefci {

// ---------------------------------------------------------------- gather --
// One block per tuple: E_core, k (pair-packed), diagonal helpers and the
// half-scaled pair matrix 1/2 (pq|rs) zero-padded for the MFMA tiles.
__global__ __launch_bounds__(256) void k_gather(Batch b) {
    const int t = blockIdx.x, tid = threadIdx.x, nth = blockDim.x;
    const ParamLayout &pl = b.pl;
    const int nA = b.nA, nC = b.nC, n = b.norb;
    double *prm = b.params + (int64_t)t * pl.stride;
    __shared__ int sA[kMaxActive], sC[64];
    __shared__ int pp[kMaxActive * (kMaxActive + 1) / 2], qq[kMaxActive * (kMaxActive + 1) / 2];
    __shared__ double heff[kMaxActive * kMaxActive];
    __shared__ double red[16];
    if (tid < nA) sA[tid] = b.act[(int64_t)t * nA + tid];
    if (tid < nC) sC[tid] = b.core[(int64_t)t * nC + tid];
    if (tid < pl.P) {
        int p, q;
        pair_of(tid, p, q);
        pp[tid] = p;
        qq[tid] = q;
    }
    __syncthreads();
    const double *h = b.h, *eri = b.eri;

    double part = 0.0;
    for (int idx = tid; idx < nC + nC * nC; idx += nth) {
        if (idx < nC) {
            const int c = sC[idx];
            part += 2.0 * h[c * n + c];
        } else {
            const int u = idx - nC, c = sC[u / nC], d = sC[u % nC];
            part += 2.0 * ERI_AT(eri, n, c, c, d, d) - ERI_AT(eri, n, c, d, d, c);
        }
    }
    const double ec = block_sum(part, red);
    if (tid == 0) prm[pl.off_ecore] = b.e_const + ec;

    for (int idx = tid; idx < nA * nA; idx += nth) {
        const int ap = sA[idx / nA], aq = sA[idx % nA];
        double v = h[ap * n + aq];
        for (int k = 0; k < nC; ++k) {
            const int c = sC[k];
            v += 2.0 * ERI_AT(eri, n, ap, aq, c, c) - ERI_AT(eri, n, ap, c, c, aq);
        }
        heff[idx] = v;
    }
    __syncthreads();
    for (int idx = tid; idx < pl.P; idx += nth) {
        const int p = pp[idx], q = qq[idx], ap = sA[p], aq = sA[q];
        double v = heff[p * nA + q];
        for (int r = 0; r < nA; ++r) v -= 0.5 * ERI_AT(eri, n, ap, sA[r], sA[r], aq);
        prm[pl.off_k + idx] = v;
    }
    for (int idx = tid; idx < nA; idx += nth) prm[pl.off_hd1 + idx] = heff[idx * nA + idx];
    for (int idx = tid; idx < nA * nA; idx += nth) {
        const int ap = sA[idx / nA], aq = sA[idx % nA];
        prm[pl.off_J + idx] = ERI_AT(eri, n, ap, ap, aq, aq);
        prm[pl.off_K + idx] = ERI_AT(eri, n, ap, aq, aq, ap);
    }
    for (int idx = tid; idx < pl.Ppad * pl.Kpad; idx += nth) {
        const int R = idx / pl.Kpad, Q = idx % pl.Kpad;
        double v = 0.0;
        if (R < pl.P && Q < pl.P)
            v = 0.5 * ERI_AT(eri, n, sA[pp[R]], sA[qq[R]], sA[pp[Q]], sA[qq[Q]]);
        prm[pl.off_eri + idx] = v;
    }
}

hipError_t launch_gather(const Batch &b, hipStream_t s) {
    hipLaunchKernelGGL(k_gather, dim3(b.B), dim3(256), 0, s, b);
    return hipGetLastError();
}

// ----------------------------------------------------------------- hdiag --
// H_II = E_a(Ia) + E_b(Ib) + sum_{i in Ia, j in Ib} (ii|jj), with
// E_s(I) = sum_{i in I} h^eff_ii + 1/2 sum_{i,j in I} [(ii|jj) - (ij|ji)].
__global__ __launch_bounds__(256) void k_hdiag(Batch b, double *out, int64_t ostride, int add_ecore) {
    const int t = blockIdx.y;
    const ParamLayout &pl = b.pl;
    const double *prm = b.params + (int64_t)t * pl.stride;
    __shared__ double hd[kMaxActive], J[kMaxActive * kMaxActive], K[kMaxActive * kMaxActive];
    const int nA = b.nA;
    for (int i = threadIdx.x; i < nA; i += blockDim.x) hd[i] = prm[pl.off_hd1 + i];
    for (int i = threadIdx.x; i < nA * nA; i += blockDim.x) {
        J[i] = prm[pl.off_J + i];
        K[i] = prm[pl.off_K + i];
    }
    __syncthreads();
    const double ec = add_ecore ? prm[pl.off_ecore] : 0.0;
    for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < b.dim;
         d += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t ma = b.strA[d / b.Nb], mb = b.strB[d % b.Nb];
        double e = 0.0;
        for (uint32_t x = ma; x; x &= x - 1) {
            const int i = __ffs(x) - 1;
            e += hd[i];
            for (uint32_t y = ma; y; y &= y - 1) {
                const int j = __ffs(y) - 1;
                e += 0.5 * (J[i * nA + j] - K[i * nA + j]);
            }
            for (uint32_t y = mb; y; y &= y - 1) e += J[i * nA + __ffs(y) - 1];
        }
        for (uint32_t x = mb; x; x &= x - 1) {
            const int i = __ffs(x) - 1;
            e += hd[i];
            for (uint32_t y = mb; y; y &= y - 1) {
                const int j = __ffs(y) - 1;
                e += 0.5 * (J[i * nA + j] - K[i * nA + j]);
            }
        }
        // level shift toward the lowest spin of the sector: lambda times the
        // diagonal of S_- S_+, n_b - (orbitals holding both spins)
        if (b.spin_shift != 0.0) e += b.spin_shift * (double)(b.nb - __popc(ma & mb));
        // level shift away from the other irreps (spatial symmetry targeting)
        if (b.sym_shift != 0.0) e += sym_pen(b, t, ma, mb);
        out[(int64_t)t * ostride + d] = e + ec;
    }
}

hipError_t launch_hdiag(const Batch &b, double *out, int64_t ostride, int add_ecore, hipStream_t s) {
    dim3 grid(grid_for(b.dim, 256, 4096), b.B);
    hipLaunchKernelGGL(k_hdiag, grid, dim3(256), 0, s, b, out, ostride, add_ecore);
    return hipGetLastError();
}

// -------------------------------------------------------------- Davidson --
// Per-tuple state lives in the Batch arrays.  Vector kernels use grid
// (nblk, B) and write block partials to part[t][blk][*]; per-tuple kernels
// (one block of 64 threads per tuple) sum them in block order.

// column sums of the partials for i < nx (thread i), fixed block order
__device__ double sum_parts(const Batch &b, int t, int i) {
    double s = 0.0;
    for (int blk = 0; blk < b.nblk; ++blk) s += parts(b, t, blk)[i];
    return s;
}

// the same plus the P-space correction block (guess norm, Ritz partials)
__device__ double sum_parts_x(const Batch &b, int t, int i) {
    const double s = sum_parts(b, t, i);
    return b.psp > 0 ? s + parts(b, t, b.nblk)[i] : s;
}

// Block-reduce up to NP (<= kParts) per-thread accumulators into partials.
template <int NP = kParts>
__device__ void store_block_partials(const Batch &b, int t, const double *acc, int nx) {
    __shared__ double sh[4][NP];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        if (i < nx) {
            const double v = wave_sum(acc[i]);
            if (lane == 0) sh[w][i] = v;
        }
    }
    __syncthreads();
    if (threadIdx.x < nx) {
        double s = 0.0;
        for (int k = 0; k < 4; ++k) s += sh[k][threadIdx.x];
        parts(b, t, blockIdx.x)[threadIdx.x] = s;
    }
}

// ------------------------------------------------------- P-space ----------
// Davidson preconditioner on the P space of the psp determinants with the
// lowest diagonal energies: the correction there solves (theta - H_PP) t_P =
// r_P exactly (H_PP = Q T Q^T, T tridiagonal, both computed once per tuple),
// elsewhere t = r / (theta - H_II).  The initial guess is the lowest
// eigenvector of H_PP plus the same 1e-3 admixture as the determinant guess
// (none when P is the whole space, where that eigenvector is exact).

// P selection, one block per tuple: histogram of H_II over [min, max] in 1024
// bins, then the determinants of the bins below the one holding the psp-th
// smallest value, and from that bin the lowest indices up to psp, in index
// order (deterministic, ties broken by index).
__global__ __launch_bounds__(256) void k_psp_select(Batch b) {
    const int t = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int n = b.psp;
    const double *hd = b.Hd + (int64_t)t * b.dim;
    int32_t *out = b.pidx + (int64_t)t * kPsp;
    __shared__ double rmin[4], rmax[4];
    __shared__ int hist[1024];
    __shared__ int sB, sC0, sNeed, wc1[4], wc2[4];
    if (b.dim <= n) {
        for (int i = tid; i < n; i += 256) out[i] = i;
        return;
    }
    double mn = 1e300, mx = -1e300;
    for (int64_t d = tid; d < b.dim; d += 256) {
        mn = fmin(mn, hd[d]);
        mx = fmax(mx, hd[d]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mn = fmin(mn, __shfl_xor(mn, o, 64));
        mx = fmax(mx, __shfl_xor(mx, o, 64));
    }
    if (lane == 0) {
        rmin[wv] = mn;
        rmax[wv] = mx;
    }
    for (int i = tid; i < 1024; i += 256) hist[i] = 0;
    __syncthreads();
    mn = fmin(fmin(rmin[0], rmin[1]), fmin(rmin[2], rmin[3]));
    mx = fmax(fmax(rmax[0], rmax[1]), fmax(rmax[2], rmax[3]));
    const double scale = mx > mn ? 1024.0 / (mx - mn) : 0.0;
    auto bin = [&](double v) -> int {
        const int k = (int)((v - mn) * scale);
        return k < 0 ? 0 : (k > 1023 ? 1023 : k);
    };
    for (int64_t d = tid; d < b.dim; d += 256) atomicAdd(&hist[bin(hd[d])], 1);
    __syncthreads();
    if (tid == 0) {
        int c = 0;
        for (int k = 0; k < 1024; ++k) {
            if (c + hist[k] >= n) {
                sB = k;
                sC0 = c;
                sNeed = n - c;
                break;
            }
            c += hist[k];
        }
    }
    __syncthreads();
    const int B = sB, C0 = sC0, need = sNeed;
    int base1 = 0, base2 = 0;
    for (int64_t d0 = 0; d0 < b.dim; d0 += 256) {
        const int64_t d = d0 + tid;
        const int k = d < b.dim ? bin(hd[d]) : 2048;
        const bool f1 = k < B, f2 = k == B;
        const uint64_t m1 = __ballot(f1), m2 = __ballot(f2);
        const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
        const int p1 = __popcll(m1 & below), p2 = __popcll(m2 & below);
        if (lane == 0) {
            wc1[wv] = __popcll(m1);
            wc2[wv] = __popcll(m2);
        }
        __syncthreads();
        int o1 = base1, o2 = base2, t1 = 0, t2 = 0;
        for (int q = 0; q < 4; ++q) {
            if (q < wv) {
                o1 += wc1[q];
                o2 += wc2[q];
            }
            t1 += wc1[q];
            t2 += wc2[q];
        }
        if (f1) out[o1 + p1] = (int32_t)d;
        if (f2 && o2 + p2 < need) out[C0 + o2 + p2] = (int32_t)d;
        base1 += t1;
        base2 += t2;
        __syncthreads();
        if (base1 >= C0 && base2 >= need) break;
    }
}

// One alpha (or beta) string pair <I|E+_P|J>: the pairs P with their
// coefficients (diagonal: the occupied orbitals of I, coefficient 1; a single
// excitation: its pair and sign; otherwise none).  Returns the count.
__device__ __forceinline__ int string_transition(uint32_t mi, uint32_t mj, int *P, double *c) {
    const uint32_t diff = mi ^ mj;
    if (diff == 0u) {
        int k = 0;
        for (uint32_t x = mi; x; x &= x - 1) {
            const int p = __ffs(x) - 1;
            P[k] = p * (p + 3) / 2;
            c[k++] = 1.0;
        }
        return k;
    }
    if (__popc(diff) != 2) return 0;
    const int p = __ffs(mi & diff) - 1, q = __ffs(mj & diff) - 1;   // created in I, annihilated from J
    const int lo = p < q ? p : q, hi = p < q ? q : p;
    const uint32_t between = mj & (((1u << hi) - 1u) & ~((1u << (lo + 1)) - 1u));
    P[0] = hi * (hi + 1) / 2 + lo;
    c[0] = (__popc(between) & 1) ? -1.0 : 1.0;
    return 1;
}

// Sign of the single excitation that turns string J into string I (one
// orbital created in I, one annihilated from J): the parity of J's occupied
// orbitals strictly between the two.
__device__ __forceinline__ double excitation_sign(uint32_t mi, uint32_t mj) {
    const uint32_t diff = mi ^ mj;
    const int p = __ffs(mi & diff) - 1, q = __ffs(mj & diff) - 1;
    const int lo = p < q ? p : q, hi = p < q ? q : p;
    const uint32_t between = mj & (((1u << hi) - 1u) & ~((1u << (lo + 1)) - 1u));
    return (__popc(between) & 1) ? -1.0 : 1.0;
}

// H_PP[i][j] = H_a[Ia][Ja] d(Ib,Jb) + H_b[Ib][Jb] d(Ia,Ja)
//            + sum_PQ (P|Q) <Ia|E+_P|Ja> <Ib|E+_Q|Jb>  (upper triangle, mirrored)
// plus, with a spin level shift, lambda <I|S_- S_+|J>: n_b - (orbitals
// holding both spins) on the diagonal, -s_a s_b where an alpha electron
// moves q <- p and a beta electron p <- q (I = E^a_qp E^b_pq J).
__global__ __launch_bounds__(256) void k_psp_build(Batch b) {
    const int t = blockIdx.x, n = b.psp;
    const ParamLayout &pl = b.pl;
    const double *prm = b.params + (int64_t)t * pl.stride;
    const int32_t *pi = b.pidx + (int64_t)t * kPsp;
    const double *Ha = b.Ha + (int64_t)t * b.Na * b.Na, *Hb = b.Hb + (int64_t)t * b.Nb * b.Nb;
    double *H = b.pQ + (int64_t)t * kPsp * kPsp;
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
        const int i = idx / n, j = idx % n;
        if (j < i) continue;
        const int64_t I = pi[i], J = pi[j];
        const int64_t ia = I / b.Nb, ib = I % b.Nb, ja = J / b.Nb, jb = J % b.Nb;
        double v = 0.0;
        if (ib == jb) v += Ha[ia * b.Na + ja];
        if (ia == ja) v += Hb[ib * b.Nb + jb];
        int Pa[kMaxActive], Pb[kMaxActive];
        double ca[kMaxActive], cb2[kMaxActive];
        const int na = string_transition(b.strA[ia], b.strA[ja], Pa, ca);
        const int nb = na ? string_transition(b.strB[ib], b.strB[jb], Pb, cb2) : 0;
        double x = 0.0;
        for (int u = 0; u < na; ++u)
            for (int w2 = 0; w2 < nb; ++w2) x += ca[u] * cb2[w2] * prm[pl.off_eri + Pa[u] * pl.Kpad + Pb[w2]];
        v += 2.0 * x;   // stored as 1/2 (P|Q)
        if (b.sym_shift != 0.0 && I == J) v += sym_pen(b, t, b.strA[ia], b.strB[ib]);
        if (b.spin_shift != 0.0) {
            const uint32_t mia = b.strA[ia], mja = b.strA[ja], mib = b.strB[ib], mjb = b.strB[jb];
            if (I == J) {
                v += b.spin_shift * (double)(b.nb - __popc(mia & mib));
            } else {
                const uint32_t da = mia ^ mja, db = mib ^ mjb;
                if (__popc(da) == 2 && __popc(db) == 2 && (mia & da) == (mjb & db) && (mja & da) == (mib & db))
                    v -= b.spin_shift * excitation_sign(mia, mja) * excitation_sign(mib, mjb);
            }
        }
        H[i * kPsp + j] = v;
        H[j * kPsp + i] = v;
    }
}

// Householder tridiagonalisation of H_PP in LDS (one block per tuple), Q
// formed explicitly, and the lowest eigenvector of H_PP (multisection on T's
// Sturm counts for the lowest eigenvalue, inverse iteration, y = Q z).  Only
// the lower triangle of the trailing block is kept; the Householder vectors
// stay below the subdiagonal, as in the usual packed storage.
__device__ double block_sum256(double v, double *sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// number of eigenvalues of the symmetric tridiagonal (d, e) below x
__device__ int sturm_count(const double *d, const double *e, int n, double x) {
    int cnt = 0;
    double q = 1.0;
    for (int i = 0; i < n; ++i) {
        q = d[i] - x - (i > 0 ? e[i - 1] * e[i - 1] / q : 0.0);
        if (q == 0.0) q = -1e-300;
        cnt += q < 0.0;
    }
    return cnt;
}

__global__ __launch_bounds__(256) void k_psp_factor(Batch b) {
    const int t = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, n = b.psp;
    constexpr int LD = kPsp + 1;
    extern __shared__ double lds[];
    double *A = lds;                 // [n][LD]
    double *vec = A + kPsp * LD;     // [kPsp] p, then a Householder vector, then z
    double *sh = vec + kPsp;         // [8]
    double *cpv = sh + 8;            // [kPsp] Thomas multipliers
    __shared__ int wcnt[4];
    double *gQ = b.pQ + (int64_t)t * kPsp * kPsp;
    double *dT = b.pT + (int64_t)t * 3 * kPsp, *eT = dT + kPsp, *yv = eT + kPsp;
    for (int i = wv; i < n; i += 4)
        for (int j = lane; j <= i; j += 64) A[i * LD + j] = gQ[i * kPsp + j];
    __syncthreads();
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;
        double *B = A + (k + 1) * LD + (k + 1);   // trailing block, B[i * LD + j] for j <= i
        double *v = A + (k + 1) * LD + k;         // column k below the diagonal, v[i * LD]
        double part = 0.0;
        for (int i = tid; i < m; i += 256) part += v[i * LD] * v[i * LD];
        const double s2 = block_sum256(part, sh);
        const double x0 = v[0];
        const double alpha = x0 > 0.0 ? -sqrt(s2) : sqrt(s2);
        const double v0 = x0 - alpha;
        const double vn2 = s2 - x0 * x0 + v0 * v0;
        __syncthreads();
        if (!(vn2 > 1e-300)) {   // column already reduced: no reflection
            if (tid == 0) eT[k] = x0;
            for (int i = tid; i < m; i += 256) v[i * LD] = 0.0;
            __syncthreads();
            continue;
        }
        if (tid == 0) eT[k] = alpha;
        const double inv = 1.0 / sqrt(vn2);
        for (int i = tid; i < m; i += 256) v[i * LD] = (i == 0 ? v0 : v[i * LD]) * inv;
        __syncthreads();
        // p = B v (B symmetric, lower triangle stored): row i by threads i and
        // i + 128, one half of the columns each (the same trip count on every
        // lane), the halves added in a fixed order
        {
            const int i = tid & 127, hf = tid >> 7, jh = (m + 1) >> 1;
            double acc = 0.0;
            if (i < m) {
                const int j0 = hf ? jh : 0, j1 = hf ? m : jh;
#pragma unroll 8
                for (int j = j0; j < j1; ++j) acc += B[j <= i ? i * LD + j : j * LD + i] * v[j * LD];
            }
            if (hf && i < m) cpv[i] = acc;
            __syncthreads();
            if (!hf && i < m) vec[i] = acc + cpv[i];
        }
        __syncthreads();
        part = 0.0;
        for (int i = tid; i < m; i += 256) part += v[i * LD] * vec[i];
        const double K = block_sum256(part, sh);
        // B -= v w^T + w v^T, w = 2 p - 2 K v (lower triangle)
        for (int i = wv; i < m; i += 4) {
            const double vi = v[i * LD], wi = 2.0 * vec[i] - 2.0 * K * vi;
            for (int j = lane; j <= i; j += 64) {
                const double vj = v[j * LD], wj = 2.0 * vec[j] - 2.0 * K * vj;
                B[i * LD + j] -= vi * wj + wi * vj;
            }
        }
        __syncthreads();
    }
    for (int i = tid; i < n; i += 256) dT[i] = A[i * LD + i];
    if (tid == 0 && n >= 2) eT[n - 2] = A[(n - 1) * LD + n - 2];
    if (tid == 0) eT[n - 1] = 0.0;
    __syncthreads();
    // Q = H_0 ... H_{n-3}, applied right to left to I and formed in place:
    // before H_k only rows and columns > k differ from I, and reflector k
    // lies in column k below the diagonal, outside that block; once H_k is
    // applied, row and column k become those of I.  The block starts as the
    // identity on rows and columns >= n - 2.
    for (int i = tid; i < 4; i += 256) {
        const int r = n - 2 + (i >> 1), c = n - 2 + (i & 1);
        if (r >= 0 && c >= 0) A[r * LD + c] = (r == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int k = n - 3; k >= 0; --k) {
        const int m = n - k - 1, rh = (m + 1) >> 1;
        const double *v = A + (k + 1) * LD + k;   // v[r * LD], r < m
        // column c of the block by threads c and c + 128 (halves of the rows):
        // a_c = 2 v . Q[:, c], then Q[:, c] -= a_c v
        const int ci = tid & 127, hf = tid >> 7, c = k + 1 + ci;
        const int r0 = hf ? rh : 0, r1 = hf ? m : rh;
        double acc = 0.0;
        if (c < n) {
#pragma unroll 8
            for (int r = r0; r < r1; ++r) acc += v[r * LD] * A[(k + 1 + r) * LD + c];
        }
        if (hf && c < n) cpv[ci] = acc;
        __syncthreads();
        if (!hf && c < n) vec[ci] = acc + cpv[ci];
        __syncthreads();
        if (c < n) {
            const double a = 2.0 * vec[ci];
#pragma unroll 8
            for (int r = r0; r < r1; ++r) A[(k + 1 + r) * LD + c] -= a * v[r * LD];
        }
        __syncthreads();
        for (int i = tid; i < n - k; i += 256) {
            A[(k + i) * LD + k] = (i == 0) ? 1.0 : 0.0;
            A[k * LD + k + i] = (i == 0) ? 1.0 : 0.0;
        }
        __syncthreads();
    }
    // lowest eigenvalue of T: Gershgorin bounds, then multisection with 256
    // Sturm counts per round (each round narrows the bracket 257 times)
    if (tid == 0) {
        double lo = 1e300, hi = -1e300;
        for (int i = 0; i < n; ++i) {
            const double r = (i > 0 ? fabs(eT[i - 1]) : 0.0) + (i + 1 < n ? fabs(eT[i]) : 0.0);
            lo = fmin(lo, dT[i] - r);
            hi = fmax(hi, dT[i] + r);
        }
        sh[4] = lo;
        sh[5] = hi;
    }
    __syncthreads();
    double lo = sh[4], hi = sh[5];
    const double span = fmax(hi - lo, 1e-300);
    for (int round = 0; round < 8 && hi - lo > 1e-15 * span; ++round) {
        const double x = lo + (hi - lo) * ((tid + 1) / 257.0);
        const bool below = sturm_count(dT, eT, n, x) < 1;   // no eigenvalue below x
        const uint64_t mk = __ballot(below);
        if (lane == 0) wcnt[wv] = __popcll(mk);
        __syncthreads();
        const int idx = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];   // first point with an eigenvalue below it
        __syncthreads();
        const double nlo = idx > 0 ? lo + (hi - lo) * (idx / 257.0) : lo;
        const double nhi = idx < 256 ? lo + (hi - lo) * ((idx + 1) / 257.0) : hi;
        lo = nlo;
        hi = nhi;
    }
    if (tid == 0) {
        // T - sigma I positive definite; scale is the size of T's entries
        // (floored, so that a zero or one-element T still gives finite pivots)
        const double scale = fmax(span + fabs(lo), 1e-30);
        const double sigma = lo - 1e-10 * scale;
        auto clampp = [scale](double p) { return fabs(p) < 1e-14 * scale ? (p >= 0.0 ? 1e-14 : -1e-14) * scale : p; };
        double *z = vec, *cp = cpv;
        for (int i = 0; i < n; ++i) z[i] = 1.0;
        for (int rep = 0; rep < 3; ++rep) {
            // Thomas on (T - sigma I) z_new = z
            double piv = clampp(dT[0] - sigma);
            cp[0] = (n > 1 ? eT[0] : 0.0) / piv;
            z[0] = z[0] / piv;
            for (int i = 1; i < n; ++i) {
                piv = clampp(dT[i] - sigma - eT[i - 1] * cp[i - 1]);
                cp[i] = (i + 1 < n ? eT[i] : 0.0) / piv;
                z[i] = (z[i] - eT[i - 1] * z[i - 1]) / piv;
            }
            for (int i = n - 2; i >= 0; --i) z[i] -= cp[i] * z[i + 1];
            double mz = 0.0;
            for (int i = 0; i < n; ++i) mz = fmax(mz, fabs(z[i]));
            double nz = 0.0;
            for (int i = 0; i < n; ++i) {
                z[i] /= mz;
                nz += z[i] * z[i];
            }
            nz = 1.0 / sqrt(nz);
            for (int i = 0; i < n; ++i) z[i] *= nz;
        }
    }
    __syncthreads();
    // y = Q z, Q to global
    for (int i = tid; i < n; i += 256) {
        double acc = 0.0;
#pragma unroll 8
        for (int j = 0; j < n; ++j) acc += A[i * LD + j] * vec[j];
        yv[i] = acc;
    }
    double *gQt = b.pQt + (int64_t)t * kPsp * kPsp;
    for (int i = wv; i < n; i += 4)
        for (int j = lane; j < n; j += 64) {
            gQ[i * kPsp + j] = A[i * LD + j];
            gQt[i * kPsp + j] = A[j * LD + i];
        }
}

size_t psp_factor_lds() { return sizeof(double) * ((size_t)kPsp * (kPsp + 1) + 2 * kPsp + 8); }

hipError_t launch_pspace(const Batch &b, hipStream_t s) {
    if (b.psp <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_psp_select, dim3(b.B), dim3(256), 0, s, b);
    hipLaunchKernelGGL(k_psp_build, dim3(b.B), dim3(256), 0, s, b);
    hipLaunchKernelGGL(k_psp_factor, dim3(b.B), dim3(256), psp_factor_lds(), s, b);
    return hipGetLastError();
}

// V_0 += lowest eigenvector of H_PP on the P determinants; the change of
// |V_0|^2 into the extra partial block.
__global__ __launch_bounds__(kPsp) void k_psp_guess(Batch b) {
    const int t = blockIdx.x, i = threadIdx.x, n = b.psp;
    double *v0 = b.V + (int64_t)t * b.max_space * b.dim;
    const double *yv = b.pT + (int64_t)t * 3 * kPsp + 2 * kPsp;
    double dn = 0.0;
    if (i < n) {
        const int64_t d = b.pidx[(int64_t)t * kPsp + i];
        const double o = v0[d], nv = o + yv[i];
        v0[d] = nv;
        dn = nv * nv - o * o;
    }
    __shared__ double sh[2];
    dn = wave_sum(dn);
    if ((i & 63) == 0) sh[i >> 6] = dn;
    __syncthreads();
    if (i == 0) {
        double *px = parts(b, t, b.nblk);
        px[0] = sh[0] + (kPsp > 64 ? sh[1] : 0.0);
    }
}

// After k_ritz: T on the P determinants <- (theta - H_PP)^-1 r_P, solved as
// Q (theta - T)^-1 Q^T r_P (Thomas, pivots kept away from zero like the
// diagonal preconditioner); the changes of |T|^2, of the projections V_i . T
// (on restart the kept vectors' x . T and x2 . T) and of the dots S_i . T
// (Ax . T, A x2 . T) go to the extra partial block.  T is the vector k_ritz
// wrote, V_m (V_restart on restart).
template <int MS>
__global__ __launch_bounds__(kPsp) void k_psp_fix(Batch b) {
    const int t = blockIdx.x, i = threadIdx.x, n = b.psp;
    if (b.status[t] != ST_RUNNING) return;
    const int m = b.m[t], rs = b.restart[t];
    const double th = b.theta[t];
    const double *yy = b.y + (int64_t)t * kMaxSpace;
    const double *V = b.V + (int64_t)t * b.max_space * b.dim;
    const double *S = b.S + (int64_t)t * b.max_space * b.dim;
    double *T = b.V + ((int64_t)t * b.max_space + (rs ? rs : m)) * b.dim;
    const double *Q = b.pQ + (int64_t)t * kPsp * kPsp, *Qt = b.pQt + (int64_t)t * kPsp * kPsp;
    const double *dT = b.pT + (int64_t)t * 3 * kPsp, *eT = dT + kPsp;
    constexpr bool SD = MS <= kSdMax;
    constexpr int NACC = SD ? kSdOff + MS : 2 + MS;
    __shared__ double r[kPsp], w[kPsp], cp[kPsp], red[2][NACC];
    int64_t d = 0;
    double x = 0.0, ax = 0.0, x2 = 0.0, a2 = 0.0, told = 0.0;
    if (i < n) {
        d = b.pidx[(int64_t)t * kPsp + i];
        if (rs) {
            x = V[d];
            ax = S[d];
            if (rs == 2) {
                x2 = V[b.dim + d];
                a2 = S[b.dim + d];
            }
        } else {
#pragma unroll
            for (int k = 0; k < MS; ++k)
                if (k < m) {
                    x += yy[k] * V[(int64_t)k * b.dim + d];
                    ax += yy[k] * S[(int64_t)k * b.dim + d];
                }
        }
        r[i] = ax - th * x;
        told = T[d];
    }
    __syncthreads();
    if (i < n) {
        double s = 0.0;
#pragma unroll 8
        for (int k = 0; k < n; ++k) s += Q[k * kPsp + i] * r[k];
        w[i] = s;
    }
    __syncthreads();
    if (i == 0) {
        auto clampp = [](double p) { return fabs(p) < 1e-8 ? (p >= 0.0 ? 1e-8 : -1e-8) : p; };
        double piv = clampp(th - dT[0]);
        cp[0] = (n > 1 ? -eT[0] : 0.0) / piv;
        w[0] = w[0] / piv;
        for (int k = 1; k < n; ++k) {
            piv = clampp(th - dT[k] + eT[k - 1] * cp[k - 1]);
            cp[k] = (k + 1 < n ? -eT[k] : 0.0) / piv;
            w[k] = (w[k] + eT[k - 1] * w[k - 1]) / piv;
        }
        for (int k = n - 2; k >= 0; --k) w[k] -= cp[k] * w[k + 1];
    }
    __syncthreads();
    double acc[NACC];
#pragma unroll
    for (int k = 0; k < NACC; ++k) acc[k] = 0.0;
    if (i < n) {
        double tv = 0.0;
#pragma unroll 8
        for (int k = 0; k < n; ++k) tv += Qt[k * kPsp + i] * w[k];
        T[d] = tv;
        const double dt = tv - told;
        acc[1] = tv * tv - told * told;
        if (rs) {
            acc[2] = x * dt;
            if (SD) acc[kSdOff] = ax * dt;
            if (rs == 2) {
                acc[3] = x2 * dt;
                if (SD) acc[kSdOff + 1] = a2 * dt;
            }
        } else {
#pragma unroll
            for (int k = 0; k < MS; ++k)
                if (k < m) {
                    acc[2 + k] = V[(int64_t)k * b.dim + d] * dt;
                    if (SD) acc[kSdOff + k] = S[(int64_t)k * b.dim + d] * dt;
                }
        }
    }
    const int nx = (SD ? kSdOff : 2) + (rs ? rs : m);
#pragma unroll
    for (int k = 0; k < NACC; ++k) {
        if (k < nx) {
            const double v = wave_sum(acc[k]);
            if ((i & 63) == 0) red[i >> 6][k] = v;
        }
    }
    __syncthreads();
    if (i < nx) parts(b, t, b.nblk)[i] = red[0][i] + (kPsp > 64 ? red[1][i] : 0.0);
}

__device__ __forceinline__ double guess_noise(int64_t d) {
    uint64_t z = (uint64_t)d + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// block-local minimum of Hd: value and index into partials 0 and 1
__global__ __launch_bounds__(256) void k_guess_min(Batch b) {
    const int t = blockIdx.y;
    const double *hd = b.Hd + (int64_t)t * b.dim;
    double best = 1e300;
    int64_t bi = INT64_MAX;
    for (int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x; d < b.dim; d += (int64_t)gridDim.x * 256) {
        const double v = hd[d];
        if (v < best || (v == best && d < bi)) { best = v; bi = d; }
    }
    __shared__ double sv[256];
    __shared__ int64_t si[256];
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            const double v2 = sv[threadIdx.x + o];
            const int64_t i2 = si[threadIdx.x + o];
            if (v2 < sv[threadIdx.x] || (v2 == sv[threadIdx.x] && i2 < si[threadIdx.x])) {
                sv[threadIdx.x] = v2;
                si[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        parts(b, t, blockIdx.x)[0] = sv[0];
        parts(b, t, blockIdx.x)[1] = (double)si[0];
    }
}

__global__ void k_guess_pick(Batch b) {
    const int t = blockIdx.x;
    if (threadIdx.x != 0) return;
    double best = 1e300, bi = 1e300;
    for (int blk = 0; blk < b.nblk; ++blk) {
        const double v = parts(b, t, blk)[0], i = parts(b, t, blk)[1];
        if (v < best || (v == best && i < bi)) { best = v; bi = i; }
    }
    b.coef[(int64_t)t * kMaxSpace] = bi;
}

// V_0 = e_imin + 1e-3 * noise(d) (with a P space: the noise alone, the P
// eigenvector follows), partial norm^2
__global__ __launch_bounds__(256) void k_guess_fill(Batch b) {
    const int t = blockIdx.y;
    const int64_t imin = (int64_t)b.coef[(int64_t)t * kMaxSpace];
    double *v0 = b.V + (int64_t)t * b.max_space * b.dim;
    // a P space that is the whole space gives the exact eigenvector: no admixture
    const double amp = (b.psp > 0 && b.psp >= b.dim) ? 0.0 : 1e-3;
    double acc[kParts];
    acc[0] = 0.0;
    for (int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x; d < b.dim; d += (int64_t)gridDim.x * 256) {
        const double v = (d == imin && b.psp <= 0 ? 1.0 : 0.0) + amp * guess_noise(d);
        v0[d] = v;
        acc[0] += v * v;
    }
    store_block_partials(b, t, acc, 1);
}

__global__ void k_guess_norm(Batch b) {
    const int t = blockIdx.x;
    if (threadIdx.x == 0) b.coef[(int64_t)t * kMaxSpace] = 1.0 / sqrt(sum_parts_x(b, t, 0));
}

__global__ __launch_bounds__(256) void k_scale_v0(Batch b) {
    const int t = blockIdx.y;
    const double s = b.coef[(int64_t)t * kMaxSpace];
    double *v0 = b.V + (int64_t)t * b.max_space * b.dim;
    for (int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x; d < b.dim; d += (int64_t)gridDim.x * 256)
        v0[d] *= s;
}

hipError_t launch_guess(const Batch &b, hipStream_t s) {
    dim3 grid(b.nblk, b.B);
    hipLaunchKernelGGL(k_guess_min, grid, dim3(256), 0, s, b);
    hipLaunchKernelGGL(k_guess_pick, dim3(b.B), dim3(64), 0, s, b);
    hipLaunchKernelGGL(k_guess_fill, grid, dim3(256), 0, s, b);
    if (b.psp > 0) hipLaunchKernelGGL(k_psp_guess, dim3(b.B), dim3(kPsp), 0, s, b);
    hipLaunchKernelGGL(k_guess_norm, dim3(b.B), dim3(64), 0, s, b);
    hipLaunchKernelGGL(k_scale_v0, grid, dim3(256), 0, s, b);
    return hipGetLastError();
}

__global__ void k_init_state(Batch b) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= b.B) return;
    b.status[t] = ST_RUNNING;
    b.m[t] = 0;              // V_0 holds the guess; its sigma follows, then m = 1
    b.iter[t] = 0;
    b.restart[t] = 0;
    b.theta[t] = 0.0;
    b.theta_prev[t] = 1e300;
    b.R[(int64_t)t * kMaxSpace * kMaxSpace] = 1.0;   // V_0 is normalised: Q_0 = V_0
    double *zp = b.zp + (int64_t)t * kMaxSpace;
    for (int i = 0; i < kMaxSpace; ++i) zp[i] = i == 0 ? 1.0 : 0.0;
    if (t == 0) b.counter[2] = 0;   // explicit Gram-Schmidt passes of the batch
}

hipError_t launch_init_state(const Batch &b, hipStream_t s) {
    hipLaunchKernelGGL(k_init_state, dim3((b.B + 255) / 256), dim3(256), 0, s, b);
    return hipGetLastError();
}

// partial dots V_i . y for i < m[t] + nx_extra (running tuples only; with
// only2, only those whose correction takes the explicit Gram-Schmidt passes)
template <int MS>
__global__ __launch_bounds__(256) void k_dots(Batch b, VecRef yref, int nx_extra, int only2) {
    const int t = blockIdx.y;
    if (b.status[t] != ST_RUNNING || (only2 && !b.cgs2[t])) return;
    const int nx = b.m[t] + nx_extra;
    const double *V = b.V + (int64_t)t * b.max_space * b.dim;
    const double *y = vref(yref, t, b.dim);
    double acc[MS + 1];
#pragma unroll
    for (int i = 0; i < MS + 1; ++i) acc[i] = 0.0;
    for (int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x; d < b.dim; d += (int64_t)gridDim.x * 256) {
        const double yv = y[d];
#pragma unroll
        for (int i = 0; i < MS + 1; ++i)
            if (i < nx) acc[i] += V[(int64_t)i * b.dim + d] * yv;
    }
    store_block_partials<MS + 1>(b, t, acc, nx);
}

// G column m: G[i][m] = G[m][i] = V_i . S_m for i <= m (partial blocks
// 0 .. nsum-1); with `sd`, the entries i < gemm_dot_first of the GEMM's
// epilogue come from the S-dots of k_ritz instead.  Then m += 1.
__global__ void k_update_G(Batch b, int nsum, int sd) {
    const int t = blockIdx.x;
    if (b.status[t] != ST_RUNNING) return;
    const int m = b.m[t];
    double *G = b.G + (int64_t)t * kMaxSpace * kMaxSpace;
    const int i0 = sd ? gemm_dot_first(b, t, m) : 0;
    if ((int)threadIdx.x <= m) {
        double v = 0.0;
        if ((int)threadIdx.x < i0) v = b.sdot[(int64_t)t * kMaxSpace + threadIdx.x];
        else
            for (int blk = 0; blk < nsum; ++blk) v += parts(b, t, blk)[threadIdx.x];
        G[threadIdx.x * kMaxSpace + m] = v;
        G[m * kMaxSpace + threadIdx.x] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) b.m[t] = m + 1;
}

hipError_t launch_dots(const Batch &b, VecRef y, int nx_extra, hipStream_t s) {
    if (b.max_space <= 12) hipLaunchKernelGGL(k_dots<12>, dim3(b.nblk, b.B), dim3(256), 0, s, b, y, nx_extra, 0);
    else hipLaunchKernelGGL(k_dots<kMaxSpace>, dim3(b.nblk, b.B), dim3(256), 0, s, b, y, nx_extra, 0);
    if (nx_extra == 1) hipLaunchKernelGGL(k_update_G, dim3(b.B), dim3(64), 0, s, b, b.nblk, 0);
    return hipGetLastError();
}

hipError_t launch_update_G(const Batch &b, int nsum, hipStream_t s) {
    hipLaunchKernelGGL(k_update_G, dim3(b.B), dim3(64), 0, s, b, nsum, 1);
    return hipGetLastError();
}

// Lowest eigenpair of the m x m projected matrix by cyclic Jacobi with a
// parallel (round-robin) rotation order; one block of 64 threads per tuple.
// The Jacobi matrix is the projection on the orthonormal basis Q = V R,
// R^T G R (upper triangle computed, mirrored); its eigenvector y becomes the
// coefficients R y on the stored basis.  Block 0 also clears the iteration's
// counters (running tuples, explicit Gram-Schmidt passes), which k_converge
// and k_coef1 count after it: no memset node in the iteration's launches.
__global__ __launch_bounds__(64) void k_small_eig(Batch b) {
    const int t = blockIdx.x;
    if (t == 0 && threadIdx.x < 2) b.counter[threadIdx.x] = 0;
    const int32_t st0 = b.status[t];
    if (st0 != ST_RUNNING && st0 != ST_RESTART) return;
    __syncthreads();
    if (threadIdx.x == 0 && st0 == ST_RESTART) b.status[t] = ST_RUNNING;
    const int m = b.m[t];
    const int mm = m + (m & 1);                  // even number of players
    __shared__ double A[kMaxSpace + 1][kMaxSpace + 2];
    __shared__ double Vv[kMaxSpace + 1][kMaxSpace + 2];
    __shared__ double Rs[kMaxSpace][kMaxSpace + 1];
    __shared__ double cs[(kMaxSpace + 2) / 2], sn[(kMaxSpace + 2) / 2];
    __shared__ int pa[(kMaxSpace + 2) / 2], pb[(kMaxSpace + 2) / 2];
    __shared__ int done;
    __shared__ double wv[kMaxSpace];
    const int tid = threadIdx.x;
    const double *G = b.G + (int64_t)t * kMaxSpace * kMaxSpace;
    const double *Rg = b.R + (int64_t)t * kMaxSpace * kMaxSpace;
    // Rs = R (upper triangle, zero below), Vv = G R, then A = R^T (G R)
    for (int i = tid; i < m * m; i += 64) {
        const int r = i / m, c = i % m;
        Rs[r][c] = (r <= c) ? Rg[r * kMaxSpace + c] : 0.0;
    }
    __syncthreads();
    for (int i = tid; i < m * m; i += 64) {
        const int r = i / m, c = i % m;
        double v = 0.0;
        for (int k = 0; k <= c; ++k) v += G[r * kMaxSpace + k] * Rs[k][c];
        Vv[r][c] = v;
    }
    __syncthreads();
    for (int i = tid; i < mm * mm; i += 64) {
        const int r = i / mm, c = i % mm;
        if (r <= c) {
            double v = 0.0;
            if (c < m)
                for (int k = 0; k <= r; ++k) v += Rs[k][r] * Vv[k][c];
            A[r][c] = v;
            A[c][r] = v;
        }
    }
    __syncthreads();
    for (int i = tid; i < mm * mm; i += 64) {
        const int r = i / mm, c = i % mm;
        Vv[r][c] = (r == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    // round-robin schedule: position 0 keeps player 0, positions 1 .. mm-1
    // rotate by one per round (period mm - 1)
    auto player = [&](int pos, int round) { return pos == 0 ? 0 : 1 + (pos - 1 + (mm - 1) - round) % (mm - 1); };
    const int half = mm / 2;
    // rotation loops: for mm <= 16 item idx is pair idx >> 4, row or column
    // idx & 15 (no integer division); larger subspaces use idx / mm, idx % mm
    const bool small = mm <= 16;
    for (int sweep = 0; sweep < 30; ++sweep) {
        {
            // off-diagonal and total squared norms (lane-parallel, fixed order)
            double off = 0.0, tot = 0.0;
            for (int i = tid; i < m * m; i += 64) {
                const int r = i / m, c = i % m;
                const double a2 = A[r][c] * A[r][c];
                tot += a2;
                if (r != c) off += a2;
            }
            off = wave_sum(off);
            tot = wave_sum(tot);
            if (tid == 0) done = (off <= 1e-30 * tot) ? 1 : 0;   // off-diagonal norm <= 1e-15 of the total
        }
        __syncthreads();
        if (done) break;
        for (int round = 0; round < mm - 1; ++round) {
            if (tid < half) {
                int p = player(tid, round), q = player(mm - 1 - tid, round);
                if (p > q) { const int x = p; p = q; q = x; }
                double c = 1.0, s = 0.0;
                if (q < m && A[p][q] != 0.0) {
                    const double apq = A[p][q];
                    const double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
                    const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + tt * tt);
                    s = tt * c;
                }
                cs[tid] = c;
                sn[tid] = s;
                pa[tid] = p;
                pb[tid] = q;
            }
            __syncthreads();
            // columns: A <- A J, V <- V J
            for (int idx = tid; idx < half * (small ? 16 : mm); idx += 64) {
                const int k = small ? idx >> 4 : idx / mm, r = small ? idx & 15 : idx % mm;
                if (r >= mm) continue;
                const int p = pa[k], q = pb[k];
                const double c = cs[k], s = sn[k];
                const double arp = A[r][p], arq = A[r][q];
                A[r][p] = c * arp - s * arq;
                A[r][q] = s * arp + c * arq;
                const double vrp = Vv[r][p], vrq = Vv[r][q];
                Vv[r][p] = c * vrp - s * vrq;
                Vv[r][q] = s * vrp + c * vrq;
            }
            __syncthreads();
            // rows: A <- J^T A
            for (int idx = tid; idx < half * (small ? 16 : mm); idx += 64) {
                const int k = small ? idx >> 4 : idx / mm, col = small ? idx & 15 : idx % mm;
                if (col >= mm) continue;
                const int p = pa[k], q = pb[k];
                const double c = cs[k], s = sn[k];
                const double apc = A[p][col], aqc = A[q][col];
                A[p][col] = c * apc - s * aqc;
                A[q][col] = s * apc + c * aqc;
            }
            __syncthreads();
        }
    }
    if (tid == 0) {
        int k = 0;
        for (int i = 1; i < m; ++i)
            if (A[i][i] < A[k][k]) k = i;
        b.theta[t] = A[k][k];
        double *y = b.y + (int64_t)t * kMaxSpace;
        for (int i = 0; i < m; ++i) {
            double v = 0.0;
            for (int j = i; j < m; ++j) v += Rs[i][j] * Vv[j][k];
            y[i] = v;
        }
        // A restart keeps the Ritz vector and, with restart_keep 2, the
        // previous iteration's Ritz vector (zp, coordinates of Q, zero past
        // its length) made orthogonal to it by two passes in these
        // coordinates; kept when that leaves a norm above 1e-6.  Its
        // Rayleigh quotient comes from the eigen-decomposition of the
        // projected matrix (A's diagonal, eigenvectors Vv), its coefficients
        // on the stored basis are R w.  The two are orthonormal and the
        // projected matrix on them is diag(theta, mu).
        const bool rs = m >= b.max_space || st0 == ST_RESTART;
        double *zp = b.zp + (int64_t)t * kMaxSpace;
        int keep = rs ? 1 : 0;
        if (rs && b.restart_keep > 1) {
            for (int i = 0; i < m; ++i) wv[i] = zp[i];
            for (int pass = 0; pass < 2; ++pass) {
                double d = 0.0;
                for (int i = 0; i < m; ++i) d += Vv[i][k] * wv[i];
                for (int i = 0; i < m; ++i) wv[i] -= d * Vv[i][k];
            }
            double nw = 0.0;
            for (int i = 0; i < m; ++i) nw += wv[i] * wv[i];
            if (nw > 1e-12) {
                const double sc = 1.0 / sqrt(nw);
                for (int i = 0; i < m; ++i) wv[i] *= sc;
                double mu = 0.0;
                for (int j = 0; j < m; ++j) {
                    double cj = 0.0;
                    for (int i = 0; i < m; ++i) cj += Vv[i][j] * wv[i];
                    mu += cj * cj * A[j][j];
                }
                b.mu[t] = mu;
                double *y2 = b.y2 + (int64_t)t * kMaxSpace;
                for (int i = 0; i < m; ++i) {
                    double v = 0.0;
                    for (int j = i; j < m; ++j) v += Rs[i][j] * wv[j];
                    y2[i] = v;
                }
                keep = 2;
            }
        }
        if (!rs)
            for (int i = 0; i < kMaxSpace; ++i) zp[i] = i < m ? Vv[i][k] : 0.0;
        b.restart[t] = keep;
    }
}

template <int MS, bool V2, bool K2>
__device__ __forceinline__ void ritz_body(const Batch &b, int t, int m, int rs) {
    const double th = b.theta[t];
    const double *yv = b.y + (int64_t)t * kMaxSpace, *zv = b.y2 + (int64_t)t * kMaxSpace;
    double yy[MS], zz[MS];
#pragma unroll
    for (int i = 0; i < MS; ++i) {
        yy[i] = (i < m) ? yv[i] : 0.0;
        zz[i] = (K2 && i < m) ? zv[i] : 0.0;
    }
    double *V = b.V + (int64_t)t * b.max_space * b.dim;
    double *S = b.S + (int64_t)t * b.max_space * b.dim;
    const double *hd = b.Hd + (int64_t)t * b.dim;
    double *T = V + (int64_t)(rs ? rs : m) * b.dim;
    constexpr bool SD = MS <= kSdMax;
    constexpr int NACC = SD ? kSdOff + MS : 2 + MS;
    double acc[NACC];
#pragma unroll
    for (int i = 0; i < NACC; ++i) acc[i] = 0.0;
    // one determinant: Ritz vector, residual, preconditioned correction, its
    // projections on the basis and its dots with the basis' sigma vectors
    auto one = [&](const double (&vd)[MS], const double (&sd)[MS], double x, double ax, double x2, double a2,
                   double h) -> double {
        const double r = ax - th * x;
        acc[0] += r * r;
        double den = th - h;
        if (fabs(den) < 1e-8) den = (den >= 0.0) ? 1e-8 : -1e-8;
        const double tv = r / den;
        acc[1] += tv * tv;
        if (rs) {
            acc[2] += x * tv;
            if (SD) acc[kSdOff] += ax * tv;
            if (K2) {
                acc[3] += x2 * tv;
                if (SD) acc[kSdOff + 1] += a2 * tv;
            }
        } else {
            // (vd[i] = sd[i] = 0 for i >= m: those sums stay unused)
#pragma unroll
            for (int i = 0; i < MS; ++i) {
                acc[2 + i] += vd[i] * tv;
                if (SD) acc[kSdOff + i] += sd[i] * tv;
            }
        }
        return tv;
    };
    // V_i and S_i, i < m, through buffer resources that end after vector m - 1:
    // the loads of vectors past m read zero, so every load of a determinant is
    // issued at once (no branch on m between them); the added terms are
    // exact zeros (yy[i] = 0 there)
    const int vbytes = (int)((int64_t)m * b.dim * (int64_t)sizeof(double));
    const __amdgpu_buffer_rsrc_t rV = __builtin_amdgcn_make_buffer_rsrc(V, (short)0, vbytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t rS = __builtin_amdgcn_make_buffer_rsrc(S, (short)0, vbytes, 0x00020000);
    const uint32_t vstride = (uint32_t)b.dim * (uint32_t)sizeof(double);
    if (V2) {
        // pairs of determinants with 16-byte loads (dim even: every vector 16-byte aligned)
        typedef double dbl2 __attribute__((ext_vector_type(2)));
        const int64_t n2 = b.dim >> 1;
        for (int64_t d2 = (int64_t)blockIdx.x * 256 + threadIdx.x; d2 < n2; d2 += (int64_t)gridDim.x * 256) {
            const int64_t d = d2 << 1;
            const uint32_t vo = (uint32_t)d * (uint32_t)sizeof(double);
            double v0[MS], v1[MS], s0[MS], s1[MS];
            double x0 = 0.0, x1 = 0.0, a0 = 0.0, a1 = 0.0, z0 = 0.0, z1 = 0.0, c0 = 0.0, c1 = 0.0;
            dbl2 vv[MS], ss[MS];
#pragma unroll
            for (int i = 0; i < MS; ++i) {
                vv[i] = __builtin_bit_cast(dbl2, __builtin_amdgcn_raw_buffer_load_b128(rV, vo, (uint32_t)i * vstride, 0));
                ss[i] = __builtin_bit_cast(dbl2, __builtin_amdgcn_raw_buffer_load_b128(rS, vo, (uint32_t)i * vstride, 0));
            }
#pragma unroll
            for (int i = 0; i < MS; ++i) {
                v0[i] = vv[i].x;
                v1[i] = vv[i].y;
                s0[i] = ss[i].x;
                s1[i] = ss[i].y;
                x0 += yy[i] * vv[i].x;
                x1 += yy[i] * vv[i].y;
                a0 += yy[i] * ss[i].x;
                a1 += yy[i] * ss[i].y;
                if (K2) {
                    z0 += zz[i] * vv[i].x;
                    z1 += zz[i] * vv[i].y;
                    c0 += zz[i] * ss[i].x;
                    c1 += zz[i] * ss[i].y;
                }
            }
            const dbl2 h = *reinterpret_cast<const dbl2 *>(hd + d);
            const double t0 = one(v0, s0, x0, a0, z0, c0, h.x);
            const double t1 = one(v1, s1, x1, a1, z1, c1, h.y);
            *reinterpret_cast<dbl2 *>(T + d) = dbl2{t0, t1};
            if (rs) {
                *reinterpret_cast<dbl2 *>(V + d) = dbl2{x0, x1};
                *reinterpret_cast<dbl2 *>(S + d) = dbl2{a0, a1};
                if (K2) {
                    *reinterpret_cast<dbl2 *>(V + b.dim + d) = dbl2{z0, z1};
                    *reinterpret_cast<dbl2 *>(S + b.dim + d) = dbl2{c0, c1};
                }
            }
        }
    } else {
        for (int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x; d < b.dim; d += (int64_t)gridDim.x * 256) {
            const uint32_t vo = (uint32_t)d * (uint32_t)sizeof(double);
            double x = 0.0, ax = 0.0, x2 = 0.0, a2 = 0.0, vd[MS], sd[MS];
#pragma unroll
            for (int i = 0; i < MS; ++i) {
                vd[i] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rV, vo, (uint32_t)i * vstride, 0));
                sd[i] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rS, vo, (uint32_t)i * vstride, 0));
            }
#pragma unroll
            for (int i = 0; i < MS; ++i) {
                x += yy[i] * vd[i];
                ax += yy[i] * sd[i];
                if (K2) {
                    x2 += zz[i] * vd[i];
                    a2 += zz[i] * sd[i];
                }
            }
            T[d] = one(vd, sd, x, ax, x2, a2, hd[d]);
            if (rs) {
                V[d] = x;
                S[d] = ax;
                if (K2) {
                    V[b.dim + d] = x2;
                    S[b.dim + d] = a2;
                }
            }
        }
    }
    store_block_partials<NACC>(b, t, acc, (SD ? kSdOff : 2) + (rs ? rs : m));
}

// x = V y, Ax = S y, r = Ax - theta x, T = r / (theta - Hd) (clamped);
// partials |r|^2, |T|^2 and the projections V_i . T on the subspace the
// correction is added to (V_i, i < m, or on restart the kept vectors: x, and
// x2 = V y2 when restart = 2), and for MS <= kSdMax the dots S_i . T (Ax . T,
// A x2 . T on restart) from partial kSdOff.  T is stored as the next basis
// vector itself: V_m, or V_restart on restart, where V_0 <- x, S_0 <- Ax (and
// V_1 <- x2, S_1 <- A x2) in place (each thread owns its d and reads every
// vector there before it writes).
template <int MS, bool V2>
__global__ __launch_bounds__(256) void k_ritz(Batch b) {
    const int t = blockIdx.y;
    if (b.status[t] != ST_RUNNING) return;
    const int m = b.m[t], rs = b.restart[t];
    if (rs == 2) ritz_body<MS, V2, true>(b, t, m, rs);
    else ritz_body<MS, V2, false>(b, t, m, rs);
}

// convergence test, restart bookkeeping, running count
__global__ void k_converge(Batch b) {
    const int t = blockIdx.x;
    if (threadIdx.x != 0 || b.status[t] != ST_RUNNING) return;
    const double rn = sqrt(sum_parts(b, t, 0));
    const double th = b.theta[t];
    b.rnorm[t] = rn;
    b.tnorm0[t] = sqrt(sum_parts_x(b, t, 1));
    int st = ST_RUNNING;
    if (!isfinite(rn) || !isfinite(th)) st = ST_NONFINITE;
    else if (rn < b.r_tol && fabs(th - b.theta_prev[t]) < b.e_tol) st = ST_DONE;
    const int it = b.iter[t] + 1;
    b.iter[t] = it;
    if (st == ST_RUNNING && it >= b.max_iter) st = ST_MAXITER;
    b.theta_prev[t] = th;
    const int keep = b.restart[t];
    if (keep) {   // V_0 = x, S_0 = A x (and V_1, S_1 the kept direction) already written
        b.m[t] = keep;
        double *G = b.G + (int64_t)t * kMaxSpace * kMaxSpace, *R = b.R + (int64_t)t * kMaxSpace * kMaxSpace;
        double *y = b.y + (int64_t)t * kMaxSpace, *zp = b.zp + (int64_t)t * kMaxSpace;
        G[0] = th;
        R[0] = 1.0;   // x = Q y has unit norm
        y[0] = 1.0;
        if (keep == 2) {
            G[1] = G[kMaxSpace] = 0.0;
            G[kMaxSpace + 1] = b.mu[t];
            R[1] = 0.0;
            R[kMaxSpace + 1] = 1.0;
            y[1] = 0.0;
        }
        for (int i = 0; i < kMaxSpace; ++i) zp[i] = i == 0 ? 1.0 : 0.0;   // x, in the new coordinates
    }
    b.status[t] = st;
    if (st == ST_RUNNING) atomicAdd(b.counter, 1);
}

// The correction T = V_m on the orthonormal basis: c = Q^T T = R^T d with d
// the projections V_i . T (partials 2..m+1 of k_ritz), and the norm outside
// the subspace, kept = |T|^2 - |c|^2.  When that keeps at least half of
// |T|^2 (Kahan's criterion for one classical Gram-Schmidt pass; the
// difference of squares is then accurate to a few ulps) T joins the basis
// unchanged: V = Q U gains the column (c, sqrt(kept)), so R = U^-1 gains
// (-R c, 1) / sqrt(kept), and no vector pass is needed.  Otherwise cgs2 is set,
// coef = R c (T - V R c is T's part outside the subspace) and the explicit
// second pass and k_tnorm decide.  One block of 64 threads (one wave) per
// tuple; every lane takes the same decision (the butterfly sums are equal in
// every lane).
__global__ void k_coef1(Batch b) {
    const int t = blockIdx.x;
    if (b.status[t] != ST_RUNNING) return;
    const int m = b.m[t], i = threadIdx.x;
    double *R = b.R + (int64_t)t * kMaxSpace * kMaxSpace;
    __shared__ double dv[kMaxSpace], cv[kMaxSpace];
    if (i < m) {
        dv[i] = sum_parts_x(b, t, 2 + i);
        if (b.max_space <= kSdMax) b.sdot[(int64_t)t * kMaxSpace + i] = sum_parts_x(b, t, kSdOff + i);
    }
    __syncthreads();
    double c = 0.0;
    if (i < m) {
        for (int j = 0; j <= i; ++j) c += R[j * kMaxSpace + i] * dv[j];
        cv[i] = c;
    }
    const double c2 = wave_sum(c * c);
    __syncthreads();
    double a = 0.0;   // (R c)_i
    if (i < m)
        for (int j = i; j < m; ++j) a += R[i * kMaxSpace + j] * cv[j];
    const double t2 = b.tnorm0[t] * b.tnorm0[t];
    const double kept = t2 - c2;
    const int two = !(kept >= 0.5 * t2);
    if (i == 0) b.cgs2[t] = two;
    if (two) {
        if (i < m) b.coef[(int64_t)t * kMaxSpace + i] = a;
        if (i == 0) {
            atomicAdd(b.counter + 1, 1);   // this iteration (the profiled loop launches the passes only then)
            atomicAdd(b.counter + 2, 1);   // the whole batch
        }
        return;
    }
    if (!(kept > 1e-300) || m >= b.max_space) {
        if (i == 0) b.status[t] = b.rnorm[t] < b.r_tol ? ST_DONE : (m > 1 ? ST_RESTART : ST_STALLED);
        return;
    }
    const double s = 1.0 / sqrt(kept);
    if (i < m) R[i * kMaxSpace + m] = -a * s;
    if (i == m) R[m * kMaxSpace + m] = s;
}

hipError_t launch_iter_head(const Batch &b, hipStream_t s) {
    hipLaunchKernelGGL(k_small_eig, dim3(b.B), dim3(64), 0, s, b);
    const bool v2 = (b.dim & 1) == 0;
    if (b.max_space <= 12) {
        if (v2) hipLaunchKernelGGL((k_ritz<12, true>), dim3(b.nblk, b.B), dim3(256), 0, s, b);
        else hipLaunchKernelGGL((k_ritz<12, false>), dim3(b.nblk, b.B), dim3(256), 0, s, b);
    } else {
        if (v2) hipLaunchKernelGGL((k_ritz<kMaxSpace, true>), dim3(b.nblk, b.B), dim3(256), 0, s, b);
        else hipLaunchKernelGGL((k_ritz<kMaxSpace, false>), dim3(b.nblk, b.B), dim3(256), 0, s, b);
    }
    if (b.psp > 0) {
        if (b.max_space <= 12) hipLaunchKernelGGL(k_psp_fix<12>, dim3(b.B), dim3(kPsp), 0, s, b);
        else hipLaunchKernelGGL(k_psp_fix<kMaxSpace>, dim3(b.B), dim3(kPsp), 0, s, b);
    }
    hipLaunchKernelGGL(k_converge, dim3(b.B), dim3(64), 0, s, b);
    hipLaunchKernelGGL(k_coef1, dim3(b.B), dim3(64), 0, s, b);
    return hipGetLastError();
}

// Coefficients of the second pass on the stored basis, coef = R R^T d with
// d_i = V_i . T the sums of partials i.  One block of 64 threads per tuple.
__global__ void k_coef(Batch b) {
    const int t = blockIdx.x;
    if (b.status[t] != ST_RUNNING || !b.cgs2[t]) return;
    const int m = b.m[t], i = threadIdx.x;
    const double *R = b.R + (int64_t)t * kMaxSpace * kMaxSpace;
    __shared__ double dv[kMaxSpace], cv[kMaxSpace];
    if (i < m) dv[i] = sum_parts(b, t, i);
    __syncthreads();
    if (i < m) {
        double c = 0.0;
        for (int j = 0; j <= i; ++j) c += R[j * kMaxSpace + i] * dv[j];
        cv[i] = c;
    }
    __syncthreads();
    if (i < m) {
        double a = 0.0;
        for (int j = i; j < m; ++j) a += R[i * kMaxSpace + j] * cv[j];
        b.coef[(int64_t)t * kMaxSpace + i] = a;
    }
}

// T -= sum_i coef_i V_i in place (T = V_m; tuples whose correction needs the
// explicit passes only), and on the second pass the partial |T|^2
template <int MS, bool V2>
__global__ __launch_bounds__(256) void k_axpy(Batch b, int second) {
    const int t = blockIdx.y;
    if (b.status[t] != ST_RUNNING || !b.cgs2[t]) return;
    const int m = b.m[t];
    double cf[MS];
    const double *cp = b.coef + (int64_t)t * kMaxSpace;
#pragma unroll
    for (int i = 0; i < MS; ++i) cf[i] = (i < m) ? cp[i] : 0.0;
    const double *V = b.V + (int64_t)t * b.max_space * b.dim;
    double *T = b.V + ((int64_t)t * b.max_space + m) * b.dim;
    double acc[1];
    acc[0] = 0.0;
    // V_i, i < m, through a buffer resource that ends after vector m - 1 (the
    // loads past it read zero, and cf[i] = 0 there): all loads at once
    const __amdgpu_buffer_rsrc_t rV = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<double *>(V), (short)0, (int)((int64_t)m * b.dim * (int64_t)sizeof(double)), 0x00020000);
    const uint32_t vstride = (uint32_t)b.dim * (uint32_t)sizeof(double);
    if (V2) {
        // pairs of determinants with 16-byte loads (dim even), all loads first
        typedef double dbl2 __attribute__((ext_vector_type(2)));
        const int64_t n2 = b.dim >> 1;
        for (int64_t d2 = (int64_t)blockIdx.x * 256 + threadIdx.x; d2 < n2; d2 += (int64_t)gridDim.x * 256) {
            const int64_t d = d2 << 1;
            const uint32_t vo = (uint32_t)d * (uint32_t)sizeof(double);
            dbl2 vv[MS];
#pragma unroll
            for (int i = 0; i < MS; ++i)
                vv[i] = __builtin_bit_cast(dbl2, __builtin_amdgcn_raw_buffer_load_b128(rV, vo, (uint32_t)i * vstride, 0));
            dbl2 v = *reinterpret_cast<const dbl2 *>(T + d);
#pragma unroll
            for (int i = 0; i < MS; ++i) {
                v.x -= cf[i] * vv[i].x;
                v.y -= cf[i] * vv[i].y;
            }
            *reinterpret_cast<dbl2 *>(T + d) = v;
            acc[0] += v.x * v.x;
            acc[0] += v.y * v.y;
        }
    } else {
        for (int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x; d < b.dim; d += (int64_t)gridDim.x * 256) {
            const uint32_t vo = (uint32_t)d * (uint32_t)sizeof(double);
            double vd[MS];
#pragma unroll
            for (int i = 0; i < MS; ++i)
                vd[i] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rV, vo, (uint32_t)i * vstride, 0));
            double v = T[d];
#pragma unroll
            for (int i = 0; i < MS; ++i) v -= cf[i] * vd[i];
            T[d] = v;
            acc[0] += v * v;
        }
    }
    if (second) store_block_partials<1>(b, t, acc, 1);   // |T|^2 after the second pass, for k_tnorm
}

// 1/|T| into coef[0] and the column of R for V_m = T/|T| (orthogonal to the
// subspace: R gains the unit column).  A correction that lies inside the subspace (its
// projection kept less than 1e-8 of its norm) adds nothing: the Ritz pair is
// converged if the residual is below r_tol (an invariant subspace, e.g. a
// one-determinant space); otherwise the tuple skips this expansion and
// restarts from its Ritz vector at the next iteration, or has stalled when the
// subspace already is that one vector.
__global__ void k_tnorm(Batch b) {
    const int t = blockIdx.x;
    if (threadIdx.x != 0 || b.status[t] != ST_RUNNING || !b.cgs2[t]) return;
    const double tn = sqrt(sum_parts(b, t, 0));
    if (!(tn > 1e-8 * b.tnorm0[t]) || !(tn > 1e-300) || b.m[t] >= b.max_space) {
        b.status[t] = b.rnorm[t] < b.r_tol ? ST_DONE : (b.m[t] > 1 ? ST_RESTART : ST_STALLED);
        return;
    }
    b.coef[(int64_t)t * kMaxSpace] = 1.0 / tn;
    const int m = b.m[t];
    double *R = b.R + (int64_t)t * kMaxSpace * kMaxSpace;
    for (int i = 0; i < m; ++i) R[i * kMaxSpace + m] = 0.0;
    R[m * kMaxSpace + m] = 1.0;
}

// V_m <- V_m / |V_m| in place (tuples that took the second pass)
__global__ __launch_bounds__(256) void k_store_t(Batch b) {
    const int t = blockIdx.y;
    if (b.status[t] != ST_RUNNING || !b.cgs2[t]) return;
    const double s = b.coef[(int64_t)t * kMaxSpace];
    double *vm = b.V + ((int64_t)t * b.max_space + b.m[t]) * b.dim;
    const double *T = vm;
    if ((b.dim & 1) == 0) {   // 16-byte pairs (every vector 16-byte aligned)
        typedef double dbl2 __attribute__((ext_vector_type(2)));
        for (int64_t d2 = (int64_t)blockIdx.x * 256 + threadIdx.x; d2 < (b.dim >> 1); d2 += (int64_t)gridDim.x * 256) {
            const dbl2 v = *reinterpret_cast<const dbl2 *>(T + 2 * d2);
            *reinterpret_cast<dbl2 *>(vm + 2 * d2) = dbl2{v.x * s, v.y * s};
        }
    } else {
        for (int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x; d < b.dim; d += (int64_t)gridDim.x * 256)
            vm[d] = T[d] * s;
    }
}

// Tuples whose correction T = V_m lies too close to the subspace: two passes
// of classical Gram-Schmidt of T against V_0..V_{m-1} (coefficients on the
// stored basis), then V_m = T/|T|.  Every other tuple returns at once.
hipError_t launch_orthonormalize(const Batch &b, hipStream_t s) {
    const dim3 grid(b.nblk, b.B);
    VecRef tr{b.V, (int64_t)b.max_space * b.dim, b.m, 0};
    // first pass: projections from k_ritz, coefficients from k_coef1
    const bool small = b.max_space <= 12, v2 = (b.dim & 1) == 0;
    auto axpy = [&](int second) {
        if (small) {
            if (v2) hipLaunchKernelGGL((k_axpy<12, true>), grid, dim3(256), 0, s, b, second);
            else hipLaunchKernelGGL((k_axpy<12, false>), grid, dim3(256), 0, s, b, second);
        } else {
            if (v2) hipLaunchKernelGGL((k_axpy<kMaxSpace, true>), grid, dim3(256), 0, s, b, second);
            else hipLaunchKernelGGL((k_axpy<kMaxSpace, false>), grid, dim3(256), 0, s, b, second);
        }
    };
    axpy(0);
    if (small) hipLaunchKernelGGL(k_dots<12>, grid, dim3(256), 0, s, b, tr, 0, 1);
    else hipLaunchKernelGGL(k_dots<kMaxSpace>, grid, dim3(256), 0, s, b, tr, 0, 1);
    hipLaunchKernelGGL(k_coef, dim3(b.B), dim3(64), 0, s, b);
    axpy(1);
    hipLaunchKernelGGL(k_tnorm, dim3(b.B), dim3(64), 0, s, b);
    hipLaunchKernelGGL(k_store_t, grid, dim3(256), 0, s, b);
    return hipGetLastError();
}

// ------------------------------------------------------------- RDMs ------
// Ritz vector x = sum_i y_i V_i (normalised) into T, for every tuple.
__global__ __launch_bounds__(256) void k_form_x(Batch b) {
    const int t = blockIdx.y;
    const int m = b.m[t];
    const double *yv = b.y + (int64_t)t * kMaxSpace;
    double yy[kMaxSpace];
#pragma unroll
    for (int i = 0; i < kMaxSpace; ++i) yy[i] = (i < m) ? yv[i] : 0.0;
    const double *V = b.V + (int64_t)t * b.max_space * b.dim;
    double *T = b.T + (int64_t)t * b.dim;
    for (int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x; d < b.dim; d += (int64_t)gridDim.x * 256) {
        double x = 0.0;
#pragma unroll
        for (int i = 0; i < kMaxSpace; ++i)
            if (i < m) x += yy[i] * V[(int64_t)i * b.dim + d];
        T[d] = x;
    }
}

hipError_t launch_form_x(const Batch &b, hipStream_t s) {
    hipLaunchKernelGGL(k_form_x, dim3(b.nblk, b.B), dim3(256), 0, s, b);
    return hipGetLastError();
}

// Gram matrix of the transition vectors: column i = p * nA + q holds
// D_pq(I) = <I|E_pq|x> (a link E_ab|I'> = s|I> of string I' adds s x_{I'} to
// D_ba(I') ... written here from the ket side: the link (a created, b
// annihilated) of string I moving I to J gives <I|E_ba|J> = s, so
// D_ba(I) += s x_J), column nA^2 holds x itself.  G = D^T D over the
// determinants, accumulated with FP64 MFMA on 32-determinant tiles staged in
// LDS; every block writes its upper tile pairs to part[t][blk][NP*NP].
constexpr int kRdmTile = 32;

__global__ __launch_bounds__(256) void k_rdm_gram(Batch b, VecRef xref, double *part, int NP, int nblk_r) {
    const int t = blockIdx.y;
    const int nA = b.nA, nn = nA * nA;
    const int ld = NP + 1;
    extern __shared__ double Dt[];                       // [32][NP+1]
    __shared__ int pp[kMaxActive * (kMaxActive + 1) / 2], qq[kMaxActive * (kMaxActive + 1) / 2];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, ar = lane & 15, kr = lane >> 4;
    if (tid < b.pl.P) {
        int p, q;
        pair_of(tid, p, q);
        pp[tid] = p;
        qq[tid] = q;
    }
    const double *x = vref(xref, t, b.dim);
    const int NT = NP / 16, npairs = NT * (NT + 1) / 2;
    dbl4 acc[kRdmMaxPairs];
#pragma unroll
    for (int u = 0; u < kRdmMaxPairs; ++u) acc[u] = dbl4{0.0, 0.0, 0.0, 0.0};
    const int64_t ntiles = (b.dim + kRdmTile - 1) / kRdmTile;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += nblk_r) {
        __syncthreads();
        for (int i = tid; i < kRdmTile * ld; i += 256) Dt[i] = 0.0;
        __syncthreads();
        const int j = tid & 31, part8 = tid >> 5;
        const int64_t d = tile * kRdmTile + j;
        if (d < b.dim) {
            const int64_t Ka = d / b.Nb, Kb = d % b.Nb;
            const uint32_t ma = b.strA[Ka], mb = b.strB[Kb];
            for (int e = part8; e < b.nentA + b.nentB; e += 8) {
                const bool alpha = e < b.nentA;
                const uint32_t L = alpha ? b.linkA[Ka * b.nentA + e] : b.linkB[Kb * b.nentB + (e - b.nentA)];
                int J, Q;
                double s;
                link_decode(L, J, Q, s);
                const int p = pp[Q], q = qq[Q];
                const uint32_t m = alpha ? ma : mb;
                // the annihilated orbital of the link is the one occupied in the string
                const int an = (m >> p & 1u) ? p : q;
                const int cr = (an == p) ? q : p;
                const double xv = alpha ? x[(int64_t)J * b.Nb + Kb] : x[Ka * b.Nb + J];
                atomicAdd(&Dt[j * ld + an * nA + cr], s * xv);
            }
            if (part8 == 0) Dt[j * ld + nn] = x[d];
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kRdmMaxPairs; ++u) {
            const int uu = wave + 4 * u;
            if (uu < npairs) {
                int ti = 0, rem = uu;
                while (rem >= NT - ti) { rem -= NT - ti; ++ti; }
                const int tj = ti + rem;
#pragma unroll
                for (int ks = 0; ks < kRdmTile / 4; ++ks) {
                    const double a = Dt[(ks * 4 + kr) * ld + ti * 16 + ar];
                    const double bb = Dt[(ks * 4 + kr) * ld + tj * 16 + ar];
                    acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc[u], 0, 0, 0);
                }
            }
        }
    }
    double *out = part + ((int64_t)t * nblk_r + blockIdx.x) * NP * NP;
#pragma unroll
    for (int u = 0; u < kRdmMaxPairs; ++u) {
        const int uu = wave + 4 * u;
        if (uu < npairs) {
            int ti = 0, rem = uu;
            while (rem >= NT - ti) { rem -= NT - ti; ++ti; }
            const int tj = ti + rem;
#pragma unroll
            for (int v = 0; v < 4; ++v) out[(int64_t)(ti * 16 + kr + 4 * v) * NP + tj * 16 + ar] = acc[u][v];
        }
    }
}

// G[t] (NP x NP, symmetric) = sum over blocks of the upper tile pairs
__global__ __launch_bounds__(256) void k_rdm_reduce(const double *part, double *G, int NP, int nblk_r) {
    const int t = blockIdx.y;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)NP * NP) return;
    int i = (int)(idx / NP), j = (int)(idx % NP);
    if (i / 16 > j / 16) { const int x = i; i = j; j = x; }
    double s = 0.0;
    for (int blk = 0; blk < nblk_r; ++blk) s += part[((int64_t)t * nblk_r + blk) * NP * NP + (int64_t)i * NP + j];
    G[(int64_t)t * NP * NP + idx] = s;
}

int rdm_np(int nA) { return round_up(nA * nA + 1, 16); }

size_t rdm_lds_bytes(int NP) { return sizeof(double) * (size_t)kRdmTile * (NP + 1); }

hipError_t launch_rdm(const Batch &b, VecRef x, double *part, double *G, int nblk_r, hipStream_t s) {
    const int NP = rdm_np(b.nA);
    hipLaunchKernelGGL(k_rdm_gram, dim3(nblk_r, b.B), dim3(256), rdm_lds_bytes(NP), s, b, x, part, NP, nblk_r);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rdm_reduce, dim3((unsigned)(((int64_t)NP * NP + 255) / 256), b.B), dim3(256), 0, s, part, G,
                       NP, nblk_r);
    return hipGetLastError();
}

// Weighted embedding of the batch's density matrices into the full-space
// gradient (n x n and n^4 doubles, row-major), w[t] the weight of tuple t:
//   grad_h[o_p, o_q] += w gamma_pq,  grad_eri[o_p, o_q, o_r, o_s] += w/2 Gamma_pqrs
// with gamma_pq = G[pq, x] and Gamma_pqrs = G[qp, rs] - d_qr gamma_ps over the
// active orbitals o, and for the doubly occupied core c, d: gamma_cc = 2,
// Gamma_cccc = 2, Gamma_ccdd = 4 and Gamma_cddc = -2 (c != d), Gamma_pqcc =
// Gamma_ccpq = 2 gamma_pq, Gamma_pccq = Gamma_cqpc = -gamma_pq.  Tuples share
// full-space entries, so the adds are atomic (their order, and the last bits
// of the sums, are not fixed).
__device__ __forceinline__ void grad_add(double *a, double v) { unsafeAtomicAdd(a, v); }

__global__ __launch_bounds__(256) void k_rdm_embed_act(Batch b, const double *w, double *ge) {
    const int t = blockIdx.y;
    const double wt = w[t];
    if (wt == 0.0 || b.status[t] != ST_DONE) return;   // unconverged: solved again, embedded then
    const int nA = b.nA, nn = nA * nA, NP = round_up(nn + 1, 16), n = b.norb;
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= nn * nn) return;
    const int p = idx / (nA * nn), q = (idx / nn) % nA, r = (idx / nA) % nA, s = idx % nA;
    const double *G = b.rdm_G + (int64_t)t * NP * NP;
    const int32_t *o = b.act + (int64_t)t * nA;
    double v = G[(int64_t)(q * nA + p) * NP + r * nA + s];
    if (q == r) v -= G[(int64_t)(p * nA + s) * NP + nn];
    grad_add(ge + (((int64_t)o[p] * n + o[q]) * n + o[r]) * n + o[s], 0.5 * wt * v);
}

__global__ __launch_bounds__(256) void k_rdm_embed_core(Batch b, const double *w, double *gh, double *ge) {
    const int t = blockIdx.x;
    const double wt = w[t];
    if (wt == 0.0 || b.status[t] != ST_DONE) return;
    const int nA = b.nA, nn = nA * nA, NP = round_up(nn + 1, 16), n = b.norb, nC = b.nC;
    const double *G = b.rdm_G + (int64_t)t * NP * NP;
    const int32_t *o = b.act + (int64_t)t * nA, *C = b.core + (int64_t)t * nC;
    const double hw = 0.5 * wt;
    auto E = [&](int p, int q, int r, int s) { return ge + (((int64_t)p * n + q) * n + r) * n + s; };
    for (int i = threadIdx.x; i < nn; i += 256) {
        const int p = i / nA, q = i % nA;
        grad_add(gh + (int64_t)o[p] * n + o[q], wt * G[(int64_t)i * NP + nn]);
    }
    for (int i = threadIdx.x; i < nC * nC; i += 256) {
        const int c = C[i / nC], d = C[i % nC];
        if (c == d) {
            grad_add(gh + (int64_t)c * n + c, 2.0 * wt);
            grad_add(E(c, c, c, c), hw * 2.0);
        } else {
            grad_add(E(c, c, d, d), hw * 4.0);
            grad_add(E(c, d, d, c), hw * -2.0);
        }
    }
    for (int i = threadIdx.x; i < nC * nn; i += 256) {
        const int c = C[i / nn], pq = i % nn, p = pq / nA, q = pq % nA;
        const double g = G[(int64_t)pq * NP + nn];
        grad_add(E(o[p], o[q], c, c), hw * 2.0 * g);
        grad_add(E(c, c, o[p], o[q]), hw * 2.0 * g);
        grad_add(E(o[p], c, c, o[q]), -hw * g);
        grad_add(E(c, o[q], o[p], c), -hw * g);
    }
}

hipError_t launch_rdm_embed(const Batch &b, const double *w, double *gh, double *ge, hipStream_t s) {
    const int n4 = b.nA * b.nA * b.nA * b.nA;
    hipLaunchKernelGGL(k_rdm_embed_act, dim3((n4 + 255) / 256, b.B), dim3(256), 0, s, b, w, ge);
    hipLaunchKernelGGL(k_rdm_embed_core, dim3(b.B), dim3(256), 0, s, b, w, gh, ge);
    return hipGetLastError();
}

__global__ void k_finalize(Batch b) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= b.B) return;
    b.out_e[t] = b.params[(int64_t)t * b.pl.stride + b.pl.off_ecore] + b.theta[t];
    b.out_status[t] = b.status[t];
}

hipError_t launch_finalize(const Batch &b, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3((b.B + 255) / 256), dim3(256), 0, s, b);
    return hipGetLastError();
}

// The workspace of the allocation-free entry point: a file-scope device array
// that the code object brings (each GPU the library runs on holds its own
// copy until the process ends).  Host code never passes its name to a kernel
// or a copy: scratch_address() resolves it once per device, with that device
// current, and callers use the returned pointer.
static __device__ __align__(256) char scratch[kScratchBytes];

hipError_t scratch_address(void **ptr) {
    *ptr = nullptr;
    return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch));
}

hipError_t init_kernels() {
    hipError_t e = init_sigma_kernels();
    if (e != hipSuccess) return e;
    if ((e = init_whole_kernels()) != hipSuccess) return e;
    return hipFuncSetAttribute((const void *)k_psp_factor, hipFuncAttributeMaxDynamicSharedMemorySize, (int)psp_factor_lds());
}

}  // namespace mbefci

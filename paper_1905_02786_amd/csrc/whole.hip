// Whole-tuple mode: one workgroup runs the complete Davidson solve of one
// small CASCI (Sec. 2: each increment needs the lowest eigenvalue of H over
// the tuple's CAS) in a single launch.  The per-iteration work of a small
// tuple is a few microseconds, far below the cost of the dozen launches of
// one batched iteration, so here the iteration loop itself runs on the
// device: Ritz pair of the projected matrix, residual and correction, two
// classical Gram-Schmidt passes and sigma, separated by workgroup barriers.
//
// The per-batch set-up is the batched path's: integral gather, string
// Hamiltonians, diagonal, P space and guess (V_0, normalised).  The basis V is
// kept orthonormal, so the projected matrix G = V^T H V is symmetric and is
// diagonalised directly.  Sigma is formed per determinant from the vector in
// LDS:
//   sigma(I_a, I_b) = sum_J_a H_a[I_a][J_a] c(J_a, I_b) + sum_J_b H_b[I_b][J_b] c(I_a, J_b)
//                   + sum over alpha links (J_a, P, s_a) of I_a and beta links (J_b, Q, s_b) of I_b
//                     of s_a s_b (P|Q) c(J_a, J_b)
// (plus lambda S_- S_+ c with a spin shift), the same operator the batched
// kernels apply.  On exit theta, status, iteration count, m and the Ritz
// coefficients y on V are written as the batched iteration leaves them.
#include "device.h"
#include "symmetry.h"

namespace mbefci {

constexpr int kWholeThreads = 512;
constexpr int kWholeWaves = kWholeThreads / 64;
constexpr int kWholeLd = kMaxSpace + 1;   // row stride of the small LDS matrices
constexpr int kWholeRed = kMaxSpace + 2;
constexpr int kWholeMaxLds = 160 * 1024;

struct WholeShared {
    double G[kMaxSpace][kWholeLd];      // projected matrix on the orthonormal basis
    double A[2][kMaxSpace][kWholeLd];   // Jacobi iterates (rounds alternate between the two)
    double Z[kMaxSpace][kWholeLd];      // eigenvectors of G in the columns (kept for a warm start)
    double W[kMaxSpace][kWholeLd];      // scratch of the warm start
    double red[kWholeWaves][kWholeRed];
    double sum[kWholeRed];
    double y[kMaxSpace], yp[kMaxSpace], z[kMaxSpace];
    double pr[kPsp], pw[kPsp], pc[kPsp];
    double pd[kPsp], pe[kPsp];   // diagonal and subdiagonal of the P-space tridiagonal factor
    unsigned short pairs[kMaxSpace - 1][kMaxSpace / 2];   // Jacobi round-robin pairs (p | q << 8)
    double rc[kMaxSpace / 2], rs[kMaxSpace / 2];          // the round's rotations
    double pp[kWholeThreads / kPsp][kPsp];   // partial sums of the P-space products
    double theta, mu;
    int done, keep, cur;
};

// Dynamic LDS: the vector of the current sigma, the pair integrals, the
// string Hamiltonians (one when both spins have the same electron count) and
// the two link tables.
size_t whole_lds_bytes(const ParamLayout &pl, int64_t dim, int64_t Na, int64_t Nb, int nentA, int nentB, bool same) {
    return 8 * (size_t)((dim + 1) & ~int64_t(1)) + 8 * (size_t)pl.P * pl.Kpad + 8 * (size_t)Nb * Nb +
           (same ? 0 : 8 * (size_t)Na * Na) + 4 * (size_t)(Na * nentA + Nb * nentB);
}

bool whole_fits(const ParamLayout &pl, int64_t dim, int64_t Na, int64_t Nb, int nentA, int nentB, bool same) {
    return pl.nA <= kWholeMaxActive && dim <= kWholeMaxDim && nentB <= kWholeMaxNent && nentA <= kWholeMaxNent &&
           whole_lds_bytes(pl, dim, Na, Nb, nentA, nentB, same) + sizeof(WholeShared) <= (size_t)kWholeMaxLds;
}

// Sums over the workgroup of acc[0 .. n-1] into w.sum[0 .. n-1] and, with
// `ext`, of x into w.sum[n] (n uniform); every thread may read w.sum after
// the call.
template <int N>
__device__ __forceinline__ void wg_sums(WholeShared &w, const double (&acc)[N], int n, bool ext = false,
                                        double x = 0.0) {
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        if (k < n) {
            const double v = wave_sum(acc[k]);
            if (l == 0) w.red[wv][k] = v;
        }
    }
    if (ext) {
        const double v = wave_sum(x);
        if (l == 0) w.red[wv][n] = v;
        ++n;
    }
    __syncthreads();
    if ((int)threadIdx.x < n) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < kWholeWaves; ++i) s += w.red[i][threadIdx.x];
        w.sum[threadIdx.x] = s;
    }
    __syncthreads();
}

// Ordering point between the phases of the single wave that runs the small
// eigenproblem: a wave executes its LDS operations in order, so only the
// compiler has to be kept from moving LDS accesses across this point.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Reciprocal and reciprocal square root: the hardware approximations refined
// by two Newton steps (to a few ulps; used for the rotations of the small
// eigenproblem and the pivots of the P-space solve).
__device__ __forceinline__ double fast_rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ double fast_rsq(double x) {
    double r = __builtin_amdgcn_rsq(x);
    r = r * fma(-0.5 * x * r, r, 1.5);
    return r * fma(-0.5 * x * r, r, 1.5);
}

// Lowest eigenpair of the symmetric m x m matrix w.G by cyclic Jacobi
// rotations, run by the first wave (the others wait at the workgroup barrier
// at the end).  The pairs of a round are disjoint (round-robin order, one
// dummy index when m is odd): the lanes first form the round's rotations,
// then apply all of them at once, each lane a fixed set of 2 x 2 blocks of
// J^T A J (A read from one buffer, written to the other) and rows of Z J.
// Warm start: w.Z holds the eigenvectors of the leading zm x zm block of G
// (the previous iteration's projected matrix), so the iteration starts from
// Z_ext^T G Z_ext, Z_ext = diag(Z, I), which is diagonal but for its new rows
// and columns.  Leaves w.theta, w.y (zero past m) and the eigenvectors in w.Z.
template <int MS>
__device__ void wg_lowest_eig(WholeShared &w, int m, int zm) {
    const int tid = threadIdx.x, mm = m + (m & 1), half = mm / 2;
    if (tid < 64) {
        for (int i = tid; i < mm * mm; i += 64) {
            const int r = i / mm, c = i - r * mm;
            w.W[r][c] = (r < zm && c < zm) ? w.Z[r][c] : (r == c ? 1.0 : 0.0);
        }
        // round r pairs position 0 with position mm - 1 and position k with
        // mm - 1 - k; the indices at positions 1 .. mm-1 rotate by one per round
        for (int i = tid; i < (mm - 1) * half; i += 64) {
            const int round = i / half, k = i - round * half;
            auto at = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + round) % (mm - 1); };
            const int a = at(k), c = at(mm - 1 - k);
            w.pairs[round][k] = (unsigned short)((a < c ? a : c) | ((a < c ? c : a) << 8));
        }
        wave_sync();
        for (int i = tid; i < mm * mm; i += 64) {   // Z <- G Z_ext (scratch)
            const int r = i / mm, c = i - r * mm;
            double v = 0.0;
            if (r < m && c < m)
                for (int k = 0; k < m; ++k) v += w.G[r][k] * w.W[k][c];
            w.Z[r][c] = v;
        }
        wave_sync();
        for (int i = tid; i < mm * mm; i += 64) {   // A = Z_ext^T G Z_ext (upper, mirrored)
            const int r = i / mm, c = i - r * mm;
            if (r <= c) {
                double v = 0.0;
                if (c < m)
                    for (int k = 0; k < m; ++k) v += w.W[k][r] * w.Z[k][c];
                w.A[0][r][c] = v;
                w.A[0][c][r] = v;
            }
        }
        wave_sync();
        for (int i = tid; i < mm * mm; i += 64) {
            const int r = i / mm, c = i - r * mm;
            w.Z[r][c] = w.W[r][c];
        }
        // this lane's items of a round: blocks (k, k2) of A, then rows r of Z
        // for pair k (bit 15 set), indices packed 5 bits each
        constexpr int NI = ((MS / 2) * (MS / 2) + (MS / 2) * MS + 63) / 64;
        const int nblk = half * half, nitem = nblk + half * mm;
        int item[NI];
#pragma unroll
        for (int j = 0; j < NI; ++j) {
            const int i = tid + 64 * j;
            int v = -1;
            if (i < nblk) v = ((i / half) << 5) | (i % half);
            else if (i < nitem) v = 0x8000 | (((i - nblk) / mm) << 5) | ((i - nblk) % mm);
            item[j] = v;
        }
        wave_sync();
        int cur = 0;
        for (int sweep = 0; sweep < 30 && mm > 1; ++sweep) {
            double off = 0.0, tot = 0.0;
            if (tid < m)
                for (int r = 0; r < m; ++r) {
                    const double a = w.A[cur][r][tid];
                    tot += a * a;
                    if (r != tid) off += a * a;
                }
            off = wave_sum(off);
            tot = wave_sum(tot);
            if (off <= 1e-24 * tot) break;   // the same sums in every lane
            for (int round = 0; round < mm - 1; ++round) {
                const double (&Ai)[kMaxSpace][kWholeLd] = w.A[cur];
                if (tid < half) {
                    // the rotation that zeroes A[p][q]: t = tan of its angle,
                    // the smaller root of t^2 + 2 tau t - 1 = 0 (identity for
                    // the dummy index and for a zero entry)
                    const unsigned pk = w.pairs[round][tid];
                    const int p = pk & 255, q = pk >> 8;
                    const double apq = Ai[p][q];
                    double c = 1.0, s = 0.0;
                    if (q < m && apq != 0.0) {
                        const double tau = (Ai[q][q] - Ai[p][p]) * fast_rcp(2.0 * apq);
                        const double at = fabs(tau);
                        double tt;
                        if (at > 1e150) tt = 0.5 * fast_rcp(tau);
                        else {
                            const double u = fma(tau, tau, 1.0);
                            tt = fast_rcp(at + u * fast_rsq(u));
                            if (tau < 0.0) tt = -tt;
                        }
                        c = fast_rsq(fma(tt, tt, 1.0));
                        s = tt * c;
                    }
                    w.rc[tid] = c;
                    w.rs[tid] = s;
                }
                wave_sync();
                double (&Ao)[kMaxSpace][kWholeLd] = w.A[cur ^ 1];
#pragma unroll
                for (int j = 0; j < NI; ++j) {
                    const int v = item[j];
                    if (v < 0) continue;
                    if (!(v & 0x8000)) {
                        // block (pair k rows, pair k2 columns) of J^T A J
                        const int k = v >> 5, k2 = v & 31;
                        const unsigned pk = w.pairs[round][k], pk2 = w.pairs[round][k2];
                        const int p = pk & 255, q = pk >> 8, p2 = pk2 & 255, q2 = pk2 >> 8;
                        const double c = w.rc[k], s = w.rs[k], c2 = w.rc[k2], s2 = w.rs[k2];
                        const double xpp = c2 * Ai[p][p2] - s2 * Ai[p][q2], xpq = s2 * Ai[p][p2] + c2 * Ai[p][q2];
                        const double xqp = c2 * Ai[q][p2] - s2 * Ai[q][q2], xqq = s2 * Ai[q][p2] + c2 * Ai[q][q2];
                        Ao[p][p2] = c * xpp - s * xqp;
                        Ao[q][p2] = s * xpp + c * xqp;
                        Ao[p][q2] = c * xpq - s * xqq;
                        Ao[q][q2] = s * xpq + c * xqq;
                    } else {
                        const int k = (v >> 5) & 31, r = v & 31;   // row r of Z J, pair k
                        const unsigned pk = w.pairs[round][k];
                        const int p = pk & 255, q = pk >> 8;
                        const double c = w.rc[k], s = w.rs[k];
                        const double zp = w.Z[r][p], zq = w.Z[r][q];
                        w.Z[r][p] = c * zp - s * zq;
                        w.Z[r][q] = s * zp + c * zq;
                    }
                }
                cur ^= 1;
                wave_sync();
            }
        }
        if (tid == 0) {
            int k = 0;
            for (int i = 1; i < m; ++i)
                if (w.A[cur][i][i] < w.A[cur][k][k]) k = i;
            w.theta = w.A[cur][k][k];
            for (int i = 0; i < kMaxSpace; ++i) w.y[i] = i < m ? w.Z[i][k] : 0.0;
        }
    }
    __syncthreads();
}

template <int MS>
__global__ __launch_bounds__(kWholeThreads) void k_whole(Batch b) {
    const int t = blockIdx.x, tid = threadIdx.x;
    const int64_t dim = b.dim;
    const int Na = (int)b.Na, Nb = (int)b.Nb, nentA = b.nentA, nentB = b.nentB;
    const ParamLayout &pl = b.pl;
    const int Kpad = pl.Kpad;
    const bool same = b.Ha == b.Hb;
    __shared__ WholeShared w;
    extern __shared__ double wlds[];
    double *cL = wlds;                                    // [dim] vector of the current sigma
    double *eri = cL + ((dim + 1) & ~int64_t(1));         // [P][Kpad] (P|Q) / 2
    double *hB = eri + pl.P * Kpad;                       // [Nb][Nb] beta string Hamiltonian
    double *hA = same ? hB : hB + Nb * Nb;                // [Na][Na] alpha string Hamiltonian
    uint32_t *lkA = reinterpret_cast<uint32_t *>(same ? hB + Nb * Nb : hA + Na * Na);   // [Na][nentA]
    uint32_t *lkB = lkA + Na * nentA;                     // [Nb][nentB]
    const double *prm = b.params + (int64_t)t * pl.stride;
    const double *Ha = b.Ha + (int64_t)t * Na * Na, *Hb = b.Hb + (int64_t)t * Nb * Nb;
    for (int i = tid; i < pl.P * Kpad; i += kWholeThreads) eri[i] = prm[pl.off_eri + i];
    for (int i = tid; i < Nb * Nb; i += kWholeThreads) hB[i] = Hb[i];
    if (!same)
        for (int i = tid; i < Na * Na; i += kWholeThreads) hA[i] = Ha[i];
    for (int i = tid; i < Na * nentA; i += kWholeThreads) lkA[i] = b.linkA[i];
    for (int i = tid; i < Nb * nentB; i += kWholeThreads) lkB[i] = b.linkB[i];
    if (b.psp > 0 && tid < b.psp) {
        w.pd[tid] = b.pT[(int64_t)t * 3 * kPsp + tid];
        w.pe[tid] = b.pT[(int64_t)t * 3 * kPsp + kPsp + tid];
    }
    double *V = b.V + (int64_t)t * b.max_space * dim;
    double *S = b.S + (int64_t)t * b.max_space * dim;
    const double *hd = b.Hd + (int64_t)t * dim;
    const int maxs = b.max_space;
    const double lam = b.spin_shift;
    // V_i and S_i, i < m, through buffer resources that end after vector
    // m - 1: loads past it read zero, so all loads of a determinant are issued
    // at once (the coefficients there are zero too)
    const uint32_t vstride = (uint32_t)dim * (uint32_t)sizeof(double);
    auto rsrc = [&](double *base, int nvec) {
        return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, (int)(nvec * vstride), 0x00020000);
    };
    auto ld = [&](__amdgpu_buffer_rsrc_t r, int64_t d, int i) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (uint32_t)d * 8u, (uint32_t)i * vstride, 0));
    };

    // out[i] = sum_k M[k][i] u[k], i < n (M row-major with stride kPsp; u,
    // out in LDS), the k range split over the workgroup's threads in
    // kWholeThreads / kPsp parts; ends with a barrier
    auto psp_product = [&](const double *Mx, const double *u, double *out) {
        constexpr int NP = kWholeThreads / kPsp;
        const int n = b.psp, i = tid % kPsp, part = tid / kPsp;
        const int k0 = part * n / NP, k1 = (part + 1) * n / NP;
        double s = 0.0;
        if (i < n) {
#pragma unroll 8
            for (int k = k0; k < k1; ++k) s += Mx[k * kPsp + i] * u[k];
        }
        w.pp[part][i] = s;
        __syncthreads();
        if (tid < n) {
            double v = 0.0;
#pragma unroll
            for (int q = 0; q < NP; ++q) v += w.pp[q][tid];
            out[tid] = v;
        }
        __syncthreads();
    };

    // sigma of the vector in cL at determinant d
    auto sigma_det = [&](int64_t d) -> double {
        const int Ia = (int)(d / Nb), Ib = (int)(d - (int64_t)Ia * Nb);
        double acc = 0.0;
        const double *ha = hA + Ia * Na;
        for (int Ja = 0; Ja < Na; ++Ja) acc += ha[Ja] * cL[Ja * Nb + Ib];
        const double *crow = cL + Ia * Nb;
        for (int Jb = 0; Jb < Nb; ++Jb) acc += hB[Jb * Nb + Ib] * crow[Jb];   // H_b symmetric
        uint32_t lb[kWholeMaxNent];
#pragma unroll
        for (int e = 0; e < kWholeMaxNent; ++e) lb[e] = e < nentB ? lkB[Ib * nentB + e] : 0u;
        double ab = 0.0;
        const uint32_t *la = lkA + Ia * nentA;
        for (int ea = 0; ea < nentA; ++ea) {
            const uint32_t L = la[ea];
            const double *er = eri + (int)((L >> 20) & 0x3FFu) * Kpad;
            const double *cr = cL + (int)(L & 0xFFFFFu) * Nb;
            double s = 0.0;
#pragma unroll
            for (int e = 0; e < kWholeMaxNent; ++e) {
                if (e < nentB) {
                    const uint32_t M = lb[e];
                    const double v = er[(M >> 20) & 0x3FFu] * cr[M & 0xFFFFFu];
                    s += (M >> 31) ? -v : v;
                }
            }
            ab += (L >> 31) ? -s : s;
        }
        acc += 2.0 * ab;   // the table holds (P|Q) / 2
        if (lam != 0.0) acc += lam * spin_ss(b, cL, Ia, Ib);
        if (b.sym_shift != 0.0) acc += sym_pen(b, t, b.strA[Ia], b.strB[Ib]) * cL[d];
        return acc;
    };

    // first basis vector: the guess, normalised by the set-up
    for (int64_t d = tid; d < dim; d += kWholeThreads) cL[d] = V[d];
    __syncthreads();
    {
        double acc[1] = {0.0};
        for (int64_t d = tid; d < dim; d += kWholeThreads) {
            const double s = sigma_det(d);
            S[d] = s;
            acc[0] += cL[d] * s;
        }
        wg_sums(w, acc, 1);
        if (tid == 0) {
            w.G[0][0] = w.sum[0];
            for (int i = 0; i < kMaxSpace; ++i) w.yp[i] = i == 0 ? 1.0 : 0.0;
        }
        __syncthreads();
    }
    int m = 1, zm = 0, iter = 0, status = ST_RUNNING, force = 0;
    double theta_prev = 1e300, theta = 0.0;
    while (true) {
        wg_lowest_eig<MS>(w, m, zm);
        zm = m;
        theta = w.theta;
        const bool restart = m >= maxs || force;
        force = 0;
        if (tid == 0) {
            int keep = restart ? 1 : 0;
            if (restart && b.restart_keep > 1) {
                // the previous Ritz vector (coordinates yp, zero past its
                // length) made orthogonal to this one by two passes
                for (int i = 0; i < m; ++i) w.z[i] = w.yp[i];
                for (int pass = 0; pass < 2; ++pass) {
                    double dd = 0.0;
                    for (int i = 0; i < m; ++i) dd += w.z[i] * w.y[i];
                    for (int i = 0; i < m; ++i) w.z[i] -= dd * w.y[i];
                }
                double nz = 0.0;
                for (int i = 0; i < m; ++i) nz += w.z[i] * w.z[i];
                if (nz > 1e-12) {
                    const double sc = 1.0 / sqrt(nz);
                    double mu = 0.0;
                    for (int i = 0; i < m; ++i) w.z[i] *= sc;
                    for (int i = 0; i < m; ++i)
                        for (int j = 0; j < m; ++j) mu += w.z[i] * w.G[i][j] * w.z[j];
                    w.mu = mu;
                    keep = 2;
                }
            }
            for (int i = m; i < kMaxSpace; ++i) w.z[i] = 0.0;
            w.keep = keep;
            if (!restart)
                for (int i = 0; i < kMaxSpace; ++i) w.yp[i] = w.y[i];
        }
        __syncthreads();
        const int keep = w.keep;
        // Ritz vector x = V y, residual r = S y - theta x, correction
        // r / (theta - H_II) (clamped) into the next basis slot; on restart x,
        // S x (and the kept direction) replace V_0, S_0 (V_1, S_1) in place
        const int slot = restart ? keep : m;
        {
            double acc[1] = {0.0};
            double *T = V + (int64_t)slot * dim;
            const __amdgpu_buffer_rsrc_t rV = rsrc(V, m), rS = rsrc(S, m);
            double yy[MS], zz[MS];
#pragma unroll
            for (int i = 0; i < MS; ++i) {
                yy[i] = w.y[i];
                zz[i] = w.z[i];
            }
            for (int64_t d = tid; d < dim; d += kWholeThreads) {
                double x = 0.0, ax = 0.0, x2 = 0.0, a2 = 0.0;
#pragma unroll
                for (int i = 0; i < MS; ++i) {
                    const double v = ld(rV, d, i), s = ld(rS, d, i);
                    x += yy[i] * v;
                    ax += yy[i] * s;
                    if (keep == 2) {
                        x2 += zz[i] * v;
                        a2 += zz[i] * s;
                    }
                }
                const double r = ax - theta * x;
                acc[0] += r * r;
                double den = theta - hd[d];
                if (fabs(den) < 1e-8) den = den >= 0.0 ? 1e-8 : -1e-8;
                if (restart) {
                    V[d] = x;
                    S[d] = ax;
                    if (keep == 2) {
                        V[dim + d] = x2;
                        S[dim + d] = a2;
                    }
                }
                T[d] = r / den;
            }
            wg_sums(w, acc, 1);
        }
        const double rn = sqrt(w.sum[0]);
        if (restart) {
            m = keep;
            zm = keep;   // G = diag(theta, mu): its eigenvectors are the unit vectors
            if (tid == 0) {
                for (int i = 0; i < kMaxSpace; ++i) {
                    w.y[i] = i == 0 ? 1.0 : 0.0;
                    w.yp[i] = w.y[i];
                }
                w.G[0][0] = theta;
                w.Z[0][0] = 1.0;
                if (keep == 2) {
                    w.G[0][1] = w.G[1][0] = 0.0;
                    w.G[1][1] = w.mu;
                    w.Z[0][1] = w.Z[1][0] = 0.0;
                    w.Z[1][1] = 1.0;
                }
            }
            __syncthreads();
        }
        double *T = V + (int64_t)m * dim;
        // P space: the correction there is the exact (theta - H_PP)^-1 r_P,
        // H_PP = Q Tr Q^T with Tr tridiagonal
        if (b.psp > 0) {
            const int n = b.psp;
            const int32_t *pidx = b.pidx + (int64_t)t * kPsp;
            const double *Q = b.pQ + (int64_t)t * kPsp * kPsp, *Qt = b.pQt + (int64_t)t * kPsp * kPsp;
            const double *dT = w.pd, *eT = w.pe;
            if (tid < n) {
                const int64_t d = pidx[tid];
                const __amdgpu_buffer_rsrc_t rV = rsrc(V, m), rS = rsrc(S, m);
                double r = 0.0;
#pragma unroll
                for (int i = 0; i < MS; ++i) r += w.y[i] * (ld(rS, d, i) - theta * ld(rV, d, i));
                w.pr[tid] = r;
            }
            __syncthreads();
            psp_product(Q, w.pr, w.pw);
            if (tid == 0) {
                // (theta - Tr) u = w: forward elimination, then back substitution
                // 1 / pivot, the pivot kept at |p| >= 1e-8
                auto inv = [](double p) { return fast_rcp(fabs(p) < 1e-8 ? (p >= 0.0 ? 1e-8 : -1e-8) : p); };
                double ip = inv(theta - dT[0]);
                double cprev = (n > 1 ? -eT[0] : 0.0) * ip, wprev = w.pw[0] * ip;
                w.pc[0] = cprev;
                w.pw[0] = wprev;
                for (int k = 1; k < n; ++k) {
                    const double e = eT[k - 1];
                    ip = inv(theta - dT[k] + e * cprev);
                    cprev = (k + 1 < n ? -eT[k] : 0.0) * ip;
                    wprev = (w.pw[k] + e * wprev) * ip;
                    w.pc[k] = cprev;
                    w.pw[k] = wprev;
                }
                for (int k = n - 2; k >= 0; --k) {
                    wprev = w.pw[k] - w.pc[k] * wprev;
                    w.pw[k] = wprev;
                }
            }
            __syncthreads();
            psp_product(Qt, w.pw, w.pr);
            if (tid < n) T[pidx[tid]] = w.pr[tid];
            __syncthreads();
        }
        ++iter;
        if (!isfinite(rn) || !isfinite(theta)) status = ST_NONFINITE;
        else if (rn < b.r_tol && fabs(theta - theta_prev) < b.e_tol) status = ST_DONE;
        else if (iter >= b.max_iter) status = ST_MAXITER;
        theta_prev = theta;
        if (status != ST_RUNNING) break;
        // two classical Gram-Schmidt passes of T against V_0 .. V_{m-1}
        double t0, tn;
        {
            const __amdgpu_buffer_rsrc_t rV = rsrc(V, m);
            double acc[MS], tt = 0.0;
#pragma unroll
            for (int i = 0; i < MS; ++i) acc[i] = 0.0;
            for (int64_t d = tid; d < dim; d += kWholeThreads) {
                const double tv = T[d];
#pragma unroll
                for (int i = 0; i < MS; ++i) acc[i] += ld(rV, d, i) * tv;
                tt += tv * tv;
            }
            wg_sums(w, acc, m, true, tt);
            t0 = sqrt(w.sum[m]);
            double cf[MS];
#pragma unroll
            for (int i = 0; i < MS; ++i) cf[i] = i < m ? w.sum[i] : 0.0;
            __syncthreads();
#pragma unroll
            for (int i = 0; i < MS; ++i) acc[i] = 0.0;
            for (int64_t d = tid; d < dim; d += kWholeThreads) {
                double vv[MS], tv = T[d];
#pragma unroll
                for (int i = 0; i < MS; ++i) vv[i] = ld(rV, d, i);
#pragma unroll
                for (int i = 0; i < MS; ++i) tv -= cf[i] * vv[i];
                T[d] = tv;
#pragma unroll
                for (int i = 0; i < MS; ++i) acc[i] += vv[i] * tv;
            }
            wg_sums(w, acc, m);
#pragma unroll
            for (int i = 0; i < MS; ++i) cf[i] = i < m ? w.sum[i] : 0.0;
            __syncthreads();
            double a2[1] = {0.0};
            for (int64_t d = tid; d < dim; d += kWholeThreads) {
                double tv = T[d];
#pragma unroll
                for (int i = 0; i < MS; ++i) tv -= cf[i] * ld(rV, d, i);
                T[d] = tv;
                a2[0] += tv * tv;
            }
            wg_sums(w, a2, 1);
            tn = sqrt(w.sum[0]);
        }
        if (!(tn > 1e-8 * t0) || !(tn > 1e-300)) {
            // the correction lies in the subspace: converged if the residual
            // is small (an invariant subspace), else restart from the Ritz
            // vector, or stalled when the subspace is that vector already
            if (rn < b.r_tol) {
                status = ST_DONE;
                break;
            }
            if (m > 1) {
                force = 1;
                continue;
            }
            status = ST_STALLED;
            break;
        }
        // V_m = T / |T|, also into LDS for its sigma
        {
            const double sc = 1.0 / tn;
            for (int64_t d = tid; d < dim; d += kWholeThreads) {
                const double v = T[d] * sc;
                T[d] = v;
                cL[d] = v;
            }
            __syncthreads();
        }
        // S_m = H V_m and the new column of G
        {
            const __amdgpu_buffer_rsrc_t rV = rsrc(V, m);
            double acc[MS], dm = 0.0;
#pragma unroll
            for (int i = 0; i < MS; ++i) acc[i] = 0.0;
            double *Sm = S + (int64_t)m * dim;
            for (int64_t d = tid; d < dim; d += kWholeThreads) {
                const double s = sigma_det(d);
                Sm[d] = s;
#pragma unroll
                for (int i = 0; i < MS; ++i) acc[i] += ld(rV, d, i) * s;
                dm += cL[d] * s;
            }
            wg_sums(w, acc, m, true, dm);
            if (tid <= m) {
                w.G[tid][m] = w.sum[tid];
                w.G[m][tid] = w.sum[tid];
            }
            __syncthreads();
            ++m;
        }
    }
    if (tid == 0) {
        b.theta[t] = theta;
        b.status[t] = status;
        b.iter[t] = iter;
        b.m[t] = m;
        double *y = b.y + (int64_t)t * kMaxSpace;
        for (int i = 0; i < kMaxSpace; ++i) y[i] = i < m ? w.y[i] : 0.0;
    }
}

hipError_t launch_whole(const Batch &b, hipStream_t s) {
    const size_t lds = whole_lds_bytes(b.pl, b.dim, b.Na, b.Nb, b.nentA, b.nentB, b.Ha == b.Hb);
    if (b.max_space <= 12) hipLaunchKernelGGL(k_whole<12>, dim3(b.B), dim3(kWholeThreads), lds, s, b);
    else hipLaunchKernelGGL(k_whole<kMaxSpace>, dim3(b.B), dim3(kWholeThreads), lds, s, b);
    return hipGetLastError();
}

hipError_t init_whole_kernels() {
    const int dyn = kWholeMaxLds - (int)sizeof(WholeShared);
    hipError_t e = hipFuncSetAttribute((const void *)k_whole<12>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void *)k_whole<kMaxSpace>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
}

}  // namespace mbefci

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
#include "internal.h"

namespace mbefci {

typedef double dbl4 __attribute__((ext_vector_type(4)));

#define ERI_AT(eri, n, p, q, r, s) (eri)[((((int64_t)(p) * (n) + (q)) * (n) + (r)) * (n) + (s))]

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the block (blockDim.x a multiple of 64, at most 1024); result valid
// in every thread.  `sh` holds >= 16 doubles.
__device__ double block_sum(double v, double *sh) {
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

__device__ __forceinline__ const double *vref(const VecRef &r, int t, int64_t dim) {
    const int32_t k = r.idx ? r.idx[t] : r.idx_const;
    return r.base + (int64_t)t * r.tstride + (int64_t)k * dim;
}

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
        out[(int64_t)t * ostride + d] = e + ec;
    }
}

static int grid_for(int64_t work, int per_block, int cap) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

hipError_t launch_hdiag(const Batch &b, double *out, int64_t ostride, int add_ecore, hipStream_t s) {
    dim3 grid(grid_for(b.dim, 256, 4096), b.B);
    hipLaunchKernelGGL(k_hdiag, grid, dim3(256), 0, s, b, out, ostride, add_ecore);
    return hipGetLastError();
}

// ----------------------------------------------------------------- sigma --
// Knowles-Handy form with pair-symmetrised operators E+_P = E_pq + E_qp (p>q),
// E+_pp = E_pp:
//   D+_Q(K) = <K|E+_Q|c>          (gather over the single-excitation links of K)
//   W_P(K)  = 1/2 sum_Q (pq|rs) D+_Q(K) + k_P c_K   (FP64 MFMA, K-tile in LDS)
//   sigma_I = sum_P <I|E+_P|K> W_P(K)                (gather, no atomics)
// Links of string I list every (p,q) with E_pq|I> = sign|J>; with the
// determinant ordering alpha-major and alpha creators left of beta creators,
// alpha links act on the row index and beta links on the column index.

__device__ __forceinline__ void link_decode(uint32_t L, int &J, int &Q, double &sg) {
    J = (int)(L & 0xFFFFFu);
    Q = (int)((L >> 20) & 0x3FFu);
    sg = (L >> 31) ? -1.0 : 1.0;
}

size_t sigma_lds_bytes(const ParamLayout &pl) {
    return sizeof(double) * ((size_t)pl.Ppad * pl.ldE + (size_t)pl.Kpad * (kTile + 1));
}

// grid: (blocks per tuple, B); block 256 = 4 waves.  Each block stages the
// tuple's 1/2 (pq|rs) in LDS once and loops over 64-determinant tiles.
__global__ __launch_bounds__(256) void k_sigma_w(Batch b, VecRef cref, int tiles_per_block, int skip_done) {
    const int t = blockIdx.y;
    if (skip_done && b.status[t] != ST_RUNNING) return;
    extern __shared__ double lds[];
    const ParamLayout &pl = b.pl;
    const int ldE = pl.ldE, ldD = kTile + 1;
    double *E = lds;
    double *D = lds + pl.Ppad * ldE;
    const double *prm = b.params + (int64_t)t * pl.stride;
    const double *c = vref(cref, t, b.dim);
    double *w = b.W + (int64_t)t * pl.P * b.dim;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < pl.Ppad * pl.Kpad; i += 256) E[(i / pl.Kpad) * ldE + (i % pl.Kpad)] = prm[pl.off_eri + i];
    const double *kp = prm + pl.off_k;
    const int64_t ntiles = (b.dim + kTile - 1) / kTile;
    const int64_t tile_end = min((int64_t)(blockIdx.x + 1) * tiles_per_block, ntiles);
    const int mtiles = pl.Ppad / 16, ksteps = pl.Kpad / 4;
    for (int64_t tile = (int64_t)blockIdx.x * tiles_per_block; tile < tile_end; ++tile) {
        const int64_t d0 = tile * kTile;
        __syncthreads();
        for (int i = tid; i < pl.Kpad * ldD; i += 256) D[i] = 0.0;
        __syncthreads();
        const int64_t d = d0 + lane;
        const bool valid = d < b.dim;
        const int64_t Ka = valid ? d / b.Nb : 0, Kb = valid ? d % b.Nb : 0;
        if (valid) {
            const uint32_t *la = b.linkA + Ka * b.nentA;
            for (int e = wave; e < b.nentA; e += 4) {
                int J, Q;
                double sg;
                link_decode(la[e], J, Q, sg);
                D[Q * ldD + lane] += sg * c[(int64_t)J * b.Nb + Kb];
            }
        }
        __syncthreads();
        if (valid) {
            const uint32_t *lb = b.linkB + Kb * b.nentB;
            const double *crow = c + Ka * b.Nb;
            for (int e = wave; e < b.nentB; e += 4) {
                int J, Q;
                double sg;
                link_decode(lb[e], J, Q, sg);
                D[Q * ldD + lane] += sg * crow[J];
            }
        }
        __syncthreads();
        // W tile: rows P (mtiles x 16), columns wave*16 .. wave*16+15
        const int col = wave * 16 + (lane & 15), kr = lane >> 4, ar = lane & 15;
        const int64_t dd = d0 + col;
        const double cv = dd < b.dim ? c[dd] : 0.0;
        for (int mt = 0; mt < mtiles; ++mt) {
            dbl4 acc = {0.0, 0.0, 0.0, 0.0};
            for (int ks = 0; ks < ksteps; ++ks) {
                const double av = E[(mt * 16 + ar) * ldE + ks * 4 + kr];
                const double bv = D[(ks * 4 + kr) * ldD + col];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
            }
            if (dd < b.dim) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = mt * 16 + kr + 4 * v;   // f64 16x16x4 output: lane>>4 + 4*item
                    if (row < pl.P) w[(int64_t)row * b.dim + dd] = acc[v] + kp[row] * cv;
                }
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_sigma_g(Batch b, VecRef cref, VecRef sref, double shift, int skip_done) {
    const int t = blockIdx.y;
    if (skip_done && b.status[t] != ST_RUNNING) return;
    const double *w = b.W + (int64_t)t * b.pl.P * b.dim;
    const double *c = vref(cref, t, b.dim);
    double *sg_out = const_cast<double *>(vref(sref, t, b.dim));
    for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < b.dim;
         d += (int64_t)gridDim.x * blockDim.x) {
        const int64_t Ka = d / b.Nb, Kb = d % b.Nb;
        double acc = 0.0;
        const uint32_t *la = b.linkA + Ka * b.nentA;
        for (int e = 0; e < b.nentA; ++e) {
            int J, Q;
            double sg;
            link_decode(la[e], J, Q, sg);
            acc += sg * w[(int64_t)Q * b.dim + (int64_t)J * b.Nb + Kb];
        }
        const uint32_t *lb = b.linkB + Kb * b.nentB;
        const double *wrow = w + Ka * b.Nb;
        for (int e = 0; e < b.nentB; ++e) {
            int J, Q;
            double sg;
            link_decode(lb[e], J, Q, sg);
            acc += sg * wrow[(int64_t)Q * b.dim + J];
        }
        sg_out[d] = acc + shift * c[d];
    }
}

// ------------------------------------------------- column-strip variant --
// With C the coefficient matrix (alpha strings x beta strings) and E^a_P,
// E^b_P the spin parts of E+_P, the Hamiltonian splits as
//   sigma = H_a C + C H_b^T + sum_PQ (P|Q) E^a_P C (E^b_Q)^T,
// where H_s = sum_P k_P E^s_P + 1/2 sum_PQ (P|Q) E^s_P E^s_Q is the dense
// string Hamiltonian of one spin (an N_s x N_s matrix per tuple, applied as
// FP64 MFMA GEMMs).  The strip kernel computes the alpha-beta term: for each
// alpha string K the beta part D^b_Q(K, I_b) = <I_b|E^b_Q|C(K, .)> uses row K
// of C only; W = 1/2 (pq|rs) (2 D^b) (FP64 MFMA) is scattered through the
// alpha links of K.  A workgroup owns 16 beta columns and keeps the sigma
// strip sigma[:, B0..B0+15] in LDS.
//
// On this GPU an FP64 MFMA keeps the SIMD's vector ALU busy for its whole
// duration, so every vector instruction of the loop costs MFMA time; the
// loop is written to need few of them: per-item addresses and multipliers are
// precomputed, the per-string parts of the load addresses are scalar, and the
// host tables already hold strip byte offsets.

// Pair order inside the strip kernel: the n_A diagonal pairs (p,p) first, then
// the pairs p > q in packed order.  Returns the packed index p(p+1)/2 + q.
__host__ __device__ inline int strip_pair_packed(int qs, int nA) {
    if (qs < nA) return qs * (qs + 3) / 2;
    const int m = qs - nA;
    int p = 1;
    while ((p + 1) * p / 2 <= m) ++p;
    return p * (p + 1) / 2 + (m - p * (p - 1) / 2);
}

// Host tables of the strip kernel (columns in the strip pair order):
//  * link form [N_s][P]: J in bits 0-19, bit 30 set when the string has a link
//    through E+_Q, bit 31 its sign (a string has at most one link per pair);
//  * scatter form [N_s + 1][P + 1]: byte offset J * 128 of the target row of
//    the sigma strip for off-diagonal links, else the discard row (N_s * 128);
//    bit 31 the sign; column P and row N_s are all discard.
constexpr uint32_t kPairJ = 0xFFFFFu, kPairValid = 1u << 30, kPairSign = 1u << 31;

// Compile-time shape of the strip kernel for n_A active orbitals.
template <int NA>
struct StripShape {
    static constexpr int P = NA * (NA + 1) / 2;
    static constexpr int Ppad = (P + 15) / 16 * 16;
    static constexpr int Kpad = (P + 3) / 4 * 4;
    static constexpr int KS = Kpad / 4;                        // MFMA K steps
    static constexpr int MT = Ppad / 16 < 4 ? Ppad / 16 : 4;   // waves, one 16-row tile each (distinct SIMDs)
    static constexpr int NX = Ppad / 16 - MT;                  // tiles past row 64, K split over the waves
    static constexpr int XR = P > 64 ? P - 64 : 0;             // pair rows past 64
    static constexpr int NTH = 64 * MT;
    static constexpr int NXI = (XR * 16 + NTH - 1) / NTH;      // items per thread on rows past 64
    static constexpr int KQ = (KS + 3) / 4;                    // K steps per wave in a tile past row 64
    static constexpr int NI = 4 + NXI;                         // D / scatter items per thread
};

// LDS of the strip kernel (doubles): sigma strip [Na + 1][16] (row Na is a
// discard row for masked-off stores), D [2][Ppad][16] (rows past Kpad are
// written with zeros and never read), per-wave partial W of rows past 64
// [2][4][XR][16].
static size_t strip_lds(const ParamLayout &pl, int64_t Na) {
    const int xr = pl.P > 64 ? pl.P - 64 : 0;
    return sizeof(double) * ((size_t)(Na + 1) * kStrip + 2 * (size_t)pl.Ppad * kStrip + 8 * (size_t)xr * kStrip);
}

size_t strip_lds_bytes(const ParamLayout &pl, int64_t Na) { return strip_lds(pl, Na); }

bool strip_fits(const ParamLayout &pl, int64_t Na, int, int) {
    return pl.nA >= 1 && pl.nA <= kMaxActive && strip_lds(pl, Na) <= 160 * 1024 && Na < (1 << 24);
}

// Workgroups are handed to the 8 XCDs round-robin by linear id; map id L to
// (tuple, strip) so that every strip of tuple t runs on XCD t % 8 and the
// strips of one tuple are dispatched back to back: its vector stays in that
// XCD's L2 while they run.
__device__ __forceinline__ bool xcd_map(int64_t L, int nstrips, int B, int &t, int &strip) {
    const int64_t xcd = L % kXcds, j = L / kXcds;
    t = (int)((j / nstrips) * kXcds + xcd);
    strip = (int)(j % nstrips);
    return t < B;
}

// Sum of x over the four lanes l, l^16, l^32, l^48 (the (lane >> 4) groups of
// an MFMA output column), as ((x0 + x1) + (x2 + x3)) in every one of them:
// row swaps of 16 and 32 lanes on the vector ALU, no LDS round trip.
__device__ __forceinline__ double sum_over_kr(double x) {
    const unsigned lo = __double2loint(x), hi = __double2hiint(x);
    const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    const double s = __hiloint2double(b[0], a[0]) + __hiloint2double(b[1], a[1]);
    const unsigned lo2 = __double2loint(s), hi2 = __double2hiint(s);
    const auto c = __builtin_amdgcn_permlane32_swap(lo2, lo2, false, false);
    const auto d = __builtin_amdgcn_permlane32_swap(hi2, hi2, false, false);
    return __hiloint2double(d[0], c[0]) + __hiloint2double(d[1], c[1]);
}

// One workgroup per (tuple, 16-column strip), MT waves.  Thread items: the
// pair rows Q = 16 w + (lane >> 4) + 4 v (v < 4) of its wave's MFMA output
// tile, column lane & 15, plus rows past 64 spread over the block.  The same
// thread writes D for its items and scatters W of those items (rows < 64
// straight from the MFMA registers).  The diagonal pairs are rows 0..n_A-1,
// all in wave 0, which sums them for the string with a lane mask and two
// cross-lane row swaps.  Software pipeline over the alpha strings, one barrier
// per step: in the step of string K the block
//   - runs the MFMA of string K on D[K & 1] (results read one step later),
//   - stores the partial rows past 64 of W(K-1) and sums its diagonal pairs,
//   - scatters W of string K-2 into the LDS strip and adds its diagonal sum,
//   - writes D of string K+1 into D[(K+1) & 1] from C row K+1,
//   - loads row K+2 of C at the beta-link columns of its items and the
//     scatter-table row of string K+2.
// Each phase touches a buffer no other phase of the same step touches, and
// the scatter of one string has no write conflicts: each link of a string
// reaches a different string, and its diagonal sum goes to the string itself.
// Masked-off stores go to the discard row, so the step has no branches
// besides wave 0's diagonal sum.
template <int NA>
__global__ __launch_bounds__(64 * StripShape<NA>::MT) void k_sigma_strip(Batch b, VecRef cref, VecRef sref,
                                                                          double shift, int skip_done) {
    using S = StripShape<NA>;
    constexpr int P = S::P, KP = S::Kpad, DR = S::Ppad, KS = S::KS, NX = S::NX, XR = S::XR, NTH = S::NTH,
                  NI = S::NI, KQ = S::KQ, NXA = NX > 0 ? NX : 1;
    constexpr uint32_t DB = DR * kStrip * sizeof(double);   // byte stride of the D buffers
    const int nstrips = (int)((b.Nb + kStrip - 1) / kStrip);
    int t, strip_id;
    if (!xcd_map(blockIdx.x, nstrips, b.B, t, strip_id)) return;
    if (skip_done && b.status[t] != ST_RUNNING) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int ar = lane & 15, kr = lane >> 4;
    // determinant indices fit 32 bits (dim <= C(13,6)^2)
    const uint32_t Na = (uint32_t)b.Na, Nb = (uint32_t)b.Nb;
    const uint32_t B0 = (uint32_t)strip_id * kStrip;
    const bool colok = B0 + ar < Nb;
    extern __shared__ double lds[];
    double *strip = lds;                   // [Na + 1][16]
    double *D = strip + (Na + 1) * kStrip; // [2][DR][16]
    double *Wx = D + 2 * DR * kStrip;      // [2][4][XR][16]
    double *const dump = strip + Na * kStrip + ar;
    const ParamLayout &pl = b.pl;
    const double *prm = b.params + (int64_t)t * pl.stride;
    const double *c = vref(cref, t, b.dim);
    double *sg = const_cast<double *>(vref(sref, t, b.dim));
    const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(c), (short)0,
                                                                        (int)(b.dim * sizeof(double)), 0x00020000);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint32_t *>(b.scatA), (short)0, (int)((Na + 1) * (P + 1) * sizeof(uint32_t)), 0x00020000);

    // A fragments of 1/2 (pq|rs) in the strip pair order: this wave's rows,
    // and its K quarter of the rows past 64
    auto eri_at = [&](int r, int k) -> double {
        return (r < P && k < P) ? prm[pl.off_eri + strip_pair_packed(r, NA) * KP + strip_pair_packed(k, NA)] : 0.0;
    };
    double af[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) af[ks] = eri_at(w * 16 + ar, ks * 4 + kr);
    double afx[NXA][KQ];
#pragma unroll
    for (int x = 0; x < NXA; ++x)
#pragma unroll
        for (int j = 0; j < KQ; ++j) {
            const int ks = w * KQ + j;
            afx[x][j] = (x < NX && ks < KS) ? eri_at(64 + 16 * x + ar, ks * 4 + kr) : 0.0;
        }
    // items: pair row, D slot (LDS byte address in buffer 0), beta link
    // (byte offset in a row of C, 2 * sign), scatter-table byte offset
    int qi[NI];
    uint32_t dsl[NI], boff[NI], qa[NI];
    double bmul[NI];
#pragma unroll
    for (int v = 0; v < 4; ++v) qi[v] = w * 16 + kr + 4 * v;
#pragma unroll
    for (int r = 0; r < NI - 4; ++r) {
        const int j = tid + NTH * r;
        qi[4 + r] = j < XR * 16 ? 64 + (j >> 4) : P;
    }
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const bool ok = colok && qi[i] < P;
        const uint32_t eb = ok ? b.pairB[(B0 + ar) * (uint32_t)P + qi[i]] : 0u;
        const bool vb = (eb & kPairValid) != 0;
        boff[i] = vb ? (eb & kPairJ) * (uint32_t)sizeof(double) : 0u;
        bmul[i] = vb ? ((eb & kPairSign) ? -2.0 : 2.0) : 0.0;
        qa[i] = (uint32_t)(qi[i] < P ? qi[i] : P) * (uint32_t)sizeof(uint32_t);
        dsl[i] = (uint32_t)(D + qi[i] * kStrip + ar - lds) * (uint32_t)sizeof(double);
    }
    for (uint32_t i = tid; i < (Na + 1) * kStrip; i += NTH) strip[i] = 0.0;
    for (int i = tid; i < 2 * DR * kStrip; i += NTH) D[i] = 0.0;

    const uint32_t rowC = Nb * (uint32_t)sizeof(double), rowS = (P + 1) * (uint32_t)sizeof(uint32_t);
    auto lds_at = [&](uint32_t byte) -> double * { return reinterpret_cast<double *>(reinterpret_cast<char *>(lds) + byte); };
    auto load_c = [&](uint32_t s, int i) -> double {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rc, boff[i], s * rowC, 0));
    };
    auto load_s = [&](uint32_t s, int i) -> uint32_t {
        return __builtin_amdgcn_raw_buffer_load_b32(rs, qa[i], s * rowS, 0);
    };

    // rows past 64: few of them (n_A = 11) go through vector FMAs on this
    // wave's K quarter instead of a mostly empty MFMA tile
    constexpr bool XV = NX == 1 && XR <= 4;
    constexpr int XVR = XV ? XR : 1;
    double axv[XVR][KQ];
#pragma unroll
    for (int r = 0; r < XVR; ++r)
#pragma unroll
        for (int j = 0; j < KQ; ++j) {
            const int ks = w * KQ + j;
            axv[r][j] = (XV && ks < KS) ? eri_at(64 + r, ks * 4 + kr) : 0.0;
        }
    const uint32_t ar8 = (uint32_t)ar * (uint32_t)sizeof(double);
    double cb[NI];
    uint32_t eA[NI], eB[NI];   // scatter entries (string K-2 is scattered, string K-1 loaded, alternately)
    double w2[4];              // W of string K-2 on this thread's wave rows
    double dg1 = 0.0;          // diagonal sum of the previous string (wave 0)
    // prologue: D of string 0 and C row 1
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        cb[i] = load_c(0, i);
        eA[i] = load_s(Na, i);   // discard row
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NI; ++i) *lds_at(dsl[i]) = bmul[i] * cb[i];
#pragma unroll
    for (int i = 0; i < NI; ++i) cb[i] = load_c(Na > 1 ? 1u : 0u, i);
#pragma unroll
    for (int v = 0; v < 4; ++v) w2[v] = 0.0;
    uint32_t sa1 = 0u;   // alpha string K-1
    dbl4 accA[1 + NXA], accB[1 + NXA];   // the wave tile, then the rows past 64
#pragma unroll
    for (int j = 0; j < 1 + NXA; ++j) accA[j] = accB[j] = dbl4{0.0, 0.0, 0.0, 0.0};
    __syncthreads();

    // Pipeline step of string K: MFMA of K into `an` (read back one step
    // later, so no wave waits for its own MFMA results), epilogue of K-1
    // from `ao`, scatter of K-2 with entries `ep` while the entries of K-1
    // load into `en`, D of K+1, C row K+2.  Steps past the last string run on
    // stale data whose results are discarded: their scatter entries come from
    // the discard row and their diagonal sums are dropped.
    auto step = [&](uint32_t K, dbl4 (&an)[1 + NXA], dbl4 (&ao)[1 + NXA], uint32_t (&ep)[NI],
                    uint32_t (&en)[NI]) {
        const double *Dk = D + (K & 1) * DR * kStrip;
        {
            double bv[KS];
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) bv[ks] = Dk[(ks * 4 + kr) * kStrip + ar];
            dbl4 a = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) a = __builtin_amdgcn_mfma_f64_16x16x4f64(af[ks], bv[ks], a, 0, 0, 0);
            an[0] = a;
        }
        if (NX > 0) {
            // rows past 64: this wave's K quarter (its own B operands)
            double bx[KQ];
#pragma unroll
            for (int j = 0; j < KQ; ++j) {
                const int ks = w * KQ + j;
                bx[j] = Dk[((ks < KS ? ks : 0) * 4 + kr) * kStrip + ar];
            }
            if (XV) {
                // lane (kr, ar): partial over k = kr (mod 4) of the quarter, then summed over kr
#pragma unroll
                for (int r = 0; r < XVR; ++r) {
                    double pr = 0.0;
#pragma unroll
                    for (int j = 0; j < KQ; ++j) pr = __builtin_fma(axv[r][j], bx[j], pr);
                    an[1][r] = sum_over_kr(pr);
                }
            } else {
#pragma unroll
                for (int x = 0; x < NXA; ++x) {
                    dbl4 a = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int j = 0; j < KQ; ++j) a = __builtin_amdgcn_mfma_f64_16x16x4f64(afx[x][j], bx[j], a, 0, 0, 0);
                    an[1 + x] = a;
                }
            }
        }
        // epilogue of string K-1: this wave's partial rows past 64 to LDS
        if (NX > 0) {
            double *wx = Wx + (((K + 1) & 1) * 4 + w) * XR * kStrip;
            if (XV) {
#pragma unroll
                for (int r = 0; r < XVR; ++r) *(kr == 0 ? wx + r * kStrip + ar : dump) = ao[1][r];
            } else {
#pragma unroll
                for (int x = 0; x < NXA; ++x)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int r = 16 * x + kr + 4 * v;
                        *(r < XR ? wx + r * kStrip + ar : dump) = ao[1 + x][v];
                    }
            }
        }
        // scatter of string K-2 through its off-diagonal alpha links
        const double *wx2 = Wx + (K & 1) * 4 * XR * kStrip;
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const uint32_t e = ep[i];
            double wv;
            if (i < 4) {
                wv = w2[i < 4 ? i : 0];
            } else {
                const int r = qi[i] < P ? qi[i] - 64 : 0;
                wv = wx2[r * kStrip + ar] + wx2[(XR + r) * kStrip + ar] + wx2[(2 * XR + r) * kStrip + ar] +
                     wx2[(3 * XR + r) * kStrip + ar];
            }
            // strip row at byte offset e & 0x7FFFFFFF (a multiple of 128), column ar; sign in bit 31
            double *d = lds_at((e & 0x7FFFFFFFu) | ar8);
            *d += __hiloint2double(__double2hiint(wv) ^ (int)(e & kPairSign), __double2loint(wv));
        }
        // D of string K+1 (C row K+1 was loaded one step ago)
#pragma unroll
        for (int i = 0; i < NI; ++i) *lds_at(dsl[i] + ((K + 1) & 1) * DB) = bmul[i] * cb[i];
        // loads: C row K+2, scatter entries of string K-1 (scattered next step)
        const uint32_t K2c = K + 2 < Na ? K + 2 : Na - 1, K1s = (K >= 1 && K - 1 < Na) ? K - 1 : Na;
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            cb[i] = load_c(K2c, i);
            en[i] = load_s(K1s, i);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) w2[v] = ao[0][v];
        // diagonal pairs: rows 0..NA-1 of wave 0.  Add the sum of string K-2,
        // then form the sum of string K-1 (lane mask of its occupied orbitals,
        // fixed order: v within the lane, then lanes (kr, kr^1), then (kr, kr^2)).
        if (w == 0) {
            if (kr == 0 && K >= 2 && K - 2 < Na) strip[(K - 2) * kStrip + ar] += dg1;
            double s = 0.0;
#pragma unroll
            for (int v = 0; v < 4; ++v)
                if (4 * v < NA) s += ((sa1 >> (kr + 4 * v)) & 1u) ? ao[0][v] : 0.0;
            dg1 = sum_over_kr(s);
        }
        const uint32_t sk = b.strA[K < Na ? K : Na - 1];
        sa1 = K < Na ? sk : 0u;
        __syncthreads();
    };
    for (uint32_t K = 0; K < Na + 2; K += 2) {
        step(K, accA, accB, eA, eB);
        step(K + 1, accB, accA, eB, eA);
    }
    for (uint32_t i = tid; i < Na * kStrip; i += NTH) {
        const uint32_t row = i / kStrip, col = i % kStrip;
        if (B0 + col < Nb) {
            const uint32_t d = row * Nb + B0 + col;
            sg[d] = strip[i] + shift * c[d];
        }
    }
}

// Dense string Hamiltonian of one spin (symmetric, N x N per tuple); thread J
// writes row J:
//   H e_J = sum_{links (Q,K,s) of J} s [ k_Q e_K + 1/2 sum_{links (P,I,s') of K} s' (P|Q) e_I ].
__global__ __launch_bounds__(64) void k_build_h(Batch b, int beta) {
    const int t = blockIdx.y;
    const int64_t N = beta ? b.Nb : b.Na;
    const int nent = beta ? b.nentB : b.nentA;
    const uint32_t *links = beta ? b.linkB : b.linkA;
    const int64_t J = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (J >= N) return;
    const ParamLayout &pl = b.pl;
    const double *prm = b.params + (int64_t)t * pl.stride;
    double *row = (beta ? b.Hb : b.Ha) + ((int64_t)t * N + J) * N;
    for (int64_t i = 0; i < N; ++i) row[i] = 0.0;
    const uint32_t *lj = links + J * nent;
    for (int e = 0; e < nent; ++e) {
        int K, Q;
        double s;
        link_decode(lj[e], K, Q, s);
        row[K] += s * prm[pl.off_k + Q];
        const uint32_t *lk = links + (int64_t)K * nent;
        for (int f = 0; f < nent; ++f) {
            int I, P;
            double s2;
            link_decode(lk[f], I, P, s2);
            row[I] += s * s2 * prm[pl.off_eri + P * pl.Kpad + Q];   // stored as 1/2 (P|Q)
        }
    }
}

hipError_t launch_build_hb(const Batch &b, hipStream_t s) {
    if (b.sigma_variant != SIGMA_STRIP) return hipSuccess;
    hipLaunchKernelGGL(k_build_h, dim3((unsigned)((b.Nb + 63) / 64), b.B), dim3(64), 0, s, b, 1);
    if (b.Ha != b.Hb)
        hipLaunchKernelGGL(k_build_h, dim3((unsigned)((b.Na + 63) / 64), b.B), dim3(64), 0, s, b, 0);
    return hipGetLastError();
}

// sigma += H_a C + C H_b per tuple (C = c as Na x Nb row-major; H_a, H_b
// symmetric): 64 x 64 output tile per block of 4 waves (2 x 2), each wave
// 32 x 32 = 2 x 2 FP64 MFMA tiles.  K runs over H_a C (K = Na) and then C H_b
// (K = Nb) in chunks of 16 staged through a double-buffered LDS tile: the
// next chunk's global loads are in flight while the current one is
// multiplied, one barrier per chunk.  Rows and columns past the matrix are
// read clamped (their results are not stored); K past the end reads as zero.
constexpr int kGK = 16;
__global__ __launch_bounds__(256) void k_gemm_h(Batch b, VecRef cref, VecRef sref, int skip_done) {
    const int t = blockIdx.z;
    if (skip_done && b.status[t] != ST_RUNNING) return;
    const int Na = (int)b.Na, Nb = (int)b.Nb;
    const double *C = vref(cref, t, b.dim);
    double *S = const_cast<double *>(vref(sref, t, b.dim));
    const double *Ha = b.Ha + (int64_t)t * Na * Na;
    const double *Hb = b.Hb + (int64_t)t * Nb * Nb;
    __shared__ double As[2][64][kGK + 1];
    __shared__ double Bs[2][kGK][64 + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wy = wave >> 1, wx = wave & 1;
    const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
    // staging: A rows (tid >> 2), 4 consecutive k from (tid & 3) * 4; B row k = tid >> 4, 4 columns from (tid & 15) * 4
    const int sa_r = tid >> 2, sa_k = (tid & 3) * 4, sb_k = tid >> 4, sb_c = (tid & 15) * 4;
    const int arow = min(r0 + sa_r, Na - 1);
    int bcol[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) bcol[e] = min(c0 + sb_c + e, Nb - 1);
    const int nc0 = (Na + kGK - 1) / kGK, nc = nc0 + (Nb + kGK - 1) / kGK;
    double ra[4], rb[4];
    auto load = [&](int j) {
        const bool p1 = j >= nc0;
        const int k0 = (p1 ? j - nc0 : j) * kGK, K = p1 ? Nb : Na;
        const double *X = p1 ? C : Ha;
        const int ldX = p1 ? Nb : Na;
        const double *Y = p1 ? Hb : C;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int ka = k0 + sa_k + e;
            ra[e] = ka < K ? X[(int64_t)arow * ldX + ka] : 0.0;
        }
        const int kb = k0 + sb_k;
#pragma unroll
        for (int e = 0; e < 4; ++e) rb[e] = kb < K ? Y[(int64_t)kb * Nb + bcol[e]] : 0.0;
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int e = 0; e < 4; ++e) As[buf][sa_r][sa_k + e] = ra[e];
#pragma unroll
        for (int e = 0; e < 4; ++e) Bs[buf][sb_k][sb_c + e] = rb[e];
    };
    dbl4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
    load(0);
    store(0);
    __syncthreads();
    for (int j = 0; j < nc; ++j) {
        const int buf = j & 1;
        if (j + 1 < nc) load(j + 1);
#pragma unroll
        for (int ks = 0; ks < kGK / 4; ++ks) {
            double af[2], bf[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) af[i] = As[buf][wy * 32 + i * 16 + (lane & 15)][ks * 4 + (lane >> 4)];
#pragma unroll
            for (int i = 0; i < 2; ++i) bf[i] = Bs[buf][ks * 4 + (lane >> 4)][wx * 32 + i * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int q = 0; q < 2; ++q) acc[i][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[q], acc[i][q], 0, 0, 0);
        }
        if (j + 1 < nc) store(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gr = r0 + wy * 32 + i * 16 + (lane >> 4) + 4 * v;
                const int gc = c0 + wx * 32 + q * 16 + (lane & 15);
                if (gr < Na && gc < Nb) S[(int64_t)gr * Nb + gc] += acc[i][q][v];
            }
}

template <int NA>
static hipError_t launch_strip_na(const Batch &b, VecRef c, VecRef sig, double shift, int skip, hipStream_t s) {
    const int64_t nstrips = (b.Nb + kStrip - 1) / kStrip;
    const dim3 grid((unsigned)(((b.B + kXcds - 1) / kXcds) * kXcds * nstrips));
    hipLaunchKernelGGL(k_sigma_strip<NA>, grid, dim3(StripShape<NA>::NTH), strip_lds(b.pl, b.Na), s, b, c, sig,
                       shift, skip);
    return hipGetLastError();
}

static hipError_t launch_strip(const Batch &b, VecRef c, VecRef sig, double shift, int skip, hipStream_t s) {
    switch (b.nA) {
        case 1: return launch_strip_na<1>(b, c, sig, shift, skip, s);
        case 2: return launch_strip_na<2>(b, c, sig, shift, skip, s);
        case 3: return launch_strip_na<3>(b, c, sig, shift, skip, s);
        case 4: return launch_strip_na<4>(b, c, sig, shift, skip, s);
        case 5: return launch_strip_na<5>(b, c, sig, shift, skip, s);
        case 6: return launch_strip_na<6>(b, c, sig, shift, skip, s);
        case 7: return launch_strip_na<7>(b, c, sig, shift, skip, s);
        case 8: return launch_strip_na<8>(b, c, sig, shift, skip, s);
        case 9: return launch_strip_na<9>(b, c, sig, shift, skip, s);
        case 10: return launch_strip_na<10>(b, c, sig, shift, skip, s);
        case 11: return launch_strip_na<11>(b, c, sig, shift, skip, s);
        case 12: return launch_strip_na<12>(b, c, sig, shift, skip, s);
        case 13: return launch_strip_na<13>(b, c, sig, shift, skip, s);
        default: return hipErrorInvalidValue;
    }
}


hipError_t launch_sigma(const Batch &b, VecRef c, VecRef sig, double shift, bool skip_done,
                        hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, hipEvent_t ev2) {
    if (b.sigma_variant == SIGMA_STRIP) {
        if (ev0) (void)hipEventRecord(ev0, s);
        hipError_t e = launch_strip(b, c, sig, shift, skip_done ? 1 : 0, s);
        if (e != hipSuccess) return e;
        if (ev1) (void)hipEventRecord(ev1, s);
        const dim3 grid((unsigned)((b.Nb + 63) / 64), (unsigned)((b.Na + 63) / 64), b.B);
        hipLaunchKernelGGL(k_gemm_h, grid, dim3(256), 0, s, b, c, sig, skip_done ? 1 : 0);
        e = hipGetLastError();
        if (ev2) (void)hipEventRecord(ev2, s);
        return e;
    }
    const int64_t ntiles = (b.dim + kTile - 1) / kTile;
    // aim for >= ~2048 blocks over the batch, at most 32 tiles per block
    int64_t want_blocks = (2048 + b.B - 1) / b.B;
    int tpb = (int)((ntiles + want_blocks - 1) / want_blocks);
    if (tpb < 1) tpb = 1;
    if (tpb > 32) tpb = 32;
    const int gx = (int)((ntiles + tpb - 1) / tpb);
    const size_t lds = sigma_lds_bytes(b.pl);
    if (ev0) (void)hipEventRecord(ev0, s);
    hipLaunchKernelGGL(k_sigma_w, dim3(gx, b.B), dim3(256), lds, s, b, c, tpb, skip_done ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev1) (void)hipEventRecord(ev1, s);
    dim3 grid(grid_for(b.dim, 256, 4096), b.B);
    hipLaunchKernelGGL(k_sigma_g, grid, dim3(256), 0, s, b, c, sig, shift, skip_done ? 1 : 0);
    e = hipGetLastError();
    if (ev2) (void)hipEventRecord(ev2, s);
    return e;
}

// -------------------------------------------------------------- Davidson --
// Per-tuple state lives in the Batch arrays.  Vector kernels use grid
// (nblk, B) and write block partials to part[t][blk][*]; per-tuple kernels
// (one block of 64 threads per tuple) sum them in block order.

__device__ __forceinline__ double *parts(const Batch &b, int t, int blk) {
    return b.part + ((int64_t)t * (b.nblk + 1) + blk) * kParts;
}

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

// H_PP[i][j] = H_a[Ia][Ja] d(Ib,Jb) + H_b[Ib][Jb] d(Ia,Ja)
//            + sum_PQ (P|Q) <Ia|E+_P|Ja> <Ib|E+_Q|Jb>  (upper triangle, mirrored)
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
        H[i * kPsp + j] = v;
        H[j * kPsp + i] = v;
    }
}

// Householder tridiagonalisation of H_PP in LDS (one block per tuple), Q
// formed explicitly, and the lowest eigenvector of H_PP (bisection on T for
// the lowest eigenvalue, inverse iteration, y = Q z).
__device__ double block_sum256(double v, double *sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ __launch_bounds__(256) void k_psp_factor(Batch b) {
    const int t = blockIdx.x, tid = threadIdx.x, n = b.psp;
    constexpr int LD = kPsp + 1;
    extern __shared__ double lds[];
    double *A = lds;                 // [n][LD]
    double *vec = A + kPsp * LD;     // [kPsp] p, then z
    double *sh = vec + kPsp;         // [8]
    double *cpv = sh + 8;            // [kPsp] Thomas multipliers
    double *gQ = b.pQ + (int64_t)t * kPsp * kPsp;
    double *dT = b.pT + (int64_t)t * 3 * kPsp, *eT = dT + kPsp, *yv = eT + kPsp;
    for (int idx = tid; idx < n * n; idx += 256) A[(idx / n) * LD + idx % n] = gQ[(idx / n) * kPsp + idx % n];
    __syncthreads();
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;
        double part = 0.0;
        for (int i = tid; i < m; i += 256) part += A[(k + 1 + i) * LD + k] * A[(k + 1 + i) * LD + k];
        const double s2 = block_sum256(part, sh);
        const double x0 = A[(k + 1) * LD + k];
        const double alpha = x0 > 0.0 ? -sqrt(s2) : sqrt(s2);
        const double v0 = x0 - alpha;
        const double vn2 = s2 - x0 * x0 + v0 * v0;
        __syncthreads();
        if (!(vn2 > 1e-300)) {   // column already reduced: no reflection
            if (tid == 0) eT[k] = x0;
            for (int i = tid; i < m; i += 256) A[(k + 1 + i) * LD + k] = 0.0;
            __syncthreads();
            continue;
        }
        if (tid == 0) eT[k] = alpha;
        const double inv = 1.0 / sqrt(vn2);
        for (int i = tid; i < m; i += 256) A[(k + 1 + i) * LD + k] = (i == 0 ? v0 : A[(k + 1 + i) * LD + k]) * inv;
        __syncthreads();
        // p = B v over the trailing block B = A[k+1.., k+1..]
        for (int i = tid; i < m; i += 256) {
            double s = 0.0;
            for (int j = 0; j < m; ++j) s += A[(k + 1 + i) * LD + k + 1 + j] * A[(k + 1 + j) * LD + k];
            vec[i] = s;
        }
        __syncthreads();
        part = 0.0;
        for (int i = tid; i < m; i += 256) part += A[(k + 1 + i) * LD + k] * vec[i];
        const double K = block_sum256(part, sh);
        // B -= v w^T + w v^T, w = 2 p - 2 K v
        for (int idx = tid; idx < m * m; idx += 256) {
            const int i = idx / m, j = idx % m;
            const double vi = A[(k + 1 + i) * LD + k], vj = A[(k + 1 + j) * LD + k];
            const double wi = 2.0 * vec[i] - 2.0 * K * vi, wj = 2.0 * vec[j] - 2.0 * K * vj;
            A[(k + 1 + i) * LD + k + 1 + j] -= vi * wj + wi * vj;
        }
        __syncthreads();
    }
    for (int i = tid; i < n; i += 256) dT[i] = A[i * LD + i];
    if (tid == 0 && n >= 2) eT[n - 2] = A[(n - 1) * LD + n - 2];
    if (tid == 0) eT[n - 1] = 0.0;
    // Householder vectors to global (lower part), then Q = H_0 ... H_{n-3} in LDS
    for (int idx = tid; idx < n * n; idx += 256) {
        const int i = idx / n, j = idx % n;
        gQ[i * kPsp + j] = (j + 2 < n && i > j) ? A[i * LD + j] : 0.0;
    }
    __syncthreads();
    for (int idx = tid; idx < n * n; idx += 256) A[(idx / n) * LD + idx % n] = (idx / n == idx % n) ? 1.0 : 0.0;
    __syncthreads();
    for (int k = n - 3; k >= 0; --k) {
        const int m = n - k - 1;
        for (int c = tid; c < n; c += 256) {
            double s = 0.0;
            for (int r = 0; r < m; ++r) s += gQ[(k + 1 + r) * kPsp + k] * A[(k + 1 + r) * LD + c];
            s *= 2.0;
            for (int r = 0; r < m; ++r) A[(k + 1 + r) * LD + c] -= s * gQ[(k + 1 + r) * kPsp + k];
        }
        __syncthreads();
    }
    // lowest eigenvalue of T by bisection (Sturm counts), then inverse iteration
    if (tid == 0) {
        double lo = 1e300, hi = -1e300;
        for (int i = 0; i < n; ++i) {
            const double r = (i > 0 ? fabs(eT[i - 1]) : 0.0) + (i + 1 < n ? fabs(eT[i]) : 0.0);
            lo = fmin(lo, dT[i] - r);
            hi = fmax(hi, dT[i] + r);
        }
        const double span = fmax(hi - lo, 1e-300);
        for (int it = 0; it < 200 && hi - lo > 1e-15 * span; ++it) {
            const double x = 0.5 * (lo + hi);
            int cnt = 0;
            double q = 1.0;
            for (int i = 0; i < n; ++i) {
                q = dT[i] - x - (i > 0 ? eT[i - 1] * eT[i - 1] / q : 0.0);
                if (q == 0.0) q = -1e-300;
                cnt += q < 0.0;
            }
            if (cnt >= 1) hi = x; else lo = x;
        }
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
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += A[i * LD + j] * vec[j];
        yv[i] = s;
    }
    for (int idx = tid; idx < n * n; idx += 256) gQ[(idx / n) * kPsp + idx % n] = A[(idx / n) * LD + idx % n];
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
// diagonal preconditioner); the changes of |T|^2 and of the projections
// V_i . T (x . T on restart) go to the extra partial block.
template <int MS>
__global__ __launch_bounds__(kPsp) void k_psp_fix(Batch b) {
    const int t = blockIdx.x, i = threadIdx.x, n = b.psp;
    if (b.status[t] != ST_RUNNING) return;
    const int m = b.m[t], rs = b.restart[t];
    const double th = b.theta[t];
    const double *yy = b.y + (int64_t)t * kMaxSpace;
    const double *V = b.V + (int64_t)t * b.max_space * b.dim;
    const double *S = b.S + (int64_t)t * b.max_space * b.dim;
    double *T = b.T + (int64_t)t * b.dim;
    const double *Q = b.pQ + (int64_t)t * kPsp * kPsp;
    const double *dT = b.pT + (int64_t)t * 3 * kPsp, *eT = dT + kPsp;
    __shared__ double r[kPsp], w[kPsp], cp[kPsp], red[2][MS + 2];
    int64_t d = 0;
    double x = 0.0, told = 0.0;
    if (i < n) {
        d = b.pidx[(int64_t)t * kPsp + i];
        double ax = 0.0;
        if (rs) {
            x = V[d];
            ax = S[d];
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
    double acc[MS + 2];
#pragma unroll
    for (int k = 0; k < MS + 2; ++k) acc[k] = 0.0;
    if (i < n) {
        double tv = 0.0;
        for (int k = 0; k < n; ++k) tv += Q[i * kPsp + k] * w[k];
        T[d] = tv;
        const double dt = tv - told;
        acc[1] = tv * tv - told * told;
        if (rs) {
            acc[2] = x * dt;
        } else {
#pragma unroll
            for (int k = 0; k < MS; ++k)
                if (k < m) acc[2 + k] = V[(int64_t)k * b.dim + d] * dt;
        }
    }
    const int nx = 2 + (rs ? 1 : m);
#pragma unroll
    for (int k = 0; k < MS + 2; ++k) {
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
}

hipError_t launch_init_state(const Batch &b, hipStream_t s) {
    hipLaunchKernelGGL(k_init_state, dim3((b.B + 255) / 256), dim3(256), 0, s, b);
    return hipGetLastError();
}

// partial dots V_i . y for i < m[t] + nx_extra (running tuples only; with
// only2, only those whose correction needs a second Gram-Schmidt pass)
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

// G column m: G[i][m] = G[m][i] = V_i . S_m for i <= m; then m += 1
__global__ void k_update_G(Batch b) {
    const int t = blockIdx.x;
    if (b.status[t] != ST_RUNNING) return;
    const int m = b.m[t];
    double *G = b.G + (int64_t)t * kMaxSpace * kMaxSpace;
    if ((int)threadIdx.x <= m) {
        const double v = sum_parts(b, t, threadIdx.x);
        G[threadIdx.x * kMaxSpace + m] = v;
        G[m * kMaxSpace + threadIdx.x] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) b.m[t] = m + 1;
}

hipError_t launch_dots(const Batch &b, VecRef y, int nx_extra, hipStream_t s) {
    if (b.max_space <= 12) hipLaunchKernelGGL(k_dots<12>, dim3(b.nblk, b.B), dim3(256), 0, s, b, y, nx_extra, 0);
    else hipLaunchKernelGGL(k_dots<kMaxSpace>, dim3(b.nblk, b.B), dim3(256), 0, s, b, y, nx_extra, 0);
    if (nx_extra == 1) hipLaunchKernelGGL(k_update_G, dim3(b.B), dim3(64), 0, s, b);
    return hipGetLastError();
}

// Lowest eigenpair of the m x m projected matrix by cyclic Jacobi with a
// parallel (round-robin) rotation order; one block of 64 threads per tuple.
__global__ __launch_bounds__(64) void k_small_eig(Batch b) {
    const int t = blockIdx.x;
    const int32_t st0 = b.status[t];
    if (st0 != ST_RUNNING && st0 != ST_RESTART) return;
    __syncthreads();
    if (threadIdx.x == 0 && st0 == ST_RESTART) b.status[t] = ST_RUNNING;
    const int m = b.m[t];
    const int mm = m + (m & 1);                  // even number of players
    __shared__ double A[kMaxSpace + 1][kMaxSpace + 2];
    __shared__ double Vv[kMaxSpace + 1][kMaxSpace + 2];
    __shared__ double cs[(kMaxSpace + 2) / 2], sn[(kMaxSpace + 2) / 2];
    __shared__ int pa[(kMaxSpace + 2) / 2], pb[(kMaxSpace + 2) / 2];
    __shared__ int order[kMaxSpace + 2];
    __shared__ int done;
    const int tid = threadIdx.x;
    const double *G = b.G + (int64_t)t * kMaxSpace * kMaxSpace;
    for (int i = tid; i < mm * mm; i += 64) {
        const int r = i / mm, c = i % mm;
        A[r][c] = (r < m && c < m) ? G[r * kMaxSpace + c] : 0.0;
        Vv[r][c] = (r == c) ? 1.0 : 0.0;
    }
    for (int i = tid; i < mm; i += 64) order[i] = i;
    __syncthreads();
    const int half = mm / 2;
    for (int sweep = 0; sweep < 30; ++sweep) {
        if (tid == 0) {
            double off = 0.0, tot = 0.0;
            for (int r = 0; r < m; ++r)
                for (int c = 0; c < m; ++c) {
                    const double a2 = A[r][c] * A[r][c];
                    tot += a2;
                    if (r != c) off += a2;
                }
            done = (off <= 1e-34 * tot) ? 1 : 0;
        }
        __syncthreads();
        if (done) break;
        for (int round = 0; round < mm - 1; ++round) {
            if (tid < half) {
                int p = order[tid], q = order[mm - 1 - tid];
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
            for (int idx = tid; idx < half * mm; idx += 64) {
                const int k = idx / mm, r = idx % mm;
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
            for (int idx = tid; idx < half * mm; idx += 64) {
                const int k = idx / mm, col = idx % mm;
                const int p = pa[k], q = pb[k];
                const double c = cs[k], s = sn[k];
                const double apc = A[p][col], aqc = A[q][col];
                A[p][col] = c * apc - s * aqc;
                A[q][col] = s * apc + c * aqc;
            }
            __syncthreads();
            // round-robin: keep order[0], rotate the others
            if (tid == 0) {
                const int last = order[mm - 1];
                for (int i = mm - 1; i > 1; --i) order[i] = order[i - 1];
                order[1] = last;
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
        for (int i = 0; i < m; ++i) y[i] = Vv[i][k];
        b.restart[t] = (m >= b.max_space || st0 == ST_RESTART) ? 1 : 0;
    }
}

// x = V y, Ax = S y, r = Ax - theta x, T = r / (theta - Hd) (clamped);
// partials |r|^2, |T|^2 and the first Gram-Schmidt projections V_i . T of the
// subspace the correction is added to (V_i, i < m, or x alone on restart).
// On restart, V_0 <- x and S_0 <- Ax in place (each thread owns its d).
template <int MS>
__global__ __launch_bounds__(256) void k_ritz(Batch b) {
    const int t = blockIdx.y;
    if (b.status[t] != ST_RUNNING) return;
    const int m = b.m[t], rs = b.restart[t];
    const double th = b.theta[t];
    const double *yv = b.y + (int64_t)t * kMaxSpace;
    double yy[MS];
#pragma unroll
    for (int i = 0; i < MS; ++i) yy[i] = (i < m) ? yv[i] : 0.0;
    double *V = b.V + (int64_t)t * b.max_space * b.dim;
    double *S = b.S + (int64_t)t * b.max_space * b.dim;
    const double *hd = b.Hd + (int64_t)t * b.dim;
    double *T = b.T + (int64_t)t * b.dim;
    double acc[MS + 2];
#pragma unroll
    for (int i = 0; i < MS + 2; ++i) acc[i] = 0.0;
    for (int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x; d < b.dim; d += (int64_t)gridDim.x * 256) {
        double x = 0.0, ax = 0.0, vd[MS];
#pragma unroll
        for (int i = 0; i < MS; ++i) {
            vd[i] = 0.0;
            if (i < m) {
                vd[i] = V[(int64_t)i * b.dim + d];
                x += yy[i] * vd[i];
                ax += yy[i] * S[(int64_t)i * b.dim + d];
            }
        }
        const double r = ax - th * x;
        acc[0] += r * r;
        double den = th - hd[d];
        if (fabs(den) < 1e-8) den = (den >= 0.0) ? 1e-8 : -1e-8;
        const double tv = r / den;
        T[d] = tv;
        acc[1] += tv * tv;
        if (rs) {
            V[d] = x;
            S[d] = ax;
            acc[2] += x * tv;
        } else {
#pragma unroll
            for (int i = 0; i < MS; ++i)
                if (i < m) acc[2 + i] += vd[i] * tv;
        }
    }
    store_block_partials<MS + 2>(b, t, acc, 2 + (rs ? 1 : m));
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
    if (b.restart[t]) {   // V_0 = x, S_0 = A x already: the subspace is {x} whatever the outcome
        b.m[t] = 1;
        b.G[(int64_t)t * kMaxSpace * kMaxSpace] = th;
        b.y[(int64_t)t * kMaxSpace] = 1.0;
    }
    b.status[t] = st;
    if (st == ST_RUNNING) atomicAdd(b.counter, 1);
}

// projection coefficients of the first Gram-Schmidt pass (partials 2..m+1 of k_ritz)
__global__ void k_coef1(Batch b) {
    const int t = blockIdx.x;
    if (b.status[t] != ST_RUNNING) return;
    const int m = b.m[t];
    if ((int)threadIdx.x < m) b.coef[(int64_t)t * kMaxSpace + threadIdx.x] = sum_parts_x(b, t, 2 + threadIdx.x);
}

hipError_t launch_iter_head(const Batch &b, hipStream_t s) {
    hipLaunchKernelGGL(k_small_eig, dim3(b.B), dim3(64), 0, s, b);
    if (b.max_space <= 12) hipLaunchKernelGGL(k_ritz<12>, dim3(b.nblk, b.B), dim3(256), 0, s, b);
    else hipLaunchKernelGGL(k_ritz<kMaxSpace>, dim3(b.nblk, b.B), dim3(256), 0, s, b);
    if (b.psp > 0) {
        if (b.max_space <= 12) hipLaunchKernelGGL(k_psp_fix<12>, dim3(b.B), dim3(kPsp), 0, s, b);
        else hipLaunchKernelGGL(k_psp_fix<kMaxSpace>, dim3(b.B), dim3(kPsp), 0, s, b);
    }
    hipLaunchKernelGGL(k_converge, dim3(b.B), dim3(64), 0, s, b);
    hipLaunchKernelGGL(k_coef1, dim3(b.B), dim3(64), 0, s, b);
    return hipGetLastError();
}

// coef[i] = sum of partials i (projection coefficients of the second pass)
__global__ void k_coef(Batch b) {
    const int t = blockIdx.x;
    if (b.status[t] != ST_RUNNING || !b.cgs2[t]) return;
    const int m = b.m[t];
    if ((int)threadIdx.x < m) b.coef[(int64_t)t * kMaxSpace + threadIdx.x] = sum_parts(b, t, threadIdx.x);
}

// T -= sum_i coef_i V_i, partial |T|^2 (second pass: flagged tuples only)
template <int MS>
__global__ __launch_bounds__(256) void k_axpy(Batch b, int only2) {
    const int t = blockIdx.y;
    if (b.status[t] != ST_RUNNING || (only2 && !b.cgs2[t])) return;
    const int m = b.m[t];
    double cf[MS];
    const double *cp = b.coef + (int64_t)t * kMaxSpace;
#pragma unroll
    for (int i = 0; i < MS; ++i) cf[i] = (i < m) ? cp[i] : 0.0;
    const double *V = b.V + (int64_t)t * b.max_space * b.dim;
    double *T = b.T + (int64_t)t * b.dim;
    double acc[1];
    acc[0] = 0.0;
    for (int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x; d < b.dim; d += (int64_t)gridDim.x * 256) {
        double v = T[d];
#pragma unroll
        for (int i = 0; i < MS; ++i)
            if (i < m) v -= cf[i] * V[(int64_t)i * b.dim + d];
        T[d] = v;
        acc[0] += v * v;
    }
    store_block_partials<1>(b, t, acc, 1);
}

// One classical Gram-Schmidt pass suffices when it kept at least 1/sqrt(2)
// of the correction's norm (Kahan's criterion); otherwise project again.
__global__ void k_cgs_check(Batch b) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= b.B || b.status[t] != ST_RUNNING) return;
    const double n1 = sqrt(sum_parts(b, t, 0));
    b.cgs2[t] = (n1 >= 0.70710678118654752 * b.tnorm0[t]) ? 0 : 1;
}

// 1/|T| into coef[0].  A correction that lies inside the subspace (its
// projection kept less than 1e-8 of its norm) adds nothing: the Ritz pair is
// converged if the residual is below r_tol (an invariant subspace, e.g. a
// one-determinant space); otherwise the tuple skips this expansion and
// restarts from its Ritz vector at the next iteration, or has stalled when the
// subspace already is that one vector.
__global__ void k_tnorm(Batch b) {
    const int t = blockIdx.x;
    if (threadIdx.x != 0 || b.status[t] != ST_RUNNING) return;
    const double tn = sqrt(sum_parts(b, t, 0));
    if (!(tn > 1e-8 * b.tnorm0[t]) || !(tn > 1e-300) || b.m[t] >= b.max_space) {
        b.status[t] = b.rnorm[t] < b.r_tol ? ST_DONE : (b.m[t] > 1 ? ST_RESTART : ST_STALLED);
        return;
    }
    b.coef[(int64_t)t * kMaxSpace] = 1.0 / tn;
}

// V_m = T / |T|
__global__ __launch_bounds__(256) void k_store_t(Batch b) {
    const int t = blockIdx.y;
    if (b.status[t] != ST_RUNNING) return;
    const double s = b.coef[(int64_t)t * kMaxSpace];
    double *vm = b.V + ((int64_t)t * b.max_space + b.m[t]) * b.dim;
    const double *T = b.T + (int64_t)t * b.dim;
    for (int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x; d < b.dim; d += (int64_t)gridDim.x * 256)
        vm[d] = T[d] * s;
}

// Classical Gram-Schmidt of T against V_0..V_{m-1} (a second pass where the
// first lost too much of the norm), then V_m = T/|T|.
hipError_t launch_orthonormalize(const Batch &b, hipStream_t s) {
    const dim3 grid(b.nblk, b.B);
    VecRef tr{b.T, b.dim, nullptr, 0};
    // first pass: projections from k_ritz, coefficients from k_coef1
    const bool small = b.max_space <= 12;
    if (small) hipLaunchKernelGGL(k_axpy<12>, grid, dim3(256), 0, s, b, 0);
    else hipLaunchKernelGGL(k_axpy<kMaxSpace>, grid, dim3(256), 0, s, b, 0);
    hipLaunchKernelGGL(k_cgs_check, dim3((b.B + 63) / 64), dim3(64), 0, s, b);
    if (small) hipLaunchKernelGGL(k_dots<12>, grid, dim3(256), 0, s, b, tr, 0, 1);
    else hipLaunchKernelGGL(k_dots<kMaxSpace>, grid, dim3(256), 0, s, b, tr, 0, 1);
    hipLaunchKernelGGL(k_coef, dim3(b.B), dim3(64), 0, s, b);
    if (small) hipLaunchKernelGGL(k_axpy<12>, grid, dim3(256), 0, s, b, 1);
    else hipLaunchKernelGGL(k_axpy<kMaxSpace>, grid, dim3(256), 0, s, b, 1);
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

hipError_t init_kernels() {
    hipError_t e = hipFuncSetAttribute((const void *)k_sigma_w, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_psp_factor, hipFuncAttributeMaxDynamicSharedMemorySize, (int)psp_factor_lds());
    if (e != hipSuccess) return e;
    const void *strips[] = {(const void *)k_sigma_strip<1>,  (const void *)k_sigma_strip<2>,
                            (const void *)k_sigma_strip<3>,  (const void *)k_sigma_strip<4>,
                            (const void *)k_sigma_strip<5>,  (const void *)k_sigma_strip<6>,
                            (const void *)k_sigma_strip<7>,  (const void *)k_sigma_strip<8>,
                            (const void *)k_sigma_strip<9>,  (const void *)k_sigma_strip<10>,
                            (const void *)k_sigma_strip<11>, (const void *)k_sigma_strip<12>,
                            (const void *)k_sigma_strip<13>};
    for (const void *f : strips) {
        e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace mbefci

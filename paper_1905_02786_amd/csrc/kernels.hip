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
// sigma = G^a( 1/2 (pq|rs) (D^a + 2 D^b) + k c ) + C H_b^T, where D^a / D^b are
// the alpha / beta parts of D+, G^a the alpha-link gather, and H_b the
// beta-string Hamiltonian sum_P k_P E+_P + 1/2 sum_PQ (P|Q) E+_P E+_Q (the
// alpha-beta coupling E^a E^b appears twice in the pair sum and is carried by
// the factor 2 on D^b).  A workgroup owns 16 beta columns: for every alpha
// string K_a it gathers D for the 16 determinants (K_a, B0..B0+15) into LDS,
// contracts with 1/2 (pq|rs) held as MFMA A fragments in registers (one
// 16-row M tile per wave), and scatters W through the alpha links of K_a
// into an LDS strip sigma[:, B0..B0+15].  Each alpha link of one string moves
// to a different string and the diagonal links all return to K_a itself, so
// the scatter of one step has no write conflicts.

// MFMA waves of the strip kernel: one 16-row M tile each, at most 4 so the
// waves of a workgroup sit on distinct SIMDs; rows beyond 64 use vector FMA.
static inline int strip_waves(const ParamLayout &pl) { return pl.Ppad / 16 < 4 ? pl.Ppad / 16 : 4; }

// M tiles past the 4 wave-owned ones (rows >= 64): each wave contracts a
// quarter of K into a partial 16x16 tile; readers sum the 4 partials.
static inline int strip_extra_tiles(const ParamLayout &pl) {
    const int x = pl.Ppad / 16 - strip_waves(pl);
    return x > 0 ? x : 0;
}

// LDS of the strip kernel; `split` keeps D^a and 2 D^b in separate tiles
// (plain stores), otherwise one tile takes both through LDS atomic adds.
static size_t strip_lds(const ParamLayout &pl, int64_t Na, bool split) {
    const int xr = pl.P > 64 ? pl.P - 64 : 0;   // rows of the extra tiles that hold pairs
    return sizeof(double) * ((size_t)Na * kStrip + (split ? 2 : 1) * (size_t)pl.Kpad * kStrip +
                             (size_t)64 * kStrip + (size_t)4 * xr * kStrip + 32);
}

// Workgroups per CU of the strip kernel (160 KiB LDS; register file: 3 waves
// per SIMD without extra tiles, 2 with).
static int strip_blocks_per_cu(const ParamLayout &pl, int64_t Na, bool split) {
    const int by_lds = (int)((160 * 1024) / strip_lds(pl, Na, split));
    const int by_regs = strip_extra_tiles(pl) ? 2 : 3;
    return by_lds < by_regs ? by_lds : by_regs;
}

static bool strip_split(const ParamLayout &pl, int64_t Na) {
    return strip_blocks_per_cu(pl, Na, true) >= strip_blocks_per_cu(pl, Na, false);
}

size_t strip_lds_bytes(const ParamLayout &pl, int64_t Na) { return strip_lds(pl, Na, strip_split(pl, Na)); }

constexpr int kMaxR = 4;   // gather items per thread: ceil(n_links * 16 / threads) <= 3 for n_A <= 13

bool strip_fits(const ParamLayout &pl, int64_t Na, int nentA, int nentB) {
    const int nth = 64 * strip_waves(pl);
    return strip_lds_bytes(pl, Na) <= 150 * 1024 && pl.Kpad / 4 <= kMaxKS && strip_extra_tiles(pl) <= 2 &&
           (nentA * kStrip + nth - 1) / nth <= kMaxR && (nentB * kStrip + nth - 1) / nth <= kMaxR;
}

// Software-pipelined: the alpha links and c values of step K_a + 1 are loaded
// into registers while step K_a runs its MFMA and scatter.  Thread items:
// alpha item (e, col) = (item >> 4, item & 15) over the alpha links of K_a
// (the same item later scatters W through that link), beta item
// (col, e) = (item / n_links_b, item % n_links_b) over the fixed beta links
// of the strip's columns.  D = D^a + 2 D^b: an entry receives at most one
// alpha and one beta term, added atomically in LDS (two-term sums commute, so
// the value does not depend on their order); writers reset their entries
// after the MFMA.
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

template <int MT, int NX, bool SPLIT>
__global__ __launch_bounds__(64 * MT) void k_sigma_strip(Batch b, VecRef cref, VecRef sref, double shift,
                                                         int skip_done) {
    const int nstrips = (int)((b.Nb + kStrip - 1) / kStrip);
    int t, strip_id;
    if (!xcd_map(blockIdx.x, nstrips, b.B, t, strip_id)) return;
    if (skip_done && b.status[t] != ST_RUNNING) return;
    constexpr int NTH = 64 * MT;
    const ParamLayout &pl = b.pl;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t Na = b.Na, Nb = b.Nb;
    const int B0 = strip_id * kStrip;
    const int ncol = (int)min((int64_t)kStrip, Nb - B0);
    const int nentA = b.nentA, nentB = b.nentB, ndiag = b.na;
    extern __shared__ double lds[];
    double *strip = lds;                               // [Na][16]
    double *D = strip + Na * kStrip;                   // [Kpad][16]  D^a (+ 2 D^b unless SPLIT)
    double *Db = SPLIT ? D + pl.Kpad * kStrip : D;     // [Kpad][16]  2 D^b when SPLIT
    double *Wt = D + (SPLIT ? 2 : 1) * pl.Kpad * kStrip;   // [64][16] rows of the wave-owned tiles
    const int XR = pl.P > 64 ? pl.P - 64 : 0;          // pair rows past 64
    double *Wp = Wt + 64 * kStrip;                     // [4][XR][16] partial rows >= 64, per wave
    double *kx = Wp + 4 * XR * kStrip;                 // [32] k of rows >= 64
    const double *prm = b.params + (int64_t)t * pl.stride;
    const double *c = vref(cref, t, b.dim);
    double *sg = const_cast<double *>(vref(sref, t, b.dim));
    const int KS = pl.Kpad / 4;
    const int ar = lane & 15, kr = lane >> 4;
    double af[kMaxKS];
#pragma unroll
    for (int ks = 0; ks < kMaxKS; ++ks)
        af[ks] = (ks < KS) ? prm[pl.off_eri + (wave * 16 + ar) * pl.Kpad + ks * 4 + kr] : 0.0;
    double kv[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int row = wave * 16 + kr + 4 * v;
        kv[v] = row < pl.P ? prm[pl.off_k + row] : 0.0;
    }
    for (int i = tid; i < Na * kStrip; i += NTH) strip[i] = 0.0;
    for (int i = tid; i < (SPLIT ? 2 : 1) * pl.Kpad * kStrip; i += NTH) D[i] = 0.0;
    // extra tiles: this wave's quarter of the K steps
    const int KQ = (KS + 3) / 4, ks0 = wave * KQ;
    double afx[NX > 0 ? NX : 1][6];
#pragma unroll
    for (int x = 0; x < NX; ++x) {
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const int ks = ks0 + j;
            afx[x][j] = (j < KQ && ks < KS) ? prm[pl.off_eri + (64 + 16 * x + ar) * pl.Kpad + ks * 4 + kr] : 0.0;
        }
    }
    for (int i = tid; i < 16 * NX; i += NTH) kx[i] = 64 + i < pl.P ? prm[pl.off_k + 64 + i] : 0.0;
    // fixed beta items: D^b offset | sign bit 31, and the source column in a c row
    int bq[kMaxR], bj[kMaxR];
#pragma unroll
    for (int r = 0; r < kMaxR; ++r) {
        const int item = tid + r * NTH;
        bq[r] = -1;
        bj[r] = 0;
        if (item < nentB * kStrip) {
            const int col = item / nentB, e = item % nentB;
            if (col < ncol) {
                const uint32_t L = b.linkB[(int64_t)(B0 + col) * nentB + e];
                bq[r] = (int)((((L >> 20) & 0x3FFu) * kStrip + col) | (L & 0x80000000u));
                bj[r] = (int)(L & 0xFFFFFu);
            }
        }
    }
    // alpha items: link e = (tid >> 4) + r * NTH / 16 of the current string, column ar (= tid & 15)
    const int ae0 = tid >> 4;
    constexpr int ESTEP = NTH / 16;
    const bool colok = ar < ncol;
    // prefetch step 0
    uint32_t lw[kMaxR];
    double ca[kMaxR], cb[kMaxR];
#pragma unroll
    for (int r = 0; r < kMaxR; ++r) {
        const bool av = colok && ae0 + r * ESTEP < nentA;
        lw[r] = av ? b.linkA[ae0 + r * ESTEP] : 0u;
        ca[r] = av ? c[(int64_t)(lw[r] & 0xFFFFFu) * Nb + B0 + ar] : 0.0;
        cb[r] = bq[r] != -1 ? c[bj[r]] : 0.0;
    }
    uint32_t sa = b.strA[0];
    double cc = ar < ncol ? c[B0 + ar] : 0.0;
    __syncthreads();
    for (int64_t Ka = 0; Ka < Na; ++Ka) {
        // P1: write D for step Ka
        uint32_t cur[kMaxR];
#pragma unroll
        for (int r = 0; r < kMaxR; ++r) {
            cur[r] = lw[r];
            if (colok && ae0 + r * ESTEP < nentA) {
                const double s = (lw[r] >> 31) ? -1.0 : 1.0;
                if (SPLIT) D[((lw[r] >> 20) & 0x3FFu) * kStrip + ar] = s * ca[r];
                else atomicAdd(&D[((lw[r] >> 20) & 0x3FFu) * kStrip + ar], s * ca[r]);
            }
            if (bq[r] != -1) {
                const double v = (bq[r] < 0 ? -2.0 : 2.0) * cb[r];
                if (SPLIT) Db[bq[r] & 0x7FFFFFFF] = v;
                else atomicAdd(&D[bq[r] & 0x7FFFFFFF], v);
            }
        }
        const uint32_t cur_sa = sa;
        const double cur_cc = cc;
        __syncthreads();
        // P2: links of step Ka+1, MFMA of step Ka, c values of step Ka+1
        const bool more = Ka + 1 < Na;
        if (more) {
#pragma unroll
            for (int r = 0; r < kMaxR; ++r)
                if (colok && ae0 + r * ESTEP < nentA) lw[r] = b.linkA[(Ka + 1) * nentA + ae0 + r * ESTEP];
            sa = b.strA[Ka + 1];
        }
        dbl4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < kMaxKS; ks += 2) {
            if (ks < KS) {
                const int o = (ks * 4 + kr) * kStrip + ar;
                acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(af[ks], SPLIT ? D[o] + Db[o] : D[o], acc0, 0, 0, 0);
            }
            if (ks + 1 < KS) {
                const int o = ((ks + 1) * 4 + kr) * kStrip + ar;
                acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(af[ks + 1], SPLIT ? D[o] + Db[o] : D[o], acc1, 0, 0, 0);
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = wave * 16 + kr + 4 * v;   // f64 16x16x4 output: lane>>4 + 4*item
            Wt[row * kStrip + ar] = acc0[v] + acc1[v] + kv[v] * cur_cc;
        }
#pragma unroll
        for (int x = 0; x < NX; ++x) {
            {
                dbl4 ax = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int j = 0; j < 6; ++j) {
                    const int ks = ks0 + j;
                    if (j < KQ && ks < KS) {
                        const int o = (ks * 4 + kr) * kStrip + ar;
                        ax = __builtin_amdgcn_mfma_f64_16x16x4f64(afx[x][j], SPLIT ? D[o] + Db[o] : D[o], ax, 0, 0, 0);
                    }
                }
                double *wp = Wp + wave * XR * kStrip;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int rr = 16 * x + kr + 4 * v;
                    if (rr < XR) wp[rr * kStrip + ar] = ax[v];
                }
            }
        }
        if (more) {
            const double *crow = c + (Ka + 1) * Nb;
#pragma unroll
            for (int r = 0; r < kMaxR; ++r) {
                if (colok && ae0 + r * ESTEP < nentA) ca[r] = c[(int64_t)(lw[r] & 0xFFFFFu) * Nb + B0 + ar];
                if (bq[r] != -1) cb[r] = crow[bj[r]];
            }
            cc = ar < ncol ? crow[B0 + ar] : 0.0;
        }
        __syncthreads();
        // P3: reset D^a, scatter W through the alpha links of Ka
        // col is always tid & 15 here, whose c value is cur_cc
        auto wval = [&](int Q, int col) -> double {
            if (NX == 0 || Q < 64) return Wt[Q * kStrip + col];
            const double *wp = Wp + (Q - 64) * kStrip + col;
            const int ws = XR * kStrip;
            return wp[0] + wp[ws] + wp[2 * ws] + wp[3 * ws] + kx[Q - 64] * cur_cc;
        };
#pragma unroll
        for (int r = 0; r < kMaxR; ++r) {
            const int e = ae0 + r * ESTEP;
            if (!SPLIT && bq[r] != -1) D[bq[r] & 0x7FFFFFFF] = 0.0;
            if (colok && e < nentA) {
                const int Q = (int)((cur[r] >> 20) & 0x3FFu);
                D[Q * kStrip + ar] = 0.0;
                if (e >= ndiag) {
                    const double s = (cur[r] >> 31) ? -1.0 : 1.0;
                    strip[(int64_t)(cur[r] & 0xFFFFFu) * kStrip + ar] += s * wval(Q, ar);
                }
            }
        }
        if (tid < kStrip) {
            double acc = 0.0;
            for (uint32_t x = cur_sa; x; x &= x - 1) {
                const int p = __ffs(x) - 1;
                acc += wval(p * (p + 3) / 2, tid);
            }
            strip[Ka * kStrip + tid] += acc;
        }
        __syncthreads();
    }
    for (int64_t i = tid; i < Na * kStrip; i += NTH) {
        const int64_t row = i / kStrip;
        const int col = (int)(i % kStrip);
        if (col < ncol) {
            const int64_t d = row * Nb + B0 + col;
            sg[d] = strip[i] + shift * c[d];
        }
    }
}

// H_b (symmetric, Nb x Nb) per tuple; thread J writes row J:
// H_b e_J = sum_{links (Q,K,s) of J} s [ k_Q e_K + 1/2 sum_{links (P,I,s') of K} s' (P|Q) e_I ].
__global__ __launch_bounds__(64) void k_build_hb(Batch b) {
    const int t = blockIdx.y;
    const int64_t J = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (J >= b.Nb) return;
    const ParamLayout &pl = b.pl;
    const double *prm = b.params + (int64_t)t * pl.stride;
    double *row = b.Hb + ((int64_t)t * b.Nb + J) * b.Nb;
    for (int64_t i = 0; i < b.Nb; ++i) row[i] = 0.0;
    const uint32_t *lj = b.linkB + J * b.nentB;
    for (int e = 0; e < b.nentB; ++e) {
        int K, Q;
        double s;
        link_decode(lj[e], K, Q, s);
        row[K] += s * prm[pl.off_k + Q];
        const uint32_t *lk = b.linkB + (int64_t)K * b.nentB;
        for (int f = 0; f < b.nentB; ++f) {
            int I, P;
            double s2;
            link_decode(lk[f], I, P, s2);
            row[I] += s * s2 * prm[pl.off_eri + P * pl.Kpad + Q];   // stored as 1/2 (P|Q)
        }
    }
}

hipError_t launch_build_hb(const Batch &b, hipStream_t s) {
    if (b.sigma_variant != SIGMA_STRIP) return hipSuccess;
    dim3 grid((unsigned)((b.Nb + 63) / 64), b.B);
    hipLaunchKernelGGL(k_build_hb, grid, dim3(64), 0, s, b);
    return hipGetLastError();
}

// sigma += C H_b per tuple (C = c as Na x Nb row-major, H_b symmetric):
// 64 x 64 output tile per block of 4 waves, each wave 32 x 32 = 2 x 2 FP64
// MFMA tiles; K in chunks of 16 staged through LDS.
__global__ __launch_bounds__(256) void k_gemm_hb(Batch b, VecRef cref, VecRef sref, int skip_done) {
    const int t = blockIdx.z;
    if (skip_done && b.status[t] != ST_RUNNING) return;
    const int64_t Na = b.Na, Nb = b.Nb;
    const double *C = vref(cref, t, b.dim);
    double *S = const_cast<double *>(vref(sref, t, b.dim));
    const double *Hb = b.Hb + (int64_t)t * Nb * Nb;
    __shared__ double As[64][17];
    __shared__ double Bs[16][65];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wy = wave >> 1, wx = wave & 1;
    const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
    dbl4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
    for (int64_t k0 = 0; k0 < Nb; k0 += 16) {
        __syncthreads();
        for (int i = tid; i < 64 * 16; i += 256) {
            const int r = i >> 4, kk = i & 15;
            const int64_t gr = r0 + r, gk = k0 + kk;
            As[r][kk] = (gr < Na && gk < Nb) ? C[gr * Nb + gk] : 0.0;
            const int kb = i >> 6, cj = i & 63;
            const int64_t gk2 = k0 + kb, gc = c0 + cj;
            Bs[kb][cj] = (gk2 < Nb && gc < Nb) ? Hb[gk2 * Nb + gc] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            double a[2], bb[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[wy * 32 + i * 16 + (lane & 15)][ks * 4 + (lane >> 4)];
#pragma unroll
            for (int j = 0; j < 2; ++j) bb[j] = Bs[ks * 4 + (lane >> 4)][wx * 32 + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bb[j], acc[i][j], 0, 0, 0);
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t gr = r0 + wy * 32 + i * 16 + (lane >> 4) + 4 * v;
                const int64_t gc = c0 + wx * 32 + j * 16 + (lane & 15);
                if (gr < Na && gc < Nb) S[gr * Nb + gc] += acc[i][j][v];
            }
}

template <int MT, int NX, bool SPLIT>
static hipError_t launch_strip_mt(const Batch &b, VecRef c, VecRef sig, double shift, int skip, hipStream_t s) {
    const int64_t nstrips = (b.Nb + kStrip - 1) / kStrip;
    const dim3 grid((unsigned)(((b.B + kXcds - 1) / kXcds) * kXcds * nstrips));
    hipLaunchKernelGGL((k_sigma_strip<MT, NX, SPLIT>), grid, dim3(64 * MT), strip_lds(b.pl, b.Na, SPLIT), s, b, c, sig, shift,
                       skip);
    return hipGetLastError();
}

static hipError_t launch_strip(const Batch &b, VecRef c, VecRef sig, double shift, int skip, hipStream_t s) {
    const bool split = strip_split(b.pl, b.Na);
    switch ((strip_waves(b.pl) * 4 + strip_extra_tiles(b.pl)) * 2 + (split ? 1 : 0)) {
        case 8: return launch_strip_mt<1, 0, false>(b, c, sig, shift, skip, s);
        case 9: return launch_strip_mt<1, 0, true>(b, c, sig, shift, skip, s);
        case 16: return launch_strip_mt<2, 0, false>(b, c, sig, shift, skip, s);
        case 17: return launch_strip_mt<2, 0, true>(b, c, sig, shift, skip, s);
        case 24: return launch_strip_mt<3, 0, false>(b, c, sig, shift, skip, s);
        case 25: return launch_strip_mt<3, 0, true>(b, c, sig, shift, skip, s);
        case 32: return launch_strip_mt<4, 0, false>(b, c, sig, shift, skip, s);
        case 33: return launch_strip_mt<4, 0, true>(b, c, sig, shift, skip, s);
        case 34: return launch_strip_mt<4, 1, false>(b, c, sig, shift, skip, s);
        case 35: return launch_strip_mt<4, 1, true>(b, c, sig, shift, skip, s);
        case 36: return launch_strip_mt<4, 2, false>(b, c, sig, shift, skip, s);
        case 37: return launch_strip_mt<4, 2, true>(b, c, sig, shift, skip, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t init_kernels() {
    hipError_t e = hipFuncSetAttribute((const void *)k_sigma_w, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    const void *strips[] = {
        (const void *)k_sigma_strip<1, 0, false>, (const void *)k_sigma_strip<1, 0, true>,
        (const void *)k_sigma_strip<2, 0, false>, (const void *)k_sigma_strip<2, 0, true>,
        (const void *)k_sigma_strip<3, 0, false>, (const void *)k_sigma_strip<3, 0, true>,
        (const void *)k_sigma_strip<4, 0, false>, (const void *)k_sigma_strip<4, 0, true>,
        (const void *)k_sigma_strip<4, 1, false>, (const void *)k_sigma_strip<4, 1, true>,
        (const void *)k_sigma_strip<4, 2, false>, (const void *)k_sigma_strip<4, 2, true>};
    for (const void *f : strips) {
        e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_sigma(const Batch &b, VecRef c, VecRef sig, double shift, bool skip_done,
                        hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, hipEvent_t ev2) {
    if (b.sigma_variant == SIGMA_STRIP) {
        if (ev0) (void)hipEventRecord(ev0, s);
        hipError_t e = launch_strip(b, c, sig, shift, skip_done ? 1 : 0, s);
        if (e != hipSuccess) return e;
        if (ev1) (void)hipEventRecord(ev1, s);
        const dim3 grid((unsigned)((b.Nb + 63) / 64), (unsigned)((b.Na + 63) / 64), b.B);
        hipLaunchKernelGGL(k_gemm_hb, grid, dim3(256), 0, s, b, c, sig, skip_done ? 1 : 0);
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
    return b.part + ((int64_t)t * b.nblk + blk) * (kMaxSpace + 1);
}

// column sums of the partials for i < nx (thread i), fixed block order
__device__ double sum_parts(const Batch &b, int t, int i) {
    double s = 0.0;
    for (int blk = 0; blk < b.nblk; ++blk) s += parts(b, t, blk)[i];
    return s;
}

// Block-reduce up to kMaxSpace+1 per-thread accumulators into partials.
__device__ void store_block_partials(const Batch &b, int t, const double *acc, int nx) {
    __shared__ double sh[4][kMaxSpace + 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < kMaxSpace + 1; ++i) {
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

// V_0 = e_imin + 1e-3 * noise(d), partial norm^2
__global__ __launch_bounds__(256) void k_guess_fill(Batch b) {
    const int t = blockIdx.y;
    const int64_t imin = (int64_t)b.coef[(int64_t)t * kMaxSpace];
    double *v0 = b.V + (int64_t)t * b.max_space * b.dim;
    double acc[kMaxSpace + 1];
    acc[0] = 0.0;
    for (int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x; d < b.dim; d += (int64_t)gridDim.x * 256) {
        const double v = (d == imin ? 1.0 : 0.0) + 1e-3 * guess_noise(d);
        v0[d] = v;
        acc[0] += v * v;
    }
    store_block_partials(b, t, acc, 1);
}

__global__ void k_guess_norm(Batch b) {
    const int t = blockIdx.x;
    if (threadIdx.x == 0) b.coef[(int64_t)t * kMaxSpace] = 1.0 / sqrt(sum_parts(b, t, 0));
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

// partial dots V_i . y for i < m[t] + nx_extra (running tuples only)
__global__ __launch_bounds__(256) void k_dots(Batch b, VecRef yref, int nx_extra) {
    const int t = blockIdx.y;
    if (b.status[t] != ST_RUNNING) return;
    const int nx = b.m[t] + nx_extra;
    const double *V = b.V + (int64_t)t * b.max_space * b.dim;
    const double *y = vref(yref, t, b.dim);
    double acc[kMaxSpace + 1];
#pragma unroll
    for (int i = 0; i < kMaxSpace + 1; ++i) acc[i] = 0.0;
    for (int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x; d < b.dim; d += (int64_t)gridDim.x * 256) {
        const double yv = y[d];
#pragma unroll
        for (int i = 0; i < kMaxSpace + 1; ++i)
            if (i < nx) acc[i] += V[(int64_t)i * b.dim + d] * yv;
    }
    store_block_partials(b, t, acc, nx);
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
    hipLaunchKernelGGL(k_dots, dim3(b.nblk, b.B), dim3(256), 0, s, b, y, nx_extra);
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

// x = V y, Ax = S y, r = Ax - theta x, T = r / (theta - Hd) (clamped), partial |r|^2.
// On restart, V_0 <- x and S_0 <- Ax in place (each thread owns its d).
__global__ __launch_bounds__(256) void k_ritz(Batch b) {
    const int t = blockIdx.y;
    if (b.status[t] != ST_RUNNING) return;
    const int m = b.m[t], rs = b.restart[t];
    const double th = b.theta[t];
    const double *yv = b.y + (int64_t)t * kMaxSpace;
    double yy[kMaxSpace];
#pragma unroll
    for (int i = 0; i < kMaxSpace; ++i) yy[i] = (i < m) ? yv[i] : 0.0;
    double *V = b.V + (int64_t)t * b.max_space * b.dim;
    double *S = b.S + (int64_t)t * b.max_space * b.dim;
    const double *hd = b.Hd + (int64_t)t * b.dim;
    double *T = b.T + (int64_t)t * b.dim;
    double acc[kMaxSpace + 1];
    acc[0] = 0.0;
    acc[1] = 0.0;
    for (int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x; d < b.dim; d += (int64_t)gridDim.x * 256) {
        double x = 0.0, ax = 0.0;
#pragma unroll
        for (int i = 0; i < kMaxSpace; ++i)
            if (i < m) {
                x += yy[i] * V[(int64_t)i * b.dim + d];
                ax += yy[i] * S[(int64_t)i * b.dim + d];
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
        }
    }
    store_block_partials(b, t, acc, 2);
}

// convergence test, restart bookkeeping, running count
__global__ void k_converge(Batch b) {
    const int t = blockIdx.x;
    if (threadIdx.x != 0 || b.status[t] != ST_RUNNING) return;
    const double rn = sqrt(sum_parts(b, t, 0));
    const double th = b.theta[t];
    b.rnorm[t] = rn;
    b.tnorm0[t] = sqrt(sum_parts(b, t, 1));
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

hipError_t launch_iter_head(const Batch &b, hipStream_t s) {
    hipLaunchKernelGGL(k_small_eig, dim3(b.B), dim3(64), 0, s, b);
    hipLaunchKernelGGL(k_ritz, dim3(b.nblk, b.B), dim3(256), 0, s, b);
    hipLaunchKernelGGL(k_converge, dim3(b.B), dim3(64), 0, s, b);
    return hipGetLastError();
}

// coef[i] = sum of partials i (projection coefficients)
__global__ void k_coef(Batch b) {
    const int t = blockIdx.x;
    if (b.status[t] != ST_RUNNING) return;
    const int m = b.m[t];
    if ((int)threadIdx.x < m) b.coef[(int64_t)t * kMaxSpace + threadIdx.x] = sum_parts(b, t, threadIdx.x);
}

// T -= sum_i coef_i V_i ; optional partial |T|^2
__global__ __launch_bounds__(256) void k_axpy(Batch b, int want_norm) {
    const int t = blockIdx.y;
    if (b.status[t] != ST_RUNNING) return;
    const int m = b.m[t];
    double cf[kMaxSpace];
    const double *cp = b.coef + (int64_t)t * kMaxSpace;
#pragma unroll
    for (int i = 0; i < kMaxSpace; ++i) cf[i] = (i < m) ? cp[i] : 0.0;
    const double *V = b.V + (int64_t)t * b.max_space * b.dim;
    double *T = b.T + (int64_t)t * b.dim;
    double acc[kMaxSpace + 1];
    acc[0] = 0.0;
    for (int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x; d < b.dim; d += (int64_t)gridDim.x * 256) {
        double v = T[d];
#pragma unroll
        for (int i = 0; i < kMaxSpace; ++i)
            if (i < m) v -= cf[i] * V[(int64_t)i * b.dim + d];
        T[d] = v;
        acc[0] += v * v;
    }
    if (want_norm) store_block_partials(b, t, acc, 1);
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

// Two rounds of classical Gram-Schmidt of T against V_0..V_{m-1}, then V_m = T/|T|.
hipError_t launch_orthonormalize(const Batch &b, hipStream_t s) {
    const dim3 grid(b.nblk, b.B);
    VecRef tr{b.T, b.dim, nullptr, 0};
    for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(k_dots, grid, dim3(256), 0, s, b, tr, 0);
        hipLaunchKernelGGL(k_coef, dim3(b.B), dim3(64), 0, s, b);
        hipLaunchKernelGGL(k_axpy, grid, dim3(256), 0, s, b, pass == 1 ? 1 : 0);
    }
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

}  // namespace mbefci

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

hipError_t init_kernels() {
    return hipFuncSetAttribute((const void *)k_sigma_w, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

hipError_t launch_sigma(const Batch &b, VecRef c, VecRef sig, double shift, bool skip_done,
                        hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, hipEvent_t ev2) {
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
    if (b.status[t] != ST_RUNNING) return;
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
        b.restart[t] = (m >= b.max_space) ? 1 : 0;
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
    if (st == ST_RUNNING && b.restart[t]) {
        b.m[t] = 1;
        b.G[(int64_t)t * kMaxSpace * kMaxSpace] = th;
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
// projection kept less than 1e-8 of its norm) ends the iteration: converged if
// the residual is within 1000 r_tol, stalled otherwise.
__global__ void k_tnorm(Batch b) {
    const int t = blockIdx.x;
    if (threadIdx.x != 0 || b.status[t] != ST_RUNNING) return;
    const double tn = sqrt(sum_parts(b, t, 0));
    if (!(tn > 1e-8 * b.tnorm0[t]) || !(tn > 1e-300) || b.m[t] >= b.max_space) {
        b.status[t] = (b.rnorm[t] < 1e3 * b.r_tol) ? ST_DONE : ST_STALLED;
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

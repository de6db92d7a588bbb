// Sigma kernels (gfx950 / CDNA4, FP64): sigma = H c for a batch of tuples of
// one shape class, in two variants (column strip with string Hamiltonians, and
// W materialised), plus the string Hamiltonians and their GEMMs.
//
// The active-space Hamiltonian (CASCI of Sec. 2 with a frozen core) is
//   H = E_core + sum_pq k_pq E_pq + 1/2 sum_pqrs (pq|rs) E_pq E_rs,
// with k and E_core as formed by k_gather.
#include "device.h"
#include "symmetry.h"

namespace mbefci {

// ----------------------------------------------------------------- sigma --
// Knowles-Handy form with pair-symmetrised operators E+_P = E_pq + E_qp (p>q),
// E+_pp = E_pp:
//   D+_Q(K) = <K|E+_Q|c>          (gather over the single-excitation links of K)
//   W_P(K)  = 1/2 sum_Q (pq|rs) D+_Q(K) + k_P c_K   (FP64 MFMA, K-tile in LDS)
//   sigma_I = sum_P <I|E+_P|K> W_P(K)                (gather, no atomics)
// Links of string I list every (p,q) with E_pq|I> = sign|J>; with the
// determinant ordering alpha-major and alpha creators left of beta creators,
// alpha links act on the row index and beta links on the column index.

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
// sigma = H_a C + C H_b^T + (alpha-beta term): the alpha-beta term is the
// strip kernel (strip.hip); the string Hamiltonians H_s and their GEMMs
// follow here.

// Dense string Hamiltonian of one spin (symmetric, N x N per tuple); lane r
// of a block accumulates row J = J0 + r in LDS:
//   H e_J = sum_{links (Q,K,s) of J} s [ k_Q e_K + 1/2 sum_{links (P,I,s') of K} s' (P|Q) e_I ].
// Only that lane adds into its row, by LDS atomic adds issued in program
// order, so every entry is summed in the link order; the block then writes
// its rows out coalesced.  rows = rows per block (dynamic LDS rows * N doubles).
__global__ __launch_bounds__(64) void k_build_h(Batch b, int beta, int rows) {
    const int t = blockIdx.y, lane = threadIdx.x;
    const int64_t N = beta ? b.Nb : b.Na;
    const int nent = beta ? b.nentB : b.nentA;
    const uint32_t *links = beta ? b.linkB : b.linkA;
    const int64_t J0 = (int64_t)blockIdx.x * rows;
    const int nr = (int)(N - J0 < rows ? N - J0 : rows);
    extern __shared__ double hrow[];   // [rows][N]
    for (int64_t i = lane; i < (int64_t)nr * N; i += 64) hrow[i] = 0.0;
    __syncthreads();
    if (lane < nr) {
        const ParamLayout &pl = b.pl;
        const double *prm = b.params + (int64_t)t * pl.stride;
        auto add = [&](int64_t col, double v) {
            __builtin_amdgcn_ds_atomic_fadd_f64((__attribute__((address_space(3))) double *)(hrow + lane * N + col), v);
        };
        const uint32_t *lj = links + (J0 + lane) * nent;
        for (int e = 0; e < nent; ++e) {
            int K, Q;
            double sg;
            link_decode(lj[e], K, Q, sg);
            add(K, sg * prm[pl.off_k + Q]);
            const uint32_t *lk = links + (int64_t)K * nent;
            for (int f = 0; f < nent; ++f) {
                int I, P;
                double s2;
                link_decode(lk[f], I, P, s2);
                add(I, sg * s2 * prm[pl.off_eri + P * pl.Kpad + Q]);   // stored as 1/2 (P|Q)
            }
        }
    }
    __syncthreads();
    double *H = (beta ? b.Hb : b.Ha) + ((int64_t)t * N + J0) * N;
    for (int64_t i = lane; i < (int64_t)nr * N; i += 64) H[i] = hrow[i];
}

// rows per block: up to 64, at most 80 KB of LDS (two blocks per CU)
static int build_h_rows(int64_t N) {
    const int64_t r = (80 * 1024) / (8 * (N > 0 ? N : 1));
    return (int)(r < 1 ? 1 : (r > 64 ? 64 : r));
}

hipError_t launch_build_hb(const Batch &b, hipStream_t s) {
    if (b.sigma_variant != SIGMA_STRIP) return hipSuccess;
    if (b.la) {
        const hipError_t e = launch_linked_a(b, s);
        if (e != hipSuccess) return e;
    }
    const int rb = build_h_rows(b.Nb), ra = build_h_rows(b.Na);
    hipLaunchKernelGGL(k_build_h, dim3((unsigned)((b.Nb + rb - 1) / rb), b.B), dim3(64), (size_t)rb * b.Nb * sizeof(double),
                       s, b, 1, rb);
    if (b.Ha != b.Hb)
        hipLaunchKernelGGL(k_build_h, dim3((unsigned)((b.Na + ra - 1) / ra), b.B), dim3(64),
                           (size_t)ra * b.Na * sizeof(double), s, b, 0, ra);
    return hipGetLastError();
}

constexpr int kGK = 16;

// sigma += H_a C + C H_b per tuple (C = c as Na x Nb row-major; H_a, H_b
// symmetric): a (32 WM) x (32 WN) output tile per block of 4 waves (2 x 2,
// each wave WM x WN FP64 MFMA tiles).  K runs over H_a C (K = Na) and then
// C H_b (K = Nb) in chunks of 16 staged through a double-buffered LDS tile:
// the next chunk's global loads are in flight while the current one is
// multiplied, one barrier per chunk.  Operands are read through
// buffer resources sized to each matrix: every per-chunk offset is a scalar
// (the K position) plus a per-thread constant, so the chunk loop does no
// vector address arithmetic.  Reads past a row's end land in the next row or
// past the matrix (zero); they only meet zero rows of the other operand (K
// past the end) or feed rows and columns that are not stored.
// With `dots` (Davidson, sigma of V_m into S_m) the block also writes the
// partial dots V_i . S_m, gemm_dot_first <= i <= m, of its finished tile to
// partial block (its tile index) of the tuple (the others come from k_ritz).
// Grid: one block per (tuple, output tile), mapped so that every tile of
// tuple t runs on XCD t % 8 and the tiles of one tuple are dispatched back to
// back: the K-chunks they all read stay in that XCD's L2.
template <int WM, int WN>
__global__ __launch_bounds__(256) void k_gemm_hx(Batch b, VecRef cref, VecRef sref, int skip_done, int dots) {
    constexpr int BM = 32 * WM, BN = 32 * WN;
    const int tx = (int)((b.Nb + BN - 1) / BN), ntiles = tx * (int)((b.Na + BM - 1) / BM);
    const int64_t L = blockIdx.x, j = L / kXcds;
    const int t = (int)((j / ntiles) * kXcds + L % kXcds), tile = (int)(j % ntiles);
    if (t >= b.B) return;
    if (skip_done && b.status[t] != ST_RUNNING) return;
    const uint32_t Na = (uint32_t)b.Na, Nb = (uint32_t)b.Nb;
    const double *C = vref(cref, t, b.dim);
    double *S = const_cast<double *>(vref(sref, t, b.dim));
    const double *Ha = b.Ha + (int64_t)t * Na * Na;
    const double *Hb = b.Hb + (int64_t)t * Nb * Nb;
    const __amdgpu_buffer_rsrc_t rC = __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(C), (short)0,
                                                                        (int)(Na * Nb * sizeof(double)), 0x00020000);
    const __amdgpu_buffer_rsrc_t rA = __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(Ha), (short)0,
                                                                        (int)(Na * Na * sizeof(double)), 0x00020000);
    const __amdgpu_buffer_rsrc_t rB = __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(Hb), (short)0,
                                                                        (int)(Nb * Nb * sizeof(double)), 0x00020000);
    __shared__ double As[2][BM][kGK + 1];
    __shared__ double Bs[2][kGK][BN + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wy = wave >> 1, wx = wave & 1;
    const uint32_t r0 = (uint32_t)(tile / tx) * BM, c0 = (uint32_t)(tile % tx) * BN;
    // staging: A element j at row (tid >> 4) + 16 j, k = tid & 15; B element j at
    // k row (tid >> 5) + 8 (j / WN), column (tid & 31) + 32 (j % WN)
    const uint32_t ar = tid >> 4, ak = tid & 15, bk = tid >> 5, bc = tid & 31;
    const uint32_t nc0 = (Na + kGK - 1) / kGK, nc = nc0 + (Nb + kGK - 1) / kGK;
    // phase 0: X = H_a (ld Na), Y = C (ld Nb); phase 1: X = C (ld Nb), Y = H_b (ld Nb)
    const uint32_t va0 = ((r0 + ar) * Na + ak) * 8u, va1 = ((r0 + ar) * Nb + ak) * 8u;
    const uint32_t vb = (bk * Nb + c0 + bc) * 8u;
    double ra[2 * WM], rb[2 * WN];
    auto load = [&](uint32_t j) {
        const bool p1 = j >= nc0;
        const uint32_t k0 = (p1 ? j - nc0 : j) * kGK;
        const __amdgpu_buffer_rsrc_t rx = p1 ? rC : rA, ry = p1 ? rB : rC;
        const uint32_t ldX = p1 ? Nb : Na, va = p1 ? va1 : va0;
#pragma unroll
        for (int e = 0; e < 2 * WM; ++e)
            ra[e] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rx, va, (k0 + 16u * e * ldX) * 8u, 0));
#pragma unroll
        for (int e = 0; e < 2 * WN; ++e)
            rb[e] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
                                                   ry, vb + 256u * (e % WN), (k0 + 8u * (e / WN)) * Nb * 8u, 0));
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int e = 0; e < 2 * WM; ++e) As[buf][ar + 16 * e][ak] = ra[e];
#pragma unroll
        for (int e = 0; e < 2 * WN; ++e) Bs[buf][bk + 8 * (e / WN)][bc + 32 * (e % WN)] = rb[e];
    };
    dbl4 acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
    load(0);
    store(0);
    __syncthreads();
    for (uint32_t j = 0; j < nc; ++j) {
        const int buf = j & 1;
        if (j + 1 < nc) load(j + 1);
#pragma unroll
        for (int ks = 0; ks < kGK / 4; ++ks) {
            double af[WM], bf[WN];
#pragma unroll
            for (int i = 0; i < WM; ++i) af[i] = As[buf][wy * 16 * WM + i * 16 + (lane & 15)][ks * 4 + (lane >> 4)];
#pragma unroll
            for (int q = 0; q < WN; ++q) bf[q] = Bs[buf][ks * 4 + (lane >> 4)][wx * 16 * WN + q * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int q = 0; q < WN; ++q) acc[i][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[q], acc[i][q], 0, 0, 0);
        }
        if (j + 1 < nc) store(buf ^ 1);
        __syncthreads();
    }
    auto elem = [&](int i, int q, int v, int64_t &idx) -> bool {
        const uint32_t gr = r0 + wy * 16 * WM + i * 16 + (lane >> 4) + 4 * v;
        const uint32_t gc = c0 + wx * 16 * WN + q * 16 + (lane & 15);
        idx = (int64_t)gr * Nb + gc;
        return gr < Na && gc < Nb;
    };
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int q = 0; q < WN; ++q)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int64_t idx;
                if (elem(i, q, v, idx)) {
                    const double sv = S[idx] + acc[i][q][v];
                    S[idx] = sv;
                    acc[i][q][v] = sv;
                } else {
                    acc[i][q][v] = 0.0;
                }
            }
    if (!dots) return;
    // acc is zero outside the matrix, so the reads there (next row, or past
    // the vectors: zero) add nothing; offsets: per (i, q) a vector part, the
    // vector k and the row step 4 v scalar
    __shared__ double red[4][kMaxSpace];
    const int m = b.m[t], k0 = gemm_dot_first(b, t, m);
    const __amdgpu_buffer_rsrc_t rV = __builtin_amdgcn_make_buffer_rsrc(
        b.V + (int64_t)t * b.max_space * b.dim, (short)0, (int)(b.max_space * b.dim * sizeof(double)), 0x00020000);
    uint32_t vo[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int q = 0; q < WN; ++q)
            vo[i][q] = ((r0 + wy * 16 * WM + i * 16 + (lane >> 4)) * Nb + c0 + wx * 16 * WN + q * 16 + (lane & 15)) * 8u;
    for (int k = k0; k <= m; ++k) {
        const uint32_t sk = (uint32_t)(k * b.dim) * 8u;
        double a = 0.0;
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
            for (int q = 0; q < WN; ++q)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    a += __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rV, vo[i][q], sk + 4u * v * Nb * 8u, 0)) *
                         acc[i][q][v];
        a = wave_sum(a);
        if (lane == 0) red[wave][k] = a;
    }
    __syncthreads();
    if (tid >= k0 && tid <= m) parts(b, t, tile)[tid] = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
}

// Tile choice: the smaller padded area of 96 x 96 and 64 x 64 tiles; on a tie
// 96 for matrices of at least 256 x 256 strings, else 64 (measured with the
// Davidson dots: 96 faster for 462 and 330 strings, 64 for 252, 210 and 165).
static int gemm_tile(const Batch &b) {
    if (b.gemm_tile == 64 || b.gemm_tile == 96) return b.gemm_tile;   // chosen by the autotuner
    auto padded = [&](int64_t t) { return ((b.Na + t - 1) / t * t) * ((b.Nb + t - 1) / t * t); };
    const int64_t p96 = padded(96), p64 = padded(64);
    if (p96 != p64) return p96 < p64 ? 96 : 64;
    return b.Na * b.Nb >= 256 * 256 ? 96 : 64;
}

int gemm_blocks(const Batch &b) {
    const int64_t t = gemm_tile(b);
    return (int)(((b.Na + t - 1) / t) * ((b.Nb + t - 1) / t));
}

template <int WM, int WN>
static void launch_gemm_hx(const Batch &b, VecRef c, VecRef sig, int skip, int dots, hipStream_t s) {
    const int64_t ntiles = ((b.Nb + 32 * WN - 1) / (32 * WN)) * ((b.Na + 32 * WM - 1) / (32 * WM));
    const dim3 grid((unsigned)(((b.B + kXcds - 1) / kXcds) * kXcds * ntiles));
    hipLaunchKernelGGL((k_gemm_hx<WM, WN>), grid, dim3(256), 0, s, b, c, sig, skip, dots);
}

static hipError_t launch_gemm_h(const Batch &b, VecRef c, VecRef sig, int skip, int dots, hipStream_t s) {
    if (gemm_tile(b) == 96) launch_gemm_hx<3, 3>(b, c, sig, skip, dots, s);
    else launch_gemm_hx<2, 2>(b, c, sig, skip, dots, s);
    return hipGetLastError();
}



// Level shift toward the lowest state of total spin S = (n_a - n_b) / 2 of
// the sector: sigma += lambda S_- S_+ c over the active orbitals (spin_ss).
// S_- S_+ vanishes on states of spin S and is positive on all others.
__global__ __launch_bounds__(256) void k_spin_sigma(Batch b, VecRef cref, VecRef sref, int skip_done) {
    const int t = blockIdx.y;
    if (skip_done && b.status[t] != ST_RUNNING) return;
    const double *c = vref(cref, t, b.dim);
    double *sg = const_cast<double *>(vref(sref, t, b.dim));
    const double lam = b.spin_shift;
    for (int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x; d < b.dim; d += (int64_t)gridDim.x * 256)
        sg[d] += lam * spin_ss(b, c, d / b.Nb, d % b.Nb);
}

static hipError_t launch_spin_sigma(const Batch &b, VecRef c, VecRef sig, bool skip_done, hipStream_t s) {
    if (b.spin_shift == 0.0) return hipSuccess;
    hipLaunchKernelGGL(k_spin_sigma, dim3(grid_for(b.dim, 256, 4096), b.B), dim3(256), 0, s, b, c, sig,
                       skip_done ? 1 : 0);
    return hipGetLastError();
}

// Level shift away from the irreps other than the target one: sigma +=
// lambda [irrep(I) != target] c(I), diagonal in the determinants (the
// Hamiltonian does not couple irreps).
__global__ __launch_bounds__(256) void k_sym_sigma(Batch b, VecRef cref, VecRef sref, int skip_done) {
    const int t = blockIdx.y;
    if (skip_done && b.status[t] != ST_RUNNING) return;
    const double *c = vref(cref, t, b.dim);
    double *sg = const_cast<double *>(vref(sref, t, b.dim));
    for (int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x; d < b.dim; d += (int64_t)gridDim.x * 256)
        sg[d] += sym_pen(b, t, b.strA[d / b.Nb], b.strB[d % b.Nb]) * c[d];
}

static hipError_t launch_sym_sigma(const Batch &b, VecRef c, VecRef sig, bool skip_done, hipStream_t s) {
    if (b.sym_shift == 0.0) return hipSuccess;
    hipLaunchKernelGGL(k_sym_sigma, dim3(grid_for(b.dim, 256, 4096), b.B), dim3(256), 0, s, b, c, sig,
                       skip_done ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_sigma(const Batch &b, VecRef c, VecRef sig, double shift, bool skip_done, bool dots,
                        hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, hipEvent_t evg, hipEvent_t ev2) {
    if (b.sigma_variant == SIGMA_STRIP) {
        if (ev0) (void)hipEventRecord(ev0, s);
        hipError_t e = launch_strip(b, c, sig, shift, skip_done ? 1 : 0, s, ev1);
        if (e != hipSuccess) return e;
        if (evg) (void)hipEventRecord(evg, s);
        // (before the GEMM, whose epilogue forms the Davidson dots of the final sigma)
        if ((e = launch_spin_sigma(b, c, sig, skip_done, s)) != hipSuccess) return e;
        if ((e = launch_sym_sigma(b, c, sig, skip_done, s)) != hipSuccess) return e;
        e = launch_gemm_h(b, c, sig, skip_done ? 1 : 0, dots ? 1 : 0, s);
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
    if (evg) (void)hipEventRecord(evg, s);
    dim3 grid(grid_for(b.dim, 256, 4096), b.B);
    hipLaunchKernelGGL(k_sigma_g, grid, dim3(256), 0, s, b, c, sig, shift, skip_done ? 1 : 0);
    e = hipGetLastError();
    if (e == hipSuccess) e = launch_spin_sigma(b, c, sig, skip_done, s);
    if (e == hipSuccess) e = launch_sym_sigma(b, c, sig, skip_done, s);
    if (ev2) (void)hipEventRecord(ev2, s);
    return e;
}

hipError_t init_sigma_kernels() {
    hipError_t e = hipFuncSetAttribute((const void *)k_sigma_w, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_build_h, hipFuncAttributeMaxDynamicSharedMemorySize, 80 * 1024);
    if (e != hipSuccess) return e;
    return init_strip_kernels();
}

}  // namespace mbefci

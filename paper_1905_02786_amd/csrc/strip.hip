// Column-strip sigma kernel (gfx950 / CDNA4, FP64): the alpha-beta term of
// sigma = H c for a batch of tuples of one shape class.
#include "device.h"

namespace mbefci {

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

// Compile-time shape of the strip kernel for n_A active orbitals.
template <int NA>
struct StripShape {
    static constexpr int P = NA * (NA + 1) / 2;
    static constexpr int Ppad = (P + 15) / 16 * 16;
    static constexpr int Kpad = (P + 3) / 4 * 4;
    static constexpr int KS = Kpad / 4;                        // MFMA K steps
    static constexpr int DR = Kpad > P ? Kpad : P + 1;         // D rows: the K rows and a discard row (P)
    static constexpr int MT = Ppad / 16 < 4 ? Ppad / 16 : 4;   // waves, one 16-row tile each (distinct SIMDs)
    static constexpr int NX = Ppad / 16 - MT;                  // tiles past row 64, K split over the waves
    static constexpr int XR = P > 64 ? P - 64 : 0;             // pair rows past 64
    static constexpr int NTH = 64 * MT;
    static constexpr int NXI = (XR * 16 + NTH - 1) / NTH;      // items per thread on rows past 64
    static constexpr int KQ = (KS + 3) / 4;                    // K steps per wave in a tile past row 64
    static constexpr int NI = 4 + NXI;                         // D / scatter items per thread
};

// LDS of the strip kernel (doubles): sigma strip [Na + 1][16] (row Na is a
// discard row for masked-off stores), D [2][DR][16] (row P takes the masked
// items' zeros; rows from P to Kpad meet zero A columns), per-wave partial W
// of rows past 64 [2][4][XR][16].  For n_A = 11 and 462 alpha strings this is
// 76.9 KB: two workgroups per CU.
static size_t strip_lds(const ParamLayout &pl, int64_t Na) {
    const int xr = pl.P > 64 ? pl.P - 64 : 0;
    const int dr = pl.Kpad > pl.P ? pl.Kpad : pl.P + 1;
    return sizeof(double) * ((size_t)(Na + 1) * kStrip + 2 * (size_t)dr * kStrip + 8 * (size_t)xr * kStrip);
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

// A compile-time flag passed to generic lambdas.
template <bool B> struct BoolC {
    static constexpr bool value = B;
};

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

// Row swaps of two values: 16-lane rows (odd rows of x with even rows of y)
// and 32-lane halves (upper half of x with lower half of y).
__device__ __forceinline__ void swap16(double &x, double &y) {
    const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(x), __double2loint(y), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(x), __double2hiint(y), false, false);
    x = __hiloint2double(hi[0], lo[0]);
    y = __hiloint2double(hi[1], lo[1]);
}
__device__ __forceinline__ void swap32(double &x, double &y) {
    const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(x), __double2loint(y), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(x), __double2hiint(y), false, false);
    x = __hiloint2double(hi[0], lo[0]);
    y = __hiloint2double(hi[1], lo[1]);
}

// Four such sums at once: lane group g (lanes 16 g .. 16 g + 15) of the result
// holds the sum of input g (a, b, c, d) over the four groups, in the same
// order ((x0 + x1) + (x2 + x3)) as sum_over_kr.
__device__ __forceinline__ double group_sums4(double a, double b, double c, double d) {
    swap16(a, b);
    swap16(c, d);
    double s = a + b, t = c + d;   // [a0+a1, b0+b1, a2+a3, b2+b3], [c0+c1, d0+d1, c2+c3, d2+d3]
    swap32(s, t);                  // [a01, b01, c01, d01], [a23, b23, c23, d23]
    return s + t;
}
// The same for two inputs (groups 0, 2: a; 1, 3: b).
__device__ __forceinline__ double group_sums2(double a, double b) {
    swap16(a, b);
    double s = a + b, t = s;
    swap32(s, t);
    return s + t;
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
    constexpr int P = S::P, KP = S::Kpad, DR = S::DR, KS = S::KS, NX = S::NX, XR = S::XR, NTH = S::NTH,
                  NI = S::NI, KQ = S::KQ, NXA = NX > 0 ? NX : 1;
    constexpr uint32_t DB = DR * kStrip * sizeof(double);   // byte stride of the D buffers
    const int nstrips = (int)((b.Nb + kStrip - 1) / kStrip);
    int t, strip_id;
    if (!xcd_map(blockIdx.x, nstrips, b.B, t, strip_id)) return;
    if (skip_done && b.status[t] != ST_RUNNING) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // the wave index as a scalar: branches on it are taken per wave, so a
    // wave does not issue the other side's instructions under an empty mask
    const int wu = __builtin_amdgcn_readfirstlane(w);
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

    // A fragments of (pq|rs) (twice the stored 1/2 (pq|rs), so that D is the
    // signed C value itself) in the strip pair order: this wave's rows, and
    // its K quarter of the rows past 64
    auto eri_at = [&](int r, int k) -> double {
        return (r < P && k < P) ? 2.0 * prm[pl.off_eri + strip_pair_packed(r, NA) * KP + strip_pair_packed(k, NA)] : 0.0;
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
    // (byte offset in a row of C, past the buffer when there is no link so
    // that the load gives zero; its sign as the bit flipped in the high
    // word), scatter-table byte offset
    int qi[NI];
    uint32_t dsl[NI], boff[NI], qa[NI], bsg[NI];
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
        boff[i] = vb ? (eb & kPairJ) * (uint32_t)sizeof(double) : 0x80000000u;
        bsg[i] = vb ? (eb & kPairSign) : 0u;
        qa[i] = (uint32_t)(qi[i] < P ? qi[i] : P) * (uint32_t)sizeof(uint32_t);
        dsl[i] = (uint32_t)(D + qi[i] * kStrip + ar - lds) * (uint32_t)sizeof(double);
    }
    for (uint32_t i = tid; i < (Na + 1) * kStrip; i += NTH) strip[i] = 0.0;
    for (int i = tid; i < 2 * DR * kStrip; i += NTH) D[i] = 0.0;

    const uint32_t rowC = Nb * (uint32_t)sizeof(double), rowS = (P + 1) * (uint32_t)sizeof(uint32_t);
    auto lds_at = [&](uint32_t byte) -> double * { return reinterpret_cast<double *>(reinterpret_cast<char *>(lds) + byte); };
    double cb[NI];
    // row byte offsets are wave-uniform: readfirstlane keeps them in scalar
    // registers (the buffer loads' scalar offset operand)
    auto load_c = [&](uint32_t s, int i) -> double {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
                                              rc, boff[i], __builtin_amdgcn_readfirstlane(s * rowC), 0));
    };
    auto load_s = [&](uint32_t s, int i) -> uint32_t {
        return __builtin_amdgcn_raw_buffer_load_b32(rs, qa[i], __builtin_amdgcn_readfirstlane(s * rowS), 0);
    };
    auto dval = [&](int i) -> double {   // D entry of item i: the signed C value
        return __hiloint2double(__double2hiint(cb[i]) ^ (int)bsg[i], __double2loint(cb[i]));
    };

    // rows past 64: few of them (n_A = 11) go through vector FMAs on this
    // wave's K quarter instead of a mostly empty MFMA tile
    constexpr bool XV = NX == 1 && XR <= 2;
    constexpr int XVR = XV ? XR : 1;
    // With XV the group sums of the rows past 64 (groups 0 and 1) and, in
    // wave 0, of the diagonal pairs (group 2) come from one exchange.
    constexpr uint32_t DGK = XV ? 2u : 0u;   // lane group holding the diagonal sum
    double axv[XVR][KQ];
#pragma unroll
    for (int r = 0; r < XVR; ++r)
#pragma unroll
        for (int j = 0; j < KQ; ++j) {
            const int ks = w * KQ + j;
            axv[r][j] = (XV && ks < KS) ? eri_at(64 + r, ks * 4 + kr) : 0.0;
        }
    const uint32_t ar8 = (uint32_t)ar * (uint32_t)sizeof(double);
    uint32_t eA[NI], eB[NI];   // scatter entries (string K-2 is scattered, string K-1 loaded, alternately)
    double w2[4];              // W of string K-2 on this thread's wave rows
    double dg1 = 0.0;          // diagonal sum of the previous string (wave 0, lane group DGK)
    double xp[2] = {0.0, 0.0}; // XV partials of the rows past 64 of the current string
    // prologue: D of string 0 and C row 1
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        cb[i] = load_c(0, i);
        eA[i] = load_s(Na, i);   // discard row
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NI; ++i) *lds_at(dsl[i]) = dval(i);
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
                // lane (kr, ar): partial over k = kr (mod 4) of the quarter,
                // summed over kr at the end of the step
#pragma unroll
                for (int r = 0; r < XVR; ++r) {
                    double pr = 0.0;
#pragma unroll
                    for (int j = 0; j < KQ; ++j) pr = __builtin_fma(axv[r][j], bx[j], pr);
                    xp[r] = pr;
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
                *(kr < XVR ? wx + kr * kStrip + ar : dump) = ao[1][0];   // row kr from lane group kr
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
            // strip row at byte offset e & 0x7FFFFFFF (a multiple of 128), column ar; sign in bit 31.
            // The add is done by the LDS unit (no address of the step is hit
            // twice, so this is the plain sum in the same order)
            // (the strip starts the dynamic LDS block, which starts at LDS
            // address 0: the kernel has no static LDS, checked at set-up)
            const uint32_t addr = (e & 0x7FFFFFFFu) | ar8;
            __builtin_amdgcn_ds_atomic_fadd_f64((__attribute__((address_space(3))) double *)(uintptr_t)addr,
                                                __hiloint2double(__double2hiint(wv) ^ (int)(e & kPairSign), __double2loint(wv)));
        }
        // D of string K+1 (C row K+1 was loaded one step ago)
#pragma unroll
        for (int i = 0; i < NI; ++i) *lds_at(dsl[i] + ((K + 1) & 1) * DB) = dval(i);
        // loads: C row K+2, scatter entries of string K-1 (scattered next step)
        // (K - 1 wraps to 2^32 - 1 at K = 0: the discard row)
        const uint32_t K2c = K + 2 < Na ? K + 2 : Na - 1, K1s = K - 1 < Na ? K - 1 : Na;
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
        if (wu == 0) {
            if (kr == DGK && K >= 2 && K - 2 < Na)
                __builtin_amdgcn_ds_atomic_fadd_f64((__attribute__((address_space(3))) double *)(strip + (K - 2) * kStrip + ar), dg1);
            double s = ((sa1 >> kr) & 1u) ? ao[0][0] : 0.0;
#pragma unroll
            for (int v = 1; v < 4; ++v)
                if (4 * v < NA) s += ((sa1 >> (kr + 4 * v)) & 1u) ? ao[0][v] : 0.0;
            if (XV) {
                const double g = group_sums4(xp[0], XVR > 1 ? xp[1] : 0.0, s, s);   // group 3 unused
                an[1][0] = g;
                dg1 = g;
            } else {
                dg1 = sum_over_kr(s);
            }
        } else if (XV) {
            an[1][0] = group_sums2(xp[0], XVR > 1 ? xp[1] : 0.0);
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

// ------------------------------------------------- linked-row variant --
// Only the rows of W whose pair links alpha string K to some string reach
// sigma: the n (n_A - n) off-diagonal pairs with one orbital occupied in K,
// and the n occupied diagonal pairs, which all land on K itself and can be
// summed before the product instead of after it:
//   sum_{p in K} W_(pp) = (sum_{p in K} A_(pp)) D.
// That leaves 1 + n (n_A - n) rows per string, at most 32 for n_A <= 11: two
// 16-row MFMA tiles where the all-pairs kernel needs ceil(P / 16) tiles.  The
// A rows of a string are gathered from a per-tuple table (A, -A with the
// alpha link sign folded into the choice of row, and the diagonal row sum of
// every alpha string), and a workgroup of four waves runs two strings per
// step, one per pair of waves.

// Rows of the per-tuple A table and the first diagonal-sum row.
__host__ __device__ static inline int64_t linked_a_rows(int P, int64_t Na) { return (kLinkedSigned ? 2 * (int64_t)P : P) + Na; }

int64_t linked_a_stride(const ParamLayout &pl, int64_t Na) {
    return (linked_a_rows(pl.P, Na) * linked_row_len(pl.Kpad) + 31) / 32 * 32;
}

// LDS: sigma strip [Na + 1][16] and D of the step's two strings [2][Kpad][16].
static size_t linked_lds_gat(const ParamLayout &pl, int64_t Na) {
    return sizeof(double) * ((size_t)(Na + 1) * kStrip + 2 * (size_t)pl.Kpad * kStrip);
}

// LDS: sigma strip [Na + 1][16], D of the three thirds' pairs
// [3][2][Kpad][16], the A rows [P][row length] and the thirds' staged
// diagonal sums [3][2].
static size_t linked_lds_res(const ParamLayout &pl, int64_t Na) {
    const size_t rl = (size_t)linked_row_len(pl.Kpad);
    return sizeof(double) * ((size_t)(Na + 1) * kStrip + 6 * (size_t)pl.Kpad * kStrip + (size_t)(pl.P + 6) * rl);
}

bool linked_fits(const ParamLayout &pl, int64_t Na, int nel) {
    return pl.nA >= 4 && pl.nA <= kMaxActive && 1 + nel * (pl.nA - nel) <= kLinkedRows &&
           linked_lds_gat(pl, Na) <= 160 * 1024 && Na < (1 << 24);
}

// LDS of the diagonal-on-vector-ALU kernel: sigma strip [Na + 1][16], D of
// the two halves' pairs [2][2][Kpad][16], the A rows [P][row length] and the
// staged diagonal-sum rows [2][2][row length].
static size_t linked_lds_dv(const ParamLayout &pl, int64_t Na) {
    const size_t rl = (size_t)linked_row_len(pl.Kpad);
    return sizeof(double) * ((size_t)(Na + 1) * kStrip + 4 * (size_t)pl.Kpad * kStrip + (size_t)(pl.P + 4) * rl);
}

bool linked_dv_fits(const ParamLayout &pl, int64_t Na, int nel) {
    return pl.nA >= 4 && pl.nA <= kMaxActive && nel * (pl.nA - nel) <= kLinkedRows &&
           linked_lds_dv(pl, Na) <= 160 * 1024 && Na < (1 << 24);
}

// The per-tuple A table.  Row r holds twice the stored 1/2 (pq|rs) of pair
// row r (strip pair order) against every pair column k, in the interleaved
// column order: column k = 4 ks + kr sits at (ks / 2) * 8 + 2 kr + (ks & 1), so
// that one 16-byte load gives a lane its values for K steps 2j and 2j + 1;
// positions past the last K step and columns k >= P are zero.  Rows: A
// [0, P), with kLinkedSigned -A [P, 2P), then for alpha string K the sum of
// the diagonal rows (p,p) over its occupied orbitals p, in ascending p.
__global__ __launch_bounds__(256) void k_linked_a(Batch b) {
    const ParamLayout &pl = b.pl;
    const int t = blockIdx.y, P = pl.P, KP = pl.Kpad, nA = b.nA, RL = linked_row_len(KP);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= linked_a_rows(P, b.Na) * RL) return;
    const int64_t r = i / RL;
    const int pos = (int)(i % RL);
    const int k = 4 * (2 * (pos >> 3) + (pos & 1)) + ((pos & 7) >> 1);
    const double *prm = b.params + (int64_t)t * pl.stride;
    auto a_at = [&](int row) -> double {
        return k < P ? 2.0 * prm[pl.off_eri + strip_pair_packed(row, nA) * KP + strip_pair_packed(k, nA)] : 0.0;
    };
    const int64_t dg = kLinkedSigned ? 2 * P : P;   // first diagonal-sum row
    double v;
    if (r < P) {
        v = a_at((int)r);
    } else if (r < dg) {
        v = -a_at((int)(r - P));
    } else {
        const uint32_t m = b.strA[r - dg];
        v = 0.0;
        for (int p = 0; p < nA; ++p)
            if (m >> p & 1u) v += a_at(p);
    }
    b.la[(int64_t)t * b.la_stride + i] = v;
}

hipError_t launch_linked_a(const Batch &b, hipStream_t s) {
    if (!b.la) return hipSuccess;
    const int64_t n = linked_a_rows(b.pl.P, b.Na) * linked_row_len(b.pl.Kpad);
    hipLaunchKernelGGL(k_linked_a, dim3((unsigned)((n + 255) / 256), b.B), dim3(256), 0, s, b);
    return hipGetLastError();
}

// Gathered-A kernel.  One workgroup per (tuple, 16-column strip), four
// waves; wave w runs row
// tile w & 1 of string g = w >> 1 of each step's pair.  Host tables per
// alpha string K, 32 slots each (row N_a: all discard): lrow = byte offset of
// the slot's row in the A table (slot 0 the diagonal sum, then the
// off-diagonal links; unused slots row 0), lscat = byte offset of its target
// row in the sigma strip (K for slot 0, the linked string J for the others,
// the discard row N_a for unused slots), bit 31 the alpha link sign, in the
// order of the MFMA output rows of a lane (linked_scat_pos).
// Step n, two phases split by a barrier:
//   1. MFMAs of string 2n + g (D[g] and this wave's gathered A rows), loads
//      of the A rows of string 2n + 2 + g, scatter of string 2n - 2 (waves
//      0, 1);
//   2. scatter of string 2n - 1 (waves 2, 3), D of strings 2n + 2 and 2n + 3
//      from the C rows loaded one step ago, loads of C rows 2n + 4, 2n + 5,
//      of the scatter entries of string 2n + g and of the A-row offsets of
//      string 2n + 6 + g.
// D is read in phase 1 and rewritten in phase 2; one string is scattered per
// phase, and its targets are distinct, so the adds into every sigma entry
// come in string order, as in the all-pairs kernel.  Strings past the last
// read clamped C rows and the discard table row.
template <int NA>
__global__ __launch_bounds__(256) void k_sigma_linked_gat(Batch b, VecRef cref, VecRef sref, double shift,
                                                      int skip_done) {
    constexpr int P = NA * (NA + 1) / 2, KP = (P + 3) / 4 * 4, KS = KP / 4, NID = (KP + 15) / 16;
    constexpr int RL = (KS + 1) / 2 * 8;   // A-table row length (linked_row_len)
    constexpr uint32_t DB = KP * kStrip * sizeof(double);   // bytes of one string's D
    const int nstrips = (int)((b.Nb + kStrip - 1) / kStrip);
    int t, strip_id;
    if (!xcd_map(blockIdx.x, nstrips, b.B, t, strip_id)) return;
    if (skip_done && b.status[t] != ST_RUNNING) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wu = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int g = wu >> 1, h = wu & 1;
    const int ar = lane & 15, kr = lane >> 4;
    const uint32_t Na = (uint32_t)b.Na, Nb = (uint32_t)b.Nb;
    const uint32_t B0 = (uint32_t)strip_id * kStrip;
    const bool colok = B0 + ar < Nb;
    extern __shared__ double lds[];
    double *strip = lds;                                                // [Na + 1][16]
    const uint32_t D0 = (Na + 1) * kStrip * (uint32_t)sizeof(double);   // LDS byte address of D [2][KP][16]
    const double *c = vref(cref, t, b.dim);
    double *sg = const_cast<double *>(vref(sref, t, b.dim));
    const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(c), (short)0,
                                                                        (int)(b.dim * sizeof(double)), 0x00020000);
    const __amdgpu_buffer_rsrc_t rl = __builtin_amdgcn_make_buffer_rsrc(
        b.la + (int64_t)t * b.la_stride, (short)0, (int)(linked_a_rows(P, Na) * RL * sizeof(double)), 0x00020000);
    const int tbytes = (int)((Na + 1) * kLinkedRows * sizeof(uint32_t));
    const __amdgpu_buffer_rsrc_t rr = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t *>(b.lrow), (short)0,
                                                                        tbytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t *>(b.lscat), (short)0,
                                                                        tbytes, 0x00020000);
    // D items: row q = 16 i + (tid >> 4) of each string, column ar; item i is
    // present in wave w when 16 i + 4 w < KP (then all four of its rows are),
    // so the items cover the rows [0, KP) exactly.  Beta link of the column
    // for pair q as a byte offset in a row of C (past the vector when there
    // is none, so that the load gives zero) and its sign bit.
    uint32_t boff[NID], bsg[NID];
#pragma unroll
    for (int i = 0; i < NID; ++i) {
        const int q = 16 * i + (tid >> 4);
        const uint32_t eb = (colok && q < P) ? b.pairB[(B0 + ar) * (uint32_t)P + q] : 0u;
        const bool vb = (eb & kPairValid) != 0;
        boff[i] = vb ? (eb & kPairJ) * (uint32_t)sizeof(double) : 0x80000000u;
        bsg[i] = vb ? (eb & kPairSign) : 0u;
    }
    // wave-uniform; only the last item can be partial
    auto item_on = [&](int i) { return 16 * i + 16 <= KP || 16 * i + 4 * wu < KP; };
    for (uint32_t i = tid; i < (Na + 1) * kStrip; i += 256) strip[i] = 0.0;

    const uint32_t rowC = Nb * (uint32_t)sizeof(double), rowT = kLinkedRows * (uint32_t)sizeof(uint32_t);
    auto lds_at = [&](uint32_t byte) -> double * { return reinterpret_cast<double *>(reinterpret_cast<char *>(lds) + byte); };
    auto crow = [&](uint32_t s) -> uint32_t { return s < Na ? s : Na - 1; };   // C row of string s
    auto trow = [&](uint32_t s) -> uint32_t { return s < Na ? s : Na; };       // table row of string s
    auto load_c = [&](uint32_t s, int i) -> double {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
                                              rc, boff[i], crow(s) * rowC, 0));
    };
    auto load_row = [&](uint32_t s) -> uint32_t {   // A-row offset of this lane's A slot 16 h + ar
        return __builtin_amdgcn_raw_buffer_load_b32(rr, (uint32_t)(16 * h + ar) * 4u,
                                                    trow(s) * rowT, 0);
    };
    // targets of this lane's output rows 16 h + kr + 4 v, v = 0..3 (stored
    // side by side at 16 h + 4 kr)
    auto load_scat = [&](uint32_t s, uint32_t (&e)[4]) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, (uint32_t)(16 * h + 4 * kr) * 4u, trow(s) * rowT, 0);
#pragma unroll
        for (int k = 0; k < 4; ++k) e[k] = v[k];
    };
    // this lane's A values for all K steps of the row at byte offset ra: one
    // 16-byte load per K-step pair (interleaved row layout)
    auto load_a = [&](uint32_t ra, double (&af)[KS]) {
        const uint32_t o = ra + (uint32_t)kr * 16u;
#pragma unroll
        for (int j = 0; j < KS / 2; ++j) {
            const auto v = __builtin_amdgcn_raw_buffer_load_b128(rl, o + (uint32_t)j * 64u, 0, 0);
            af[2 * j] = __hiloint2double((int)v[1], (int)v[0]);
            af[2 * j + 1] = __hiloint2double((int)v[3], (int)v[2]);
        }
        if (KS & 1)
            af[KS - 1] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rl, o + (uint32_t)(KS / 2) * 64u, 0, 0));
    };
    auto dval = [&](double x, int i) -> double {   // D entry: the C value with the beta link sign
        return __hiloint2double(__double2hiint(x) ^ (int)bsg[i], __double2loint(x));
    };
    const uint32_t dw = D0 + (uint32_t)tid * (uint32_t)sizeof(double);   // D item 0 of string 0
    const uint32_t dr = D0 + (uint32_t)g * DB + (uint32_t)(kr * kStrip + ar) * (uint32_t)sizeof(double);
    const uint32_t ar8 = (uint32_t)ar * (uint32_t)sizeof(double);

    // Loads run two steps ahead of their use (A rows one step), in register
    // sets that alternate between even (A) and odd (B) steps.
    double afA[KS], afB[KS], cbA[2][NID], cbB[2][NID];
    uint32_t eA[4], eB[4];
    dbl4 accA = {0.0, 0.0, 0.0, 0.0}, accB = {0.0, 0.0, 0.0, 0.0};
    // prologue: A rows of string g, D of strings 0 and 1, C rows 2 to 5,
    // scatter entries of strings g - 2 (discard) and g
    {
        const uint32_t r0 = load_row(g);
        load_a(r0, afA);
    }
    uint32_t raA = load_row(2 + g), raB = load_row(4 + g);
    load_scat(Na, eA);
    load_scat(g, eB);
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
        for (int i = 0; i < NID; ++i)
            if (item_on(i)) *lds_at(dw + s2 * DB + i * 2048u) = dval(load_c(s2, i), i);
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
        for (int i = 0; i < NID; ++i) {
            cbA[s2][i] = item_on(i) ? load_c(2 + s2, i) : 0.0;
            cbB[s2][i] = item_on(i) ? load_c(4 + s2, i) : 0.0;
        }
    __syncthreads();

    auto scatter = [&](const dbl4 &w, const uint32_t (&e)[4]) {
        // target row e (a multiple of 128 bytes), column ar; the add is done
        // by the LDS unit (the strip starts the dynamic LDS block at address
        // 0: the kernel has no static LDS, checked at set-up)
        // (without kLinkedSigned the link sign is bit 31 of the entry)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const double x = kLinkedSigned ? w[v]
                                           : __hiloint2double(__double2hiint(w[v]) ^ (int)(e[v] & kPairSign),
                                                              __double2loint(w[v]));
            __builtin_amdgcn_ds_atomic_fadd_f64(
                (__attribute__((address_space(3))) double *)(uintptr_t)((e[v] & 0x7FFFFFFFu) | ar8), x);
        }
    };
    // step n: MFMAs of string 2n + g into `an`, scatter of string 2n - 2 + g
    // from `ao` with entries `e`, D of strings 2n + 2, 2n + 3 from `cb`;
    // reloads: A rows of string 2n + 2 + g into `afn` (with `ra`), then `ra`
    // for string 2n + 6 + g, `e` for string 2n + 2 + g, `cb` with C rows
    // 2n + 6, 2n + 7
    auto step = [&](uint32_t n, double (&afc)[KS], double (&afn)[KS], dbl4 &an, dbl4 &ao, uint32_t (&e)[4],
                    uint32_t &ra, double (&cb)[2][NID]) {
        {
            double bv[KS];
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) bv[ks] = *lds_at(dr + ks * 4u * kStrip * (uint32_t)sizeof(double));
            dbl4 a = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) a = __builtin_amdgcn_mfma_f64_16x16x4f64(afc[ks], bv[ks], a, 0, 0, 0);
            an = a;
        }
        load_a(ra, afn);
        ra = load_row(2 * n + 6 + g);
        if (g == 0) scatter(ao, e);
        __syncthreads();
        if (g == 1) scatter(ao, e);
        load_scat(2 * n + 2 + g, e);
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
            for (int i = 0; i < NID; ++i)
                if (item_on(i)) *lds_at(dw + s2 * DB + i * 2048u) = dval(cb[s2][i], i);
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
            for (int i = 0; i < NID; ++i)
                if (item_on(i)) cb[s2][i] = load_c(2 * n + 6 + s2, i);
        __syncthreads();
    };
    const uint32_t nsteps = (Na + 1) / 2 + 1;
    for (uint32_t n = 0; n < nsteps; n += 2) {
        step(n, afA, afB, accA, accB, eA, raA, cbA);
        step(n + 1, afB, afA, accB, accA, eB, raB, cbB);
    }
    for (uint32_t i = tid; i < Na * kStrip; i += 256) {
        const uint32_t row = i / kStrip, col = i % kStrip;
        if (B0 + col < Nb) {
            const uint32_t d = row * Nb + B0 + col;
            sg[d] = strip[i] + shift * c[d];
        }
    }
}

// Resident-A kernel.  One workgroup of twelve waves per (tuple, 16-column
// strip), in three thirds of four (waves 0-3, 4-7, 8-11: one wave of each
// third per SIMD).  The alpha strings are taken in pairs (lperm, host order:
// the two strings of a pair differ in at least three orbitals, so they share
// no scatter target), and pair q belongs to third q % 3.  In phase p (one
// barrier after each) third z does, by (p - z) mod 3:
//   0. the MFMAs of pair p: wave 4z + 2g + h computes row tile h of string g
//      of the pair, with its B operand from the pair's D tile and its A
//      operand from the A rows held in LDS for the whole strip (the slot-0
//      lanes from the pair's staged diagonal sums);
//   1. the scatter of pair p - 1 from the MFMA registers, and the A-row
//      offsets of its next pair p + 2;
//   2. D and the diagonal sums of its next pair p + 1 (from values loaded
//      three phases earlier), then the loads for the cycle after: C values
//      and diagonal sums of pair p + 4, scatter entries of pair p + 1.
// So on every SIMD one wave feeds the matrix pipe while two others share the
// memory work of two phases; one pair is scattered per phase, in pair order,
// so every sigma entry gets its adds in a fixed order.  Host tables per alpha
// string K, 32 slots each (row N_a: all discard): lrow = byte offset of the
// slot's A row (slot 0, the diagonal sum, is read from the staged row
// instead; unused slots row 0), lscat = byte offset of its target row in the
// sigma strip (K for slot 0, the linked string J for the others, the discard
// row N_a for unused slots), bit 31 the alpha link sign, in the order of the
// MFMA output rows of a lane (linked_scat_pos).  Dummy strings (index N_a)
// pad the last pair and the pairs past it.
template <int NA>
__global__ __launch_bounds__(768) void k_sigma_linked_res(Batch b, VecRef cref, VecRef sref, double shift,
                                                          int skip_done) {
    constexpr int P = NA * (NA + 1) / 2, KP = (P + 3) / 4 * 4, KS = KP / 4;
    constexpr int RL = (KS + 1) / 2 * 8;                      // A-table row length (linked_row_len)
    constexpr uint32_t RLB = RL * sizeof(double);
    constexpr uint32_t DB = KP * kStrip * sizeof(double);     // bytes of one string's D
    constexpr int NDI = (2 * KP * kStrip + 255) / 256;        // D items per thread of a third
    const int nstrips = (int)((b.Nb + kStrip - 1) / kStrip);
    int t, strip_id;
    if (!xcd_map(blockIdx.x, nstrips, b.B, t, strip_id)) return;
    if (skip_done && b.status[t] != ST_RUNNING) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wu = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int z = wu >> 2, lw = wu & 3, g = lw >> 1, h = lw & 1;   // third, wave in third, string, tile
    const int th = tid & 255;                                      // thread in third
    const int ar = lane & 15, kr = lane >> 4;
    const uint32_t Na = (uint32_t)b.Na, Nb = (uint32_t)b.Nb;
    const uint32_t B0 = (uint32_t)strip_id * kStrip;
    const bool colok = B0 + ar < Nb;
    extern __shared__ double lds[];
    double *strip = lds;                                                // [Na + 1][16]
    const uint32_t D0 = (Na + 1) * kStrip * (uint32_t)sizeof(double);   // D [3 thirds][2][KP][16]
    const uint32_t A0 = D0 + 6 * DB;                                    // A rows [P][RL]
    const uint32_t G0 = A0 + P * RLB;                                   // diagonal sums [3 thirds][2][RL]
    const double *c = vref(cref, t, b.dim);
    double *sg = const_cast<double *>(vref(sref, t, b.dim));
    const int32_t *perm = b.lperm;
    const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(c), (short)0,
                                                                        (int)(b.dim * sizeof(double)), 0x00020000);
    const __amdgpu_buffer_rsrc_t rl = __builtin_amdgcn_make_buffer_rsrc(
        b.la + (int64_t)t * b.la_stride, (short)0, (int)(linked_a_rows(P, Na) * RLB), 0x00020000);
    const int tbytes = (int)((Na + 1) * kLinkedRows * sizeof(uint32_t));
    const __amdgpu_buffer_rsrc_t rr = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t *>(b.lrow), (short)0,
                                                                        tbytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t *>(b.lscat), (short)0,
                                                                        tbytes, 0x00020000);
    // D items of a third: element j = th + 256 i of its D [2][KP][16] (string
    // j / (16 KP), row (j / 16) % KP, column ar).  A wave's 64 elements of an
    // item lie in one string (16 KP is a multiple of 64), so the string is
    // wave-uniform, and so is the presence of the last item.  Beta link of
    // the column for the item's pair as a byte offset in a row of C (past the
    // vector when there is none, so that the load gives zero) and its sign.
    uint32_t boff[NDI], bsg[NDI];
#pragma unroll
    for (int i = 0; i < NDI; ++i) {
        const int j = th + 256 * i, q = (j >> 4) % KP;
        const uint32_t eb = (colok && j < 2 * KP * kStrip && q < P) ? b.pairB[(B0 + ar) * (uint32_t)P + q] : 0u;
        const bool vb = (eb & kPairValid) != 0;
        boff[i] = vb ? (eb & kPairJ) * (uint32_t)sizeof(double) : 0x80000000u;
        bsg[i] = vb ? (eb & kPairSign) : 0u;
    }
    // wave-uniform; only the last item can be partial
    auto item_on = [&](int i) { return 256 * (i + 1) <= 2 * KP * kStrip || 64 * lw + 256 * i < 2 * KP * kStrip; };
    auto item_str = [&](int i) { return (64 * lw + 256 * i) / (KP * kStrip); };

    const uint32_t rowC = Nb * (uint32_t)sizeof(double), rowT = kLinkedRows * (uint32_t)sizeof(uint32_t);
    auto lds_at = [&](uint32_t byte) -> double * { return reinterpret_cast<double *>(reinterpret_cast<char *>(lds) + byte); };
    auto str = [&](uint32_t q, int k) -> uint32_t { return (uint32_t)perm[2 * q + k]; };   // string k of pair q
    auto crow = [&](uint32_t s) -> uint32_t { return s < Na ? s : 0u; };   // C row (dummy: any row)
    auto trow = [&](uint32_t s) -> uint32_t { return s < Na ? s : Na; };   // table row (dummy: discard)
    auto load_c = [&](uint32_t s, int i) -> double {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rc, boff[i], crow(s) * rowC, 0));
    };
    auto load_row = [&](uint32_t s) -> uint32_t {   // A-row offset of this lane's A slot 16 h + ar
        return __builtin_amdgcn_raw_buffer_load_b32(rr, (uint32_t)(16 * h + ar) * 4u, trow(s) * rowT, 0);
    };
    // targets of this lane's output rows 16 h + kr + 4 v, v = 0..3 (stored
    // side by side at 16 h + 4 kr)
    auto load_scat = [&](uint32_t s, uint32_t (&e)[4]) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, (uint32_t)(16 * h + 4 * kr) * 4u, trow(s) * rowT, 0);
#pragma unroll
        for (int k = 0; k < 4; ++k) e[k] = v[k];
    };
    // diagonal sum of string s: 16 bytes per lane, lanes < RL / 2 of waves
    // 2g of a third (one wave per string of the pair)
    const bool dgl = h == 0 && lane < RL / 2;
    auto load_dg = [&](uint32_t s) -> dbl2v {
        const uint32_t r = (uint32_t)P + (s < Na ? s : 0u);
        return __builtin_bit_cast(dbl2v, __builtin_amdgcn_raw_buffer_load_b128(rl, (uint32_t)lane * 16u, r * RLB, 0));
    };
    auto dval = [&](double v, int i) -> double {   // D entry: the C value with the beta link sign
        return __hiloint2double(__double2hiint(v) ^ (int)bsg[i], __double2loint(v));
    };
    const uint32_t dw = D0 + (uint32_t)z * 2 * DB + (uint32_t)th * (uint32_t)sizeof(double);   // D element th of the third
    const uint32_t dr = D0 + (uint32_t)(2 * z + g) * DB + (uint32_t)(kr * kStrip + ar) * (uint32_t)sizeof(double);
    const uint32_t gd = G0 + (uint32_t)(2 * z + g) * RLB;                  // staged diagonal sum of string g
    const uint32_t gw = gd + (uint32_t)lane * 16u;
    const bool isdg = h == 0 && ar == 0;                                   // lanes of slot 0
    const uint32_t ar8 = (uint32_t)ar * (uint32_t)sizeof(double);

    // prologue: sigma strip zero, A rows into LDS; third 0: D and diagonal
    // sums of pair 0; the registers of each third's first phases (third z
    // prepares pair 3 if z = 0, else pair z)
    for (uint32_t i = tid; i < (Na + 1) * kStrip; i += 768) strip[i] = 0.0;
    for (uint32_t i = tid; i < (uint32_t)P * RL / 2; i += 768)
        *reinterpret_cast<dbl2v *>(lds_at(A0 + 16u * i)) =
            __builtin_bit_cast(dbl2v, __builtin_amdgcn_raw_buffer_load_b128(rl, 16u * i, 0, 0));
    if (z == 0) {
#pragma unroll
        for (int i = 0; i < NDI; ++i)
            if (item_on(i)) *lds_at(dw + 2048u * i) = dval(load_c(str(0, item_str(i)), i), i);
        if (dgl) *reinterpret_cast<dbl2v *>(lds_at(gw)) = load_dg(str(0, g));
    }
    const uint32_t q0 = z == 0 ? 3u : (uint32_t)z;
    uint32_t ra = load_row(z == 2 ? Na : str((uint32_t)z, g));
    uint32_t e[4];
    load_scat(z == 0 ? str(0, g) : Na, e);
    double cb[NDI];
#pragma unroll
    for (int i = 0; i < NDI; ++i) cb[i] = item_on(i) ? load_c(str(q0, item_str(i)), i) : 0.0;
    dbl2v dg = {0.0, 0.0};
    if (dgl) dg = load_dg(str(q0, g));
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
    __syncthreads();

    // 0: the MFMAs of this third's pair
    auto mphase = [&]() {
        double bv[KS], af[KS];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) bv[ks] = *lds_at(dr + ks * 4u * kStrip * (uint32_t)sizeof(double));
        const uint32_t arow = (isdg ? gd : A0 + ra) + (uint32_t)kr * 16u;
#pragma unroll
        for (int j = 0; j < KS / 2; ++j) {
            const dbl2v v = *reinterpret_cast<const dbl2v *>(lds_at(arow + 64u * j));
            af[2 * j] = v[0];
            af[2 * j + 1] = v[1];
        }
        if (KS & 1) af[KS - 1] = *lds_at(arow + 64u * (KS / 2));
        dbl4 a = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) a = __builtin_amdgcn_mfma_f64_16x16x4f64(af[ks], bv[ks], a, 0, 0, 0);
        acc = a;
    };
    // 1 (phase p): scatter of pair p - 1, A-row offsets of pair p + 2
    auto n1phase = [&](uint32_t p) {
        ra = load_row(str(p + 2, g));
        // target row e & 0x7FFFFFFF (a multiple of 128 bytes), column ar, link
        // sign in bit 31; the add is done by the LDS unit (the strip starts the
        // dynamic LDS block at address 0: the kernel has no static LDS, checked
        // at set-up)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            __builtin_amdgcn_ds_atomic_fadd_f64(
                (__attribute__((address_space(3))) double *)(uintptr_t)((e[v] & 0x7FFFFFFFu) | ar8),
                __hiloint2double(__double2hiint(acc[v]) ^ (int)(e[v] & kPairSign), __double2loint(acc[v])));
    };
    // 2 (phase p): D and diagonal sums of pair p + 1; loads of pair p + 4 and
    // of the scatter entries of pair p + 1
    auto n2phase = [&](uint32_t p) {
#pragma unroll
        for (int i = 0; i < NDI; ++i)
            if (item_on(i)) *lds_at(dw + 2048u * i) = dval(cb[i], i);
        if (dgl) *reinterpret_cast<dbl2v *>(lds_at(gw)) = dg;
        load_scat(str(p + 1, g), e);
#pragma unroll
        for (int i = 0; i < NDI; ++i)
            if (item_on(i)) cb[i] = load_c(str(p + 4, item_str(i)), i);
        if (dgl) dg = load_dg(str(p + 4, g));
    };
    // one loop per third (straight-line bodies, three barriers each); phases
    // 0 .. 3k - 1 cover the last pair's scatter in phase lpairs
    const uint32_t nph = (uint32_t)b.lpairs + 1;
    if (z == 0) {
        for (uint32_t p = 0; p < nph; p += 3) {
            mphase();
            __syncthreads();
            n1phase(p + 1);
            __syncthreads();
            n2phase(p + 2);
            __syncthreads();
        }
    } else if (z == 1) {
        for (uint32_t p = 0; p < nph; p += 3) {
            n2phase(p);
            __syncthreads();
            mphase();
            __syncthreads();
            n1phase(p + 2);
            __syncthreads();
        }
    } else {
        for (uint32_t p = 0; p < nph; p += 3) {
            n1phase(p);
            __syncthreads();
            n2phase(p + 1);
            __syncthreads();
            mphase();
            __syncthreads();
        }
    }
    for (uint32_t i = tid; i < Na * kStrip; i += 768) {
        const uint32_t row = i / kStrip, col = i % kStrip;
        if (B0 + col < Nb) {
            const uint32_t d = row * Nb + B0 + col;
            sg[d] = strip[i] + shift * c[d];
        }
    }
}

// Diagonal-on-vector-ALU kernel: for strings with n (n_A - n) = 32
// off-diagonal links (n_A = 12 at four or eight electrons of the spin) the
// 32 row slots hold the off-diagonal links only, and the diagonal-sum row of
// each string, (sum_{p in K} A_(pp)) D, is formed on the vector ALU from the
// B operands the MFMA wave already holds: lane (kr, ar) sums the K steps
// congruent to kr, and the four lane groups are added with row swaps.  The A
// rows stay in LDS for the whole strip; for lack of room for a third set of
// D tiles, eight waves run in two halves of four (one wave of each half per
// SIMD) in ping-pong.  Pair q of the string order (lperm) belongs to half
// q % 2, and in phase p (one barrier after each):
//   * half p % 2 runs the MFMAs of pair p (wave 4z + 2g + h: row tile h of
//     string g) and, in its h = 0 waves, the diagonal sum of string g;
//   * the other half scatters its pair p - 1 from the MFMA registers and adds
//     the two diagonal sums to their own strings' rows, writes D and the
//     diagonal-sum row of its next pair p + 1 (values loaded two phases
//     earlier), and loads the C values, diagonal-sum rows and A-row offsets of
//     pair p + 3 and the scatter entries of pair p + 1.
// One pair is scattered per phase, in pair order; the two strings of a pair
// differ in at least three orbitals, so neither they nor any of their links
// coincide, and every sigma entry gets its adds in a fixed order.  Host
// tables per alpha string K, 32 slots each (row N_a: all discard): lrow =
// byte offset of the slot's A row, lscat = byte offset of its target row in
// the sigma strip (the linked string J, or the discard row N_a for unused
// slots), bit 31 the alpha link sign, in the order of the MFMA output rows of
// a lane (linked_scat_pos).
template <int NA>
__global__ __launch_bounds__(512) void k_sigma_linked_dv(Batch b, VecRef cref, VecRef sref, double shift,
                                                         int skip_done) {
    constexpr int P = NA * (NA + 1) / 2, KP = (P + 3) / 4 * 4, KS = KP / 4;
    constexpr int RL = (KS + 1) / 2 * 8;                      // A-table row length (linked_row_len)
    constexpr uint32_t RLB = RL * sizeof(double);
    constexpr uint32_t DB = KP * kStrip * sizeof(double);     // bytes of one string's D
    constexpr int NDI = (2 * KP * kStrip + 255) / 256;        // D items per thread of a half
    const int nstrips = (int)((b.Nb + kStrip - 1) / kStrip);
    int t, strip_id;
    if (!xcd_map(blockIdx.x, nstrips, b.B, t, strip_id)) return;
    if (skip_done && b.status[t] != ST_RUNNING) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wu = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int z = wu >> 2, lw = wu & 3, g = lw >> 1, h = lw & 1;   // half, wave in half, string, tile
    const int th = tid & 255;                                      // thread in half
    const int ar = lane & 15, kr = lane >> 4;
    const uint32_t Na = (uint32_t)b.Na, Nb = (uint32_t)b.Nb;
    const uint32_t B0 = (uint32_t)strip_id * kStrip;
    const bool colok = B0 + ar < Nb;
    extern __shared__ double lds[];
    double *strip = lds;                                                // [Na + 1][16]
    const uint32_t D0 = (Na + 1) * kStrip * (uint32_t)sizeof(double);   // D [2 halves][2][KP][16]
    const uint32_t A0 = D0 + 4 * DB;                                    // A rows [P][RL]
    const uint32_t G0 = A0 + P * RLB;                                   // diagonal-sum rows [2 halves][2][RL]
    const double *c = vref(cref, t, b.dim);
    double *sg = const_cast<double *>(vref(sref, t, b.dim));
    const int32_t *perm = b.lperm;
    const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(c), (short)0,
                                                                        (int)(b.dim * sizeof(double)), 0x00020000);
    const __amdgpu_buffer_rsrc_t rl = __builtin_amdgcn_make_buffer_rsrc(
        b.la + (int64_t)t * b.la_stride, (short)0, (int)(linked_a_rows(P, Na) * RLB), 0x00020000);
    const int tbytes = (int)((Na + 1) * kLinkedRows * sizeof(uint32_t));
    const __amdgpu_buffer_rsrc_t rr = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t *>(b.lrow), (short)0,
                                                                        tbytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t *>(b.lscat), (short)0,
                                                                        tbytes, 0x00020000);
    // D items of a half: element j = th + 256 i of its D [2][KP][16] (string
    // j / (16 KP), row (j / 16) % KP, column ar); wave-uniform string and
    // presence, as in the resident-A kernel
    uint32_t boff[NDI], bsg[NDI];
#pragma unroll
    for (int i = 0; i < NDI; ++i) {
        const int j = th + 256 * i, q = (j >> 4) % KP;
        const uint32_t eb = (colok && j < 2 * KP * kStrip && q < P) ? b.pairB[(B0 + ar) * (uint32_t)P + q] : 0u;
        const bool vb = (eb & kPairValid) != 0;
        boff[i] = vb ? (eb & kPairJ) * (uint32_t)sizeof(double) : 0x80000000u;
        bsg[i] = vb ? (eb & kPairSign) : 0u;
    }
    auto item_on = [&](int i) { return 256 * (i + 1) <= 2 * KP * kStrip || 64 * lw + 256 * i < 2 * KP * kStrip; };
    auto item_str = [&](int i) { return (64 * lw + 256 * i) / (KP * kStrip); };

    const uint32_t rowC = Nb * (uint32_t)sizeof(double), rowT = kLinkedRows * (uint32_t)sizeof(uint32_t);
    auto lds_at = [&](uint32_t byte) -> double * { return reinterpret_cast<double *>(reinterpret_cast<char *>(lds) + byte); };
    auto str = [&](uint32_t q, int k) -> uint32_t { return (uint32_t)perm[2 * q + k]; };   // string k of pair q
    auto crow = [&](uint32_t s) -> uint32_t { return s < Na ? s : 0u; };   // C row (dummy: any row)
    auto trow = [&](uint32_t s) -> uint32_t { return s < Na ? s : Na; };   // table row (dummy: discard)
    auto load_c = [&](uint32_t s, int i) -> double {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rc, boff[i], crow(s) * rowC, 0));
    };
    auto load_row = [&](uint32_t s) -> uint32_t {   // A-row offset of this lane's slot 16 h + ar
        return __builtin_amdgcn_raw_buffer_load_b32(rr, (uint32_t)(16 * h + ar) * 4u, trow(s) * rowT, 0);
    };
    auto load_scat = [&](uint32_t s, uint32_t (&e)[4]) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, (uint32_t)(16 * h + 4 * kr) * 4u, trow(s) * rowT, 0);
#pragma unroll
        for (int k = 0; k < 4; ++k) e[k] = v[k];
    };
    // diagonal-sum row of string s: 16 bytes per lane, lanes < RL / 2 of the
    // h = 0 wave of each string
    const bool dgl = h == 0 && lane < RL / 2;
    auto load_dg = [&](uint32_t s) -> dbl2v {
        const uint32_t r = (uint32_t)P + (s < Na ? s : 0u);
        return __builtin_bit_cast(dbl2v, __builtin_amdgcn_raw_buffer_load_b128(rl, (uint32_t)lane * 16u, r * RLB, 0));
    };
    auto dval = [&](double v, int i) -> double {
        return __hiloint2double(__double2hiint(v) ^ (int)bsg[i], __double2loint(v));
    };
    const uint32_t dw = D0 + (uint32_t)z * 2 * DB + (uint32_t)th * (uint32_t)sizeof(double);
    const uint32_t dr = D0 + (uint32_t)(2 * z + g) * DB + (uint32_t)(kr * kStrip + ar) * (uint32_t)sizeof(double);
    const uint32_t gd = G0 + (uint32_t)(2 * z + g) * RLB;                  // staged diagonal-sum row of string g
    const uint32_t gw = gd + (uint32_t)lane * 16u;
    const uint32_t ar8 = (uint32_t)ar * (uint32_t)sizeof(double);

    for (uint32_t i = tid; i < (Na + 1) * kStrip; i += 512) strip[i] = 0.0;
    for (uint32_t i = tid; i < (uint32_t)P * RL / 2; i += 512)
        *reinterpret_cast<dbl2v *>(lds_at(A0 + 16u * i)) =
            __builtin_bit_cast(dbl2v, __builtin_amdgcn_raw_buffer_load_b128(rl, 16u * i, 0, 0));
    // prologue: half 0 stages pair 0 and holds the loads of pair 2; half 1
    // holds the loads of pair 1 (staged in its first phase)
    uint32_t ra = 0u, rap = 0u, e[4];
    double cb[NDI];
    dbl2v dg = {0.0, 0.0};
    if (z == 0) {
#pragma unroll
        for (int i = 0; i < NDI; ++i)
            if (item_on(i)) *lds_at(dw + 2048u * i) = dval(load_c(str(0, item_str(i)), i), i);
        if (dgl) *reinterpret_cast<dbl2v *>(lds_at(gw)) = load_dg(str(0, g));
        ra = load_row(str(0, g));
        load_scat(str(0, g), e);
    } else {
        load_scat(Na, e);
    }
    const uint32_t q0 = z == 0 ? 2u : 1u;
#pragma unroll
    for (int i = 0; i < NDI; ++i) cb[i] = item_on(i) ? load_c(str(q0, item_str(i)), i) : 0.0;
    if (dgl) dg = load_dg(str(q0, g));
    rap = load_row(str(q0, g));
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
    double dsum = 0.0;     // diagonal sum of this wave's string (h = 0 waves), column ar
    uint32_t dtgt = Na;    // its target row (the string itself; the discard row before the first pair)
    __syncthreads();

    // MFMAs of pair q, and in the h = 0 waves (DG) the diagonal sum of string
    // g.  The diagonal sum's LDS reads are issued together ahead of the
    // chain's operands (taken one at a time after the chain, each one's
    // latency delayed the barrier that ends the phase); the scheduling
    // barriers keep them there and keep the chain ahead of that barrier.
    auto mphase = [&](uint32_t q, auto dgc) {
        constexpr bool DG = decltype(dgc)::value;
        constexpr int NG = DG ? (KS + 1) / 2 : 1;
        double bv[KS], af[KS];
        dbl2v gv[NG];
        if constexpr (DG) {
            const uint32_t grow = gd + (uint32_t)kr * 16u;
#pragma unroll
            for (int j = 0; j < KS / 2; ++j) gv[j] = *reinterpret_cast<const dbl2v *>(lds_at(grow + 64u * j));
            if (KS & 1) gv[NG - 1][0] = *lds_at(grow + 64u * (KS / 2));
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) bv[ks] = *lds_at(dr + ks * 4u * kStrip * (uint32_t)sizeof(double));
        const uint32_t arow = A0 + ra + (uint32_t)kr * 16u;
#pragma unroll
        for (int j = 0; j < KS / 2; ++j) {
            const dbl2v v = *reinterpret_cast<const dbl2v *>(lds_at(arow + 64u * j));
            af[2 * j] = v[0];
            af[2 * j + 1] = v[1];
        }
        if (KS & 1) af[KS - 1] = *lds_at(arow + 64u * (KS / 2));
        dbl4 a = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) a = __builtin_amdgcn_mfma_f64_16x16x4f64(af[ks], bv[ks], a, 0, 0, 0);
        acc = a;
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (DG) {
            // lane (kr, ar): sum over k = 4 ks + kr of G_k D_k(ar), in ks order
            double s = 0.0;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) s = __builtin_fma(gv[ks / 2][ks & 1], bv[ks], s);
            dsum = sum_over_kr(s);
            dtgt = trow(str(q, g));
        }
    };
    // phase p of the other half: scatter of pair p - 1 and its diagonal
    // sums; D and diagonal-sum rows of pair p + 1; loads of pairs p + 1, p + 3
    auto nphase = [&](uint32_t p) {
#pragma unroll
        for (int v = 0; v < 4; ++v)
            __builtin_amdgcn_ds_atomic_fadd_f64(
                (__attribute__((address_space(3))) double *)(uintptr_t)((e[v] & 0x7FFFFFFFu) | ar8),
                __hiloint2double(__double2hiint(acc[v]) ^ (int)(e[v] & kPairSign), __double2loint(acc[v])));
        if (h == 0 && kr == 0)
            __builtin_amdgcn_ds_atomic_fadd_f64(
                (__attribute__((address_space(3))) double *)(uintptr_t)(dtgt * 128u | ar8), dsum);
#pragma unroll
        for (int i = 0; i < NDI; ++i)
            if (item_on(i)) *lds_at(dw + 2048u * i) = dval(cb[i], i);
        if (dgl) *reinterpret_cast<dbl2v *>(lds_at(gw)) = dg;
        ra = rap;
        load_scat(str(p + 1, g), e);
#pragma unroll
        for (int i = 0; i < NDI; ++i)
            if (item_on(i)) cb[i] = load_c(str(p + 3, item_str(i)), i);
        // the string index as a scalar, so that the row load's offset is one
        // (a vector offset there costs a waterfall loop and a register copy
        // that waits for every load just issued)
        const uint32_t s3 = (uint32_t)__builtin_amdgcn_readfirstlane((int)str(p + 3, g));
        if (dgl) dg = load_dg(s3);
        rap = load_row(s3);
    };
    // phases 0 .. 2k - 1 cover the last pair's scatter in phase lpairs; the
    // loop is compiled once with the diagonal sum (h = 0 waves) and once
    // without
    const uint32_t nph = (uint32_t)b.lpairs + 1;
    auto run = [&](auto dgc) {
        if (z == 0) {
            for (uint32_t p = 0; p < nph; p += 2) {
                mphase(p, dgc);
                __syncthreads();
                nphase(p + 1);
                __syncthreads();
            }
        } else {
            for (uint32_t p = 0; p < nph; p += 2) {
                nphase(p);
                __syncthreads();
                mphase(p + 1, dgc);
                __syncthreads();
            }
        }
    };
    if (h == 0)
        run(BoolC<true>{});
    else
        run(BoolC<false>{});
    for (uint32_t i = tid; i < Na * kStrip; i += 512) {
        const uint32_t row = i / kStrip, col = i % kStrip;
        if (B0 + col < Nb) {
            const uint32_t d = row * Nb + B0 + col;
            sg[d] = strip[i] + shift * c[d];
        }
    }
}

// ---------------------------------------------- linked rows, W in HBM --
// For alpha-string counts whose sigma strip leaves no LDS for the A rows
// (n_A = 12 at 5 or 6 electrons of the spin: 792 and 924 strings) the linked
// rows of W = A D are written to HBM instead of being scattered into an LDS
// strip, and a second kernel gathers them: for target string J and column
// I_b, sigma(J, I_b) = sum over the links K -> J of the link sign times
// W(K, slot of the link)(I_b), plus its own diagonal-sum row.  Each W element
// is written once and read once; the sum over the incoming links of J runs in
// a fixed order.  Slots per string: 0 the diagonal sum, then the off-diagonal
// links in link order, up to 48 (three MFMA row tiles).
//
// W kernel: one workgroup of four waves per (tuple, 16-column strip, part of
// the strings), the A rows resident in LDS (staged once, the only barrier).
// Each wave then takes every fourth string of the
// part on its own: it loads the string's D straight into its MFMA B operands
// (lane (ar, kr) of K step ks holds the signed c(K, J) of the beta link of
// column B0 + ar and pair 4 ks + kr), stages the string's diagonal-sum row in
// an LDS slot of its own, runs the three row tiles and stores the W rows;
// the loads of its next string are issued before the MFMAs of this one.  Two
// workgroups per CU: while one wave of a SIMD runs its MFMAs the other's
// loads and stores proceed.  Every W element is written by one lane, so the
// result does not depend on the order in which the waves run.
template <int NA>
__global__ __launch_bounds__(256) void k_linked_wr(Batch b, VecRef cref, int skip_done, int aparts) {
    constexpr int P = NA * (NA + 1) / 2, KP = (P + 3) / 4 * 4, KS = KP / 4;
    constexpr int RL = (KS + 1) / 2 * 8;
    constexpr uint32_t RLB = RL * sizeof(double);
    const int nstrips = (int)((b.Nb + kStrip - 1) / kStrip);
    int t, sp;
    if (!xcd_map(blockIdx.x, nstrips * aparts, b.B, t, sp)) return;
    if (skip_done && b.status[t] != ST_RUNNING) return;
    const int strip_id = sp / aparts, part = sp % aparts;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int ar = lane & 15, kr = lane >> 4;
    const uint32_t Na = (uint32_t)b.Na, Nb = (uint32_t)b.Nb, SW = (uint32_t)b.lw_slots;
    const uint32_t B0 = (uint32_t)strip_id * kStrip;
    const bool colok = B0 + ar < Nb;
    const uint32_t per = (Na + (uint32_t)aparts - 1) / (uint32_t)aparts;
    const uint32_t S0 = (uint32_t)part * per, S1 = S0 + per < Na ? S0 + per : Na;   // strings [S0, S1)
    if (S0 >= S1) return;   // an empty part (the whole workgroup)
    extern __shared__ double lds[];
    const uint32_t G0 = P * RLB;   // after the A rows [P][RL]: diagonal-sum rows [4 waves][2][RL]
    const double *c = vref(cref, t, b.dim);
    double *W = b.lw + (int64_t)t * b.lw_stride;
    const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(c), (short)0,
                                                                        (int)(b.dim * sizeof(double)), 0x00020000);
    const __amdgpu_buffer_rsrc_t rl = __builtin_amdgcn_make_buffer_rsrc(
        b.la + (int64_t)t * b.la_stride, (short)0, (int)(linked_a_rows(P, Na) * RLB), 0x00020000);
    const uint32_t rowT = kLinkedRowsW * (uint32_t)sizeof(uint32_t);
    const __amdgpu_buffer_rsrc_t rr = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint32_t *>(b.lrow_w), (short)0, (int)((Na + 1) * rowT), 0x00020000);
    // this lane's D elements: byte offset of c(., J) in a C row (out of range:
    // an absent link, the load returns 0) and the link sign
    uint32_t boff[KS], bsg[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const int q = 4 * ks + kr;
        const uint32_t eb = (colok && q < P) ? b.pairB[(B0 + ar) * (uint32_t)P + q] : 0u;
        const bool vb = (eb & kPairValid) != 0;
        boff[ks] = vb ? (eb & kPairJ) * (uint32_t)sizeof(double) : 0x80000000u;
        bsg[ks] = vb ? (eb & kPairSign) : 0u;
    }
    const uint32_t rowC = Nb * (uint32_t)sizeof(double);
    auto lds_at = [&](uint32_t byte) -> double * { return reinterpret_cast<double *>(reinterpret_cast<char *>(lds) + byte); };
    // the C value of this lane's D element (unsigned), and with its sign
    auto load_d = [&](uint32_t K, int ks) -> double {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rc, boff[ks], K * rowC, 0));
    };
    auto sign_d = [&](double v, int ks) -> double {
        return __hiloint2double(__double2hiint(v) ^ (int)bsg[ks], __double2loint(v));
    };
    auto load_row = [&](uint32_t K, int h) -> uint32_t {   // A-row offset of this lane's slot 16 h + ar
        return __builtin_amdgcn_raw_buffer_load_b32(rr, (uint32_t)(16 * h + ar) * 4u, K * rowT, 0);
    };
    const bool dgl = lane < RL / 2;
    // lanes past the row read out of range (zero): no branch around the load
    const uint32_t dgo = dgl ? (uint32_t)lane * 16u : 0x80000000u;
    auto load_dg = [&](uint32_t K) -> dbl2v {
        return __builtin_bit_cast(dbl2v, __builtin_amdgcn_raw_buffer_load_b128(rl, dgo, ((uint32_t)P + K) * RLB, 0));
    };
    // W rows through a buffer resource: this lane's element of output row
    // 16 h + kr + 4 v at a fixed offset (out of range, so the store is
    // dropped, for slots past the string's and columns past N_b), the string
    // as the scalar offset.  No branch around the stores: the compiler's wait
    // counts then cover them, and the next string's loads need not wait for
    // them.
    const __amdgpu_buffer_rsrc_t rw = __builtin_amdgcn_make_buffer_rsrc(
        W, (short)0, (int)((int64_t)Na * SW * Nb * (int64_t)sizeof(double)), 0x00020000);
    uint32_t wo[3][4];
#pragma unroll
    for (int h = 0; h < 3; ++h)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const uint32_t slot = 16 * h + kr + 4 * v;
            wo[h][v] = (colok && slot < SW) ? (slot * Nb + B0 + ar) * (uint32_t)sizeof(double) : 0x80000000u;
        }
    const uint32_t rowW = SW * Nb * (uint32_t)sizeof(double);

    for (uint32_t i = tid; i < (uint32_t)P * RL / 2; i += 256)
        *reinterpret_cast<dbl2v *>(lds_at(16u * i)) =
            __builtin_bit_cast(dbl2v, __builtin_amdgcn_raw_buffer_load_b128(rl, 16u * i, 0, 0));
    __syncthreads();

    uint32_t s = S0 + (uint32_t)wv;
    if (s >= S1) return;
    // Loads run one string ahead in two register sets used in turn (no
    // copies between them), kept unsigned: the signs are applied when the
    // string's MFMAs start, so the wait is for loads issued one string before.
    // The prologue issues twelve stores that the bounds check drops, so that
    // the compiler's wait counts on entering the loop match those of later
    // iterations (a string's loads, then its stores).
    double blA[KS], blB[KS];
    dbl2v dgA, dgB;
    uint32_t raA[3], raB[3];
    auto issue = [&](uint32_t K, double (&bl)[KS], dbl2v &dgv, uint32_t (&rav)[3]) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) bl[ks] = load_d(K, ks);
        dgv = load_dg(K);
#pragma unroll
        for (int h = 0; h < 3; ++h) rav[h] = load_row(K, h);
    };
    issue(s, blA, dgA, raA);
#pragma unroll
    for (int v = 0; v < 12; ++v)   // (distinct offsets, or the compiler would keep one)
        __builtin_amdgcn_raw_buffer_store_b64(u32x2{0u, 0u}, rw, 0x80000000u + 8u * (uint32_t)v, 0, 0);
    const uint32_t gb0 = G0 + (uint32_t)(2 * wv) * RLB;
    // string s from the set (bl, dgv, rav) while the next string's loads go
    // to the other set
    auto string = [&](uint32_t s, uint32_t gbuf, const double (&bl)[KS], const dbl2v &dgv, const uint32_t (&rav)[3],
                      double (&bo)[KS], dbl2v &dgo_, uint32_t (&rao)[3]) {
        s = __builtin_amdgcn_readfirstlane(s);   // wave-uniform: scalar offsets
        double bv[KS];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) bv[ks] = sign_d(bl[ks], ks);
        const dbl2v dg = dgv;
        uint32_t ra[3];
#pragma unroll
        for (int h = 0; h < 3; ++h) ra[h] = rav[h];
        __builtin_amdgcn_sched_barrier(0);
        // the next string's loads (the last string loads itself again, unused)
        issue(s + 4 < S1 ? s + 4 : s, bo, dgo_, rao);
        __builtin_amdgcn_sched_barrier(0);
        // this string's diagonal-sum row in the wave's own slot (LDS accesses
        // of one wave complete in order: the reads below see it)
        if (dgl) *reinterpret_cast<dbl2v *>(lds_at(gbuf + (uint32_t)lane * 16u)) = dg;
        dbl4 acc[3];
#pragma unroll
        for (int h = 0; h < 3; ++h) {
            double af[KS];
            const uint32_t arow = ((h == 0 && ar == 0) ? gbuf : ra[h]) + (uint32_t)kr * 16u;
#pragma unroll
            for (int j = 0; j < KS / 2; ++j) {
                const dbl2v v = *reinterpret_cast<const dbl2v *>(lds_at(arow + 64u * j));
                af[2 * j] = v[0];
                af[2 * j + 1] = v[1];
            }
            if (KS & 1) af[KS - 1] = *lds_at(arow + 64u * (KS / 2));
            dbl4 a = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) a = __builtin_amdgcn_mfma_f64_16x16x4f64(af[ks], bv[ks], a, 0, 0, 0);
            acc[h] = a;
        }
#pragma unroll
        for (int h = 0; h < 3; ++h)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                // (the element copied out first: a bit cast of the vector
                // element expression itself stored element 0 four times)
                const double x = acc[h][v];
                __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), rw, wo[h][v], s * rowW, 0);
            }
    };
    for (;;) {
        string(s, gb0, blA, dgA, raA, blB, dgB, raB);
        s += 4;
        if (s >= S1) break;
        string(s, gb0 + RLB, blB, dgB, raB, blA, dgA, raA);
        s += 4;
        if (s >= S1) break;
    }
}

// Gather: sigma(J, I_b) = sum_i sign_i W(row_i)(I_b) + shift c(J, I_b) over the
// incoming rows of J (table linc [N_a][ninc]: W row index K * SW + slot, bit
// 31 the link sign; entry 0 is J's own diagonal-sum row), in table order.
// One block per (512 columns, target string, tuple), two columns per thread
// (16-byte loads when N_b is even, so that every W row starts 16-byte
// aligned); the table row is staged in LDS and all loads of a column pair
// are issued before the ordered sum.
template <bool V2>
__global__ __launch_bounds__(256) void k_linked_gw(Batch b, VecRef cref, VecRef sref, double shift, int skip_done) {
    const int t = blockIdx.z;
    if (skip_done && b.status[t] != ST_RUNNING) return;
    const uint32_t J = blockIdx.y, Nb = (uint32_t)b.Nb;
    const int ninc = b.lw_ninc;
    __shared__ uint32_t sinc[kLinkedRowsW];
    if ((int)threadIdx.x < ninc) sinc[threadIdx.x] = b.linc[(size_t)J * ninc + threadIdx.x];
    __syncthreads();
    const uint32_t ib = blockIdx.x * 512u + 2u * threadIdx.x;
    if (ib >= Nb) return;
    const double *W = b.lw + (int64_t)t * b.lw_stride;
    const double *c = vref(cref, t, b.dim);
    double *sg = const_cast<double *>(vref(sref, t, b.dim));
    const int64_t d = (int64_t)J * Nb + ib;
    if (V2) {
        dbl2v w[kLinkedRowsW];
#pragma unroll
        for (int i = 0; i < kLinkedRowsW; ++i)
            if (i < ninc) w[i] = *reinterpret_cast<const dbl2v *>(W + (int64_t)(sinc[i] & 0x7FFFFFFFu) * Nb + ib);
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int i = 0; i < kLinkedRowsW; ++i)
            if (i < ninc) {
                const bool neg = sinc[i] >> 31;
                a0 += neg ? -w[i][0] : w[i][0];
                a1 += neg ? -w[i][1] : w[i][1];
            }
        const dbl2v cv = *reinterpret_cast<const dbl2v *>(c + d);
        *reinterpret_cast<dbl2v *>(sg + d) = dbl2v{a0 + shift * cv[0], a1 + shift * cv[1]};
    } else {
        const bool two = ib + 1 < Nb;
        double w0[kLinkedRowsW], w1[kLinkedRowsW];
#pragma unroll
        for (int i = 0; i < kLinkedRowsW; ++i)
            if (i < ninc) {
                const double *r = W + (int64_t)(sinc[i] & 0x7FFFFFFFu) * Nb + ib;
                w0[i] = r[0];
                w1[i] = two ? r[1] : 0.0;
            }
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int i = 0; i < kLinkedRowsW; ++i)
            if (i < ninc) {
                const bool neg = sinc[i] >> 31;
                a0 += neg ? -w0[i] : w0[i];
                a1 += neg ? -w1[i] : w1[i];
            }
        sg[d] = a0 + shift * c[d];
        if (two) sg[d + 1] = a1 + shift * c[d + 1];
    }
}

static size_t linked_lds_w(const ParamLayout &pl) {
    return sizeof(double) * (size_t)(pl.P + 8) * (size_t)linked_row_len(pl.Kpad);
}

bool linked_w_fits(const ParamLayout &pl, int64_t Na, int nel) {
    return pl.nA >= 4 && pl.nA <= kMaxActive && 1 + nel * (pl.nA - nel) <= kLinkedRowsW &&
           linked_lds_w(pl) <= 160 * 1024 && Na < (1 << 24);
}

template <int NA>
static hipError_t launch_linked_w_na(const Batch &b, VecRef c, VecRef sig, double shift, int skip, hipStream_t s,
                                     hipEvent_t ev_mid) {
    const int64_t nstrips = (b.Nb + kStrip - 1) / kStrip;
    // two workgroups run per CU: small batches split the strings of a strip
    // over up to eight workgroups, until there are 2048 (four per slot)
    int aparts = 1;
    while (aparts < 8 && (int64_t)b.B * nstrips * aparts < 2048 && b.Na >= 32 * (aparts + 1)) ++aparts;
    const dim3 grid((unsigned)(((b.B + kXcds - 1) / kXcds) * kXcds * nstrips * aparts));
    hipLaunchKernelGGL(k_linked_wr<NA>, grid, dim3(256), linked_lds_w(b.pl), s, b, c, skip, aparts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev_mid) (void)hipEventRecord(ev_mid, s);
    const dim3 gg((unsigned)((b.Nb + 511) / 512), (unsigned)b.Na, (unsigned)b.B);
    if ((b.Nb & 1) == 0) hipLaunchKernelGGL(k_linked_gw<true>, gg, dim3(256), 0, s, b, c, sig, shift, skip);
    else hipLaunchKernelGGL(k_linked_gw<false>, gg, dim3(256), 0, s, b, c, sig, shift, skip);
    return hipGetLastError();
}

// The resident-A kernel (A rows in LDS, one twelve-wave workgroup in three
// thirds) needs more LDS than the gathered-A kernel (four waves, A rows
// loaded through the vector memory path, which they saturate).  It runs
// wherever it fits and there are at least as many alpha strings as pairs (its
// A rows are staged once per strip): the faster of the two, or within 1 %,
// on every n_A = 9..13 class measured.
static bool use_resident(const Batch &b) {
    const bool res_fits = linked_lds_res(b.pl, b.Na) <= 160 * 1024,
               gat_fits = linked_lds_gat(b.pl, b.Na) <= 160 * 1024;
    if (b.linked_mode == 3) return res_fits;
    if (b.linked_mode == 2 || !res_fits) return !gat_fits;
    return b.Na >= b.pl.P;
}

int alpha_beta_kernel(const Batch &b) {
    if (b.sigma_variant != SIGMA_STRIP) return 4;
    if (!b.la) return 0;
    if (b.lw) return 5;
    if (b.linked_dv) return 3;
    return use_resident(b) ? 2 : 1;
}

template <int NA>
static hipError_t launch_linked_na(const Batch &b, VecRef c, VecRef sig, double shift, int skip, hipStream_t s) {
    const int64_t nstrips = (b.Nb + kStrip - 1) / kStrip;
    const dim3 grid((unsigned)(((b.B + kXcds - 1) / kXcds) * kXcds * nstrips));
    if (b.linked_dv)
        hipLaunchKernelGGL(k_sigma_linked_dv<NA>, grid, dim3(512), linked_lds_dv(b.pl, b.Na), s, b, c, sig, shift,
                           skip);
    else if (use_resident(b))
        hipLaunchKernelGGL(k_sigma_linked_res<NA>, grid, dim3(768), linked_lds_res(b.pl, b.Na), s, b, c, sig,
                           shift, skip);
    else
        hipLaunchKernelGGL(k_sigma_linked_gat<NA>, grid, dim3(256), linked_lds_gat(b.pl, b.Na), s, b, c, sig,
                           shift, skip);
    return hipGetLastError();
}

template <int NA>
static hipError_t launch_strip_na(const Batch &b, VecRef c, VecRef sig, double shift, int skip, hipStream_t s) {
    const int64_t nstrips = (b.Nb + kStrip - 1) / kStrip;
    const dim3 grid((unsigned)(((b.B + kXcds - 1) / kXcds) * kXcds * nstrips));
    hipLaunchKernelGGL(k_sigma_strip<NA>, grid, dim3(StripShape<NA>::NTH), strip_lds(b.pl, b.Na), s, b, c, sig,
                       shift, skip);
    return hipGetLastError();
}

static hipError_t launch_strip_one(const Batch &b, VecRef c, VecRef sig, double shift, int skip, hipStream_t s);

hipError_t launch_strip(const Batch &b, VecRef c, VecRef sig, double shift, int skip, hipStream_t s,
                        hipEvent_t ev_mid) {
    if (b.lw) {   // linked rows through W in HBM (the planner checked linked_w_fits)
        switch (b.nA) {
            case 4: return launch_linked_w_na<4>(b, c, sig, shift, skip, s, ev_mid);
            case 5: return launch_linked_w_na<5>(b, c, sig, shift, skip, s, ev_mid);
            case 6: return launch_linked_w_na<6>(b, c, sig, shift, skip, s, ev_mid);
            case 7: return launch_linked_w_na<7>(b, c, sig, shift, skip, s, ev_mid);
            case 8: return launch_linked_w_na<8>(b, c, sig, shift, skip, s, ev_mid);
            case 9: return launch_linked_w_na<9>(b, c, sig, shift, skip, s, ev_mid);
            case 10: return launch_linked_w_na<10>(b, c, sig, shift, skip, s, ev_mid);
            case 11: return launch_linked_w_na<11>(b, c, sig, shift, skip, s, ev_mid);
            case 12: return launch_linked_w_na<12>(b, c, sig, shift, skip, s, ev_mid);
            case 13: return launch_linked_w_na<13>(b, c, sig, shift, skip, s, ev_mid);
            default: return hipErrorInvalidValue;
        }
    }
    hipError_t e = launch_strip_one(b, c, sig, shift, skip, s);
    if (e == hipSuccess && ev_mid) (void)hipEventRecord(ev_mid, s);
    return e;
}

static hipError_t launch_strip_one(const Batch &b, VecRef c, VecRef sig, double shift, int skip, hipStream_t s) {
    if (b.la) {   // linked-row variant (the planner checked linked_fits)
        switch (b.nA) {
            case 4: return launch_linked_na<4>(b, c, sig, shift, skip, s);
            case 5: return launch_linked_na<5>(b, c, sig, shift, skip, s);
            case 6: return launch_linked_na<6>(b, c, sig, shift, skip, s);
            case 7: return launch_linked_na<7>(b, c, sig, shift, skip, s);
            case 8: return launch_linked_na<8>(b, c, sig, shift, skip, s);
            case 9: return launch_linked_na<9>(b, c, sig, shift, skip, s);
            case 10: return launch_linked_na<10>(b, c, sig, shift, skip, s);
            case 11: return launch_linked_na<11>(b, c, sig, shift, skip, s);
            case 12: return launch_linked_na<12>(b, c, sig, shift, skip, s);
            case 13: return launch_linked_na<13>(b, c, sig, shift, skip, s);
            default: return hipErrorInvalidValue;
        }
    }
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

hipError_t init_strip_kernels() {
    hipError_t e = hipSuccess;
    const void *strips[] = {(const void *)k_sigma_strip<1>,  (const void *)k_sigma_strip<2>,
                            (const void *)k_sigma_strip<3>,  (const void *)k_sigma_strip<4>,
                            (const void *)k_sigma_strip<5>,  (const void *)k_sigma_strip<6>,
                            (const void *)k_sigma_strip<7>,  (const void *)k_sigma_strip<8>,
                            (const void *)k_sigma_strip<9>,  (const void *)k_sigma_strip<10>,
                            (const void *)k_sigma_strip<11>, (const void *)k_sigma_strip<12>,
                            (const void *)k_sigma_strip<13>,
                            (const void *)k_sigma_linked_res<4>,  (const void *)k_sigma_linked_gat<4>,
                            (const void *)k_sigma_linked_res<5>,  (const void *)k_sigma_linked_gat<5>,
                            (const void *)k_sigma_linked_res<6>,  (const void *)k_sigma_linked_gat<6>,
                            (const void *)k_sigma_linked_res<7>,  (const void *)k_sigma_linked_gat<7>,
                            (const void *)k_sigma_linked_res<8>,  (const void *)k_sigma_linked_gat<8>,
                            (const void *)k_sigma_linked_res<9>,  (const void *)k_sigma_linked_gat<9>,
                            (const void *)k_sigma_linked_res<10>, (const void *)k_sigma_linked_gat<10>,
                            (const void *)k_sigma_linked_res<11>, (const void *)k_sigma_linked_gat<11>,
                            (const void *)k_sigma_linked_res<12>, (const void *)k_sigma_linked_gat<12>,
                            (const void *)k_sigma_linked_res<13>, (const void *)k_sigma_linked_gat<13>,
                            (const void *)k_sigma_linked_dv<4>,  (const void *)k_sigma_linked_dv<5>,
                            (const void *)k_sigma_linked_dv<6>,  (const void *)k_sigma_linked_dv<7>,
                            (const void *)k_sigma_linked_dv<8>,  (const void *)k_sigma_linked_dv<9>,
                            (const void *)k_sigma_linked_dv<10>, (const void *)k_sigma_linked_dv<11>,
                            (const void *)k_sigma_linked_dv<12>, (const void *)k_sigma_linked_dv<13>,
                            (const void *)k_linked_wr<4>,  (const void *)k_linked_wr<5>,
                            (const void *)k_linked_wr<6>,  (const void *)k_linked_wr<7>,
                            (const void *)k_linked_wr<8>,  (const void *)k_linked_wr<9>,
                            (const void *)k_linked_wr<10>, (const void *)k_linked_wr<11>,
                            (const void *)k_linked_wr<12>, (const void *)k_linked_wr<13>};
    for (const void *f : strips) {
        e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        // the scatter addresses the strip by raw LDS address: no static LDS
        hipFuncAttributes fa;
        e = hipFuncGetAttributes(&fa, f);
        if (e != hipSuccess) return e;
        if (fa.sharedSizeBytes != 0) return hipErrorInvalidKernelFile;
    }
    return hipSuccess;
}

}  // namespace mbefci

// Internal declarations shared by the host planner (mbefci.cpp) and the HIP
// kernels (kernels.hip, sigma.hip, strip.hip) of libmbefci.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mbefci {

constexpr int kMaxActive = 13;     // n_A limit: the sigma kernel stages (P x P) in LDS
constexpr int kMaxSpace = 32;      // Davidson subspace limit
constexpr int kParts = kMaxSpace + 2;   // block partial sums per tuple and block
// With a subspace bound of at most kSdMax, k_ritz also forms the dots S_i . T
// of the new basis vector (partials kSdOff + i): they are the new column of
// the projected matrix above the diagonal (H symmetric: V_i^T H V_m =
// S_i . V_m), so that the GEMM's epilogue only forms the diagonal entry
constexpr int kSdMax = 12;
constexpr int kSdOff = 2 + kSdMax;
static_assert(kSdOff + kSdMax <= kParts, "S-dot partials past the partial block");
constexpr int kPsp = 128;          // largest P space of the Davidson preconditioner
constexpr int kTile = 64;          // determinants per sigma tile (materialised-W variant)
constexpr int kStrip = 16;         // beta columns per workgroup (column-strip variant)
// dense pair table entries (pairB): linked string J, link present, link sign
constexpr uint32_t kPairJ = 0xFFFFFu, kPairValid = 1u << 30, kPairSign = 1u << 31;
constexpr int kXcds = 8;           // accelerator complex dies, each with its own L2
constexpr int kMaxKS = 24;         // K steps of 4 covering the padded pair count (<= 92)
constexpr int kRdmMaxPairs = 16;   // upper 16x16 tile pairs of the RDM Gram per wave (n_A <= 12)
constexpr int kRdmMaxActive = 12;

// sigma variants: the column strip (W stays in LDS, beta-beta part as a GEMM
// with the dense beta-string Hamiltonian) and the materialised W (W in HBM,
// gathered back).  0 picks the strip whenever its LDS footprint fits.
enum : int32_t { SIGMA_AUTO = 0, SIGMA_STRIP = 1, SIGMA_WMAT = 2 };

// Davidson per-tuple status codes (device side); the public codes are derived.
enum : int32_t { ST_RUNNING = 0, ST_DONE = 1, ST_MAXITER = 2, ST_NONFINITE = 3, ST_STALLED = 4,
                 ST_RESTART = 5 /* running; skips this expansion, restarts from its Ritz vector next */ };

__host__ __device__ inline int pair_count(int n) { return n * (n + 1) / 2; }
__host__ __device__ inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// Offsets (in doubles) inside one tuple's parameter block.
struct ParamLayout {
    int nA, P, Ppad, Kpad, ldE;
    int off_ecore, off_k, off_hd1, off_J, off_K, off_eri, stride;
    void init(int nA_) {
        nA = nA_;
        P = pair_count(nA);
        Ppad = round_up(P > 0 ? P : 1, 16);
        Kpad = round_up(P > 0 ? P : 1, 4);
        ldE = Kpad + 1;                       // odd row stride against LDS bank conflicts
        off_ecore = 0;
        off_k = 1;
        off_hd1 = off_k + P;
        off_J = off_hd1 + nA;
        off_K = off_J + nA * nA;
        off_eri = round_up(off_K + nA * nA, 2);
        stride = round_up(off_eri + Ppad * Kpad, 32);
    }
};

// A reference to one vector per tuple: base + t*tstride + idx[t]*dim (idx may
// be null, then idx_const is used).
struct VecRef {
    double *base;
    int64_t tstride;
    const int32_t *idx;
    int32_t idx_const;
};

// Everything the kernels of one batch need (device pointers).
struct Batch {
    int B;                  // tuples in the batch
    int nA, na, nb, nC;     // active orbitals, active electrons, core orbitals
    int64_t Na, Nb, dim;    // strings and determinants
    int nentA, nentB;       // link entries per string
    ParamLayout pl;
    int norb;
    double e_const;
    const double *h, *eri;  // resident integrals (n^2, n^4)
    const uint32_t *strA, *strB, *linkA, *linkB;
    const uint32_t *scatA, *pairB;   // column-strip sigma: alpha scatter table, beta pair links
    // linked-row strip sigma (null la: the all-pairs strip kernel): per alpha
    // string the A-row offsets and sigma-strip targets of its 32 row slots
    // [Na + 1][32], the per-tuple A table [B][la_stride] and the string order
    const uint32_t *lrow, *lscat;
    double *la;
    int64_t la_stride;
    const int32_t *lperm;   // [2 (lpairs + 8)] alpha strings in pairs (N_a: dummy)
    int lpairs;
    int linked_mode;        // 1: variant by occupancy, 2: gathered A, 3: resident A (where it fits)
    int linked_dv;          // slots hold the off-diagonal links only; diagonal sums on the vector ALU
    int gemm_tile;          // string-Hamiltonian GEMM output tile (64, 96; 0: by padding)
    // linked rows through W in HBM (null lw: not this form): per alpha string
    // the A-row offsets of its 48 slots [Na + 1][48], W [B][Na * lw_slots * Nb],
    // and per target string its incoming W rows [Na][lw_ninc]
    const uint32_t *lrow_w, *linc;
    double *lw;
    int64_t lw_stride;
    int lw_slots, lw_ninc;
    const int32_t *act;     // [B * nA] active orbitals (ascending)
    const int32_t *core;    // [B * nC] core orbitals
    double *params;         // [B * pl.stride]
    // Davidson state
    int max_space, max_iter;
    double e_tol, r_tol;
    double *V, *S;          // [B][max_space][dim]
    double *Hd, *T;         // [B][dim]; T: the Ritz vector for the RDMs
    int sigma_variant;      // SIGMA_STRIP or SIGMA_WMAT
    double *W;              // [B][P][dim] sigma intermediate (SIGMA_WMAT)
    double *Ha, *Hb;        // [B][Na][Na], [B][Nb][Nb] string Hamiltonians (SIGMA_STRIP; Ha == Hb when na == nb)
    int nblk;               // blocks per tuple for vector kernels
    double *part;           // [B][nblk + 1][kParts] block partial sums (the last block: P-space corrections)
    double *G;              // [B][kMaxSpace*kMaxSpace] projected matrix V^T H V of the stored basis
    // The stored basis V is not orthonormal: V = Q U with Q orthonormal and U
    // upper triangular; R = U^-1 (upper triangular, R[i][j] at i*kMaxSpace+j,
    // entries j >= i used), so Q = V R
    double *R;              // [B][kMaxSpace*kMaxSpace]
    double *y, *coef;       // [B][kMaxSpace]; y: Ritz coefficients on the stored basis V
    // restarts that keep the previous Ritz vector (restart_keep 2): zp the
    // previous iteration's Ritz vector in the coordinates of Q (zero past its
    // length), y2 the coefficients on V of the kept direction, mu its Rayleigh
    // quotient
    int restart_keep;
    double spin_shift;      // lambda of the level shift lambda S_- S_+ (0: none)
    int whole;              // whole-tuple mode: one workgroup per tuple runs the whole Davidson solve
    double *y2, *zp;        // [B][kMaxSpace]
    double *mu;             // [B]
    double *sdot;           // [B][kMaxSpace] S_i . V_m, i < m, of the basis vector V_m being added
    double *theta, *theta_prev, *rnorm, *tnorm0, *out_e;   // [B]; tnorm0 = |T| before projection
    int32_t *status, *m, *iter, *out_status; // [B]
    int32_t *restart;       // [B] 0, or the vectors this iteration's restart keeps (1 or 2)
    int32_t *cgs2;          // [B] correction takes two explicit Gram-Schmidt passes
    // P-space preconditioner: the psp determinants of lowest diagonal energy
    // (0: diagonal preconditioner only); H_PP = Q T Q^T with T tridiagonal
    int psp;
    int32_t *pidx;          // [B][kPsp] determinant indices
    double *pQ;             // [B][kPsp][kPsp] H_PP, then Q
    double *pQt;            // [B][kPsp][kPsp] Q transposed (coalesced reads of Q w)
    double *pT;             // [B][3][kPsp] diagonal, subdiagonal of T, lowest eigenvector of H_PP
    int32_t *counter;       // [2] running tuples, tuples whose correction needs the explicit passes
    // RDM pass (backward): Gram partials and sums
    int nblk_r;
    double *rdm_part;       // [B][nblk_r][NP*NP]
    double *rdm_G;          // [B][NP*NP]
    double *rdm_w;          // [B] weights of the device embedding into the gradient
    // spatial symmetry targeting
    double sym_shift;       // lambda of the level shift away from other irreps (0: none)
    int irrep;              // target irrep label
    const int32_t *orb_irrep;   // [n] irrep labels of the orbitals (device)
};

// kernels.hip, sigma.hip and strip.hip
hipError_t init_kernels();
// Static device workspace of mbefci_solve_tuples_noalloc: 128 MiB per device.
constexpr size_t kScratchBytes = (size_t)128 << 20;
// Its device address on the current device (hipGetSymbolAddress).
hipError_t scratch_address(void **ptr);
hipError_t init_sigma_kernels();   // LDS limits of the sigma kernels (called by init_kernels)
hipError_t init_strip_kernels();   // the same for the strip kernels (called by init_sigma_kernels)
// alpha-beta term of sigma (column strip, strip.hip): sig = X + shift c
// (ev_mid, if given, is recorded after the MFMA kernel, before the gather of
// the W-in-HBM form)
hipError_t launch_strip(const Batch &b, VecRef c, VecRef sig, double shift, int skip, hipStream_t s,
                        hipEvent_t ev_mid = nullptr);
// which alpha-beta kernel launch_sigma runs for the batch (0 all pair rows,
// 1 linked gathered, 2 linked resident, 3 linked with the vector-ALU
// diagonal, 4 W materialised, 5 linked rows through W in HBM)
int alpha_beta_kernel(const Batch &b);
// linked-row strip kernel: row slots per alpha string, fit check, per-tuple
// A-table size (doubles) and its build (once per batch, after the gather)
constexpr int kLinkedRows = 32;
constexpr int kLinkedRowsW = 48;       // slots of the form with W in HBM (three MFMA row tiles)
constexpr int kLinkedMinActive = 9;    // smallest n_A that uses the linked-row kernel
// Per-tuple A table of the linked-row kernel: with kLinkedSigned the rows are
// A, -A (the alpha link sign picked by the row), then the diagonal sums;
// without it A, then the diagonal sums, and the sign rides on the scatter
// entry (bit 31).  Row length (doubles) for a padded pair count Kpad: the
// columns of two consecutive MFMA K steps are interleaved (linked_pos), 8
// doubles per K-step pair.
constexpr bool kLinkedSigned = false;
__host__ __device__ inline int linked_row_len(int Kpad) { return (Kpad / 4 + 1) / 2 * 8; }
// Position of row slot s = 16 h + kr + 4 v (MFMA output row of tile h held by
// lanes kr in register v) in a string's scatter-entry row: 16 h + 4 kr + v.
inline int linked_scat_pos(int s) { return (s & 16) | ((s & 3) << 2) | ((s >> 2) & 3); }
bool linked_fits(const ParamLayout &pl, int64_t Na, int nel);
// the form whose 32 slots hold only the n (n_A - n) off-diagonal links (the
// diagonal sums on the vector ALU, A resident in LDS, two halves of four waves)
bool linked_dv_fits(const ParamLayout &pl, int64_t Na, int nel);
// the form that writes the linked rows of W to HBM and gathers them (no sigma
// strip in LDS; 1 + n (n_A - n) <= 48 rows)
bool linked_w_fits(const ParamLayout &pl, int64_t Na, int nel);
int64_t linked_a_stride(const ParamLayout &pl, int64_t Na);
hipError_t launch_linked_a(const Batch &b, hipStream_t s);
hipError_t launch_gather(const Batch &b, hipStream_t s);
hipError_t launch_hdiag(const Batch &b, double *out, int64_t ostride, int add_ecore, hipStream_t s);
// sigma = (H + shift) c; with `dots` and the column-strip variant the GEMM
// also leaves the partial dots V_i . sig, i <= m, in partial blocks
// 0 .. gemm_blocks(b) - 1 (sigma_fuses_dots)
hipError_t launch_sigma(const Batch &b, VecRef c, VecRef sig, double shift, bool skip_done, bool dots,
                        hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, hipEvent_t evg, hipEvent_t ev2);
inline bool sigma_fuses_dots(const Batch &b) { return b.sigma_variant == SIGMA_STRIP; }
int gemm_blocks(const Batch &b);
hipError_t launch_update_G(const Batch &b, int nsum, hipStream_t s);
hipError_t launch_guess(const Batch &b, hipStream_t s);
hipError_t launch_init_state(const Batch &b, hipStream_t s);
hipError_t launch_dots(const Batch &b, VecRef y, int nx_extra, hipStream_t s);
hipError_t launch_iter_head(const Batch &b, hipStream_t s);
hipError_t launch_orthonormalize(const Batch &b, hipStream_t s);
hipError_t launch_finalize(const Batch &b, hipStream_t s);
size_t sigma_lds_bytes(const ParamLayout &pl);
size_t strip_lds_bytes(const ParamLayout &pl, int64_t Na);
bool strip_fits(const ParamLayout &pl, int64_t Na, int nentA, int nentB);
// per-batch set-up of the column-strip sigma: string Hamiltonians and, for
// the linked-row kernel, the per-tuple A tables (after the gather)
hipError_t launch_build_hb(const Batch &b, hipStream_t s);
hipError_t launch_form_x(const Batch &b, hipStream_t s);
hipError_t launch_pspace(const Batch &b, hipStream_t s);
int rdm_np(int nA);
size_t rdm_lds_bytes(int NP);
hipError_t launch_rdm(const Batch &b, VecRef x, double *part, double *G, int nblk_r, hipStream_t s);
// weighted embedding of the batch's density matrices (b.rdm_G) into the
// full-space gradient gh [n^2], ge [n^4] (device), weights w [B] (device)
hipError_t launch_rdm_embed(const Batch &b, const double *w, double *gh, double *ge, hipStream_t s);

// whole-tuple mode (whole.hip): classes of at most kWholeMaxDim determinants
// and kWholeMaxActive orbitals, with the vector of each sigma, the pair
// integrals, the string Hamiltonians and both link tables in LDS
constexpr int kWholeMaxDim = 4900;
constexpr int kWholeDefaultDim = 1225;   // default options.whole_dim (measured crossover)
constexpr int kWholeMaxActive = 10;
constexpr int kWholeMaxNent = 32;
constexpr int kWholePsp = 32;      // P space of the whole-tuple mode (at most options.pspace)   // link entries per string (n (n_A - n + 1) <= 30 for n_A <= 10)
// (same: both spins have the same electron count and share one string Hamiltonian)
bool whole_fits(const ParamLayout &pl, int64_t dim, int64_t Na, int64_t Nb, int nentA, int nentB, bool same);
// after the set-up (gather, string Hamiltonians, diagonal, P space, guess):
// every iteration of every tuple, then theta, status, iter, m and y as the
// batched iteration leaves them
hipError_t launch_whole(const Batch &b, hipStream_t s);
hipError_t init_whole_kernels();

// base-model energies (base.hip): eps_base of ntup tuples, one workgroup
// each; act/core: per tuple (stride sa, sc) the active and core orbitals,
// nact/ncore their counts; NaN for a tuple with a non-positive denominator
hipError_t launch_base(const double *h, const double *eri, int n, const int32_t *act, const int32_t *nact, int sa,
                       const int32_t *core, const int32_t *ncore, int sc, int nalpha, int nbeta, double e_const,
                       int ntup, double *out, hipStream_t s);
// coupled-cluster base (cc.hip): CCSD / CCSD(T) per tuple, one workgroup each
constexpr int kCcMaxActive = 32;        // active orbitals of a tuple (the whole space of a base energy included)
constexpr int kCcMaxIter = 300;         // amplitude iterations
constexpr double kCcTol = 1e-11;        // largest amplitude change at convergence
constexpr double kCanonTol = 1e-10;     // off-diagonal Fock elements allowed with (T)
constexpr int kCcCoopActive = 10;       // tuples of at least this many active orbitals: one cooperative launch each
constexpr int kCcMaxWgs = 256;          // workgroups of such a launch
int64_t cc_slice_doubles(int o, int v);
int ccsd_coop_wgs();
hipError_t launch_ccsd_coop(const double *h, const double *eri, int n, const int32_t *act, const int32_t *nact,
                            const int32_t *core, const int32_t *ncore, int stride, int nalpha, int nbeta,
                            double e_const, double *work, int64_t slice, int triples, int max_iter, double tol,
                            double *out, int32_t *status, int wgs, double *part, hipStream_t s);
hipError_t launch_ccsd(const double *h, const double *eri, int n, const int32_t *act, const int32_t *nact,
                       const int32_t *core, const int32_t *ncore, int stride, int nalpha, int nbeta, double e_const,
                       int ntup, double *work, int64_t slice, int triples, int max_iter, double tol, double *out,
                       int32_t *status, hipStream_t s);

// CASSCF expansion reference (casscf.hip)
constexpr int kMaxOrb = 64;         // orbital limit of the library
// h = U^T h0 U and eri = the four-index transformation of eri0 (full n^4
// layouts; tmp: n^4 doubles of scratch)
hipError_t launch_rotate_integrals(const double *h0, const double *eri0, const double *U, double *h, double *eri,
                                   double *tmp, int n, hipStream_t s);
// generalised Fock matrix F and Fock matrix f (n x n) from the full-space
// gamma and Gamma / 2 (g2h); occ: the no orbitals with density
hipError_t launch_fock(const double *h, const double *eri, const double *g1, const double *g2h, const int32_t *occ,
                       int no, int n, double *F, double *f, hipStream_t s);

}  // namespace mbefci

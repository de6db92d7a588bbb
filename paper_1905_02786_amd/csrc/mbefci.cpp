// Host side of libmbefci.so: context, validation, string tables, the MBE
// planner (tuple generation, screening, increment assembly; Eq. 1-3) and the
// batch driver of the Davidson solver whose kernels live in kernels.hip,
// sigma.hip and strip.hip.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/mbefci.h"
#include "internal.h"

using namespace mbefci;

namespace {

struct Tables {
    int nA = 0, nel = 0, nent = 0;
    int64_t nstr = 0;
    std::vector<uint32_t> strings;   // ascending bit masks
    std::vector<uint32_t> links;     // [nstr][nent]
    std::vector<uint32_t> pairs;     // [nstr][P]: link of each string per pair, strip pair order
    std::vector<uint32_t> scat;      // [nstr + 1][P + 1]: scatter form for the strip kernel
    std::vector<uint32_t> lrow, lscat;   // [nstr + 1][32]: linked-row form (empty if the links need more slots)
    std::vector<uint32_t> lrow_v, lscat_v;   // the same without the diagonal slot (diagonal on the vector ALU)
    // linked rows through W in HBM: A-row offsets of 48 slots per string
    // [nstr + 1][48] (slot 0 the diagonal sum), and per target string its
    // incoming W rows [nstr][1 + n (n_A - n)] (row K * slots + slot, bit 31 sign)
    std::vector<uint32_t> lrow_w, linc;
    int w_slots = 0;
    std::vector<int32_t> lperm;          // [2 (lpairs + 8)]: string order of the linked-row kernel
    int lpairs = 0;
};

// Order of the alpha strings for the linked-row kernel: pairs of strings
// that differ in at least three orbitals (then neither reaches the other,
// nor a common string, by one replacement: they share no scatter target),
// padded with the dummy index nstr, plus eight dummy pairs at the end.
// Greedy, most constrained first: a pair starts with the unplaced string
// that has the fewest unplaced compatible strings and takes the compatible
// one with the fewest (lowest index on ties).
void pair_strings(Tables &T) {
    const int64_t N = T.nstr;
    const size_t W = (size_t)(N + 63) / 64;
    std::vector<uint64_t> comp((size_t)N * W, 0), avail(W, 0), cand(W);
    std::vector<int64_t> deg(N, 0);
    for (int64_t i = 0; i < N; ++i) {
        avail[i / 64] |= 1ull << (i % 64);
        for (int64_t j = 0; j < N; ++j)
            if (j != i && __builtin_popcount(T.strings[i] & T.strings[j]) <= T.nel - 3) {
                comp[(size_t)i * W + j / 64] |= 1ull << (j % 64);
                ++deg[i];
            }
    }
    auto pick = [&](const std::vector<uint64_t> &set) -> int64_t {
        int64_t best = -1;
        for (size_t w = 0; w < W; ++w)
            for (uint64_t m = set[w]; m; m &= m - 1) {
                const int64_t i = (int64_t)(w * 64 + __builtin_ctzll(m));
                if (best < 0 || deg[i] < deg[best]) best = i;
            }
        return best;
    };
    auto take = [&](int64_t i) {
        avail[i / 64] &= ~(1ull << (i % 64));
        for (size_t w = 0; w < W; ++w)
            for (uint64_t m = comp[(size_t)i * W + w]; m; m &= m - 1) --deg[w * 64 + __builtin_ctzll(m)];
    };
    T.lperm.clear();
    for (int64_t left = N; left > 0;) {
        const int64_t a = pick(avail);
        take(a);
        for (size_t w = 0; w < W; ++w) cand[w] = avail[w] & comp[(size_t)a * W + w];
        const int64_t b = pick(cand);
        if (b >= 0) take(b);
        T.lperm.push_back((int32_t)a);
        T.lperm.push_back(b >= 0 ? (int32_t)b : (int32_t)N);
        left -= b >= 0 ? 2 : 1;
    }
    T.lpairs = (int)(T.lperm.size() / 2);
    T.lperm.resize(T.lperm.size() + 16, (int32_t)N);
}

// Strings with `nel` of `nA` bits set, ascending; for each string I the
// entries (p, q) with q in I and (p not in I or p == q): diagonal entries
// first (p ascending), then q ascending, p ascending.  E_pq|I> = sign |J> with
// sign = (-1)^(number of occupied orbitals strictly between p and q).
void build_tables(int nA, int nel, Tables &T) {
    T.nA = nA;
    T.nel = nel;
    T.nent = nel * (nA - nel) + nel;
    std::vector<int32_t> rank((size_t)1 << nA, -1);
    T.strings.clear();
    for (uint32_t m = 0; m < (1u << nA); ++m)
        if (__builtin_popcount(m) == nel) {
            rank[m] = (int32_t)T.strings.size();
            T.strings.push_back(m);
        }
    T.nstr = (int64_t)T.strings.size();
    T.links.assign((size_t)T.nstr * T.nent, 0);
    for (int64_t I = 0; I < T.nstr; ++I) {
        const uint32_t m = T.strings[I];
        uint32_t *out = &T.links[(size_t)I * T.nent];
        int e = 0;
        for (int p = 0; p < nA; ++p)
            if (m >> p & 1u) out[e++] = (uint32_t)I | ((uint32_t)(p * (p + 1) / 2 + p) << 20);
        for (int q = 0; q < nA; ++q) {
            if (!(m >> q & 1u)) continue;
            for (int p = 0; p < nA; ++p) {
                if (m >> p & 1u) continue;
                const uint32_t J = (m & ~(1u << q)) | (1u << p);
                const int lo = std::min(p, q), hi = std::max(p, q);
                const uint32_t between = m & (((1u << hi) - 1u) & ~((1u << (lo + 1)) - 1u));
                const uint32_t neg = (uint32_t)(__builtin_popcount(between) & 1);
                const int P = hi * (hi + 1) / 2 + lo;
                out[e++] = (uint32_t)rank[J] | ((uint32_t)P << 20) | (neg << 31);
            }
        }
    }
    // Dense forms for the column-strip sigma kernel, columns in its pair order
    // (diagonal pairs (p,p) first as column p, then p > q in packed order; a
    // string has at most one link per pair):
    //   pairs[I][Q] = J | bit 30 (link exists) | bit 31 (sign);
    //   scat[I][Q]  = J * 128 (byte offset of the sigma-strip row) | bit 31
    //                 for off-diagonal links, else nstr * 128 (discard row);
    //                 column np and row nstr are all discard.
    const int np = nA * (nA + 1) / 2;
    const uint32_t discard = (uint32_t)T.nstr * 128u;
    T.pairs.assign((size_t)T.nstr * np, 0u);
    T.scat.assign((size_t)(T.nstr + 1) * (np + 1), discard);
    for (int64_t I = 0; I < T.nstr; ++I) {
        for (int e = 0; e < T.nent; ++e) {
            const uint32_t L = T.links[(size_t)I * T.nent + e];
            const int P = (int)((L >> 20) & 0x3FFu);
            int p = 0;
            while ((p + 1) * (p + 2) / 2 <= P) ++p;
            const int q = P - p * (p + 1) / 2;
            const int col = p == q ? p : nA + P - p;
            const uint32_t J = L & 0xFFFFFu, sign = L & 0x80000000u;
            T.pairs[(size_t)I * np + col] = J | sign | (1u << 30);
            if (p != q) T.scat[(size_t)I * (np + 1) + col] = J * 128u | sign;
        }
    }
    // Linked-row form for the linked-row strip kernel, 32 slots per string
    // (row nstr all discard), as byte offsets: lrow = the slot's row of the
    // per-tuple A table (rows of Kpad doubles: pair col, np + col for the
    // negated row, 2 np + I for the diagonal sum of string I), lscat = its
    // target row of the sigma strip (128 bytes a row).  Slot 0 is the
    // diagonal sum (target I), then the off-diagonal links in link order
    // (target J, the negated row for a negative sign); unused slots read row
    // 0 and go to the discard row nstr.  lscat is stored in the order of the
    // MFMA output rows of a lane (linked_scat_pos), so that a lane's four
    // entries are one 16-byte load.
    T.lrow.clear();
    T.lscat.clear();
    T.lrow_v.clear();
    T.lscat_v.clear();
    T.lperm.clear();
    T.lpairs = 0;
    // both forms where they fit: with the diagonal sum in slot 0 (1 + n (n_A - n)
    // rows) and, for the vector-ALU diagonal, the off-diagonal links alone
    for (int form = 0; form < 2; ++form) {
        const bool dv = form == 1;
        if ((dv ? 0 : 1) + nel * (nA - nel) > kLinkedRows) continue;
        const uint32_t kp8 = (uint32_t)linked_row_len((np + 3) / 4 * 4) * 8u;
        const uint32_t dg = kLinkedSigned ? 2 * np : np;   // first diagonal-sum row
        std::vector<uint32_t> &LR = dv ? T.lrow_v : T.lrow, &LS = dv ? T.lscat_v : T.lscat;
        LR.assign((size_t)(T.nstr + 1) * kLinkedRows, 0u);
        LS.assign((size_t)(T.nstr + 1) * kLinkedRows, discard);
        for (int64_t I = 0; I < T.nstr; ++I) {
            uint32_t *lr = &LR[(size_t)I * kLinkedRows], *ls = &LS[(size_t)I * kLinkedRows];
            int slot = 0;
            if (!dv) {
                lr[0] = (uint32_t)(dg + I) * kp8;
                ls[linked_scat_pos(0)] = (uint32_t)I * 128u;
                slot = 1;
            }
            for (int e = 0; e < T.nent; ++e) {
                const uint32_t L = T.links[(size_t)I * T.nent + e];
                const int P = (int)((L >> 20) & 0x3FFu);
                int p = 0;
                while ((p + 1) * (p + 2) / 2 <= P) ++p;
                const int q = P - p * (p + 1) / 2;
                if (p == q) continue;
                const int col = nA + P - p;
                const uint32_t neg = L & 0x80000000u;
                lr[slot] = (uint32_t)(col + ((kLinkedSigned && neg) ? np : 0)) * kp8;
                ls[linked_scat_pos(slot)] = (L & 0xFFFFFu) * 128u | (kLinkedSigned ? 0u : neg);
                ++slot;
            }
        }
    }
    if (!T.lrow.empty() || !T.lrow_v.empty()) pair_strings(T);
    // the W-in-HBM form: slot 0 the diagonal sum, then the off-diagonal links
    // in link order; the gather table lists for target J its own diagonal row
    // first, then the rows (K, slot) of the links K -> J by ascending K
    T.lrow_w.clear();
    T.linc.clear();
    T.w_slots = 0;
    const int offd = nel * (nA - nel);
    if (1 + offd <= kLinkedRowsW && T.nstr > 0) {
        const int S = 1 + offd;
        const uint32_t kp8 = (uint32_t)linked_row_len((np + 3) / 4 * 4) * 8u;
        T.w_slots = S;
        T.lrow_w.assign((size_t)(T.nstr + 1) * kLinkedRowsW, 0u);
        std::vector<std::vector<uint32_t>> inc((size_t)T.nstr);
        for (int64_t J = 0; J < T.nstr; ++J) inc[J].push_back((uint32_t)(J * S));
        for (int64_t K = 0; K < T.nstr; ++K) {
            int slot = 1;
            for (int e = 0; e < T.nent; ++e) {
                const uint32_t L = T.links[(size_t)K * T.nent + e];
                const int P = (int)((L >> 20) & 0x3FFu);
                int p = 0;
                while ((p + 1) * (p + 2) / 2 <= P) ++p;
                const int q = P - p * (p + 1) / 2;
                if (p == q) continue;
                T.lrow_w[(size_t)K * kLinkedRowsW + slot] = (uint32_t)(nA + P - p) * kp8;
                const int64_t J = (int64_t)(L & 0xFFFFFu);
                inc[J].push_back((uint32_t)(K * S + slot) | (L & 0x80000000u));
                ++slot;
            }
        }
        T.linc.reserve((size_t)T.nstr * S);
        for (int64_t J = 0; J < T.nstr; ++J) T.linc.insert(T.linc.end(), inc[J].begin(), inc[J].end());
    }
}

struct ClassKey {
    int nA, na, nb;
    bool operator<(const ClassKey &o) const {
        if (nA != o.nA) return nA < o.nA;
        if (na != o.na) return na < o.na;
        return nb < o.nb;
    }
};

struct Result {
    struct Order {
        int k;
        std::vector<int16_t> tuples;
        std::vector<double> eps, dinc;
        std::vector<int32_t> status;
        double sum = 0.0, wall_ms = 0.0;
    };
    std::vector<Order> orders;
    double total = 0.0;
    // base model (options.base_model): the orders hold eps - eps_base, and
    // the total includes the base energy of the whole space
    double e_base = 0.0;
    // gradient of the total formed by the forward run (options.gradient = 1):
    // dE/dh [n^2] and dE/d(pq|rs) [n^4], entries as independent variables
    bool has_grad = false;
    std::vector<double> grad_h, grad_eri;
    // streamed last order (options.stream_last): listed but solved in slices
    // by mbefci_order_solve; its increments need the lower orders' d_eps
    bool open = false;
    std::vector<char> solved;
    std::unordered_map<uint64_t, double> dinc_map;
};

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

double now_ms() {
    return std::chrono::duration<double, std::milli>(
               std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct mbefci_result {
    Result r;
};

struct mbefci_ctx {
    int device = -1;
    bool host_only = true;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;   // private stream the Davidson iteration is captured on (graph mode)
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};   // sigma start, MFMA kernel end, gather end, end
    std::string err;
    // Hamiltonian
    int norb = 0;
    bool ham_set = false;
    bool sym_checked = false;   // the Hamiltonian checked against the irrep labels
    std::vector<double> h, eri;
    std::vector<int32_t> irr;          // orbital irrep labels (empty: not set)
    int32_t *d_irr = nullptr;
    double e_const = 0.0;
    double *d_h = nullptr, *d_eri = nullptr;
    mbefci_eri_layout eri_layout = MBEFCI_ERI_FULL;
    // device gradient accumulators of the running gradient pass (in the
    // caller's workspace, past the part the batches use)
    double *d_gh = nullptr, *d_ge = nullptr;
    // the static device workspace of this context's device (resolved at creation)
    void *scratch = nullptr;
    int gemm_tile = 0;   // GEMM tile of the batches being carved (autotuner choice; 0: by padding)
    // spaces
    bool spaces_set = false;
    int nalpha = 0, nbeta = 0, nfrozen = 0;
    std::vector<int> ref, X;
    std::vector<char> inX;
    std::vector<std::pair<int, int>> pi;   // degenerate pairs of the expansion space (pi-pruning)
    mbefci_options opt{};
    mbefci_stats stats{};
    std::map<std::tuple<int, int, int>, mbefci_class_stats> cstats;   // per shape class, last call
    mbefci_class_stats *sigma_cls = nullptr;   // class of the sigma whose events are pending
    bool sigma_pending = false;   // profile: events of the last sigma not read yet
    std::map<std::pair<int, int>, Tables> tables;

    mbefci_status fail(mbefci_status s, const std::string &m) {
        err = m;
        return s;
    }
    const Tables &table(int nA, int nel) {
        auto key = std::make_pair(nA, nel);
        auto it = tables.find(key);
        if (it != tables.end()) return it->second;
        Tables &T = tables[key];
        build_tables(nA, nel, T);
        return T;
    }
};

#define HIPCHK(x)                                                                     \
    do {                                                                              \
        hipError_t e_ = (x);                                                          \
        if (e_ != hipSuccess)                                                         \
            return ctx->fail(MBEFCI_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

namespace {

// Shape of one tuple's CAS (Sec. 2 partition).
struct TupleShape {
    ClassKey key;
    int nC;
    std::vector<int32_t> act, core;
};

mbefci_status check_symmetry(mbefci_ctx *ctx, int order, int64_t ntup, const std::vector<TupleShape> &shapes);

mbefci_status tuple_shape(mbefci_ctx *ctx, int order, const int16_t *tup, TupleShape &ts) {
    for (int i = 0; i < order; ++i) {
        const int p = tup[i];
        if (p < 0 || p >= ctx->norb || !ctx->inX[p])
            return ctx->fail(MBEFCI_EINVAL, "tuple orbital " + std::to_string(p) + " is not an expansion orbital");
        if (i > 0 && tup[i - 1] >= p) return ctx->fail(MBEFCI_EINVAL, "tuple not strictly ascending");
    }
    ts.act.clear();
    std::vector<char> inA(ctx->norb, 0);
    for (int p : ctx->ref) inA[p] = 1;
    for (int i = 0; i < order; ++i) inA[tup[i]] = 1;
    for (int p = 0; p < ctx->norb; ++p)
        if (inA[p]) ts.act.push_back(p);
    ts.core.clear();
    for (int p = 0; p < ctx->nbeta; ++p)
        if (!inA[p]) ts.core.push_back(p);   // frozen orbitals are < nbeta and never active
    int na = 0, nb = 0;
    for (int p : ts.act) {
        na += p < ctx->nalpha;
        nb += p < ctx->nbeta;
    }
    ts.key = ClassKey{(int)ts.act.size(), na, nb};
    ts.nC = (int)ts.core.size();
    if (ts.key.nA > kMaxActive)
        return ctx->fail(MBEFCI_ETOOLARGE, "CAS with " + std::to_string(ts.key.nA) + " active orbitals exceeds " +
                                               std::to_string(kMaxActive));
    return MBEFCI_OK;
}

// Blocks per tuple of the Davidson vector kernels: about 4096 determinants
// (16 per thread) per block; the per-tuple kernels then sum few partials.
int nblk_for(int64_t dim) {
    int64_t g = (dim + 4095) / 4096;
    return (int)std::max<int64_t>(1, std::min<int64_t>(256, g));
}

struct ClassPlan {
    ClassKey key;
    int nC;
    const Tables *ta, *tb;
    int64_t dim;
    ParamLayout pl;
    int nblk;
    int variant;
    int psp;   // P-space size of the Davidson preconditioner (0: diagonal only)
    bool linked;   // linked-row strip kernel
    bool linked_dv;   // its form without the diagonal slot (diagonal sums on the vector ALU)
    bool linked_w;    // linked rows through W in HBM (no sigma strip in LDS)
    bool whole;       // whole-tuple mode (one workgroup per tuple, the Davidson loop on the device)
    bool rdm;
    int nblk_r, NP;
    size_t fixed_bytes, per_tuple;
};

int nblk_rdm(int64_t dim) {
    const int64_t tiles = (dim + 31) / 32;
    return (int)std::max<int64_t>(1, std::min<int64_t>(32, (tiles + 7) / 8));
}

void plan_class(mbefci_ctx *ctx, const ClassKey &key, int nC, ClassPlan &cp, bool davidson, bool rdm = false) {
    cp.key = key;
    cp.nC = nC;
    cp.ta = &ctx->table(key.nA, key.na);
    cp.tb = &ctx->table(key.nA, key.nb);
    cp.dim = cp.ta->nstr * cp.tb->nstr;
    cp.pl.init(key.nA);
    cp.nblk = nblk_for(cp.dim);
    // the strip variant's GEMM writes one partial block per output tile (at
    // most this many: 64 x 64 tiles)
    cp.nblk = std::max<int64_t>(cp.nblk, ((cp.ta->nstr + 63) / 64) * ((cp.tb->nstr + 63) / 64));
    const int want = ctx->opt.sigma_variant;
    const bool fits = strip_fits(cp.pl, cp.ta->nstr, cp.ta->nent, cp.tb->nent);
    cp.variant = (want == SIGMA_WMAT || !fits) ? SIGMA_WMAT : SIGMA_STRIP;
    cp.psp = (davidson && cp.variant == SIGMA_STRIP && ctx->opt.pspace > 0)
                 ? (int)std::min<int64_t>(ctx->opt.pspace, cp.dim) : 0;
    // linked rows pay off where they replace at least three MFMA row tiles;
    // the form with the diagonal slot wherever it fits (linked_rows 1-3), else
    // (or always with linked_rows 4) the form with the diagonal sums on the
    // vector ALU
    const int lm = ctx->opt.linked_rows;
    const bool lin_ok = cp.variant == SIGMA_STRIP && lm != 0 && key.nA >= (lm == 1 ? kLinkedMinActive : 4);
    const bool classic = lin_ok && !cp.ta->lrow.empty() && linked_fits(cp.pl, cp.ta->nstr, key.na);
    const bool dvf = lin_ok && !cp.ta->lrow_v.empty() && linked_dv_fits(cp.pl, cp.ta->nstr, key.na);
    cp.linked_dv = dvf && (lm == 4 || !classic);
    // linked rows through W in HBM where neither LDS form fits (or always with
    // linked_rows 5)
    // (the W kernel addresses a tuple's W rows through a 32-bit buffer offset)
    const bool wf = lin_ok && cp.ta->w_slots > 0 && linked_w_fits(cp.pl, cp.ta->nstr, key.na) &&
                    (double)cp.dim * cp.ta->w_slots * sizeof(double) < 2147483647.0;
    cp.linked_w = wf && (lm == 5 || (!classic && !cp.linked_dv));
    if (lm == 5 && cp.linked_w) cp.linked_dv = false;
    const bool cls = classic && !cp.linked_dv && !cp.linked_w;
    cp.linked = cls || cp.linked_dv || cp.linked_w;
    // whole-tuple mode for small classes (not with per-launch sigma timing)
    cp.whole = davidson && cp.variant == SIGMA_STRIP && !ctx->opt.profile && cp.dim <= ctx->opt.whole_dim &&
               whole_fits(cp.pl, cp.dim, cp.ta->nstr, cp.tb->nstr, cp.ta->nent, cp.tb->nent,
                          key.na == key.nb);
    // a smaller P space there unless it holds the whole CAS: its
    // factorisation is part of every class's set-up, and the iterations it
    // saves are cheap in that mode
    if (cp.whole && cp.dim > kPsp) cp.psp = std::min(cp.psp, kWholePsp);
    cp.fixed_bytes = align256(4 * (cp.ta->nstr + cp.tb->nstr)) +
                     align256(4 * (size_t)cp.ta->nstr * cp.ta->nent) +
                     align256(4 * (size_t)cp.tb->nstr * cp.tb->nent) +
                     align256(4 * (size_t)(cp.ta->nstr + 1) * (cp.pl.P + 1)) +
                     align256(4 * (size_t)cp.tb->nstr * cp.pl.P) +
                     (cp.linked ? 2 * align256(4 * (size_t)(cp.ta->nstr + 1) * kLinkedRows) +
                                      align256(4 * cp.ta->lperm.size()) : 0) +
                     (cp.linked_w ? align256(4 * (size_t)(cp.ta->nstr + 1) * kLinkedRowsW) +
                                        align256(4 * cp.ta->linc.size()) : 0) +
                     64 * 256;
    const int ms = davidson ? ctx->opt.max_space : 0;
    size_t pt = 0;
    pt += 8 * (size_t)cp.pl.stride;                          // params
    pt += 4 * (size_t)(key.nA + nC + 2);                      // act, core
    pt += 8 * (size_t)cp.dim * (2 * ms + (davidson ? 2 : 0)); // V, S, Hd, T
    if (cp.variant == SIGMA_WMAT) pt += 8 * (size_t)cp.pl.P * cp.dim;            // W
    else pt += 8 * (size_t)cp.tb->nstr * cp.tb->nstr +                             // H_b, H_a
               (key.na != key.nb ? 8 * (size_t)cp.ta->nstr * cp.ta->nstr : 0);
    pt += 8 * (size_t)(cp.nblk + 1) * kParts;                // partials (+ P-space block)
    if (cp.linked) pt += 8 * (size_t)linked_a_stride(cp.pl, cp.ta->nstr);   // A table
    if (cp.linked_w) pt += 8 * (size_t)cp.dim * cp.ta->w_slots + 256;          // W rows
    if (cp.psp > 0) pt += 4 * (size_t)kPsp + 16 * (size_t)kPsp * kPsp + 24 * (size_t)kPsp + 4 * 256;
    cp.rdm = rdm;
    cp.NP = rdm_np(key.nA);
    cp.nblk_r = nblk_rdm(cp.dim);
    if (rdm) pt += 8 * (size_t)(cp.nblk_r + 1) * cp.NP * cp.NP + 8 + 256;  // RDM Gram partials, sum, weight
    pt += 8 * (size_t)(2 * kMaxSpace * kMaxSpace + 5 * kMaxSpace + 7) + 4 * 7;
    cp.per_tuple = pt + 256;
}

// Bump allocator over the caller's workspace.
struct Carver {
    char *base;
    size_t size, off = 0;
    bool ok = true;
    template <class T> T *take(size_t count) {
        size_t bytes = align256(count * sizeof(T));
        if (off + bytes > size) {
            ok = false;
            return nullptr;
        }
        T *p = reinterpret_cast<T *>(base + off);
        off += bytes;
        return p;
    }
};

// Fill the table and batch pointers; returns false if it does not fit.
bool carve_batch(mbefci_ctx *ctx, const ClassPlan &cp, int B, Carver &cv, Batch &b, bool davidson) {
    b = Batch{};
    b.B = B;
    b.nA = cp.key.nA;
    b.na = cp.key.na;
    b.nb = cp.key.nb;
    b.nC = cp.nC;
    b.Na = cp.ta->nstr;
    b.Nb = cp.tb->nstr;
    b.dim = cp.dim;
    b.nentA = cp.ta->nent;
    b.nentB = cp.tb->nent;
    b.pl = cp.pl;
    b.norb = ctx->norb;
    b.e_const = ctx->e_const;
    b.h = ctx->d_h;
    b.eri = ctx->d_eri;
    b.strA = cv.take<uint32_t>(b.Na);
    b.strB = cv.take<uint32_t>(b.Nb);
    b.linkA = cv.take<uint32_t>((size_t)b.Na * b.nentA);
    b.linkB = cv.take<uint32_t>((size_t)b.Nb * b.nentB);
    b.scatA = cv.take<uint32_t>((size_t)(b.Na + 1) * (cp.pl.P + 1));
    b.pairB = cv.take<uint32_t>((size_t)b.Nb * cp.pl.P);
    if (cp.linked) {
        b.lrow = cv.take<uint32_t>((size_t)(b.Na + 1) * kLinkedRows);
        b.lscat = cv.take<uint32_t>((size_t)(b.Na + 1) * kLinkedRows);
        b.la_stride = linked_a_stride(cp.pl, b.Na);
        b.la = cv.take<double>((size_t)B * b.la_stride);
        b.lperm = cv.take<int32_t>(cp.ta->lperm.size() + 1);
        b.lpairs = cp.ta->lpairs;
        b.linked_mode = ctx->opt.linked_rows;
        b.linked_dv = cp.linked_dv ? 1 : 0;
        if (cp.linked_w) {
            b.lrow_w = cv.take<uint32_t>((size_t)(b.Na + 1) * kLinkedRowsW);
            b.linc = cv.take<uint32_t>(cp.ta->linc.size());
            b.lw_slots = cp.ta->w_slots;
            b.lw_ninc = cp.ta->w_slots;
            b.lw_stride = (int64_t)b.dim * cp.ta->w_slots;
            b.lw = cv.take<double>((size_t)B * b.lw_stride);
        }
    } else {
        b.lrow = b.lscat = nullptr;
        b.la = nullptr;
        b.la_stride = 0;
        b.lperm = nullptr;
        b.lpairs = 0;
    }
    b.act = cv.take<int32_t>((size_t)B * b.nA + 1);
    b.core = cv.take<int32_t>((size_t)B * b.nC + 1);
    b.params = cv.take<double>((size_t)B * cp.pl.stride);
    b.max_space = davidson ? ctx->opt.max_space : 0;
    b.restart_keep = ctx->opt.max_space >= 3 ? ctx->opt.restart_keep : 1;
    b.spin_shift = ctx->opt.spin_shift;
    b.sym_shift = ctx->opt.sym_shift;
    b.irrep = ctx->opt.irrep;
    b.orb_irrep = ctx->d_irr;
    b.whole = cp.whole ? 1 : 0;
    b.max_iter = ctx->opt.max_iter;
    b.e_tol = ctx->opt.e_tol;
    b.r_tol = ctx->opt.r_tol;
    if (davidson) {
        b.V = cv.take<double>((size_t)B * b.max_space * b.dim);
        b.S = cv.take<double>((size_t)B * b.max_space * b.dim);
        b.Hd = cv.take<double>((size_t)B * b.dim);
        b.T = cv.take<double>((size_t)B * b.dim);
    }
    b.sigma_variant = cp.variant;
    if (cp.variant == SIGMA_WMAT) {
        b.W = cv.take<double>((size_t)B * cp.pl.P * b.dim + 1);
        b.Ha = b.Hb = nullptr;
    } else {
        b.W = nullptr;
        b.Hb = cv.take<double>((size_t)B * b.Nb * b.Nb);
        // equal electron counts share tables and integrals, hence the string Hamiltonian
        b.Ha = b.na == b.nb ? b.Hb : cv.take<double>((size_t)B * b.Na * b.Na);
    }
    b.nblk = cp.nblk;
    b.gemm_tile = ctx->gemm_tile;
    b.part = cv.take<double>((size_t)B * (b.nblk + 1) * kParts);
    b.psp = cp.psp;
    if (cp.psp > 0) {
        b.pidx = cv.take<int32_t>((size_t)B * kPsp);
        b.pQ = cv.take<double>((size_t)B * kPsp * kPsp);
        b.pQt = cv.take<double>((size_t)B * kPsp * kPsp);
        b.pT = cv.take<double>((size_t)B * 3 * kPsp);
    } else {
        b.pidx = nullptr;
        b.pQ = b.pQt = b.pT = nullptr;
    }
    b.G = cv.take<double>((size_t)B * kMaxSpace * kMaxSpace);
    b.R = cv.take<double>((size_t)B * kMaxSpace * kMaxSpace);
    b.y = cv.take<double>((size_t)B * kMaxSpace);
    b.y2 = cv.take<double>((size_t)B * kMaxSpace);
    b.zp = cv.take<double>((size_t)B * kMaxSpace);
    b.mu = cv.take<double>(B);
    b.coef = cv.take<double>((size_t)B * kMaxSpace);
    b.sdot = cv.take<double>((size_t)B * kMaxSpace);
    b.theta = cv.take<double>(B);
    b.theta_prev = cv.take<double>(B);
    b.rnorm = cv.take<double>(B);
    b.tnorm0 = cv.take<double>(B);
    b.out_e = cv.take<double>(B);
    b.status = cv.take<int32_t>(B);
    b.m = cv.take<int32_t>(B);
    b.iter = cv.take<int32_t>(B);
    b.restart = cv.take<int32_t>(B);
    b.out_status = cv.take<int32_t>(B);
    b.cgs2 = cv.take<int32_t>(B);
    b.counter = cv.take<int32_t>(3);
    b.nblk_r = cp.nblk_r;
    if (cp.rdm) {
        b.rdm_part = cv.take<double>((size_t)B * cp.nblk_r * cp.NP * cp.NP);
        b.rdm_G = cv.take<double>((size_t)B * cp.NP * cp.NP);
        b.rdm_w = cv.take<double>(B);
    } else {
        b.rdm_part = b.rdm_G = b.rdm_w = nullptr;
    }
    return cv.ok;
}

mbefci_status upload_tables(mbefci_ctx *ctx, const ClassPlan &cp, const Batch &b) {
    HIPCHK(hipMemcpyAsync((void *)b.strA, cp.ta->strings.data(), 4 * b.Na, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync((void *)b.strB, cp.tb->strings.data(), 4 * b.Nb, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync((void *)b.linkA, cp.ta->links.data(), 4 * (size_t)b.Na * b.nentA, hipMemcpyHostToDevice,
                          ctx->stream));
    HIPCHK(hipMemcpyAsync((void *)b.linkB, cp.tb->links.data(), 4 * (size_t)b.Nb * b.nentB, hipMemcpyHostToDevice,
                          ctx->stream));
    HIPCHK(hipMemcpyAsync((void *)b.scatA, cp.ta->scat.data(), 4 * (size_t)(b.Na + 1) * (b.pl.P + 1),
                          hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync((void *)b.pairB, cp.tb->pairs.data(), 4 * (size_t)b.Nb * b.pl.P, hipMemcpyHostToDevice,
                          ctx->stream));
    if (b.la) {
        // the slot tables of the LDS forms (not read by the W-in-HBM form,
        // whose class may have none)
        const std::vector<uint32_t> &lr = b.linked_dv ? cp.ta->lrow_v : cp.ta->lrow,
                                    &ls = b.linked_dv ? cp.ta->lscat_v : cp.ta->lscat;
        if (!b.lw) {
            HIPCHK(hipMemcpyAsync((void *)b.lrow, lr.data(), 4 * (size_t)(b.Na + 1) * kLinkedRows,
                                  hipMemcpyHostToDevice, ctx->stream));
            HIPCHK(hipMemcpyAsync((void *)b.lscat, ls.data(), 4 * (size_t)(b.Na + 1) * kLinkedRows,
                                  hipMemcpyHostToDevice, ctx->stream));
            HIPCHK(hipMemcpyAsync((void *)b.lperm, cp.ta->lperm.data(), 4 * cp.ta->lperm.size(),
                                  hipMemcpyHostToDevice, ctx->stream));
        }
        if (b.lw) {
            HIPCHK(hipMemcpyAsync((void *)b.lrow_w, cp.ta->lrow_w.data(), 4 * cp.ta->lrow_w.size(),
                                  hipMemcpyHostToDevice, ctx->stream));
            HIPCHK(hipMemcpyAsync((void *)b.linc, cp.ta->linc.data(), 4 * cp.ta->linc.size(), hipMemcpyHostToDevice,
                                  ctx->stream));
        }
    }
    return MBEFCI_OK;
}

mbefci_status upload_shapes(mbefci_ctx *ctx, const Batch &b, const std::vector<const TupleShape *> &shapes) {
    std::vector<int32_t> act((size_t)b.B * b.nA + 1, 0), core((size_t)b.B * b.nC + 1, 0);
    for (int t = 0; t < b.B; ++t) {
        std::copy(shapes[t]->act.begin(), shapes[t]->act.end(), act.begin() + (size_t)t * b.nA);
        std::copy(shapes[t]->core.begin(), shapes[t]->core.end(), core.begin() + (size_t)t * b.nC);
    }
    HIPCHK(hipMemcpyAsync((void *)b.act, act.data(), 4 * act.size(), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync((void *)b.core, core.data(), 4 * core.size(), hipMemcpyHostToDevice, ctx->stream));
    return MBEFCI_OK;
}

// W = A D on the rows the kernel must form: all P pair rows, or with the
// linked-row kernel the 1 + n_a (n_A - n_a) rows that link each alpha string
double sigma_flops(const Batch &b) {
    const double rows = b.la ? 1.0 + (double)b.na * (b.nA - b.na) : (double)b.pl.P;
    return 2.0 * rows * b.pl.P * (double)b.dim;
}
double sigma_bytes(const Batch &b) { return 16.0 * (double)b.dim + 8.0 * (double)b.pl.P * b.pl.P; }

// Accumulate the HIP-event time of the last sigma launch pair (profile mode).
// Called only after a stream synchronisation, so the events are complete.
void flush_sigma_time(mbefci_ctx *ctx) {
    if (!ctx->sigma_pending) return;
    ctx->sigma_pending = false;
    float ms_w = 0.f, ms_g = 0.f, ms_all = 0.f;
    if (hipEventElapsedTime(&ms_w, ctx->ev[0], ctx->ev[1]) == hipSuccess &&
        hipEventElapsedTime(&ms_g, ctx->ev[1], ctx->ev[2]) == hipSuccess &&
        hipEventElapsedTime(&ms_all, ctx->ev[0], ctx->ev[3]) == hipSuccess) {
        ctx->stats.sigma_ms += ms_w;
        ctx->stats.gather_ms += ms_g;
        ctx->stats.sigma_total_ms += ms_all;
        if (ctx->sigma_cls) {
            ctx->sigma_cls->sigma_ms += ms_w;
            ctx->sigma_cls->gather_ms += ms_g;
            ctx->sigma_cls->sigma_total_ms += ms_all;
        }
    }
}

mbefci_class_stats &class_stats(mbefci_ctx *ctx, const Batch &b) {
    mbefci_class_stats &c = ctx->cstats[std::make_tuple(b.nA, b.na, b.nb)];
    c.n_active = b.nA;
    c.n_alpha = b.na;
    c.n_beta = b.nb;
    c.dim = b.dim;
    c.kernel = b.whole ? 6 : alpha_beta_kernel(b);
    return c;
}

mbefci_status run_sigma(mbefci_ctx *ctx, const Batch &b, VecRef c, VecRef s, double shift, bool skip_done,
                        int64_t napps, bool dots = false) {
    const bool prof = ctx->opt.profile != 0;
    if (prof && ctx->sigma_pending) {   // a sigma whose events were not read yet
        HIPCHK(hipEventSynchronize(ctx->ev[3]));
        flush_sigma_time(ctx);
    }
    hipError_t e = launch_sigma(b, c, s, shift, skip_done, dots, ctx->stream, prof ? ctx->ev[0] : nullptr,
                                prof ? ctx->ev[1] : nullptr, prof ? ctx->ev[2] : nullptr,
                                prof ? ctx->ev[3] : nullptr);
    if (e != hipSuccess) return ctx->fail(MBEFCI_EDEVICE, std::string("sigma launch: ") + hipGetErrorString(e));
    ctx->stats.sigma_launches += 1;
    ctx->stats.sigma_calls += napps;
    ctx->stats.sigma_flops += napps * sigma_flops(b);
    ctx->stats.sigma_bytes += napps * sigma_bytes(b);
    mbefci_class_stats &cs = class_stats(ctx, b);
    cs.sigma_launches += 1;
    cs.sigma_calls += napps;
    cs.sigma_flops += napps * sigma_flops(b);
    ctx->sigma_cls = &cs;
    ctx->sigma_pending = prof;
    return MBEFCI_OK;
}

// What happens to the density matrices of a batch's converged vectors:
// copied to the host as Gram matrices (gram), or embedded on the device into
// the gradient accumulators ctx->d_gh, d_ge with the weights w (host, [B]).
struct RdmOut {
    std::vector<double> *gram = nullptr;
    const double *w = nullptr;
};

mbefci_status davidson_finish(mbefci_ctx *ctx, const Batch &b, double *e_out, int32_t *st_out, const RdmOut *ro);

// Davidson for one batch; energies/status (public codes) written at out[t].
mbefci_status davidson_batch(mbefci_ctx *ctx, const Batch &b, double *e_out, int32_t *st_out,
                             const RdmOut *ro = nullptr) {
    hipStream_t s = ctx->stream;
    hipError_t e;
    if ((e = launch_gather(b, s)) != hipSuccess) return ctx->fail(MBEFCI_EDEVICE, hipGetErrorString(e));
    if ((e = launch_build_hb(b, s)) != hipSuccess) return ctx->fail(MBEFCI_EDEVICE, hipGetErrorString(e));
    if ((e = launch_hdiag(b, b.Hd, b.dim, 0, s)) != hipSuccess) return ctx->fail(MBEFCI_EDEVICE, hipGetErrorString(e));
    if ((e = launch_init_state(b, s)) != hipSuccess) return ctx->fail(MBEFCI_EDEVICE, hipGetErrorString(e));
    if ((e = launch_pspace(b, s)) != hipSuccess) return ctx->fail(MBEFCI_EDEVICE, hipGetErrorString(e));
    if ((e = launch_guess(b, s)) != hipSuccess) return ctx->fail(MBEFCI_EDEVICE, hipGetErrorString(e));
    const int64_t tstride = (int64_t)b.max_space * b.dim;
    VecRef vm{b.V, tstride, b.m, 0}, sm{b.S, tstride, b.m, 0};
    if (b.whole) {
        // every iteration of every tuple in one launch
        if ((e = launch_whole(b, s)) != hipSuccess) return ctx->fail(MBEFCI_EDEVICE, hipGetErrorString(e));
        ++ctx->stats.whole_batches;
        return davidson_finish(ctx, b, e_out, st_out, ro);
    }
    // sigma of V_m into S_m, then column m of G (from the GEMM's partial dots
    // where the sigma variant computes them)
    auto sigma_and_G = [&](int64_t napps) -> mbefci_status {
        const bool fused = sigma_fuses_dots(b);
        mbefci_status r = run_sigma(ctx, b, vm, sm, 0.0, true, napps, fused);
        if (r != MBEFCI_OK) return r;
        hipError_t e2 = fused ? launch_update_G(b, gemm_blocks(b), s) : launch_dots(b, sm, 1, s);
        return e2 == hipSuccess ? MBEFCI_OK : ctx->fail(MBEFCI_EDEVICE, hipGetErrorString(e2));
    };
    mbefci_status rc = sigma_and_G(b.B);
    if (rc != MBEFCI_OK) return rc;
    int32_t cnt[3] = {b.B, 0, 0};   // running tuples; of them those that need the explicit Gram-Schmidt
                                    // passes; explicit passes of the whole batch
    const bool prof = ctx->opt.profile != 0;
    if (prof) {
        // one iteration per host round trip: the sigma launch of every
        // iteration is timed with events, and the explicit Gram-Schmidt
        // passes are launched only when some tuple needs them
        for (int it = 0; it <= b.max_iter; ++it) {
            if ((e = launch_iter_head(b, s)) != hipSuccess) return ctx->fail(MBEFCI_EDEVICE, hipGetErrorString(e));
            HIPCHK(hipMemcpyAsync(cnt, b.counter, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            flush_sigma_time(ctx);
            if (cnt[0] == 0) break;
            if (cnt[1] > 0 && (e = launch_orthonormalize(b, s)) != hipSuccess)
                return ctx->fail(MBEFCI_EDEVICE, hipGetErrorString(e));
            rc = sigma_and_G(cnt[0]);
            if (rc != MBEFCI_OK) return rc;
        }
    } else {
        // Iterations in blocks launched back to back, the running count read
        // once per block: every kernel skips the tuples that are no longer
        // running (the explicit Gram-Schmidt kernels also those whose
        // correction does not need them), so the result is that of one
        // iteration per round trip.  With options.graph the iteration's
        // launches are captured once per batch in a hipGraph (on a private
        // stream) and the graph is replayed on the context's stream.
        const bool fused = sigma_fuses_dots(b);
        auto one_iter = [&](hipStream_t st) -> hipError_t {
            hipError_t e1 = launch_iter_head(b, st);
            if (e1 != hipSuccess) return e1;
            if ((e1 = launch_orthonormalize(b, st)) != hipSuccess) return e1;
            if ((e1 = launch_sigma(b, vm, sm, 0.0, true, fused, st, nullptr, nullptr, nullptr, nullptr)) != hipSuccess)
                return e1;
            return fused ? launch_update_G(b, gemm_blocks(b), st) : launch_dots(b, sm, 1, st);
        };
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        if (ctx->opt.graph && ctx->cap_stream) {
            if (hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeRelaxed) == hipSuccess) {
                const hipError_t ec = one_iter(ctx->cap_stream);
                const hipError_t ee = hipStreamEndCapture(ctx->cap_stream, &graph);
                if (ec == hipSuccess && ee == hipSuccess && graph &&
                    hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
                    exec = nullptr;
            }
            (void)hipGetLastError();   // a capture that did not work leaves the direct launches
            if (exec) ++ctx->stats.graph_batches;
        }
        int block = 4;
        for (int it = 0; it <= b.max_iter + block; it += block) {
            for (int j = 0; j < block; ++j) {
                e = exec ? hipGraphLaunch(exec, s) : one_iter(s);
                if (e != hipSuccess) break;
            }
            if (e == hipSuccess) e = hipMemcpyAsync(cnt, b.counter, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess || cnt[0] == 0) break;
            block = std::min(block + 2, 8);
        }
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return ctx->fail(MBEFCI_EDEVICE, std::string("Davidson iterations: ") + hipGetErrorString(e));
    }
    return davidson_finish(ctx, b, e_out, st_out, ro);
}

// Energies, statuses and counters of a solved batch (and its density
// matrices for an RDM run).
mbefci_status davidson_finish(mbefci_ctx *ctx, const Batch &b, double *e_out, int32_t *st_out, const RdmOut *ro) {
    hipStream_t s = ctx->stream;
    hipError_t e;
    const bool prof = ctx->opt.profile != 0;
    if ((e = launch_finalize(b, s)) != hipSuccess) return ctx->fail(MBEFCI_EDEVICE, hipGetErrorString(e));
    if (ro) {
        const int NP = rdm_np(b.nA);
        if ((e = launch_form_x(b, s)) != hipSuccess) return ctx->fail(MBEFCI_EDEVICE, hipGetErrorString(e));
        VecRef xr{b.T, b.dim, nullptr, 0};
        if ((e = launch_rdm(b, xr, b.rdm_part, b.rdm_G, b.nblk_r, s)) != hipSuccess)
            return ctx->fail(MBEFCI_EDEVICE, hipGetErrorString(e));
        if (ro->gram) {
            ro->gram->resize((size_t)b.B * NP * NP);
            HIPCHK(hipMemcpyAsync(ro->gram->data(), b.rdm_G, 8 * ro->gram->size(), hipMemcpyDeviceToHost, s));
        }
        if (ro->w) {
            HIPCHK(hipMemcpyAsync(b.rdm_w, ro->w, 8 * (size_t)b.B, hipMemcpyHostToDevice, s));
            if ((e = launch_rdm_embed(b, b.rdm_w, ctx->d_gh, ctx->d_ge, s)) != hipSuccess)
                return ctx->fail(MBEFCI_EDEVICE, hipGetErrorString(e));
        }
    }
    std::vector<int32_t> dst(b.B), dit(b.B);
    HIPCHK(hipMemcpyAsync(e_out, b.out_e, 8 * (size_t)b.B, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(dst.data(), b.out_status, 4 * (size_t)b.B, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(dit.data(), b.iter, 4 * (size_t)b.B, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    flush_sigma_time(ctx);
    mbefci_class_stats &cs = class_stats(ctx, b);
    cs.tuples += b.B;
    for (int t = 0; t < b.B; ++t) cs.iterations += dit[t];
    {
        int32_t gs = 0;
        HIPCHK(hipMemcpy(&gs, b.counter + 2, sizeof(int32_t), hipMemcpyDeviceToHost));
        ctx->stats.gs_second_pass += gs;
    }
    if (!prof) {
        // sigma applications: the first, then one per iteration that a tuple
        // leaves still running (counted by run_sigma in the profiled loop)
        int64_t apps = 0;
        for (int t = 0; t < b.B; ++t) apps += std::max(0, dit[t] - 1);
        ctx->stats.sigma_calls += apps;
        ctx->stats.sigma_flops += (double)apps * sigma_flops(b);
        ctx->stats.sigma_bytes += (double)apps * sigma_bytes(b);
        cs.sigma_calls += apps;
        cs.sigma_flops += (double)apps * sigma_flops(b);
    }
    for (int t = 0; t < b.B; ++t) {
        const int32_t d = dst[t];
        st_out[t] = d == ST_DONE ? MBEFCI_TUPLE_OK
                    : d == ST_MAXITER ? MBEFCI_TUPLE_MAXITER
                    : d == ST_NONFINITE ? MBEFCI_TUPLE_NONFINITE
                    : d == ST_STALLED ? MBEFCI_TUPLE_STALLED : MBEFCI_TUPLE_MAXITER;
        ctx->stats.iterations_total += dit[t];
        ctx->stats.iterations_max = std::max<int64_t>(ctx->stats.iterations_max, dit[t]);
    }
    return MBEFCI_OK;
}

mbefci_status check_device(mbefci_ctx *ctx) {
    if (!ctx) return MBEFCI_EINVAL;
    if (ctx->host_only) return ctx->fail(MBEFCI_ESTATE, "host-only context");
    if (!ctx->ham_set) return ctx->fail(MBEFCI_ESTATE, "no Hamiltonian set");
    if (!ctx->spaces_set) return ctx->fail(MBEFCI_ESTATE, "no spaces set");
    HIPCHK(hipSetDevice(ctx->device));
    return MBEFCI_OK;
}

// Density matrices of solved tuples: embedded on the device with a weight
// per tuple (device() true; the caller has set ctx->d_gh, d_ge), or their Gram
// matrices handed over on the host (input index, its shape).
struct RdmSink {
    virtual bool device() const { return false; }
    virtual double weight(int64_t) const { return 1.0; }
    virtual void take(int64_t, const TupleShape &, const double *, int) {}
    virtual ~RdmSink() = default;
};

// Solve a list of tuples (device).  Groups by shape class, batches within
// the workspace, writes energies/status in input order.
// ------------------------------------------------------------ autotuner --
// Per shape class, once per process and device: the alpha-beta sigma form
// (all pair rows, linked rows with the A rows gathered or resident, the
// vector-ALU diagonal, W in HBM) and the string-Hamiltonian GEMM tile (64 or
// 96) are chosen by timing one sigma of every candidate that fits on up to 16
// tuples of the class (HIP events, the second of two launches), the fastest
// whole sigma winning.  The choice is kept for the process, so that repeated
// runs stay bitwise identical; processes whose measurements differ can differ
// in the last bits (the forms sum in different orders).
struct TuneChoice {
    int linked_rows;   // the linked_rows setting that selects the form
    int gemm_tile;
};
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, TuneChoice> g_tune;   // (device, n_A, n_a, n_b)

mbefci_status autotune_class(mbefci_ctx *ctx, const ClassKey &key, int nC, const std::vector<const TupleShape *> &sample,
                             void *ws, size_t wsb, TuneChoice &out) {
    const auto gk = std::make_tuple(ctx->device, key.nA, key.na, key.nb);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(gk);
        if (it != g_tune.end()) {
            out = it->second;
            return MBEFCI_OK;
        }
    }
    const mbefci_options saved = ctx->opt;
    const int saved_tile = ctx->gemm_tile;
    hipStream_t s = ctx->stream;
    float best = 1e30f;
    TuneChoice bestc{saved.linked_rows, 0};
    std::vector<int> seen;
    mbefci_status rc = MBEFCI_OK;
    for (int lm : {1, 0, 2, 3, 4, 5}) {
        for (int tile : {64, 96}) {
            ctx->opt = saved;
            ctx->opt.linked_rows = lm;
            ctx->gemm_tile = tile;
            ClassPlan cp;
            plan_class(ctx, key, nC, cp, true, false);
            const int B = (int)std::min<size_t>(sample.size(), 16);
            if (cp.fixed_bytes + cp.per_tuple * (size_t)B > wsb) continue;
            Carver cv{(char *)ws, wsb};
            Batch b;
            if (!carve_batch(ctx, cp, B, cv, b, true)) continue;
            const int kid = alpha_beta_kernel(b) * 1000 + tile;
            if (std::find(seen.begin(), seen.end(), kid) != seen.end()) continue;
            seen.push_back(kid);
            if ((rc = upload_tables(ctx, cp, b)) != MBEFCI_OK) break;
            std::vector<const TupleShape *> sh(sample.begin(), sample.begin() + B);
            if ((rc = upload_shapes(ctx, b, sh)) != MBEFCI_OK) break;
            hipError_t e = launch_gather(b, s);
            if (e == hipSuccess) e = launch_build_hb(b, s);
            if (e == hipSuccess) e = launch_hdiag(b, b.Hd, b.dim, 0, s);
            VecRef cin{b.Hd, b.dim, nullptr, 0}, sout{b.S, (int64_t)b.max_space * b.dim, nullptr, 0};
            float ms = 0.f;
            for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
                e = hipEventRecord(ctx->ev[0], s);
                if (e == hipSuccess) e = launch_sigma(b, cin, sout, 0.0, false, false, s, nullptr, nullptr, nullptr, nullptr);
                if (e == hipSuccess) e = hipEventRecord(ctx->ev[3], s);
                if (e == hipSuccess) e = hipEventSynchronize(ctx->ev[3]);
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[3]);
            }
            if (e != hipSuccess) {
                rc = ctx->fail(MBEFCI_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
                break;
            }
            if (ms < best) {
                best = ms;
                bestc = TuneChoice{lm, tile};
            }
        }
        if (rc != MBEFCI_OK) break;
    }
    ctx->opt = saved;
    ctx->gemm_tile = saved_tile;
    if (rc != MBEFCI_OK) return rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto ins = g_tune.emplace(gk, bestc);
        out = ins.first->second;   // another thread may have tuned the class first
    }
    ctx->stats.tuned_classes += 1;
    return MBEFCI_OK;
}

// The same sink seen through a list of input indices (second pass).
struct SubsetSink : RdmSink {
    RdmSink *inner;
    const std::vector<int64_t> *map;
    bool device() const override { return inner->device(); }
    double weight(int64_t i) const override { return inner->weight((*map)[i]); }
    void take(int64_t i, const TupleShape &ts, const double *G, int NP) override { inner->take((*map)[i], ts, G, NP); }
};

// Davidson settings of the second pass: tuples that fail the first (iteration
// limit, stalled) are solved again with the largest subspace and without the
// P space.  In the strongly spin-coupled classes a small subspace with
// restarts to the Ritz vector can stagnate above the lowest state, which 32
// vectors resolve; a class whose first batch sends at least a quarter of its
// tuples to the second pass runs the rest of its batches with these settings.
void second_pass_options(mbefci_options &o) {
    o.max_space = kMaxSpace;
    o.pspace = 0;
    o.max_iter = std::max(10 * o.max_iter, 3000);
}

mbefci_status solve_device(mbefci_ctx *ctx, int order, int64_t ntup, const int16_t *tuples, void *ws, size_t wsb,
                           double *energies, int32_t *status, RdmSink *sink = nullptr, bool second = false) {
    mbefci_status rc = check_device(ctx);
    if (rc != MBEFCI_OK) return rc;
    if (ntup < 0 || (ntup > 0 && order > 0 && !tuples)) return ctx->fail(MBEFCI_EINVAL, "bad tuple list");
    if (!ws) return ctx->fail(MBEFCI_EINVAL, "null workspace");
    std::vector<TupleShape> shapes(ntup);
    std::map<std::pair<ClassKey, int>, std::vector<int64_t>> groups;
    for (int64_t i = 0; i < ntup; ++i) {
        rc = tuple_shape(ctx, order, tuples + (size_t)i * order, shapes[i]);
        if (rc != MBEFCI_OK) return rc;
        groups[{shapes[i].key, shapes[i].nC}].push_back(i);
    }
    if (ctx->opt.sym_shift != 0.0 && (rc = check_symmetry(ctx, order, ntup, shapes)) != MBEFCI_OK) return rc;
    const mbefci_options first_opt = ctx->opt;
    std::vector<int64_t> retry;
    for (auto &g : groups) {
        if (sink && g.first.first.nA > kRdmMaxActive)
            return ctx->fail(MBEFCI_ETOOLARGE, "RDMs need at most 12 active orbitals");
        bool hard = false;   // this class runs with the second-pass settings
        const std::vector<int64_t> &idx = g.second;
        // the sigma form and GEMM tile of the class: automatic settings only
        // (linked_rows 1, sigma_variant 0), classes of at least 10^4 determinants
        TuneChoice tc{first_opt.linked_rows, 0};
        bool tuned = false;
        if (first_opt.autotune && first_opt.linked_rows == 1 && first_opt.sigma_variant == SIGMA_AUTO) {
            const Tables &ta = ctx->table(g.first.first.nA, g.first.first.na),
                         &tb = ctx->table(g.first.first.nA, g.first.first.nb);
            if (ta.nstr * tb.nstr >= 10000) {
                std::vector<const TupleShape *> sample;
                for (size_t j = 0; j < idx.size() && j < 16; ++j) sample.push_back(&shapes[idx[j]]);
                if ((rc = autotune_class(ctx, g.first.first, g.first.second, sample, ws, wsb, tc)) != MBEFCI_OK) {
                    ctx->opt = first_opt;
                    return rc;
                }
                tuned = true;
            }
        }
        for (size_t start = 0; start < idx.size();) {
            ctx->opt = first_opt;
            if (hard) second_pass_options(ctx->opt);
            if (tuned) {
                ctx->opt.linked_rows = tc.linked_rows;
                ctx->gemm_tile = tc.gemm_tile;
            }
            ClassPlan cp;
            plan_class(ctx, g.first.first, g.first.second, cp, true, sink != nullptr);
            if (cp.fixed_bytes + cp.per_tuple > wsb) {
                ctx->opt = first_opt;
                return ctx->fail(MBEFCI_ENOMEM, "workspace of " + std::to_string(wsb) + " bytes cannot hold one tuple (" +
                                                    std::to_string(cp.fixed_bytes + cp.per_tuple) + " needed)");
            }
            int64_t Bmax = ctx->opt.batched ? (int64_t)((wsb - cp.fixed_bytes) / cp.per_tuple) : 1;
            Bmax = std::max<int64_t>(1, std::min<int64_t>(Bmax, 65535));
            const int B = (int)std::min<size_t>(Bmax, idx.size() - start);
            Carver cv{(char *)ws, wsb};
            Batch b;
            if (!carve_batch(ctx, cp, B, cv, b, true)) {
                ctx->opt = first_opt;
                return ctx->fail(MBEFCI_ENOMEM, "workspace carve failed");
            }
            if ((rc = upload_tables(ctx, cp, b)) != MBEFCI_OK) break;
            std::vector<const TupleShape *> sh(B);
            for (int t = 0; t < B; ++t) sh[t] = &shapes[idx[start + t]];
            if ((rc = upload_shapes(ctx, b, sh)) != MBEFCI_OK) break;
            std::vector<double> e(B), gram, wts;
            std::vector<int32_t> st(B);
            const double tb0 = now_ms();
            RdmOut ro;
            if (sink && sink->device()) {
                wts.resize(B);
                for (int t = 0; t < B; ++t) wts[t] = sink->weight(idx[start + t]);
                ro.w = wts.data();
            } else if (sink) {
                ro.gram = &gram;
            }
            if ((rc = davidson_batch(ctx, b, e.data(), st.data(), sink ? &ro : nullptr)) != MBEFCI_OK) break;
            class_stats(ctx, b).wall_ms += now_ms() - tb0;
            int nfail = 0;
            for (int t = 0; t < B; ++t) {
                const int64_t i = idx[start + t];
                energies[i] = e[t];
                status[i] = st[t];
                if (st[t] != MBEFCI_TUPLE_OK) {   // not embedded on the device (k_rdm_embed skips it)
                    ++nfail;
                    retry.push_back(i);
                    continue;
                }
                if (sink && !sink->device()) sink->take(i, shapes[i], gram.data() + (size_t)t * cp.NP * cp.NP, cp.NP);
            }
            if (start == 0 && !second && 4 * nfail >= B && B >= 4) hard = true;
            start += B;
        }
        ctx->opt = first_opt;
        ctx->gemm_tile = 0;
        if (rc != MBEFCI_OK) return rc;
    }
    ctx->stats.ntuples += ntup;
    if (!retry.empty() && !second) {
        std::sort(retry.begin(), retry.end());
        ctx->stats.second_pass += (int64_t)retry.size();
        std::vector<int16_t> tl(retry.size() * (size_t)order);
        for (size_t j = 0; j < retry.size(); ++j)
            std::copy(tuples + retry[j] * order, tuples + (retry[j] + 1) * order, tl.begin() + j * order);
        std::vector<double> e2(retry.size());
        std::vector<int32_t> st2(retry.size());
        SubsetSink sub;
        sub.inner = sink;
        sub.map = &retry;
        second_pass_options(ctx->opt);
        rc = solve_device(ctx, order, (int64_t)retry.size(), tl.data(), ws, wsb, e2.data(), st2.data(),
                          sink ? &sub : nullptr, true);
        ctx->opt = first_opt;
        ctx->stats.ntuples -= (int64_t)retry.size();
        if (rc != MBEFCI_OK && rc != MBEFCI_ENOCONV) return rc;
        for (size_t j = 0; j < retry.size(); ++j) {
            energies[retry[j]] = e2[j];
            status[retry[j]] = st2[j];
        }
        for (int32_t x : st2)
            if (x != MBEFCI_TUPLE_OK) return ctx->fail(MBEFCI_ENOCONV, "at least one tuple did not converge");
        return MBEFCI_OK;
    }
    for (int64_t i = 0; i < ntup; ++i)
        if (status[i] != MBEFCI_TUPLE_OK) return ctx->fail(MBEFCI_ENOCONV, "at least one tuple did not converge");
    return MBEFCI_OK;
}

// ----------------------------------------------------------------- planner --

// all k-combinations of X in lexicographic order
void combinations(const std::vector<int> &X, int k, std::vector<int16_t> &out) {
    out.clear();
    const int n = (int)X.size();
    if (k > n) return;
    std::vector<int> ix(k);
    for (int i = 0; i < k; ++i) ix[i] = i;
    while (true) {
        for (int i = 0; i < k; ++i) out.push_back((int16_t)X[ix[i]]);
        int i = k - 1;
        while (i >= 0 && ix[i] == n - k + i) --i;
        if (i < 0) break;
        ++ix[i];
        for (int j = i + 1; j < k; ++j) ix[j] = ix[j - 1] + 1;
    }
}

uint64_t tuple_mask(const int16_t *t, int k) {
    uint64_t m = 0;
    for (int i = 0; i < k; ++i) m |= (uint64_t)1 << t[i];
    return m;
}

double screen_threshold(double a, int k) { return 1.0e-10 * std::pow(a, (double)(k - 1)); }

// Children of the order-(k-1) tuples with |d_eps| >= tau: every T u {x},
// x in X \ T, deduplicated, lexicographic.
void children(const Result::Order &prev, const std::vector<int> &X, double tau, std::vector<int16_t> &out) {
    const int kp = prev.k, k = kp + 1;
    const int64_t np = (int64_t)prev.dinc.size();
    std::vector<uint64_t> masks;
    for (int64_t i = 0; i < np; ++i) {
        if (!(std::fabs(prev.dinc[i]) >= tau)) continue;
        const int16_t *T = prev.tuples.data() + (size_t)i * kp;
        const uint64_t mT = tuple_mask(T, kp);
        for (int x : X)
            if (!(mT >> x & 1)) masks.push_back(mT | ((uint64_t)1 << x));
    }
    std::sort(masks.begin(), masks.end());
    masks.erase(std::unique(masks.begin(), masks.end()), masks.end());
    std::vector<int16_t> rows(masks.size() * k);
    for (size_t i = 0; i < masks.size(); ++i) {
        int j = 0;
        for (uint64_t m = masks[i]; m; m &= m - 1) rows[i * k + j++] = (int16_t)__builtin_ctzll(m);
    }
    std::vector<size_t> ord(masks.size());
    for (size_t i = 0; i < ord.size(); ++i) ord[i] = i;
    std::sort(ord.begin(), ord.end(), [&](size_t a, size_t b) {
        return std::lexicographical_compare(rows.begin() + a * k, rows.begin() + (a + 1) * k, rows.begin() + b * k,
                                            rows.begin() + (b + 1) * k);
    });
    out.resize(rows.size());
    for (size_t i = 0; i < ord.size(); ++i) std::copy(rows.begin() + ord[i] * k, rows.begin() + (ord[i] + 1) * k,
                                                      out.begin() + i * k);
}

// Pi-pruning (Sec. 3, Table 2): a tuple holds both components of every
// degenerate pair or neither.
bool pi_complete(uint64_t m, const std::vector<std::pair<int, int>> &pi) {
    for (const auto &pr : pi)
        if (((m >> pr.first) & 1u) != ((m >> pr.second) & 1u)) return false;
    return true;
}

// Lexicographic rows of k orbitals from sorted, unique masks.
void rows_from_masks(std::vector<uint64_t> &masks, int k, std::vector<int16_t> &out) {
    std::sort(masks.begin(), masks.end());
    masks.erase(std::unique(masks.begin(), masks.end()), masks.end());
    std::vector<int16_t> rows(masks.size() * k);
    for (size_t i = 0; i < masks.size(); ++i) {
        int j = 0;
        for (uint64_t m = masks[i]; m; m &= m - 1) rows[i * k + j++] = (int16_t)__builtin_ctzll(m);
    }
    std::vector<size_t> ord(masks.size());
    for (size_t i = 0; i < ord.size(); ++i) ord[i] = i;
    std::sort(ord.begin(), ord.end(), [&](size_t a, size_t b) {
        return std::lexicographical_compare(rows.begin() + a * k, rows.begin() + (a + 1) * k, rows.begin() + b * k,
                                            rows.begin() + (b + 1) * k);
    });
    out.resize(rows.size());
    for (size_t i = 0; i < ord.size(); ++i)
        std::copy(rows.begin() + ord[i] * k, rows.begin() + (ord[i] + 1) * k, out.begin() + i * k);
}

// Order-k candidates under pi-pruning and screening: an unpaired orbital added
// to an order-(k-1) tuple with |d_eps| >= tau_{k-1}, or a whole pair added to
// an order-(k-2) tuple with |d_eps| >= tau_{k-2} (the empty tuple always
// counts).  Without screening this reaches every pi-complete tuple.
void pi_children(const std::vector<Result::Order> &orders, int k, const std::vector<int> &X,
                 const std::vector<std::pair<int, int>> &pi, double a, std::vector<int16_t> &out) {
    std::vector<char> paired(64, 0);
    for (const auto &pr : pi) paired[pr.first] = paired[pr.second] = 1;
    std::vector<uint64_t> masks;
    if (k - 1 >= 1) {
        const Result::Order &o = orders[k - 1];
        const double tau = screen_threshold(a, k - 1);
        for (size_t i = 0; i < o.dinc.size(); ++i) {
            if (!(std::fabs(o.dinc[i]) >= tau)) continue;
            const uint64_t mT = tuple_mask(o.tuples.data() + i * o.k, o.k);
            for (int x : X)
                if (!paired[x] && !(mT >> x & 1)) masks.push_back(mT | ((uint64_t)1 << x));
        }
    }
    if (k - 2 >= 0) {
        const Result::Order &o = orders[k - 2];
        const double tau = screen_threshold(a, k - 2);
        const size_t nt = k - 2 == 0 ? 1 : o.dinc.size();
        for (size_t i = 0; i < nt; ++i) {
            if (k - 2 > 0 && !(std::fabs(o.dinc[i]) >= tau)) continue;
            const uint64_t mT = k - 2 == 0 ? 0 : tuple_mask(o.tuples.data() + i * o.k, o.k);
            for (const auto &pr : pi)
                if (!(mT >> pr.first & 1) && !(mT >> pr.second & 1))
                    masks.push_back(mT | ((uint64_t)1 << pr.first) | ((uint64_t)1 << pr.second));
        }
    }
    rows_from_masks(masks, k, out);
}

// Eq. 3 for one tuple: subtuples in (size, lexicographic) order from 0.0.
double increment(const int16_t *S, int k, double eps, const std::unordered_map<uint64_t, double> &dinc) {
    double acc = 0.0;
    std::vector<int> ix(k);
    for (int m = 0; m < k; ++m) {
        for (int i = 0; i < m; ++i) ix[i] = i;
        while (true) {
            uint64_t mask = 0;
            for (int i = 0; i < m; ++i) mask |= (uint64_t)1 << S[ix[i]];
            auto it = dinc.find(mask);
            if (it != dinc.end()) acc += it->second;
            int i = m - 1;
            while (i >= 0 && ix[i] == k - m + i) --i;
            if (i < 0) break;
            ++ix[i];
            for (int j = i + 1; j < m; ++j) ix[j] = ix[j - 1] + 1;
        }
    }
    return eps - acc;
}

mbefci_status check_canonical(mbefci_ctx *ctx);

// Base-model energies eps_base(S) of nt tuples of order k (k = |X| with the
// whole expansion space gives the base energy of the whole space): per tuple
// the active and core orbital lists, one workgroup each (launch_base).
mbefci_status base_energies(mbefci_ctx *ctx, int k, int64_t nt, const int16_t *tuples, void *ws, size_t wsb,
                            double *out) {
    const int n = ctx->norb;
    std::vector<int32_t> act((size_t)nt * n), core((size_t)nt * n), na((size_t)nt), nc((size_t)nt);
    for (int64_t t = 0; t < nt; ++t) {
        std::vector<char> inA(n, 0);
        for (int p : ctx->ref) inA[p] = 1;
        for (int i = 0; i < k; ++i) inA[tuples[t * k + i]] = 1;
        int a = 0, c = 0;
        for (int p = 0; p < n; ++p) {
            if (inA[p]) act[(size_t)t * n + a++] = p;
            else if (p < ctx->nbeta) core[(size_t)t * n + c++] = p;
        }
        na[t] = a;
        nc[t] = c;
    }
    const int model = std::max(1, (int)ctx->opt.base_model);
    Carver cv{(char *)ws, wsb};
    int32_t *d_act = cv.take<int32_t>(act.size()), *d_core = cv.take<int32_t>(core.size());
    int32_t *d_na = cv.take<int32_t>(na.size()), *d_nc = cv.take<int32_t>(nc.size());
    double *d_out = cv.take<double>((size_t)nt);
    if (!cv.ok) return ctx->fail(MBEFCI_ENOMEM, "workspace too small for the base-model energies");
    if (model >= 2) {
        // coupled cluster: one workspace slice per tuple of a launch.  When a
        // call holds few tuples (fewer than a quarter of the workgroups one
        // cooperative launch gets), those of at least kCcCoopActive active
        // orbitals run one at a time on many workgroups (a cooperative launch,
        // typically the base energy of the whole space); otherwise every tuple
        // runs batched, one workgroup each, with slices sized for the largest
        const int coop_wgs = ccsd_coop_wgs();
        const bool few = nt * 4 < coop_wgs;
        auto coop = [&](int64_t t) { return few && na[t] >= kCcCoopActive; };
        int omax = 0, vmax = 0;
        int64_t big_slice = 0;
        for (int64_t t = 0; t < nt; ++t) {
            int o = 0;
            for (int i = 0; i < na[t]; ++i) o += (act[(size_t)t * n + i] < ctx->nalpha) + (act[(size_t)t * n + i] < ctx->nbeta);
            if (na[t] > kCcMaxActive)
                return ctx->fail(MBEFCI_EINVAL, "coupled-cluster base: more than 32 active orbitals in a tuple");
            if (coop(t)) {
                big_slice = std::max(big_slice, cc_slice_doubles(o, 2 * na[t] - o));
            } else {
                omax = std::max(omax, o);
                vmax = std::max(vmax, 2 * na[t] - o);
            }
        }
        if (model == 3) {
            const mbefci_status rc = check_canonical(ctx);
            if (rc != MBEFCI_OK) return rc;
        }
        int32_t *d_st = cv.take<int32_t>((size_t)nt);
        double *d_part = cv.take<double>(2 * (size_t)kCcMaxWgs);
        // (at least one aligned unit: a call may hold only large tuples)
        const int64_t slice = std::max<int64_t>(32, (cc_slice_doubles(omax, vmax) + 31) / 32 * 32);
        const size_t room = cv.ok && cv.size - cv.off > 256 ? (cv.size - cv.off - 256) / 8 : 0;
        const int64_t per = (int64_t)std::min<size_t>(room / (size_t)slice, 4096);
        if (!cv.ok || per < 1 || (size_t)big_slice > room)
            return ctx->fail(MBEFCI_ENOMEM, "workspace too small for the coupled-cluster base");
        double *d_work = cv.take<double>(std::max((size_t)(per * slice), (size_t)big_slice));
        const int wgs = coop_wgs;
        HIPCHK(hipMemcpyAsync(d_act, act.data(), 4 * act.size(), hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(hipMemcpyAsync(d_core, core.data(), 4 * core.size(), hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(hipMemcpyAsync(d_na, na.data(), 4 * na.size(), hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(hipMemcpyAsync(d_nc, nc.data(), 4 * nc.size(), hipMemcpyHostToDevice, ctx->stream));
        for (int64_t t0 = 0; t0 < nt;) {
            hipError_t e;
            if (coop(t0)) {
                e = launch_ccsd_coop(ctx->d_h, ctx->d_eri, n, d_act + t0 * n, d_na + t0, d_core + t0 * n, d_nc + t0, n,
                                     ctx->nalpha, ctx->nbeta, ctx->e_const, d_work, big_slice, model == 3, kCcMaxIter,
                                     kCcTol, d_out + t0, d_st + t0, wgs, d_part, ctx->stream);
                ++t0;
            } else {
                int cnt = 0;   // a run of small tuples
                while (t0 + cnt < nt && cnt < per && !coop(t0 + cnt)) ++cnt;
                e = launch_ccsd(ctx->d_h, ctx->d_eri, n, d_act + t0 * n, d_na + t0, d_core + t0 * n, d_nc + t0, n,
                                ctx->nalpha, ctx->nbeta, ctx->e_const, cnt, d_work, slice, model == 3, kCcMaxIter,
                                kCcTol, d_out + t0, d_st + t0, ctx->stream);
                t0 += cnt;
            }
            if (e != hipSuccess) return ctx->fail(MBEFCI_EDEVICE, hipGetErrorString(e));
        }
        std::vector<int32_t> st((size_t)nt);
        HIPCHK(hipMemcpyAsync(out, d_out, 8 * (size_t)nt, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipMemcpyAsync(st.data(), d_st, 4 * (size_t)nt, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        for (int64_t t = 0; t < nt; ++t) {
            if (st[t] == 1)
                return ctx->fail(MBEFCI_EINVAL, "coupled-cluster base: an orbital energy difference of the reference "
                                                "determinant is not negative (intruder)");
            if (st[t] != 0 || !std::isfinite(out[t]))
                return ctx->fail(MBEFCI_ENOCONV, "coupled-cluster base: the amplitude equations did not converge");
        }
        return MBEFCI_OK;
    }
    HIPCHK(hipMemcpyAsync(d_act, act.data(), 4 * act.size(), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(d_core, core.data(), 4 * core.size(), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(d_na, na.data(), 4 * na.size(), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(d_nc, nc.data(), 4 * nc.size(), hipMemcpyHostToDevice, ctx->stream));
    hipError_t e = launch_base(ctx->d_h, ctx->d_eri, n, d_act, d_na, n, d_core, d_nc, n, ctx->nalpha, ctx->nbeta,
                               ctx->e_const, (int)nt, d_out, ctx->stream);
    if (e != hipSuccess) return ctx->fail(MBEFCI_EDEVICE, hipGetErrorString(e));
    HIPCHK(hipMemcpyAsync(out, d_out, 8 * (size_t)nt, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (int64_t t = 0; t < nt; ++t)
        if (!std::isfinite(out[t]))
            return ctx->fail(MBEFCI_EINVAL, "base model: an excitation of the reference determinant does not raise "
                                            "the zeroth-order energy (intruder)");
    return MBEFCI_OK;
}

// The (T) correction assumes canonical orbitals: the Fock operator of the
// reference determinant (every orbital below n_alpha / n_beta occupied: the
// same determinant for every tuple) diagonal on the orbitals a tuple can hold.
mbefci_status check_canonical(mbefci_ctx *ctx) {
    const int n = ctx->norb;
    std::vector<int> orbs(ctx->ref.begin(), ctx->ref.end());
    orbs.insert(orbs.end(), ctx->X.begin(), ctx->X.end());
    auto E = [&](int p, int q, int r, int s) { return ctx->eri[(((size_t)p * n + q) * n + r) * n + s]; };
    for (int spin = 0; spin < 2; ++spin)
        for (int p : orbs)
            for (int q : orbs) {
                if (p == q) continue;
                double f = ctx->h[(size_t)p * n + q];
                for (int k = 0; k < ctx->nalpha; ++k) f += E(p, q, k, k) - (spin == 0 ? E(p, k, k, q) : 0.0);
                for (int k = 0; k < ctx->nbeta; ++k) f += E(p, q, k, k) - (spin == 1 ? E(p, k, k, q) : 0.0);
                if (std::fabs(f) > kCanonTol)
                    return ctx->fail(MBEFCI_EINVAL, "CCSD(T) base needs canonical orbitals: the Fock operator of the "
                                                    "reference determinant is not diagonal");
            }
    return MBEFCI_OK;
}

// tuple energies minus their base-model energies (after a solve)
mbefci_status subtract_base(mbefci_ctx *ctx, int k, int64_t nt, const int16_t *tuples, void *ws, size_t wsb, double *e) {
    std::vector<double> b((size_t)nt);
    mbefci_status rc = base_energies(ctx, k, nt, tuples, ws, wsb, b.data());
    if (rc != MBEFCI_OK) return rc;
    for (int64_t i = 0; i < nt; ++i) e[i] -= b[i];
    return MBEFCI_OK;
}

template <class EnergyFn>
mbefci_status run_planner(mbefci_ctx *ctx, EnergyFn energy, Result &R) {
    const int nX = (int)ctx->X.size();
    int kmax = ctx->opt.max_order > 0 ? std::min(ctx->opt.max_order, nX) : nX;
    std::unordered_map<uint64_t, double> dinc;
    bool failed = false;
    R.orders.clear();
    R.total = 0.0;
    for (int k = 0; k <= kmax; ++k) {
        Result::Order o;
        o.k = k;
        const bool pi = !ctx->pi.empty();
        if (k == 0) {
            o.tuples.clear();
        } else if (k == 1 || ctx->opt.a <= 0.0) {
            combinations(ctx->X, k, o.tuples);
            if (pi) {   // keep the pi-complete tuples, in the same order
                size_t w = 0;
                for (size_t i = 0; i < o.tuples.size() / k; ++i)
                    if (pi_complete(tuple_mask(o.tuples.data() + i * k, k), ctx->pi)) {
                        std::copy(o.tuples.begin() + i * k, o.tuples.begin() + (i + 1) * k, o.tuples.begin() + w * k);
                        ++w;
                    }
                o.tuples.resize(w * k);
            }
        } else if (pi) {
            pi_children(R.orders, k, ctx->X, ctx->pi, ctx->opt.a, o.tuples);
        } else {
            children(R.orders.back(), ctx->X, screen_threshold(ctx->opt.a, k - 1), o.tuples);
        }
        const int64_t nt = k == 0 ? 1 : (int64_t)(o.tuples.size() / k);
        if (nt == 0) {
            // under pi-pruning a pair added to the order before may still follow
            if (pi && !R.orders.back().eps.empty()) {
                R.orders.push_back(std::move(o));
                continue;
            }
            break;
        }
        if (k == kmax && k >= 1 && ctx->opt.stream_last) {
            // the last order is only listed; mbefci_order_solve fills it slice by slice
            o.eps.assign(nt, std::nan(""));
            o.dinc.assign(nt, std::nan(""));
            o.status.assign(nt, MBEFCI_TUPLE_PENDING);
            R.orders.push_back(std::move(o));
            R.open = true;
            R.solved.assign(nt, 0);
            R.dinc_map = std::move(dinc);
            break;
        }
        const double t0 = now_ms();
        o.eps.assign(nt, 0.0);
        o.status.assign(nt, 0);
        mbefci_status rc = energy(k, nt, o.tuples.data(), o.eps.data(), o.status.data());
        if (rc == MBEFCI_ENOCONV) failed = true;
        else if (rc != MBEFCI_OK) return rc;
        o.dinc.resize(nt);
        for (int64_t i = 0; i < nt; ++i) o.dinc[i] = increment(o.tuples.data() + (size_t)i * k, k, o.eps[i], dinc);
        for (int64_t i = 0; i < nt; ++i) dinc[tuple_mask(o.tuples.data() + (size_t)i * k, k)] = o.dinc[i];
        double s = 0.0;
        for (double d : o.dinc) s += d;
        o.sum = s;
        o.wall_ms = now_ms() - t0;
        R.orders.push_back(std::move(o));
    }
    double tot = 0.0;
    for (auto &o : R.orders) tot += o.sum;
    R.total = tot;
    return failed ? ctx->fail(MBEFCI_ENOCONV, "at least one tuple did not converge") : MBEFCI_OK;
}

// The status code of a listed tuple of a streamed order not solved yet.
static_assert(MBEFCI_TUPLE_PENDING == 4, "status codes");

// Full-space density matrices of one CASCI vector from its Gram matrix G
// (columns p*nA+q: D_pq = <I|E_pq|x>, column nA^2: x), accumulated with
// weight w into gh (n*n, receives w gamma) and ge (n^4, receives w Gamma / 2):
//   gamma_pq = G[pq, x],  Gamma_pqrs = G[qp, rs] - delta_qr gamma_ps  (active);
//   core c (doubly occupied): gamma_cc = 2, Gamma_ccdd = 4, Gamma_cddc = -2
//   (c != d), Gamma_cccc = 2, and with active p, q: Gamma_pqcc = Gamma_ccpq =
//   2 gamma_pq, Gamma_pccq = Gamma_cqpc = -gamma_pq.
void accumulate_rdm(int n, const TupleShape &ts, const double *G, int NP, double w, double *gh, double *ge) {
    const int nA = (int)ts.act.size(), nn = nA * nA;
    const std::vector<int32_t> &o = ts.act, &C = ts.core;
    std::vector<double> gam(nn);
    for (int p = 0; p < nA; ++p)
        for (int q = 0; q < nA; ++q) gam[p * nA + q] = G[(size_t)(p * nA + q) * NP + nn];
    auto E = [&](int p, int q, int r, int s) -> double & { return ge[(((size_t)p * n + q) * n + r) * n + s]; };
    const double hw = 0.5 * w;
    for (int p = 0; p < nA; ++p)
        for (int q = 0; q < nA; ++q) gh[(size_t)o[p] * n + o[q]] += w * gam[p * nA + q];
    for (int cc : C) gh[(size_t)cc * n + cc] += 2.0 * w;
    for (int p = 0; p < nA; ++p)
        for (int q = 0; q < nA; ++q)
            for (int r = 0; r < nA; ++r)
                for (int s = 0; s < nA; ++s) {
                    double v = G[(size_t)(q * nA + p) * NP + (r * nA + s)];
                    if (q == r) v -= gam[p * nA + s];
                    E(o[p], o[q], o[r], o[s]) += hw * v;
                }
    for (int cc : C)
        for (int d : C) {
            if (cc == d) {
                E(cc, cc, cc, cc) += hw * 2.0;
            } else {
                E(cc, cc, d, d) += hw * 4.0;
                E(cc, d, d, cc) += hw * -2.0;
            }
        }
    for (int cc : C)
        for (int p = 0; p < nA; ++p)
            for (int q = 0; q < nA; ++q) {
                const double g = gam[p * nA + q];
                E(o[p], o[q], cc, cc) += hw * 2.0 * g;
                E(cc, cc, o[p], o[q]) += hw * 2.0 * g;
                E(o[p], cc, cc, o[q]) -= hw * g;
                E(cc, o[q], o[p], cc) -= hw * g;
            }
}

// dE_total / d eps(S) = w_S for the summed increments of Eq. 3 with the tuple
// set fixed: w_S = 1 - sum_{U computed, U proper superset of S} w_U (integers),
// evaluated from the highest order down.
std::vector<std::vector<int64_t>> adjoint_weights(const Result &R) {
    std::unordered_map<uint64_t, int64_t> acc;
    for (auto &o : R.orders) {
        const size_t nt = o.eps.size();
        for (size_t i = 0; i < nt; ++i) acc[tuple_mask(o.tuples.data() + i * o.k, o.k)] = 0;
    }
    std::vector<std::vector<int64_t>> w(R.orders.size());
    std::vector<int> ix;
    for (int oi = (int)R.orders.size() - 1; oi >= 0; --oi) {
        const auto &o = R.orders[oi];
        const int k = o.k;
        const size_t nt = o.eps.size();
        w[oi].resize(nt);
        for (size_t i = 0; i < nt; ++i) {
            const int16_t *U = o.tuples.data() + i * k;
            const int64_t wu = 1 - acc[tuple_mask(U, k)];
            w[oi][i] = wu;
            if (wu == 0) continue;
            for (uint32_t sub = 0; sub + 1 < (1u << k); ++sub) {   // proper subsets, by bit pattern
                uint64_t m = 0;
                for (int j = 0; j < k; ++j)
                    if (sub >> j & 1u) m |= (uint64_t)1 << U[j];
                auto it = acc.find(m);
                if (it != acc.end()) it->second += wu;
            }
        }
    }
    return w;
}

// Host accumulation of Gram matrices with integer weights (one tuple's
// density matrices, mbefci_tuple_rdm).
struct GradSink : RdmSink {
    int n;
    const std::vector<int64_t> *w;
    double *gh, *ge;
    void take(int64_t index, const TupleShape &ts, const double *G, int NP) override {
        const double wi = (double)(*w)[index];
        if (wi != 0.0) accumulate_rdm(n, ts, G, NP, wi, gh, ge);
    }
};

// Device embedding with the weight of each tuple of the list being solved.
struct WeightSink : RdmSink {
    const std::vector<double> *w;
    bool device() const override { return true; }
    double weight(int64_t index) const override { return (*w)[index]; }
};

// Gram matrices of one order kept on the host until the weights are known.
struct StoreSink : RdmSink {
    std::vector<std::vector<double>> G;
    std::vector<TupleShape> shape;
    std::vector<int> NP;
    void take(int64_t index, const TupleShape &ts, const double *g, int np) override {
        G[index].assign(g, g + (size_t)np * np);
        shape[index] = ts;
        NP[index] = np;
    }
};

// Davidson tolerances of a density-matrix pass: density matrices are first
// order in the residual, so |r| <= 1e-9 (and |d theta| <= 1e-12) whatever the
// energy-only settings are.
struct TightTol {
    mbefci_ctx *ctx;
    mbefci_options saved;
    explicit TightTol(mbefci_ctx *c) : ctx(c), saved(c->opt) {
        ctx->opt.r_tol = std::min(ctx->opt.r_tol, 1e-9);
        ctx->opt.e_tol = std::min(ctx->opt.e_tol, 1e-12);
        ctx->opt.max_iter = std::max(ctx->opt.max_iter, 300);
    }
    ~TightTol() { ctx->opt = saved; }
};

// The device gradient accumulators (n^2 + n^4 doubles) at the end of the
// caller's workspace, cleared; *wsb shrinks to the part left for batches.
mbefci_status grad_region(mbefci_ctx *ctx, void *ws, size_t *wsb) {
    const size_t n2 = (size_t)ctx->norb * ctx->norb, n4 = n2 * n2;
    const size_t bytes = align256(8 * n2) + align256(8 * n4);
    if (!ws || *wsb < bytes + ((size_t)1 << 20))
        return ctx->fail(MBEFCI_ENOMEM, "workspace too small for the gradient accumulators (" +
                                            std::to_string(bytes) + " bytes)");
    const size_t off = (*wsb - bytes) / 256 * 256;
    ctx->d_gh = reinterpret_cast<double *>(static_cast<char *>(ws) + off);
    ctx->d_ge = reinterpret_cast<double *>(static_cast<char *>(ws) + off + align256(8 * n2));
    HIPCHK(hipMemsetAsync(ctx->d_gh, 0, bytes, ctx->stream));
    *wsb = off;
    return MBEFCI_OK;
}

// Device accumulators added into host arrays gh [n^2], ge [n^4].
mbefci_status grad_fetch(mbefci_ctx *ctx, std::vector<double> &gh, std::vector<double> &ge) {
    const size_t n2 = (size_t)ctx->norb * ctx->norb, n4 = n2 * n2;
    std::vector<double> dh(n2), de(n4);
    HIPCHK(hipMemcpyAsync(dh.data(), ctx->d_gh, 8 * n2, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(de.data(), ctx->d_ge, 8 * n4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->d_gh = ctx->d_ge = nullptr;
    gh.resize(n2, 0.0);
    ge.resize(n4, 0.0);
    for (size_t i = 0; i < n2; ++i) gh[i] += dh[i];
    for (size_t i = 0; i < n4; ++i) ge[i] += de[i];
    return MBEFCI_OK;
}

// grad_eri in the layout the integrals were given in: the full array, or per
// packed element the sum over its distinct equivalent index quadruples.
void write_grad(const mbefci_ctx *ctx, const std::vector<double> &gh, const std::vector<double> &ge, double gE,
                double *grad_h1, double *grad_eri) {
    const int n = ctx->norb;
    const size_t n2 = (size_t)n * n, n4 = n2 * n2;
    for (size_t i = 0; i < n2; ++i) grad_h1[i] = gE * gh[i];
    if (ctx->eri_layout == MBEFCI_ERI_FULL) {
        for (size_t i = 0; i < n4; ++i) grad_eri[i] = gE * ge[i];
        return;
    }
    const size_t np = n2 / 2 + (size_t)n / 2 + (n % 2 ? 1 : 0);   // n (n + 1) / 2
    std::fill(grad_eri, grad_eri + np * (np + 1) / 2, 0.0);
    auto pr = [](int p, int q) -> size_t { return p >= q ? (size_t)p * (p + 1) / 2 + q : (size_t)q * (q + 1) / 2 + p; };
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q)
            for (int r = 0; r < n; ++r)
                for (int s2 = 0; s2 < n; ++s2) {
                    const size_t P = pr(p, q), R = pr(r, s2);
                    const size_t k = P >= R ? P * (P + 1) / 2 + R : R * (R + 1) / 2 + P;
                    grad_eri[k] += gE * ge[(((size_t)p * n + q) * n + r) * n + s2];
                }
}

}  // namespace

// ====================================================================== ABI


namespace {

// ------------------------------------------------- CASSCF (host algebra) --
// Small dense helpers on n x n row-major matrices (n <= 64): the orbital
// rotation exp(K) of an antisymmetric K, products, and symmetric
// eigenvectors.  The integrals, the CASCI and the Fock matrices are on the
// device.
using Mat = std::vector<double>;

Mat mat_mul(const Mat &A, const Mat &B, int n) {
    Mat C((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) {
            const double a = A[(size_t)i * n + k];
            if (a == 0.0) continue;
            for (int j = 0; j < n; ++j) C[(size_t)i * n + j] += a * B[(size_t)k * n + j];
        }
    return C;
}

// exp(K) by scaling and squaring: K / 2^s with norm below 1/4, its Taylor
// series to 16 terms, then s squarings.
Mat mat_exp(const Mat &K, int n) {
    double nrm = 0.0;
    for (double v : K) nrm += v * v;
    nrm = std::sqrt(nrm);
    int sq = 0;
    while (nrm > 0.25) {
        nrm *= 0.5;
        ++sq;
    }
    const double sc = std::ldexp(1.0, -sq);
    Mat A(K);
    for (double &v : A) v *= sc;
    Mat E((size_t)n * n, 0.0), T((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) E[(size_t)i * n + i] = T[(size_t)i * n + i] = 1.0;
    for (int k = 1; k <= 16; ++k) {
        T = mat_mul(T, A, n);
        for (double &v : T) v /= k;
        for (size_t i = 0; i < E.size(); ++i) E[i] += T[i];
    }
    for (int k = 0; k < sq; ++k) E = mat_mul(E, E, n);
    return E;
}

// Eigenvectors of the symmetric m x m matrix A (cyclic Jacobi); columns of V
// in the order of ascending (or descending) eigenvalues.
void sym_eig(Mat A, int m, bool descending, std::vector<double> &w, Mat &V) {
    V.assign((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) V[(size_t)i * m + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                const double a = A[(size_t)i * m + j] * A[(size_t)i * m + j];
                tot += a;
                if (i != j) off += a;
            }
        if (off <= 1e-32 * tot || off == 0.0) break;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) {
                const double apq = A[(size_t)p * m + q];
                if (apq == 0.0) continue;
                const double tau = (A[(size_t)q * m + q] - A[(size_t)p * m + p]) / (2.0 * apq);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                for (int k = 0; k < m; ++k) {   // columns p, q
                    const double akp = A[(size_t)k * m + p], akq = A[(size_t)k * m + q];
                    A[(size_t)k * m + p] = c * akp - s * akq;
                    A[(size_t)k * m + q] = s * akp + c * akq;
                    const double vkp = V[(size_t)k * m + p], vkq = V[(size_t)k * m + q];
                    V[(size_t)k * m + p] = c * vkp - s * vkq;
                    V[(size_t)k * m + q] = s * vkp + c * vkq;
                }
                for (int k = 0; k < m; ++k) {   // rows p, q
                    const double apk = A[(size_t)p * m + k], aqk = A[(size_t)q * m + k];
                    A[(size_t)p * m + k] = c * apk - s * aqk;
                    A[(size_t)q * m + k] = s * apk + c * aqk;
                }
            }
    }
    std::vector<int> ord(m);
    for (int i = 0; i < m; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
        const double da = A[(size_t)a * m + a], db = A[(size_t)b * m + b];
        return descending ? da > db : da < db;
    });
    Mat Vs((size_t)m * m);
    w.resize(m);
    for (int j = 0; j < m; ++j) {
        w[j] = A[(size_t)ord[j] * m + ord[j]];
        for (int i = 0; i < m; ++i) Vs[(size_t)i * m + j] = V[(size_t)i * m + ord[j]];
    }
    V.swap(Vs);
}

}  // namespace

extern "C" {

const char *mbefci_version(void) { return "mbefci 0.1 (gfx950, FP64)"; }

void mbefci_default_options(mbefci_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->a = 0.0;
    o->max_order = 0;
    o->e_tol = 1e-11;
    o->r_tol = 1e-6;
    o->max_iter = 300;
    o->max_space = 12;
    o->pspace = kPsp;
    o->linked_rows = 1;
    o->batched = 1;
    o->gradient = 0;
    o->profile = 0;
    o->graph = 1;
    o->autotune = 1;
    o->restart_keep = 2;
    o->spin_shift = 0.0;
    o->whole_dim = kWholeDefaultDim;
    o->base_model = 0;
    o->sym_shift = 0.0;
    o->irrep = 0;
}

mbefci_status mbefci_create(mbefci_ctx **out, int32_t dev, void *stream) {
    if (!out) return MBEFCI_EINVAL;
    *out = nullptr;
    auto ctx = std::make_unique<mbefci_ctx>();
    mbefci_default_options(&ctx->opt);
    if (dev >= 0) {
        int n = 0;
        if (hipGetDeviceCount(&n) != hipSuccess || dev >= n) return MBEFCI_EDEVICE;
        if (hipSetDevice(dev) != hipSuccess) return MBEFCI_EDEVICE;
        ctx->device = dev;
        ctx->host_only = false;
        ctx->stream = (hipStream_t)stream;
        for (auto &e : ctx->ev)
            if (hipEventCreate(&e) != hipSuccess) return MBEFCI_EDEVICE;
        if (init_kernels() != hipSuccess) return MBEFCI_EDEVICE;
        if (scratch_address(&ctx->scratch) != hipSuccess || !ctx->scratch) return MBEFCI_EDEVICE;
        if (hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess) return MBEFCI_EDEVICE;
    }
    *out = ctx.release();
    return MBEFCI_OK;
}

void mbefci_destroy(mbefci_ctx *ctx) {
    if (!ctx) return;
    if (!ctx->host_only) {
        (void)hipSetDevice(ctx->device);
        if (ctx->d_irr) (void)hipFree(ctx->d_irr);
        if (ctx->d_h) (void)hipFree(ctx->d_h);
        if (ctx->d_eri) (void)hipFree(ctx->d_eri);
        for (auto e : ctx->ev)
            if (e) (void)hipEventDestroy(e);
        if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    }
    delete ctx;
}

const char *mbefci_last_error(const mbefci_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

mbefci_status mbefci_set_hamiltonian(mbefci_ctx *ctx, int32_t n, const double *h1, const double *eri,
                                     mbefci_eri_layout layout, double e_const) {
    if (!ctx) return MBEFCI_EINVAL;
    if (n < 1 || n > 64) return ctx->fail(MBEFCI_EINVAL, "norb must be in 1..64");
    if (!h1 || !eri) return ctx->fail(MBEFCI_EINVAL, "null integrals");
    if (!std::isfinite(e_const)) return ctx->fail(MBEFCI_EINVAL, "non-finite constant");
    const size_t n2 = (size_t)n * n, n4 = n2 * n2;
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q) {
            const double a = h1[p * n + q], b = h1[q * n + p];
            if (!std::isfinite(a)) return ctx->fail(MBEFCI_EINVAL, "non-finite h1");
            if (std::fabs(a - b) > 1e-12) return ctx->fail(MBEFCI_EINVAL, "h1 not symmetric");
        }
    std::vector<double> full(n4);
    if (layout == MBEFCI_ERI_FULL) {
        std::memcpy(full.data(), eri, n4 * sizeof(double));
        // 8-fold symmetry: the kernels read one element per orbit
        for (int p = 0; p < n; ++p)
            for (int q = 0; q < n; ++q)
                for (int r = 0; r < n; ++r)
                    for (int s2 = 0; s2 < n; ++s2) {
                        auto at = [&](int a, int b, int c, int d) { return eri[(((size_t)a * n + b) * n + c) * n + d]; };
                        const double v = at(p, q, r, s2);
                        if (!std::isfinite(v)) return ctx->fail(MBEFCI_EINVAL, "non-finite eri");
                        if (std::fabs(v - at(q, p, r, s2)) > 1e-12 || std::fabs(v - at(p, q, s2, r)) > 1e-12 ||
                            std::fabs(v - at(r, s2, p, q)) > 1e-12)
                            return ctx->fail(MBEFCI_EINVAL, "eri not 8-fold symmetric (pq|rs) = (qp|rs) = (pq|sr) = "
                                                            "(rs|pq) within 1e-12");
                    }
    } else if (layout == MBEFCI_ERI_PACKED8) {
        auto pr = [](int p, int q) { return p >= q ? p * (p + 1) / 2 + q : q * (q + 1) / 2 + p; };
        for (int p = 0; p < n; ++p)
            for (int q = 0; q < n; ++q)
                for (int r = 0; r < n; ++r)
                    for (int s = 0; s < n; ++s) {
                        const size_t P = pr(p, q), R = pr(r, s);
                        const size_t k = P >= R ? P * (P + 1) / 2 + R : R * (R + 1) / 2 + P;
                        full[((size_t)(p * n + q) * n + r) * n + s] = eri[k];
                    }
    } else {
        return ctx->fail(MBEFCI_EINVAL, "unknown eri layout");
    }
    for (double v : full)
        if (!std::isfinite(v)) return ctx->fail(MBEFCI_EINVAL, "non-finite eri");
    ctx->norb = n;
    ctx->eri_layout = layout;
    ctx->h.assign(h1, h1 + n2);
    ctx->eri.swap(full);
    ctx->e_const = e_const;
    ctx->ham_set = true;
    ctx->sym_checked = false;
    if (!ctx->host_only) {
        HIPCHK(hipSetDevice(ctx->device));
        if (ctx->d_h) (void)hipFree(ctx->d_h);
        if (ctx->d_eri) (void)hipFree(ctx->d_eri);
        ctx->d_h = ctx->d_eri = nullptr;
        HIPCHK(hipMalloc((void **)&ctx->d_h, n2 * sizeof(double)));
        HIPCHK(hipMalloc((void **)&ctx->d_eri, n4 * sizeof(double)));
        HIPCHK(hipMemcpy(ctx->d_h, ctx->h.data(), n2 * sizeof(double), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(ctx->d_eri, ctx->eri.data(), n4 * sizeof(double), hipMemcpyHostToDevice));
    }
    if (ctx->spaces_set && (int)ctx->inX.size() != n) ctx->spaces_set = false;
    return MBEFCI_OK;
}

mbefci_status mbefci_set_spaces(mbefci_ctx *ctx, int32_t nalpha, int32_t nbeta, int32_t nfrozen,
                                const int32_t *ref, int32_t nref) {
    if (!ctx) return MBEFCI_EINVAL;
    if (!ctx->ham_set) return ctx->fail(MBEFCI_ESTATE, "set the Hamiltonian first");
    const int n = ctx->norb;
    if (nbeta < 0 || nalpha < nbeta || nalpha > n) return ctx->fail(MBEFCI_EINVAL, "need 0 <= nbeta <= nalpha <= norb");
    if (nfrozen < 0 || nfrozen > nbeta) return ctx->fail(MBEFCI_EINVAL, "frozen orbitals must be doubly occupied");
    if (nref < 0 || (nref > 0 && !ref)) return ctx->fail(MBEFCI_EINVAL, "bad reference space");
    std::vector<char> inref(n, 0);
    for (int i = 0; i < nref; ++i) {
        const int p = ref[i];
        if (p < 0 || p >= n) return ctx->fail(MBEFCI_EINVAL, "reference orbital out of range");
        if (p < nfrozen) return ctx->fail(MBEFCI_EINVAL, "reference orbital is frozen");
        if (inref[p]) return ctx->fail(MBEFCI_EINVAL, "duplicate reference orbital");
        inref[p] = 1;
    }
    for (int p = nbeta; p < nalpha; ++p)
        if (!inref[p]) return ctx->fail(MBEFCI_EINVAL, "singly occupied orbitals must lie in the reference space");
    ctx->nalpha = nalpha;
    ctx->nbeta = nbeta;
    ctx->nfrozen = nfrozen;
    ctx->ref.clear();
    for (int p = 0; p < n; ++p)
        if (inref[p]) ctx->ref.push_back(p);
    ctx->X.clear();
    ctx->inX.assign(n, 0);
    for (int p = nfrozen; p < n; ++p)
        if (!inref[p]) {
            ctx->X.push_back(p);
            ctx->inX[p] = 1;
        }
    if ((int)ctx->ref.size() > kMaxActive)
        return ctx->fail(MBEFCI_ETOOLARGE, "reference space exceeds the active-orbital limit");
    ctx->pi.clear();
    ctx->spaces_set = true;
    return MBEFCI_OK;
}

mbefci_status mbefci_set_pi_pairs(mbefci_ctx *ctx, const int32_t *orbs, int32_t npairs) {
    if (!ctx) return MBEFCI_EINVAL;
    if (!ctx->spaces_set) return ctx->fail(MBEFCI_ESTATE, "set the spaces first");
    if (npairs < 0 || (npairs > 0 && !orbs)) return ctx->fail(MBEFCI_EINVAL, "bad pair list");
    std::vector<char> used(ctx->norb, 0);
    std::vector<std::pair<int, int>> pi;
    for (int i = 0; i < npairs; ++i) {
        const int x = orbs[2 * i], y = orbs[2 * i + 1];
        for (int p : {x, y}) {
            if (p < 0 || p >= ctx->norb || !ctx->inX[p])
                return ctx->fail(MBEFCI_EINVAL, "pair orbital " + std::to_string(p) + " is not an expansion orbital");
            if (used[p]) return ctx->fail(MBEFCI_EINVAL, "orbital " + std::to_string(p) + " in two pairs");
            used[p] = 1;
        }
        if (x == y) return ctx->fail(MBEFCI_EINVAL, "a pair needs two orbitals");
        pi.emplace_back(std::min(x, y), std::max(x, y));
    }
    ctx->pi.swap(pi);
    return MBEFCI_OK;
}

mbefci_status mbefci_set_orbital_irreps(mbefci_ctx *ctx, const int32_t *labels) {
    if (!ctx || !labels) return MBEFCI_EINVAL;
    if (!ctx->ham_set) return ctx->fail(MBEFCI_ESTATE, "set the Hamiltonian first");
    for (int p = 0; p < ctx->norb; ++p)
        if (labels[p] < 0 || labels[p] > 7) return ctx->fail(MBEFCI_EINVAL, "irrep labels must be 0..7");
    ctx->irr.assign(labels, labels + ctx->norb);
    ctx->sym_checked = false;
    if (ctx->device >= 0) {
        if (!ctx->d_irr) HIPCHK(hipMalloc(&ctx->d_irr, sizeof(int32_t) * kMaxOrb));
        HIPCHK(hipMemcpy(ctx->d_irr, ctx->irr.data(), sizeof(int32_t) * ctx->norb, hipMemcpyHostToDevice));
    }
    return MBEFCI_OK;
}

namespace {

// Symmetry targeting needs labels that the Hamiltonian respects, and a
// determinant of the target irrep in every tuple's CAS (the irreps that a
// spin's electrons can reach on the active orbitals, by counting).
mbefci_status check_symmetry(mbefci_ctx *ctx, int order, int64_t ntup, const std::vector<TupleShape> &shapes) {
    if (ctx->irr.size() != (size_t)ctx->norb)
        return ctx->fail(MBEFCI_EINVAL, "sym_shift needs orbital irrep labels (mbefci_set_orbital_irreps)");
    if (!ctx->sym_checked) {
        const int n = ctx->norb;
        const std::vector<int32_t> &g = ctx->irr;
        for (int p = 0; p < n; ++p)
            for (int q = 0; q < n; ++q) {
                if (g[p] != g[q] && std::fabs(ctx->h[(size_t)p * n + q]) > 1e-12)
                    return ctx->fail(MBEFCI_EINVAL, "the Hamiltonian does not respect the irrep labels (h)");
                for (int r = 0; r < n; ++r)
                    for (int s = 0; s < n; ++s)
                        if ((g[p] ^ g[q] ^ g[r] ^ g[s]) != 0 &&
                            std::fabs(ctx->eri[(((size_t)p * n + q) * n + r) * n + s]) > 1e-12)
                            return ctx->fail(MBEFCI_EINVAL, "the Hamiltonian does not respect the irrep labels (eri)");
            }
        ctx->sym_checked = true;
    }
    for (int64_t i = 0; i < ntup; ++i) {
        const TupleShape &ts = shapes[i];
        // reach[k] = bit set of irreps of k electrons on the active orbitals seen so far
        auto reach = [&](int ne) {
            std::vector<uint32_t> r(ne + 1, 0u);
            r[0] = 1u;
            for (int32_t p : ts.act)
                for (int k = ne; k >= 1; --k)
                    for (int x = 0; x < 8; ++x)
                        if (r[k - 1] >> x & 1u) r[k] |= 1u << (x ^ ctx->irr[p]);
            return r[ne];
        };
        const uint32_t ra = reach(ts.key.na), rb = reach(ts.key.nb);
        bool ok = false;
        for (int x = 0; x < 8 && !ok; ++x)
            for (int y = 0; y < 8 && !ok; ++y)
                ok = (ra >> x & 1u) && (rb >> y & 1u) && (x ^ y) == ctx->opt.irrep;
        if (!ok) return ctx->fail(MBEFCI_EINVAL, "no determinant of the target irrep in the CAS of a tuple of order " +
                                                 std::to_string(order));
    }
    return MBEFCI_OK;
}

}  // namespace

mbefci_status mbefci_set_options(mbefci_ctx *ctx, const mbefci_options *o) {
    if (!ctx || !o) return MBEFCI_EINVAL;
    if (!(o->sym_shift >= 0.0) || !std::isfinite(o->sym_shift))
        return ctx->fail(MBEFCI_EINVAL, "sym_shift must be finite and >= 0");
    if (o->irrep < 0 || o->irrep > 7) return ctx->fail(MBEFCI_EINVAL, "irrep must be 0..7");
    if (!std::isfinite(o->a)) return ctx->fail(MBEFCI_EINVAL, "non-finite a");
    if (o->max_space < 2 || o->max_space > kMaxSpace) return ctx->fail(MBEFCI_EINVAL, "max_space must be in 2..32");
    if (o->max_iter < 1) return ctx->fail(MBEFCI_EINVAL, "max_iter must be >= 1");
    if (!(o->e_tol > 0) || !(o->r_tol > 0)) return ctx->fail(MBEFCI_EINVAL, "tolerances must be positive");
    if (o->sigma_variant < 0 || o->sigma_variant > 2) return ctx->fail(MBEFCI_EINVAL, "sigma_variant must be 0, 1 or 2");
    if (o->pspace < 0 || o->pspace > kPsp) return ctx->fail(MBEFCI_EINVAL, "pspace must be in 0..128");
    if (o->linked_rows < 0 || o->linked_rows > 5) return ctx->fail(MBEFCI_EINVAL, "linked_rows must be in 0..5");
    if (o->restart_keep < 1 || o->restart_keep > 2) return ctx->fail(MBEFCI_EINVAL, "restart_keep must be 1 or 2");
    if (!(o->spin_shift >= 0.0) || !std::isfinite(o->spin_shift))
        return ctx->fail(MBEFCI_EINVAL, "spin_shift must be finite and >= 0");
    if (o->base_model < 0 || o->base_model > 3) return ctx->fail(MBEFCI_EINVAL, "base_model must be 0, 1, 2 or 3");
    if (o->whole_dim < 0 || o->whole_dim > kWholeMaxDim)
        return ctx->fail(MBEFCI_EINVAL, "whole_dim must be in 0.." + std::to_string(kWholeMaxDim));
    ctx->opt = *o;
    return MBEFCI_OK;
}

mbefci_status mbefci_workspace_query(mbefci_ctx *ctx, int32_t order, int64_t ntup, const int16_t *tuples,
                                     size_t *min_bytes, size_t *want_bytes) {
    if (!ctx || !min_bytes || !want_bytes) return MBEFCI_EINVAL;
    if (!ctx->spaces_set) return ctx->fail(MBEFCI_ESTATE, "no spaces set");
    std::map<std::pair<ClassKey, int>, int64_t> count;
    for (int64_t i = 0; i < ntup; ++i) {
        TupleShape ts;
        mbefci_status rc = tuple_shape(ctx, order, tuples + (size_t)i * order, ts);
        if (rc != MBEFCI_OK) return rc;
        count[{ts.key, ts.nC}]++;
    }
    size_t mn = 0, wt = 0;
    for (auto &c : count) {
        ClassPlan cp;
        plan_class(ctx, c.first.first, c.first.second, cp, true);
        mn = std::max(mn, cp.fixed_bytes + cp.per_tuple);
        wt = std::max(wt, cp.fixed_bytes + cp.per_tuple * (size_t)c.second);
    }
    *min_bytes = mn;
    *want_bytes = wt;
    return MBEFCI_OK;
}

mbefci_status mbefci_solve_tuples(mbefci_ctx *ctx, int32_t order, int64_t ntup, const int16_t *tuples, void *ws,
                                  size_t wsb, double *energies, int32_t *status) {
    if (!ctx) return MBEFCI_EINVAL;
    if (!energies || !status || order < 0) return ctx->fail(MBEFCI_EINVAL, "null output");
    ctx->stats = mbefci_stats{};
    ctx->cstats.clear();
    ctx->sigma_cls = nullptr;
    const double t0 = now_ms();
    mbefci_status rc = solve_device(ctx, order, ntup, tuples, ws, wsb, energies, status);
    ctx->stats.solve_ms = now_ms() - t0;
    return rc;
}

mbefci_status mbefci_solve_tuples_noalloc(mbefci_ctx *ctx, int32_t order, int64_t ntup, const int16_t *tuples,
                                          double *energies, int32_t *status) {
    if (!ctx) return MBEFCI_EINVAL;
    if (ctx->host_only || !ctx->scratch) return ctx->fail(MBEFCI_ESTATE, "host-only context");
    if (!energies || !status || order < 0) return ctx->fail(MBEFCI_EINVAL, "null output");
    if (!ctx->spaces_set) return ctx->fail(MBEFCI_ESTATE, "no spaces set");
    if (ntup > 0) {
        size_t mn = 0, want = 0;
        mbefci_status rq = mbefci_workspace_query(ctx, order, ntup, tuples, &mn, &want);
        if (rq != MBEFCI_OK) return rq;
        if (mn > kScratchBytes)
            return ctx->fail(MBEFCI_ENOMEM, "a tuple needs " + std::to_string(mn) + " bytes of workspace; the static "
                                            "workspace holds " + std::to_string(kScratchBytes));
    }
    ctx->stats = mbefci_stats{};
    ctx->cstats.clear();
    ctx->sigma_cls = nullptr;
    const double t0 = now_ms();
    mbefci_status rc = solve_device(ctx, order, ntup, tuples, ctx->scratch, kScratchBytes, energies, status);
    ctx->stats.solve_ms = now_ms() - t0;
    return rc;
}

mbefci_status mbefci_run(mbefci_ctx *ctx, void *ws, size_t wsb, mbefci_result **out) {
    if (!ctx || !out) return MBEFCI_EINVAL;
    *out = nullptr;
    mbefci_status rc = check_device(ctx);
    if (rc != MBEFCI_OK) return rc;
    ctx->stats = mbefci_stats{};
    ctx->cstats.clear();
    ctx->sigma_cls = nullptr;
    const double t0 = now_ms();
    auto res = std::make_unique<mbefci_result>();
    const bool grad = ctx->opt.gradient != 0;
    const bool base = ctx->opt.base_model != 0;
    if (grad && base) return ctx->fail(MBEFCI_EINVAL, "the gradient is not available with a base model");
    if (base) {
        // the base energy of the whole space (the tuple of every expansion orbital)
        std::vector<int16_t> all(ctx->X.begin(), ctx->X.end());
        if ((rc = base_energies(ctx, (int)all.size(), 1, all.data(), ws, wsb, &res->r.e_base)) != MBEFCI_OK) return rc;
    }
    if (!grad) {
        rc = run_planner(ctx,
                         [&](int k, int64_t nt, const int16_t *tup, double *e, int32_t *st) {
                             mbefci_status r = solve_device(ctx, k, nt, tup, ws, wsb, e, st);
                             if (base && (r == MBEFCI_OK || r == MBEFCI_ENOCONV)) {
                                 const mbefci_status rb = subtract_base(ctx, k, nt, tup, ws, wsb, e);
                                 if (rb != MBEFCI_OK) return rb;
                             }
                             return r;
                         },
                         res->r);
        res->r.total += res->r.e_base;
        ctx->stats.solve_ms = now_ms() - t0;
        if (rc == MBEFCI_OK || rc == MBEFCI_ENOCONV) *out = res.release();
        return rc;
    }
    // Forward run that also forms the gradient of the total (tuple set fixed).
    // The adjoint weight of every tuple of the last order is 1 (no computed
    // superset), so those density matrices are embedded on the device as they
    // converge; the Gram matrices of the lower orders wait on the host until
    // the tuple lists, and with them the weights w = (I + L^T)^-1 1, are known.
    TightTol tight(ctx);
    size_t wsb_run = wsb;
    if ((rc = grad_region(ctx, ws, &wsb_run)) != MBEFCI_OK) return rc;
    const int nX = (int)ctx->X.size();
    const int kmax = ctx->opt.max_order > 0 ? std::min(ctx->opt.max_order, nX) : nX;
    std::vector<std::unique_ptr<StoreSink>> stores;
    rc = run_planner(ctx,
                     [&](int k, int64_t nt, const int16_t *tup, double *e, int32_t *st) {
                         if (k == kmax) {
                             std::vector<double> ones((size_t)nt, 1.0);
                             WeightSink unit;
                             unit.w = &ones;
                             stores.emplace_back(nullptr);
                             return solve_device(ctx, k, nt, tup, ws, wsb_run, e, st, &unit);
                         }
                         auto sk = std::make_unique<StoreSink>();
                         sk->G.resize(nt);
                         sk->shape.resize(nt);
                         sk->NP.resize(nt, 0);
                         mbefci_status r = solve_device(ctx, k, nt, tup, ws, wsb_run, e, st, sk.get());
                         stores.push_back(std::move(sk));
                         return r;
                     },
                     res->r);
    if (rc != MBEFCI_OK && rc != MBEFCI_ENOCONV) {
        ctx->d_gh = ctx->d_ge = nullptr;
        return rc;
    }
    const auto w = adjoint_weights(res->r);
    const int n = ctx->norb;
    std::vector<double> gh((size_t)n * n, 0.0), ge((size_t)n * n * n * n, 0.0);
    for (size_t oi = 0; oi < stores.size() && oi < w.size(); ++oi) {
        if (!stores[oi]) continue;
        StoreSink &sk = *stores[oi];
        for (size_t i = 0; i < sk.G.size(); ++i) {
            if (w[oi][i] != 0 && sk.NP[i] > 0) accumulate_rdm(n, sk.shape[i], sk.G[i].data(), sk.NP[i], (double)w[oi][i],
                                                              gh.data(), ge.data());
            std::vector<double>().swap(sk.G[i]);
        }
    }
    mbefci_status rf = grad_fetch(ctx, gh, ge);
    if (rf != MBEFCI_OK) return rf;
    res->r.has_grad = true;
    res->r.grad_h.swap(gh);
    res->r.grad_eri.swap(ge);
    ctx->stats.solve_ms = now_ms() - t0;
    *out = res.release();
    return rc;
}

mbefci_status mbefci_run_host(mbefci_ctx *ctx, mbefci_energy_fn fn, void *user, mbefci_result **out) {
    if (!ctx || !fn || !out) return MBEFCI_EINVAL;
    *out = nullptr;
    if (!ctx->spaces_set) return ctx->fail(MBEFCI_ESTATE, "no spaces set");
    auto res = std::make_unique<mbefci_result>();
    mbefci_status rc = run_planner(ctx,
                                   [&](int k, int64_t nt, const int16_t *tup, double *e, int32_t *st) {
                                       for (int64_t i = 0; i < nt; ++i) st[i] = 0;
                                       if (fn(user, k, nt, tup, e) != 0)
                                           return ctx->fail(MBEFCI_EINVAL, "energy callback failed");
                                       return MBEFCI_OK;
                                   },
                                   res->r);
    if (rc == MBEFCI_OK) *out = res.release();
    return rc;
}

int32_t mbefci_result_norders(const mbefci_result *res) { return res ? (int32_t)res->r.orders.size() : 0; }

mbefci_status mbefci_result_order(const mbefci_result *res, int32_t k, int64_t *ntup, const int16_t **tuples,
                                  const double **eps, const double **dinc, const int32_t **status,
                                  double *order_sum, double *wall_ms) {
    if (!res || k < 0 || k >= (int32_t)res->r.orders.size()) return MBEFCI_EINVAL;
    const auto &o = res->r.orders[k];
    if (ntup) *ntup = (int64_t)o.eps.size();
    if (tuples) *tuples = o.tuples.data();
    if (eps) *eps = o.eps.data();
    if (dinc) *dinc = o.dinc.data();
    if (status) *status = o.status.data();
    if (order_sum) *order_sum = o.sum;
    if (wall_ms) *wall_ms = o.wall_ms;
    return MBEFCI_OK;
}

double mbefci_result_total(const mbefci_result *res) { return res ? res->r.total : 0.0; }
double mbefci_result_base(const mbefci_result *res) { return res ? res->r.e_base : 0.0; }

void mbefci_result_free(mbefci_result *res) { delete res; }

static mbefci_status single_tuple_batch(mbefci_ctx *ctx, int32_t order, const int16_t *tuple, void *ws, size_t wsb,
                                        Batch &b) {
    mbefci_status rc = check_device(ctx);
    if (rc != MBEFCI_OK) return rc;
    if (order < 0 || (order > 0 && !tuple) || !ws) return ctx->fail(MBEFCI_EINVAL, "bad arguments");
    TupleShape ts;
    if ((rc = tuple_shape(ctx, order, tuple, ts)) != MBEFCI_OK) return rc;
    ClassPlan cp;
    plan_class(ctx, ts.key, ts.nC, cp, false);
    Carver cv{(char *)ws, wsb};
    if (!carve_batch(ctx, cp, 1, cv, b, false)) return ctx->fail(MBEFCI_ENOMEM, "workspace too small");
    if ((rc = upload_tables(ctx, cp, b)) != MBEFCI_OK) return rc;
    std::vector<const TupleShape *> sh{&ts};
    if ((rc = upload_shapes(ctx, b, sh)) != MBEFCI_OK) return rc;
    hipError_t e = launch_gather(b, ctx->stream);
    if (e != hipSuccess) return ctx->fail(MBEFCI_EDEVICE, hipGetErrorString(e));
    e = launch_build_hb(b, ctx->stream);
    if (e != hipSuccess) return ctx->fail(MBEFCI_EDEVICE, hipGetErrorString(e));
    return MBEFCI_OK;
}

mbefci_status mbefci_tuple_sigma(mbefci_ctx *ctx, int32_t order, const int16_t *tuple, void *ws, size_t wsb,
                                 const double *d_c, double *d_sigma, int32_t nvec) {
    if (!ctx) return MBEFCI_EINVAL;
    if (!d_c || !d_sigma || nvec < 1) return ctx->fail(MBEFCI_EINVAL, "bad vectors");
    Batch b;
    mbefci_status rc = single_tuple_batch(ctx, order, tuple, ws, wsb, b);
    if (rc != MBEFCI_OK) return rc;
    // energy shift E_core: read back from the gathered parameters
    double ecore = 0.0;
    HIPCHK(hipMemcpyAsync(&ecore, b.params + b.pl.off_ecore, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (int v = 0; v < nvec; ++v) {
        VecRef c{const_cast<double *>(d_c), 0, nullptr, v};
        VecRef s{d_sigma, 0, nullptr, v};
        hipError_t e = launch_sigma(b, c, s, ecore, false, false, ctx->stream, nullptr, nullptr, nullptr, nullptr);
        if (e != hipSuccess) return ctx->fail(MBEFCI_EDEVICE, hipGetErrorString(e));
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return MBEFCI_OK;
}

mbefci_status mbefci_tuple_hdiag(mbefci_ctx *ctx, int32_t order, const int16_t *tuple, void *ws, size_t wsb,
                                 double *d_hdiag) {
    if (!ctx) return MBEFCI_EINVAL;
    if (!d_hdiag) return ctx->fail(MBEFCI_EINVAL, "null output");
    Batch b;
    mbefci_status rc = single_tuple_batch(ctx, order, tuple, ws, wsb, b);
    if (rc != MBEFCI_OK) return rc;
    hipError_t e = launch_hdiag(b, d_hdiag, b.dim, 1, ctx->stream);
    if (e != hipSuccess) return ctx->fail(MBEFCI_EDEVICE, hipGetErrorString(e));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return MBEFCI_OK;
}

mbefci_status mbefci_tuple_shape(mbefci_ctx *ctx, int32_t order, const int16_t *tuple, int64_t *na_str,
                                 int64_t *nb_str, int32_t *n_act, int32_t *na_act, int32_t *nb_act) {
    if (!ctx) return MBEFCI_EINVAL;
    if (!ctx->spaces_set) return ctx->fail(MBEFCI_ESTATE, "no spaces set");
    if (order < 0 || (order > 0 && !tuple)) return ctx->fail(MBEFCI_EINVAL, "bad tuple");
    TupleShape ts;
    mbefci_status rc = tuple_shape(ctx, order, tuple, ts);
    if (rc != MBEFCI_OK) return rc;
    const Tables &ta = ctx->table(ts.key.nA, ts.key.na), &tb = ctx->table(ts.key.nA, ts.key.nb);
    if (na_str) *na_str = ta.nstr;
    if (nb_str) *nb_str = tb.nstr;
    if (n_act) *n_act = ts.key.nA;
    if (na_act) *na_act = ts.key.na;
    if (nb_act) *nb_act = ts.key.nb;
    return MBEFCI_OK;
}

mbefci_status mbefci_string_tables(int32_t nA, int32_t nel, int64_t *n_strings, int32_t *n_entries,
                                   uint32_t *strings, uint32_t *links) {
    if (nA < 0 || nA > 20 || nel < 0 || nel > nA) return MBEFCI_EINVAL;
    Tables T;
    build_tables(nA, nel, T);
    if (n_strings) *n_strings = T.nstr;
    if (n_entries) *n_entries = T.nent;
    if (strings) std::memcpy(strings, T.strings.data(), 4 * T.strings.size());
    if (links) std::memcpy(links, T.links.data(), 4 * T.links.size());
    return MBEFCI_OK;
}

mbefci_status mbefci_backward(mbefci_ctx *ctx, const mbefci_result *res, double gE, void *ws, size_t wsb,
                              double *grad_h1, double *grad_eri) {
    if (!ctx || !res || !grad_h1 || !grad_eri) return MBEFCI_EINVAL;
    if (!std::isfinite(gE)) return ctx->fail(MBEFCI_EINVAL, "non-finite gE");
    if (!ctx->ham_set) return ctx->fail(MBEFCI_ESTATE, "no Hamiltonian set");
    const int n = ctx->norb;
    const size_t n2 = (size_t)n * n, n4 = n2 * n2;
    if (res->r.open) return ctx->fail(MBEFCI_ESTATE, "the last order is still open (mbefci_order_close)");
    if (res->r.has_grad) {   // formed by the forward run
        if (res->r.grad_h.size() != n2 || res->r.grad_eri.size() != n4)
            return ctx->fail(MBEFCI_ESTATE, "result was computed for another orbital count");
        write_grad(ctx, res->r.grad_h, res->r.grad_eri, gE, grad_h1, grad_eri);
        return MBEFCI_OK;
    }
    mbefci_status rc = check_device(ctx);
    if (rc != MBEFCI_OK) return rc;
    const double t0 = now_ms();
    ctx->stats = mbefci_stats{};
    ctx->cstats.clear();
    ctx->sigma_cls = nullptr;
    TightTol tight(ctx);
    size_t wsb_run = wsb;
    if ((rc = grad_region(ctx, ws, &wsb_run)) != MBEFCI_OK) return rc;
    const auto w = adjoint_weights(res->r);
    for (size_t oi = 0; oi < res->r.orders.size(); ++oi) {
        const auto &o = res->r.orders[oi];
        // tuples with a non-zero weight only, solved again and embedded on the device
        std::vector<int16_t> tl;
        std::vector<double> wl;
        for (size_t i = 0; i < o.eps.size(); ++i)
            if (w[oi][i] != 0) {
                tl.insert(tl.end(), o.tuples.begin() + i * o.k, o.tuples.begin() + (i + 1) * o.k);
                wl.push_back((double)w[oi][i]);
            }
        if (wl.empty()) continue;
        std::vector<double> e(wl.size());
        std::vector<int32_t> st(wl.size());
        WeightSink sink;
        sink.w = &wl;
        rc = solve_device(ctx, o.k, (int64_t)wl.size(), tl.data(), ws, wsb_run, e.data(), st.data(), &sink);
        if (rc != MBEFCI_OK) {
            ctx->d_gh = ctx->d_ge = nullptr;
            return rc;
        }
    }
    std::vector<double> gh, ge;
    if ((rc = grad_fetch(ctx, gh, ge)) != MBEFCI_OK) return rc;
    write_grad(ctx, gh, ge, gE, grad_h1, grad_eri);
    ctx->stats.solve_ms = now_ms() - t0;
    return MBEFCI_OK;
}

mbefci_status mbefci_casscf(mbefci_ctx *ctx, void *ws, size_t wsb, int32_t max_iter, double g_tol, double *U_out,
                            double *e_out, int32_t *iter_out) {
    if (!ctx) return MBEFCI_EINVAL;
    mbefci_status rc = check_device(ctx);
    if (rc != MBEFCI_OK) return rc;
    if (!ctx->ham_set || !ctx->spaces_set) return ctx->fail(MBEFCI_EINVAL, "Hamiltonian and spaces must be set");
    if (max_iter < 1 || !(g_tol > 0.0)) return ctx->fail(MBEFCI_EINVAL, "max_iter >= 1 and g_tol > 0 required");
    if ((int)ctx->ref.size() > kRdmMaxActive)
        return ctx->fail(MBEFCI_ETOOLARGE, "reference space above " + std::to_string(kRdmMaxActive) + " orbitals");
    const double t0 = now_ms();
    const int n = ctx->norb;
    const size_t n2 = (size_t)n * n, n4 = n2 * n2;
    // spaces: frozen (never rotated), core, active = [Pi], virtual
    std::vector<int> kind(n, 3);   // 0 frozen, 1 core, 2 active, 3 virtual
    for (int p = 0; p < ctx->nbeta; ++p) kind[p] = 1;
    for (int p = 0; p < ctx->nfrozen; ++p) kind[p] = 0;
    for (int p : ctx->ref) kind[p] = 2;
    std::vector<int> C, A, V, occ;
    for (int p = 0; p < n; ++p) {
        if (kind[p] == 1) C.push_back(p);
        if (kind[p] == 2) A.push_back(p);
        if (kind[p] == 3) V.push_back(p);
        if (kind[p] != 3) occ.push_back(p);
    }
    std::vector<std::pair<int, int>> pairs;
    for (int p : C)
        for (int q : A) pairs.emplace_back(p, q);
    for (int p : C)
        for (int q : V) pairs.emplace_back(p, q);
    for (int p : A)
        for (int q : V) pairs.emplace_back(p, q);
    const int np = (int)pairs.size();
    // workspace: the starting integrals, one n^4 scratch, U, F, f, occ; the
    // rest for the reference CASCI and its density matrices
    Carver cv{(char *)ws, wsb};
    double *d_eri0 = cv.take<double>(n4), *d_tmp = cv.take<double>(n4), *d_h0 = cv.take<double>(n2);
    double *d_U = cv.take<double>(n2), *d_F = cv.take<double>(n2), *d_f = cv.take<double>(n2);
    int32_t *d_occ = cv.take<int32_t>(occ.size() + 1);
    if (!cv.ok) return ctx->fail(MBEFCI_ENOMEM, "workspace too small for the integral transformation");
    char *ws2 = (char *)ws + cv.off;
    const size_t wsb2 = wsb - cv.off;
    HIPCHK(hipMemcpyAsync(d_eri0, ctx->eri.data(), 8 * n4, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(d_h0, ctx->h.data(), 8 * n2, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(d_occ, occ.data(), 4 * occ.size(), hipMemcpyHostToDevice, ctx->stream));
    // the reference CASCI converged tightly: the gradient comes from its
    // density matrices, which carry the residual to first order
    const mbefci_options saved = ctx->opt;
    ctx->opt.r_tol = std::min(ctx->opt.r_tol, 1e-11);
    ctx->opt.e_tol = std::min(ctx->opt.e_tol, 1e-13);
    ctx->opt.max_iter = std::max(ctx->opt.max_iter, 600);
    struct Restore {
        mbefci_ctx *c;
        const mbefci_options &o;
        ~Restore() { c->opt = o; }
    } restore{ctx, saved};
    Mat F(n2), f(n2), g1(n2);
    // integrals in the orbitals U, the reference energy, F, f and gamma
    auto evaluate = [&](const Mat &U, double &E) -> mbefci_status {
        HIPCHK(hipMemcpyAsync(d_U, U.data(), 8 * n2, hipMemcpyHostToDevice, ctx->stream));
        hipError_t e = launch_rotate_integrals(d_h0, d_eri0, d_U, ctx->d_h, ctx->d_eri, d_tmp, n, ctx->stream);
        if (e != hipSuccess) return ctx->fail(MBEFCI_EDEVICE, hipGetErrorString(e));
        size_t wsr = wsb2;
        mbefci_status r = grad_region(ctx, ws2, &wsr);
        if (r != MBEFCI_OK) return r;
        std::vector<double> w1{1.0};
        WeightSink sink;
        sink.w = &w1;
        int32_t st = 0;
        r = solve_device(ctx, 0, 1, nullptr, ws2, wsr, &E, &st, &sink);
        if (r != MBEFCI_OK) {
            ctx->d_gh = ctx->d_ge = nullptr;
            return r;
        }
        if (st != MBEFCI_TUPLE_OK) {
            ctx->d_gh = ctx->d_ge = nullptr;
            return ctx->fail(MBEFCI_ENOCONV, "reference CASCI did not converge");
        }
        e = launch_fock(ctx->d_h, ctx->d_eri, ctx->d_gh, ctx->d_ge, d_occ, (int)occ.size(), n, d_F, d_f, ctx->stream);
        if (e != hipSuccess) return ctx->fail(MBEFCI_EDEVICE, hipGetErrorString(e));
        HIPCHK(hipMemcpyAsync(F.data(), d_F, 8 * n2, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipMemcpyAsync(f.data(), d_f, 8 * n2, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipMemcpyAsync(g1.data(), ctx->d_gh, 8 * n2, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        ctx->d_gh = ctx->d_ge = nullptr;
        return MBEFCI_OK;
    };
    // dE/dkappa_pq of the local rotation U exp(K), K_pq = kappa = -K_qp:
    // 2 (F_qp - F_pq)
    auto gradient = [&](std::vector<double> &g) {
        g.resize(np);
        for (int k = 0; k < np; ++k) {
            const int p = pairs[k].first, q = pairs[k].second;
            g[k] = 2.0 * (F[(size_t)q * n + p] - F[(size_t)p * n + q]);
        }
    };
    auto rotation = [&](const std::vector<double> &d) {
        Mat K(n2, 0.0);
        for (int k = 0; k < np; ++k) {
            K[(size_t)pairs[k].first * n + pairs[k].second] = d[k];
            K[(size_t)pairs[k].second * n + pairs[k].first] = -d[k];
        }
        return mat_exp(K, n);
    };
    Mat U(n2, 0.0);
    for (int i = 0; i < n; ++i) U[(size_t)i * n + i] = 1.0;
    double E = 0.0;
    if ((rc = evaluate(U, E)) != MBEFCI_OK) return rc;
    std::vector<double> g;
    gradient(g);
    // quasi-Newton in the frame of the current orbitals: limited-memory BFGS
    // (8 pairs) on a diagonal estimate of the Hessian,
    // 2 gamma_pp f_qq + 2 gamma_qq f_pp - 2 F_pp - 2 F_qq (at least 0.05),
    // steps of at most 0.5 per rotation, halved until the energy falls by a
    // fraction of the predicted decrease
    std::vector<std::vector<double>> hs, hy;
    int it = 0;
    double gmax = 0.0;
    for (; it < max_iter; ++it) {
        gmax = 0.0;
        for (double v : g) gmax = std::max(gmax, std::fabs(v));
        if (gmax < g_tol || np == 0) break;
        std::vector<double> H(np);
        for (int k = 0; k < np; ++k) {
            const size_t p = pairs[k].first, q = pairs[k].second;
            const double h = 2.0 * g1[p * n + p] * f[q * n + q] + 2.0 * g1[q * n + q] * f[p * n + p] -
                             2.0 * F[p * n + p] - 2.0 * F[q * n + q];
            H[k] = std::max(std::fabs(h), 0.05);
        }
        std::vector<double> r(g), al(hs.size());
        for (int m = (int)hs.size() - 1; m >= 0; --m) {
            double ys = 0.0, sr = 0.0;
            for (int k = 0; k < np; ++k) {
                ys += hy[m][k] * hs[m][k];
                sr += hs[m][k] * r[k];
            }
            al[m] = sr / ys;
            for (int k = 0; k < np; ++k) r[k] -= al[m] * hy[m][k];
        }
        for (int k = 0; k < np; ++k) r[k] /= H[k];
        for (size_t m = 0; m < hs.size(); ++m) {
            double ys = 0.0, yr = 0.0;
            for (int k = 0; k < np; ++k) {
                ys += hy[m][k] * hs[m][k];
                yr += hy[m][k] * r[k];
            }
            const double be = yr / ys;
            for (int k = 0; k < np; ++k) r[k] += hs[m][k] * (al[m] - be);
        }
        std::vector<double> d(np);
        double dg = 0.0, dmax = 0.0;
        for (int k = 0; k < np; ++k) {
            d[k] = -r[k];
            dg += d[k] * g[k];
        }
        if (!(dg < 0.0)) {   // not a descent direction: the preconditioned gradient
            hs.clear();
            hy.clear();
            dg = 0.0;
            for (int k = 0; k < np; ++k) {
                d[k] = -g[k] / H[k];
                dg += d[k] * g[k];
            }
        }
        for (double v : d) dmax = std::max(dmax, std::fabs(v));
        if (dmax > 0.5) {
            for (double &v : d) v *= 0.5 / dmax;
            dg *= 0.5 / dmax;
        }
        double alpha = 1.0, En = 0.0;
        Mat Un;
        for (;;) {
            std::vector<double> ds(d);
            for (double &v : ds) v *= alpha;
            Un = mat_mul(U, rotation(ds), n);
            if ((rc = evaluate(Un, En)) != MBEFCI_OK) return rc;
            // (a predicted decrease below the energy's own rounding cannot be
            // checked: near convergence the quasi-Newton step is taken as it is)
            if (En <= E + 1e-4 * alpha * dg || alpha < 1e-3 ||
                std::fabs(alpha * dg) < 1e-12 * std::max(1.0, std::fabs(E)))
                break;
            alpha *= 0.5;
        }
        std::vector<double> gn;
        gradient(gn);
        std::vector<double> sv(np), yv(np);
        double ys = 0.0;
        for (int k = 0; k < np; ++k) {
            sv[k] = alpha * d[k];
            yv[k] = gn[k] - g[k];
            ys += sv[k] * yv[k];
        }
        if (ys > 1e-14) {
            hs.push_back(sv);
            hy.push_back(yv);
            if (hs.size() > 8) {
                hs.erase(hs.begin());
                hy.erase(hy.begin());
            }
        }
        U.swap(Un);
        E = En;
        g.swap(gn);
    }
    // canonical orbitals: Fock eigenvectors in the core and virtual blocks
    // (ascending), natural orbitals in the active block (descending
    // occupation), each at its space's own positions; every column signed so
    // that its largest entry is positive
    Mat R(n2, 0.0);
    for (int i = 0; i < n; ++i) R[(size_t)i * n + i] = 1.0;
    auto block = [&](const std::vector<int> &B, const Mat &M, bool desc) {
        const int m = (int)B.size();
        if (m == 0) return;
        Mat S((size_t)m * m), Vb;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) S[(size_t)i * m + j] = 0.5 * (M[(size_t)B[i] * n + B[j]] + M[(size_t)B[j] * n + B[i]]);
        std::vector<double> w;
        sym_eig(S, m, desc, w, Vb);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) R[(size_t)B[i] * n + B[j]] = Vb[(size_t)i * m + j];
    };
    block(C, f, false);
    block(V, f, false);
    block(A, g1, true);
    Mat Uc = mat_mul(U, R, n);
    for (int j = 0; j < n; ++j) {
        int im = 0;
        for (int i = 1; i < n; ++i)
            if (std::fabs(Uc[(size_t)i * n + j]) > std::fabs(Uc[(size_t)im * n + j])) im = i;
        if (Uc[(size_t)im * n + j] < 0.0)
            for (int i = 0; i < n; ++i) Uc[(size_t)i * n + j] = -Uc[(size_t)i * n + j];
    }
    // the context's Hamiltonian in the canonical orbitals (device and host)
    HIPCHK(hipMemcpyAsync(d_U, Uc.data(), 8 * n2, hipMemcpyHostToDevice, ctx->stream));
    hipError_t e = launch_rotate_integrals(d_h0, d_eri0, d_U, ctx->d_h, ctx->d_eri, d_tmp, n, ctx->stream);
    if (e != hipSuccess) return ctx->fail(MBEFCI_EDEVICE, hipGetErrorString(e));
    HIPCHK(hipMemcpyAsync(ctx->h.data(), ctx->d_h, 8 * n2, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->eri.data(), ctx->d_eri, 8 * n4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (int p = 0; p < n; ++p)   // exact symmetry of h (rounding of the two products)
        for (int q = 0; q < p; ++q) {
            const double v = 0.5 * (ctx->h[(size_t)p * n + q] + ctx->h[(size_t)q * n + p]);
            ctx->h[(size_t)p * n + q] = ctx->h[(size_t)q * n + p] = v;
        }
    HIPCHK(hipMemcpy(ctx->d_h, ctx->h.data(), 8 * n2, hipMemcpyHostToDevice));
    ctx->sym_checked = false;
    if (U_out) std::memcpy(U_out, Uc.data(), 8 * n2);
    if (e_out) *e_out = E;
    if (iter_out) *iter_out = it;
    ctx->stats.solve_ms = now_ms() - t0;
    if (gmax >= g_tol && np > 0) return ctx->fail(MBEFCI_ENOCONV, "orbital gradient above g_tol after max_iter");
    return MBEFCI_OK;
}

// Restricted closed-shell Hartree-Fock orbitals (the paper's expansion
// orbitals, Sec. 1 and 2, and the reference of its CCSD(T) base, Sec. 4.2.1).
// Energy descent over the occupied-virtual rotations C <- C exp(K): the
// gradient in the current orbitals is 4 f_ai, f the closed-shell Fock matrix
// of D = C_occ C_occ^T (built on the device from the starting integrals);
// limited-memory BFGS steps (8 pairs, in the frame of the current orbitals)
// on the diagonal Hessian estimate 4 (f_aa - f_ii) floored at 0.05, at most
// 0.5 per element, halved until the energy does not rise; once the gradient
// is below 1e-5, Newton steps on the Hessian from central differences of the
// gradient (at most six; the quasi-Newton steps converge slowly there).
// Then the Fock matrix diagonalised in the occupied and the virtual block,
// each ascending, occupied orbitals first; every column signed so that its
// largest entry is positive; the context's Hamiltonian replaced by the one in
// these orbitals.
mbefci_status mbefci_hf(mbefci_ctx *ctx, void *ws, size_t wsb, int32_t max_iter, double g_tol, double *U_out,
                        double *e_out, int32_t *iter_out) {
    if (!ctx) return MBEFCI_EINVAL;
    mbefci_status rc = check_device(ctx);
    if (rc != MBEFCI_OK) return rc;
    if (!ctx->ham_set || !ctx->spaces_set) return ctx->fail(MBEFCI_EINVAL, "Hamiltonian and spaces must be set");
    if (max_iter < 1 || !(g_tol > 0.0)) return ctx->fail(MBEFCI_EINVAL, "max_iter >= 1 and g_tol > 0 required");
    if (ctx->nalpha != ctx->nbeta) return ctx->fail(MBEFCI_EINVAL, "Hartree-Fock orbitals need a closed shell");
    const double t0 = now_ms();
    const int n = ctx->norb, no = ctx->nalpha, nv = n - no;
    const size_t n2 = (size_t)n * n, n4 = n2 * n2;
    Carver cv{(char *)ws, wsb};
    double *d_eri0 = cv.take<double>(n4), *d_tmp = cv.take<double>(n4), *d_h0 = cv.take<double>(n2);
    double *d_U = cv.take<double>(n2), *d_f = cv.take<double>(n2), *d_g1 = cv.take<double>(n2);
    int32_t *d_all = cv.take<int32_t>((size_t)n);
    if (!cv.ok) return ctx->fail(MBEFCI_ENOMEM, "workspace too small for the Hartree-Fock orbitals");
    std::vector<int32_t> all(n);
    for (int p = 0; p < n; ++p) all[p] = p;
    const Mat h0 = ctx->h;
    HIPCHK(hipMemcpyAsync(d_eri0, ctx->eri.data(), 8 * n4, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(d_h0, ctx->h.data(), 8 * n2, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(d_all, all.data(), 4 * (size_t)n, hipMemcpyHostToDevice, ctx->stream));
    // energy and the Fock matrix in the orbitals C (columns; row-major n x n)
    Mat g1(n2), fao(n2);
    auto evaluate = [&](const Mat &C, double &E, Mat &Fm) -> mbefci_status {
        for (int p = 0; p < n; ++p)
            for (int q = 0; q < n; ++q) {
                double d = 0.0;
                for (int i = 0; i < no; ++i) d += C[(size_t)p * n + i] * C[(size_t)q * n + i];
                g1[(size_t)p * n + q] = 2.0 * d;
            }
        HIPCHK(hipMemcpyAsync(d_g1, g1.data(), 8 * n2, hipMemcpyHostToDevice, ctx->stream));
        hipError_t e = launch_fock(d_h0, d_eri0, d_g1, nullptr, d_all, n, n, d_f, d_f, ctx->stream);
        if (e != hipSuccess) return ctx->fail(MBEFCI_EDEVICE, hipGetErrorString(e));
        HIPCHK(hipMemcpyAsync(fao.data(), d_f, 8 * n2, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        E = ctx->e_const;
        for (size_t k = 0; k < n2; ++k) E += 0.5 * g1[k] * (h0[k] + fao[k]);
        Mat T = mat_mul(fao, C, n), Ct(n2);
        for (int p = 0; p < n; ++p)
            for (int q = 0; q < n; ++q) Ct[(size_t)q * n + p] = C[(size_t)p * n + q];
        Fm = mat_mul(Ct, T, n);
        return MBEFCI_OK;
    };
    // start: the eigenvectors of h, ascending
    Mat C;
    {
        std::vector<double> w;
        sym_eig(h0, n, false, w, C);
    }
    double E = 0.0;
    Mat Fm;
    if ((rc = evaluate(C, E, Fm)) != MBEFCI_OK) return rc;
    const int np = no * nv;
    auto grad = [&](const Mat &F) {
        std::vector<double> g((size_t)np);
        for (int a = 0; a < nv; ++a)
            for (int i = 0; i < no; ++i) g[(size_t)a * no + i] = 4.0 * F[(size_t)(no + a) * n + i];
        return g;
    };
    std::vector<double> g = grad(Fm), g_old, step_old;
    std::vector<std::vector<double>> Ss, Ys;
    auto dot = [](const std::vector<double> &x, const std::vector<double> &y) {
        double s = 0.0;
        for (size_t k = 0; k < x.size(); ++k) s += x[k] * y[k];
        return s;
    };
    // C exp(K(x)) for rotation parameters x[a * no + i]
    auto rotate = [&](const Mat &Cx, const std::vector<double> &x) {
        Mat K(n2, 0.0);
        for (int a = 0; a < nv; ++a)
            for (int i = 0; i < no; ++i) {
                K[(size_t)(no + a) * n + i] = x[(size_t)a * no + i];
                K[(size_t)i * n + no + a] = -x[(size_t)a * no + i];
            }
        return mat_mul(Cx, mat_exp(K, n), n);
    };
    // Newton step on the Hessian from central differences of the gradient;
    // ok = false (and nothing changed) when that Hessian is not positive definite
    auto newton_step = [&](bool &ok) -> mbefci_status {
        const double hs = 1e-4;
        std::vector<double> H((size_t)np * np), x(np, 0.0);
        for (int kk = 0; kk < np; ++kk) {
            double Ep, Em;
            Mat Fp, Fmn;
            x[kk] = hs;
            if ((rc = evaluate(rotate(C, x), Ep, Fp)) != MBEFCI_OK) return rc;
            x[kk] = -hs;
            if ((rc = evaluate(rotate(C, x), Em, Fmn)) != MBEFCI_OK) return rc;
            x[kk] = 0.0;
            const std::vector<double> gp = grad(Fp), gm = grad(Fmn);
            for (int j = 0; j < np; ++j) H[(size_t)j * np + kk] = (gp[j] - gm[j]) / (2.0 * hs);
        }
        // symmetrise into the lower triangle, then Cholesky H = L L^T in place
        for (int a = 0; a < np; ++a)
            for (int b = 0; b < a; ++b) H[(size_t)a * np + b] = 0.5 * (H[(size_t)a * np + b] + H[(size_t)b * np + a]);
        for (int j = 0; j < np; ++j) {
            double d = H[(size_t)j * np + j];
            for (int q = 0; q < j; ++q) d -= H[(size_t)j * np + q] * H[(size_t)j * np + q];
            if (!(d > 0.0)) {
                ok = false;
                return MBEFCI_OK;
            }
            d = std::sqrt(d);
            H[(size_t)j * np + j] = d;
            for (int r = j + 1; r < np; ++r) {
                double v = H[(size_t)r * np + j];
                for (int q = 0; q < j; ++q) v -= H[(size_t)r * np + q] * H[(size_t)j * np + q];
                H[(size_t)r * np + j] = v / d;
            }
        }
        std::vector<double> y(np);
        for (int r = 0; r < np; ++r) {   // L y = -g, then L^T x = y
            double v = -g[r];
            for (int q = 0; q < r; ++q) v -= H[(size_t)r * np + q] * y[q];
            y[r] = v / H[(size_t)r * np + r];
        }
        for (int r = np - 1; r >= 0; --r) {
            double v = y[r];
            for (int q = r + 1; q < np; ++q) v -= H[(size_t)q * np + r] * x[q];
            x[r] = v / H[(size_t)r * np + r];
        }
        C = rotate(C, x);
        if ((rc = evaluate(C, E, Fm)) != MBEFCI_OK) return rc;
        ok = true;
        return MBEFCI_OK;
    };
    double gmax = 0.0;
    int it = 0, newton = 0;
    for (; it < max_iter; ++it) {
        gmax = 0.0;
        for (double x : g) gmax = std::max(gmax, std::fabs(x));
        if (gmax < g_tol || np == 0) break;
        if (gmax < 1e-5 && newton < 6) {   // quasi-Newton converges slowly here
            bool ok = false;
            if ((rc = newton_step(ok)) != MBEFCI_OK) return rc;
            if (ok) {
                ++newton;
                g = grad(Fm);
                g_old.clear();
                Ss.clear();
                Ys.clear();
                continue;
            }
            newton = 6;   // not positive definite: keep descending
        }
        if (!g_old.empty()) {
            std::vector<double> y(np);
            for (int k = 0; k < np; ++k) y[k] = g[k] - g_old[k];
            if (dot(step_old, y) > 1e-16) {
                Ss.push_back(step_old);
                Ys.push_back(y);
                if (Ss.size() > 8) {
                    Ss.erase(Ss.begin());
                    Ys.erase(Ys.begin());
                }
            }
        }
        std::vector<double> hd(np), q = g, al;
        for (int a = 0; a < nv; ++a)
            for (int i = 0; i < no; ++i)
                hd[(size_t)a * no + i] =
                    std::max(4.0 * (Fm[(size_t)(no + a) * n + no + a] - Fm[(size_t)i * n + i]), 0.05);
        for (int k = (int)Ss.size() - 1; k >= 0; --k) {
            const double a = dot(Ss[k], q) / dot(Ss[k], Ys[k]);
            al.push_back(a);
            for (int j = 0; j < np; ++j) q[j] -= a * Ys[k][j];
        }
        for (int j = 0; j < np; ++j) q[j] /= hd[j];
        for (size_t k = 0; k < Ss.size(); ++k) {
            const double b = dot(Ys[k], q) / dot(Ss[k], Ys[k]);
            const double a = al[Ss.size() - 1 - k];
            for (int j = 0; j < np; ++j) q[j] += (a - b) * Ss[k][j];
        }
        std::vector<double> step(np);
        for (int j = 0; j < np; ++j) step[j] = -q[j];
        if (dot(step, g) >= 0.0) {   // not a descent direction: the preconditioned gradient
            for (int j = 0; j < np; ++j) step[j] = -g[j] / hd[j];
            Ss.clear();
            Ys.clear();
        }
        for (double &x : step) x = std::min(0.5, std::max(-0.5, x));
        double alpha = 1.0, En = 0.0;
        Mat Cn, Fn;
        for (;;) {
            Mat K(n2, 0.0);
            for (int a = 0; a < nv; ++a)
                for (int i = 0; i < no; ++i) {
                    const double k = alpha * step[(size_t)a * no + i];
                    K[(size_t)(no + a) * n + i] = k;
                    K[(size_t)i * n + no + a] = -k;
                }
            Cn = mat_mul(C, mat_exp(K, n), n);
            if ((rc = evaluate(Cn, En, Fn)) != MBEFCI_OK) return rc;
            if (En <= E + 1e-13 * std::max(1.0, std::fabs(E)) || alpha < 1e-6 || gmax < 1e-5) break;
            alpha *= 0.5;
        }
        g_old = g;
        step_old = step;
        for (double &x : step_old) x *= alpha;
        C.swap(Cn);
        Fm.swap(Fn);
        E = En;
        g = grad(Fm);
    }
    // canonical orbitals
    Mat R(n2, 0.0);
    auto block = [&](int b0, int m) {
        if (m == 0) return;
        Mat S((size_t)m * m), Vb;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j)
                S[(size_t)i * m + j] = 0.5 * (Fm[(size_t)(b0 + i) * n + b0 + j] + Fm[(size_t)(b0 + j) * n + b0 + i]);
        std::vector<double> w;
        sym_eig(S, m, false, w, Vb);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) R[(size_t)(b0 + i) * n + b0 + j] = Vb[(size_t)i * m + j];
    };
    block(0, no);
    block(no, nv);
    Mat Uc = mat_mul(C, R, n);
    for (int j = 0; j < n; ++j) {
        int im = 0;
        for (int i = 1; i < n; ++i)
            if (std::fabs(Uc[(size_t)i * n + j]) > std::fabs(Uc[(size_t)im * n + j])) im = i;
        if (Uc[(size_t)im * n + j] < 0.0)
            for (int i = 0; i < n; ++i) Uc[(size_t)i * n + j] = -Uc[(size_t)i * n + j];
    }
    HIPCHK(hipMemcpyAsync(d_U, Uc.data(), 8 * n2, hipMemcpyHostToDevice, ctx->stream));
    hipError_t e = launch_rotate_integrals(d_h0, d_eri0, d_U, ctx->d_h, ctx->d_eri, d_tmp, n, ctx->stream);
    if (e != hipSuccess) return ctx->fail(MBEFCI_EDEVICE, hipGetErrorString(e));
    HIPCHK(hipMemcpyAsync(ctx->h.data(), ctx->d_h, 8 * n2, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->eri.data(), ctx->d_eri, 8 * n4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (int p = 0; p < n; ++p)   // exact symmetry of h (rounding of the two products)
        for (int q = 0; q < p; ++q) {
            const double v = 0.5 * (ctx->h[(size_t)p * n + q] + ctx->h[(size_t)q * n + p]);
            ctx->h[(size_t)p * n + q] = ctx->h[(size_t)q * n + p] = v;
        }
    HIPCHK(hipMemcpy(ctx->d_h, ctx->h.data(), 8 * n2, hipMemcpyHostToDevice));
    ctx->sym_checked = false;
    if (U_out) std::memcpy(U_out, Uc.data(), 8 * n2);
    if (e_out) *e_out = E;
    if (iter_out) *iter_out = it;
    ctx->stats.solve_ms = now_ms() - t0;
    if (gmax >= g_tol && np > 0) return ctx->fail(MBEFCI_ENOCONV, "orbital gradient above g_tol after max_iter");
    return MBEFCI_OK;
}

mbefci_status mbefci_tuple_base(mbefci_ctx *ctx, int32_t order, int64_t ntup, const int16_t *tuples, void *ws,
                                size_t wsb, double *energies) {
    if (!ctx || !energies || ntup < 0 || order < 0 || (order > 0 && ntup > 0 && !tuples)) return MBEFCI_EINVAL;
    mbefci_status rc = check_device(ctx);
    if (rc != MBEFCI_OK) return rc;
    if (!ctx->ham_set || !ctx->spaces_set) return ctx->fail(MBEFCI_EINVAL, "Hamiltonian and spaces must be set");
    for (int64_t t = 0; t < ntup; ++t)
        for (int i = 0; i < order; ++i) {
            const int p = tuples[t * order + i];
            if (p < 0 || p >= ctx->norb || !ctx->inX[p] || (i > 0 && tuples[t * order + i - 1] >= p))
                return ctx->fail(MBEFCI_EINVAL, "tuple orbitals must be ascending expansion orbitals");
        }
    return base_energies(ctx, order, ntup, tuples, ws, wsb, energies);
}

mbefci_status mbefci_get_hamiltonian(const mbefci_ctx *ctx, double *h1, double *eri, double *e_const) {
    if (!ctx || !ctx->ham_set) return MBEFCI_EINVAL;
    const size_t n2 = (size_t)ctx->norb * ctx->norb;
    if (h1) std::memcpy(h1, ctx->h.data(), 8 * n2);
    if (eri) std::memcpy(eri, ctx->eri.data(), 8 * n2 * n2);
    if (e_const) *e_const = ctx->e_const;
    return MBEFCI_OK;
}

mbefci_status mbefci_tuple_rdm(mbefci_ctx *ctx, int32_t order, const int16_t *tuple, void *ws, size_t wsb,
                               double *energy, double *gamma, double *Gamma) {
    if (!ctx || !energy || !gamma || !Gamma) return MBEFCI_EINVAL;
    const int n = ctx->norb;
    const size_t n2 = (size_t)n * n;
    std::memset(gamma, 0, 8 * n2);
    std::memset(Gamma, 0, 8 * n2 * n2);
    TightTol tight(ctx);
    std::vector<int64_t> w1{1};
    GradSink sink;
    sink.n = n;
    sink.w = &w1;
    sink.gh = gamma;
    sink.ge = Gamma;
    int32_t st = 0;
    mbefci_status rc = solve_device(ctx, order, 1, tuple, ws, wsb, energy, &st, &sink);
    if (rc != MBEFCI_OK) return rc;
    for (size_t i = 0; i < n2 * n2; ++i) Gamma[i] *= 2.0;   // the sink stores Gamma / 2
    return MBEFCI_OK;
}

mbefci_status mbefci_order_solve(mbefci_ctx *ctx, mbefci_result *res, int64_t first, int64_t stride, int64_t count,
                                 void *ws, size_t wsb) {
    if (!ctx || !res) return MBEFCI_EINVAL;
    Result &R = res->r;
    if (!R.open) return ctx->fail(MBEFCI_ESTATE, "no open order");
    mbefci_status rc = check_device(ctx);
    if (rc != MBEFCI_OK) return rc;
    Result::Order &o = R.orders.back();
    const int k = o.k;
    const int64_t nt = (int64_t)o.eps.size();
    if (first < 0 || stride < 1 || count < 0 || (count > 0 && first + (count - 1) * stride >= nt))
        return ctx->fail(MBEFCI_EINVAL, "slice outside the open order");
    if (count == 0) return MBEFCI_OK;
    std::vector<int64_t> idx((size_t)count);
    std::vector<int16_t> tl((size_t)count * k);
    for (int64_t i = 0; i < count; ++i) {
        idx[i] = first + i * stride;
        if (R.solved[idx[i]]) return ctx->fail(MBEFCI_EINVAL, "tuple " + std::to_string(idx[i]) + " already solved");
        std::copy(o.tuples.begin() + idx[i] * k, o.tuples.begin() + (idx[i] + 1) * k, tl.begin() + i * k);
    }
    ctx->stats = mbefci_stats{};
    ctx->cstats.clear();
    ctx->sigma_cls = nullptr;
    const double t0 = now_ms();
    std::vector<double> e((size_t)count);
    std::vector<int32_t> st((size_t)count);
    const bool grad = ctx->opt.gradient != 0 && R.has_grad;
    if (grad) {
        // the last order's adjoint weights are 1: density matrices embedded on
        // the device as they converge, then added to the result's gradient
        TightTol tight(ctx);
        size_t wsb_run = wsb;
        if ((rc = grad_region(ctx, ws, &wsb_run)) != MBEFCI_OK) return rc;
        std::vector<double> ones((size_t)count, 1.0);
        WeightSink unit;
        unit.w = &ones;
        rc = solve_device(ctx, k, count, tl.data(), ws, wsb_run, e.data(), st.data(), &unit);
        if (rc != MBEFCI_OK && rc != MBEFCI_ENOCONV) {
            ctx->d_gh = ctx->d_ge = nullptr;
            return rc;
        }
        mbefci_status rf = grad_fetch(ctx, R.grad_h, R.grad_eri);
        if (rf != MBEFCI_OK) return rf;
    } else {
        rc = solve_device(ctx, k, count, tl.data(), ws, wsb, e.data(), st.data());
        if (rc != MBEFCI_OK && rc != MBEFCI_ENOCONV) return rc;
        if (ctx->opt.base_model) {
            const mbefci_status rb = subtract_base(ctx, k, count, tl.data(), ws, wsb, e.data());
            if (rb != MBEFCI_OK) return rb;
        }
    }
    // Eq. 3 against the completed lower orders (no tuple of the open order is
    // a subtuple of another)
    for (int64_t i = 0; i < count; ++i) {
        const int64_t j = idx[i];
        o.eps[j] = e[i];
        o.status[j] = st[i];
        o.dinc[j] = increment(o.tuples.data() + (size_t)j * k, k, e[i], R.dinc_map);
        R.solved[j] = 1;
    }
    o.wall_ms += now_ms() - t0;
    ctx->stats.solve_ms = now_ms() - t0;
    return rc;
}

mbefci_status mbefci_order_close(mbefci_ctx *ctx, mbefci_result *res) {
    if (!ctx || !res) return MBEFCI_EINVAL;
    Result &R = res->r;
    if (!R.open) return ctx->fail(MBEFCI_ESTATE, "no open order");
    Result::Order &o = R.orders.back();
    for (size_t i = 0; i < R.solved.size(); ++i)
        if (!R.solved[i]) return ctx->fail(MBEFCI_ESTATE, "tuple " + std::to_string(i) + " of the open order not solved");
    double s = 0.0;
    for (double d : o.dinc) s += d;
    o.sum = s;
    double tot = 0.0;
    for (auto &oo : R.orders) tot += oo.sum;
    R.total = tot + R.e_base;
    R.open = false;
    R.solved.clear();
    std::unordered_map<uint64_t, double>().swap(R.dinc_map);
    bool failed = false;
    for (int32_t st : o.status) failed |= st != MBEFCI_TUPLE_OK;
    return failed ? ctx->fail(MBEFCI_ENOCONV, "at least one tuple of the closed order did not converge") : MBEFCI_OK;
}

mbefci_status mbefci_get_class_stats(const mbefci_ctx *ctx, int32_t *nclass, mbefci_class_stats *out) {
    if (!ctx || !nclass) return MBEFCI_EINVAL;
    const int32_t cap = *nclass;
    *nclass = (int32_t)ctx->cstats.size();
    if (out) {
        int32_t i = 0;
        for (const auto &kv : ctx->cstats) {
            if (i >= cap) break;
            out[i++] = kv.second;
        }
    }
    return MBEFCI_OK;
}

mbefci_status mbefci_get_stats(const mbefci_ctx *ctx, mbefci_stats *s) {
    if (!ctx || !s) return MBEFCI_EINVAL;
    *s = ctx->stats;
    return MBEFCI_OK;
}

}  // extern "C"

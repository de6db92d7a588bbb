// Coupled-cluster base energies of tuples: CCSD and CCSD(T) on the reference
// determinant Phi(S) of each tuple's CAS, the base of MBE-FCI-b (Sec. 4.2.1,
// Table 3; Sec. 1 on coupled-cluster base models).
//
// Spin-orbital CCSD in the intermediate form of Stanton and Gauss (J. Chem.
// Phys. 94, 4334 (1991)), valid for non-canonical orbitals: the occupied
// spin-orbitals are the core-free active ones of Phi (alpha: active orbitals of
// index below n_alpha, beta: below n_beta), the frozen core enters through the
// Fock operator of Phi and the reference energy.  Amplitudes are updated by
// t = RHS / D with the Fock diagonal in D, accelerated by DIIS over the last
// kCcDiis updates.  The (T) correction (Raghavachari et al., Chem. Phys. Lett.
// 157, 479 (1989)) assumes canonical orbitals (the host checks the Fock
// operator): over the unique triples i<j<k, a<b<c,
//   D x = P(i/jk) P(a/bc) [sum_e t_jk^ae <ei||bc> - sum_m t_im^bc <ma||jk>],
//   D y = P(i/jk) P(a/bc) t_i^a <jk||bc>,   E_(T) = sum x (x + y) D.
// One workgroup per tuple runs the whole iteration; amplitudes, intermediates
// and the DIIS history live in a slice of the workspace per tuple.
#include "device.h"

#include <hip/hip_cooperative_groups.h>

namespace mbefci {

constexpr int kCcThreads = 1024;
constexpr int kCcDiis = 6;
constexpr int kCcMaxSo = 2 * kCcMaxActive;   // spin-orbitals of one CAS

// Doubles of one tuple's slice for o occupied and v virtual spin-orbitals.
int64_t cc_slice_doubles(int o, int v) {
    const int64_t L = (int64_t)o * v + (int64_t)o * o * v * v;
    const int64_t o2v2 = (int64_t)o * o * v * v;
    const int64_t N = o + v;
    return L * (2 + 2 * kCcDiis) + 3 * o2v2 + 2 * ((int64_t)v * v + (int64_t)o * o) + (int64_t)o * v +
           (int64_t)o * o * o * o + (int64_t)v * v * v * v + o2v2 + N * N * N * N + o2v2 + (int64_t)v * v * v * o;
}

__device__ __forceinline__ double block_max(double v, double *sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = blockDim.x >> 6;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    for (int i = 0; i < nw; ++i) r = fmax(r, sh[i]);
    return r;
}

struct CcArgs {
    const double *h, *eri;
    int n;
    const int32_t *act, *nact, *core, *ncore;
    int stride;            // entries per tuple of act / core
    int nalpha, nbeta;
    double e_const;
    double *work;          // slice per tuple
    int64_t slice;         // doubles per slice
    int triples;           // add (T)
    int max_iter;
    double tol;            // on the largest amplitude change
    double *out;           // energies (NaN on failure)
    int32_t *status;       // 0 ok, 1 non-negative denominator, 2 not converged
    int wgs;               // workgroups per tuple
    double *part;          // [2][wgs] reduction partials (wgs > 1)
};

__global__ __launch_bounds__(kCcThreads) void k_ccsd(CcArgs A) {
    // A.wgs workgroups per tuple (more than one: a cooperative launch of one
    // tuple, the workgroups joined by grid barriers)
    const int t = blockIdx.x / A.wgs, rk = blockIdx.x % A.wgs, tid = threadIdx.x, nth = kCcThreads;
    const int64_t gid = (int64_t)rk * nth + tid, gst = (int64_t)A.wgs * nth;
    auto gsync = [&]() {
        if (A.wgs > 1) {
            __threadfence();
            cooperative_groups::this_grid().sync();
        } else {
            __syncthreads();
        }
    };
    const int n = A.n, nA = A.nact[t], nC = A.ncore[t];
    const int32_t *act = A.act + (int64_t)t * A.stride, *core = A.core + (int64_t)t * A.stride;
    const double *eri = A.eri, *h = A.h;
    const int64_t n2 = (int64_t)n * n, n3 = n2 * n;
    auto E = [&](int p, int q, int r, int s) { return eri[p * n3 + q * n2 + r * n + s]; };

    __shared__ int so_orb[kCcMaxSo], so_spin[kCcMaxSo];
    __shared__ int lc[kMaxOrb];
    __shared__ double f[kCcMaxSo][kCcMaxSo];
    __shared__ double sh[16];
    __shared__ double B[kCcDiis + 1][kCcDiis + 1], coef[kCcDiis + 1];
    __shared__ int no_sh, nv_sh, bad_sh;
    // sum (or max) over the tuple's threads in a fixed order: workgroup sums,
    // then, across workgroups, their partials in two alternating slots
    int red_cnt = 0;
    auto grid_red = [&](double x, bool mx) -> double {
        const double w = mx ? block_max(x, sh) : block_sum(x, sh);
        if (A.wgs == 1) return w;
        double *pp = A.part + (size_t)(red_cnt & 1) * A.wgs;
        ++red_cnt;
        if (tid == 0) pp[rk] = w;
        gsync();
        double r = 0.0;
        for (int q = 0; q < A.wgs; ++q) r = mx ? fmax(r, pp[q]) : r + pp[q];
        return r;
    };
    if (tid == 0) {
        int o = 0;
        for (int s = 0; s < 2; ++s)
            for (int k = 0; k < nA; ++k)
                if (act[k] < (s ? A.nbeta : A.nalpha)) {
                    so_orb[o] = act[k];
                    so_spin[o++] = s;
                }
        int N = o;
        for (int s = 0; s < 2; ++s)
            for (int k = 0; k < nA; ++k)
                if (act[k] >= (s ? A.nbeta : A.nalpha)) {
                    so_orb[N] = act[k];
                    so_spin[N++] = s;
                }
        no_sh = o;
        nv_sh = N - o;
        bad_sh = 0;
    }
    for (int i = tid; i < nC; i += nth) lc[i] = core[i];
    __syncthreads();
    const int o = no_sh, v = nv_sh, N = o + v;
    // <PQ||RS> over spin-orbitals (chemists' (pr|qs) with spin deltas), from
    // the resident integrals; tabulated per tuple below
    auto asy_raw = [&](int P, int Q, int R, int S) {
        const int sp = so_spin[P], sq = so_spin[Q], sr = so_spin[R], ss = so_spin[S];
        double x = 0.0;
        if (sp == sr && sq == ss) x += E(so_orb[P], so_orb[R], so_orb[Q], so_orb[S]);
        if (sp == ss && sq == sr) x -= E(so_orb[P], so_orb[S], so_orb[Q], so_orb[R]);
        return x;
    };
    // an excitation conserves spin when the spins of the holes and of the
    // particles agree as multisets
    auto spin_ok2 = [&](int i, int j, int a, int b) {
        return so_spin[i] + so_spin[j] == so_spin[a] + so_spin[b];
    };
    // Fock operator of Phi on the active spin-orbitals
    for (int k = tid; k < N * N; k += nth) {
        const int P = k / N, Q = k % N;
        double x = 0.0;
        if (so_spin[P] == so_spin[Q]) {
            const int p = so_orb[P], q = so_orb[Q];
            x = h[p * n + q];
            for (int c = 0; c < nC; ++c) x += 2.0 * E(p, q, lc[c], lc[c]) - E(p, lc[c], lc[c], q);
            for (int m = 0; m < o; ++m) x += asy_raw(P, m, Q, m);
        }
        f[P][Q] = x;
    }
    // reference energy <Phi|H|Phi>
    double eref = 0.0;
    {
        const int nocc = 2 * nC + o;    // core spin-orbitals (both spins) then the active occupied ones
        auto orb = [&](int k, int &p, int &s) {
            if (k < 2 * nC) {
                p = lc[k >> 1];
                s = k & 1;
            } else {
                p = so_orb[k - 2 * nC];
                s = so_spin[k - 2 * nC];
            }
        };
        for (int k = tid; k < nocc; k += nth) {
            int p, s;
            orb(k, p, s);
            eref += h[p * n + p];
        }
        for (int kk = tid; kk < nocc * nocc; kk += nth) {
            int p, s, q, s2;
            orb(kk / nocc, p, s);
            orb(kk % nocc, q, s2);
            eref += 0.5 * (E(p, p, q, q) - (s == s2 ? E(p, q, q, p) : 0.0));
        }
    }
    eref = block_sum(eref, sh);
    __syncthreads();
    // denominators of the spin-conserving excitations must be negative
    for (int k = tid; k < o * v; k += nth)
        if (so_spin[k / v] == so_spin[o + k % v] && !(f[k / v][k / v] - f[o + k % v][o + k % v] < 0.0)) bad_sh = 1;
    __syncthreads();
    if (bad_sh) {
        if (tid == 0 && rk == 0) {
            A.out[t] = __builtin_nan("");
            A.status[t] = 1;
        }
        return;
    }

    // workspace slice
    const int64_t ov = (int64_t)o * v, o2v2 = ov * ov, L = ov + o2v2;
    double *w = A.work + (int64_t)t * A.slice;
    double *T = w;               // current amplitudes: t1[i][a] then t2[i][j][a][b]
    double *Tn = T + L;          // new amplitudes
    double *Hist = Tn + L;       // kCcDiis amplitude vectors
    double *Err = Hist + kCcDiis * L;
    double *tau = Err + kCcDiis * L, *taut = tau + o2v2, *Ioovv = taut + o2v2;
    double *Fae = Ioovv + o2v2, *Fmi = Fae + (int64_t)v * v, *Fme = Fmi + (int64_t)o * o;
    double *Wmnij = Fme + ov, *Wabef = Wmnij + (int64_t)o * o * o * o, *Wmbej = Wabef + (int64_t)v * v * v * v;
    double *Fbe2 = Wmbej + o2v2, *Fmj2 = Fbe2 + (int64_t)v * v;   // F_be - t_m^b F_me / 2, F_mj + t_j^e F_me / 2
    double *G = Fmj2 + (int64_t)o * o;                            // <PQ||RS>, N^4
    double *RQ = G + (int64_t)N * N * N * N;                      // ring term [i][a][j][b]
    double *Y = RQ + o2v2;                                        // sum_m t_m^a <mb||ej>, [a][b][e][j]
    auto asy = [&](int P, int Q, int R, int S) { return G[((P * N + Q) * N + R) * N + S]; };
    auto t1 = [&](int i, int a) -> double & { return T[i * v + a]; };
    auto t2 = [&](int i, int j, int a, int b) -> double & { return T[ov + ((i * o + j) * v + a) * v + b]; };
    auto iovv = [&](int m, int n_, int e, int f_) { return Ioovv[((m * o + n_) * v + e) * v + f_]; };
    const int V0 = o;   // spin-orbital index of virtual 0

    for (int64_t k = gid; k < L; k += gst) T[k] = 0.0;
    const int64_t N4 = (int64_t)N * N * N * N;
    for (int64_t k = gid; k < N4; k += gst)
        G[k] = asy_raw((int)(k / N / N / N), (int)(k / N / N % N), (int)(k / N % N), (int)(k % N));
    gsync();
    for (int64_t k = gid; k < o2v2; k += gst) {
        const int b = k % v, a = (k / v) % v, j = (k / v / v) % o, i = k / v / v / o;
        Ioovv[k] = asy(i, j, V0 + a, V0 + b);
    }
    gsync();

    double e_cc = 0.0, e_old = 0.0;
    int it = 0, nh = 0, conv = 0;
    for (; it < A.max_iter && L > 0; ++it) {
        // tau, tau~
        for (int64_t k = gid; k < o2v2; k += gst) {
            const int b = k % v, a = (k / v) % v, j = (k / v / v) % o, i = k / v / v / o;
            const double x = t1(i, a) * t1(j, b) - t1(i, b) * t1(j, a);
            tau[k] = T[ov + k] + x;
            taut[k] = T[ov + k] + 0.5 * x;
        }
        gsync();
        // one-body intermediates
        for (int k = (int)gid; k < v * v + o * o + o * v; k += (int)gst) {
            if (k < v * v) {
                const int a = k / v, e = k % v;
                double x = (a != e) ? f[V0 + a][V0 + e] : 0.0;
                #pragma unroll 4
                for (int m = 0; m < o; ++m) x -= 0.5 * f[m][V0 + e] * t1(m, a);
                for (int m = 0; m < o; ++m)
                    #pragma unroll 4
                    for (int ff = 0; ff < v; ++ff) x += t1(m, ff) * asy(m, V0 + a, V0 + ff, V0 + e);
                for (int m = 0; m < o; ++m)
                    for (int nn = 0; nn < o; ++nn)
                        #pragma unroll 4
                        for (int ff = 0; ff < v; ++ff)
                            x -= 0.5 * taut[((m * o + nn) * v + a) * v + ff] * iovv(m, nn, e, ff);
                Fae[k] = x;
            } else if (k < v * v + o * o) {
                const int kk = k - v * v, m = kk / o, i = kk % o;
                double x = (m != i) ? f[m][i] : 0.0;
                #pragma unroll 4
                for (int e = 0; e < v; ++e) x += 0.5 * t1(i, e) * f[m][V0 + e];
                for (int nn = 0; nn < o; ++nn)
                    #pragma unroll 4
                    for (int e = 0; e < v; ++e) x += t1(nn, e) * asy(m, nn, i, V0 + e);
                for (int nn = 0; nn < o; ++nn)
                    for (int e = 0; e < v; ++e)
                        #pragma unroll 4
                        for (int ff = 0; ff < v; ++ff)
                            x += 0.5 * taut[((i * o + nn) * v + e) * v + ff] * iovv(m, nn, e, ff);
                Fmi[kk] = x;
            } else {
                const int kk = k - v * v - o * o, m = kk / v, e = kk % v;
                double x = f[m][V0 + e];
                for (int nn = 0; nn < o; ++nn)
                    #pragma unroll 4
                    for (int ff = 0; ff < v; ++ff) x += t1(nn, ff) * iovv(m, nn, e, ff);
                Fme[kk] = x;
            }
        }
        gsync();
        // two-body intermediates, and the one-body ones dressed for the T2 equation
        const int64_t o4 = (int64_t)o * o * o * o, v4 = (int64_t)v * v * v * v;
        for (int k = (int)gid; k < v * v + o * o; k += (int)gst) {
            if (k < v * v) {
                const int b = k / v, e = k % v;
                double x = Fae[k];
                #pragma unroll 4
                for (int m = 0; m < o; ++m) x -= 0.5 * t1(m, b) * Fme[m * v + e];
                Fbe2[k] = x;
            } else {
                const int kk = k - v * v, m = kk / o, j = kk % o;
                double x = Fmi[kk];
                #pragma unroll 4
                for (int e = 0; e < v; ++e) x += 0.5 * t1(j, e) * Fme[m * v + e];
                Fmj2[kk] = x;
            }
        }
        const int64_t v3o = (int64_t)v * v * v * o;
        for (int64_t k = gid; k < o4 + v4 + o2v2 + v3o; k += gst) {
            if (k >= o4 + v4 + o2v2) {
                const int64_t kk = k - o4 - v4 - o2v2;
                const int j = kk % o, e = (kk / o) % v, b = (kk / o / v) % v, a = kk / o / v / v;
                double x = 0.0;
                #pragma unroll 4
                for (int m = 0; m < o; ++m) x += t1(m, a) * asy(m, V0 + b, V0 + e, j);
                Y[kk] = x;
            } else if (k < o4) {
                const int j = k % o, i = (k / o) % o, nn = (k / o / o) % o, m = k / o / o / o;
                double x = asy(m, nn, i, j);
                #pragma unroll 4
                for (int e = 0; e < v; ++e)
                    x += t1(j, e) * asy(m, nn, i, V0 + e) - t1(i, e) * asy(m, nn, j, V0 + e);
                for (int e = 0; e < v; ++e)
                    #pragma unroll 4
                    for (int ff = 0; ff < v; ++ff) x += 0.25 * tau[((i * o + j) * v + e) * v + ff] * iovv(m, nn, e, ff);
                Wmnij[k] = x;
            } else if (k < o4 + v4) {
                const int64_t kk = k - o4;
                const int ff = kk % v, e = (kk / v) % v, b = (kk / v / v) % v, a = kk / v / v / v;
                double x = asy(V0 + a, V0 + b, V0 + e, V0 + ff);
                #pragma unroll 4
                for (int m = 0; m < o; ++m)
                    x -= t1(m, b) * asy(V0 + a, m, V0 + e, V0 + ff) - t1(m, a) * asy(V0 + b, m, V0 + e, V0 + ff);
                for (int m = 0; m < o; ++m)
                    #pragma unroll 4
                    for (int nn = 0; nn < o; ++nn) x += 0.25 * tau[((m * o + nn) * v + a) * v + b] * iovv(m, nn, e, ff);
                Wabef[kk] = x;
            } else {
                // W_mbej stored as [m][b][e][j]
                const int64_t kk = k - o4 - v4;
                const int j = kk % o, e = (kk / o) % v, b = (kk / o / v) % v, m = kk / o / v / v;
                double x = asy(m, V0 + b, V0 + e, j);
                #pragma unroll 4
                for (int ff = 0; ff < v; ++ff) x += t1(j, ff) * asy(m, V0 + b, V0 + e, V0 + ff);
                #pragma unroll 4
                for (int nn = 0; nn < o; ++nn) x -= t1(nn, b) * asy(m, nn, V0 + e, j);
                for (int nn = 0; nn < o; ++nn)
                    #pragma unroll 4
                    for (int ff = 0; ff < v; ++ff)
                        x -= (0.5 * t2(j, nn, ff, b) + t1(j, ff) * t1(nn, b)) * iovv(m, nn, e, ff);
                Wmbej[kk] = x;
            }
        }
        gsync();
        auto wmbej = [&](int m, int b, int e, int j) { return Wmbej[((m * v + b) * v + e) * o + j]; };
        // ring term before its permutations:
        //   RQ(i,a,j,b) = sum_me t_im^ae W_mbej - sum_e t_i^e sum_m t_m^a <mb||ej>
        for (int64_t k = gid; k < o2v2; k += gst) {
            const int b = k % v, j = (k / v) % o, a = (k / v / o) % v, i = k / v / o / v;
            double x = 0.0;
            for (int m = 0; m < o; ++m)
                #pragma unroll 4
                for (int e = 0; e < v; ++e) x += t2(i, m, a, e) * wmbej(m, b, e, j);
            #pragma unroll 4
            for (int e = 0; e < v; ++e) x -= t1(i, e) * Y[((a * v + b) * v + e) * o + j];
            RQ[k] = x;
        }
        gsync();
        auto rq = [&](int i, int a, int j, int b) { return RQ[((i * v + a) * o + j) * v + b]; };
        // new amplitudes
        for (int64_t k = gid; k < L; k += gst) {
            if (k < ov) {
                const int i = k / v, a = k % v;
                if (so_spin[i] != so_spin[V0 + a]) {   // spin-forbidden: stays zero
                    Tn[k] = 0.0;
                    continue;
                }
                double x = f[i][V0 + a];
                #pragma unroll 4
                for (int e = 0; e < v; ++e) x += t1(i, e) * Fae[a * v + e];
                #pragma unroll 4
                for (int m = 0; m < o; ++m) x -= t1(m, a) * Fmi[m * o + i];
                for (int m = 0; m < o; ++m)
                    #pragma unroll 4
                    for (int e = 0; e < v; ++e) x += t2(i, m, a, e) * Fme[m * v + e];
                for (int nn = 0; nn < o; ++nn)
                    #pragma unroll 4
                    for (int ff = 0; ff < v; ++ff) x -= t1(nn, ff) * asy(nn, V0 + a, i, V0 + ff);
                for (int m = 0; m < o; ++m)
                    for (int e = 0; e < v; ++e)
                        #pragma unroll 4
                        for (int ff = 0; ff < v; ++ff) x -= 0.5 * t2(i, m, e, ff) * asy(m, V0 + a, V0 + e, V0 + ff);
                for (int m = 0; m < o; ++m)
                    for (int e = 0; e < v; ++e)
                        #pragma unroll 4
                        for (int nn = 0; nn < o; ++nn) x -= 0.5 * t2(m, nn, a, e) * asy(nn, m, V0 + e, i);
                Tn[k] = x / (f[i][i] - f[V0 + a][V0 + a]);
            } else {
                const int64_t kk = k - ov;
                const int b = kk % v, a = (kk / v) % v, j = (kk / v / v) % o, i = kk / v / v / o;
                if (i == j || a == b || !spin_ok2(i, j, V0 + a, V0 + b)) {
                    Tn[k] = 0.0;
                    continue;
                }
                double x = iovv(i, j, a, b);
                // P(ab) sum_e t_ij^ae (F_be - 1/2 sum_m t_m^b F_me)
                #pragma unroll 4
                for (int e = 0; e < v; ++e) x += t2(i, j, a, e) * Fbe2[b * v + e] - t2(i, j, b, e) * Fbe2[a * v + e];
                // -P(ij) sum_m t_im^ab (F_mj + 1/2 sum_e t_j^e F_me)
                #pragma unroll 4
                for (int m = 0; m < o; ++m) x -= t2(i, m, a, b) * Fmj2[m * o + j] - t2(j, m, a, b) * Fmj2[m * o + i];
                for (int m = 0; m < o; ++m)
                    #pragma unroll 4
                    for (int nn = 0; nn < o; ++nn)
                        x += 0.5 * tau[((m * o + nn) * v + a) * v + b] * Wmnij[((m * o + nn) * o + i) * o + j];
                for (int e = 0; e < v; ++e)
                    #pragma unroll 4
                    for (int ff = 0; ff < v; ++ff)
                        x += 0.5 * tau[((i * o + j) * v + e) * v + ff] * Wabef[((a * v + b) * v + e) * v + ff];
                // P(ij) P(ab) sum_me (t_im^ae W_mbej - t_i^e t_m^a <mb||ej>)
                x += rq(i, a, j, b) - rq(j, a, i, b) - rq(i, b, j, a) + rq(j, b, i, a);
                // P(ij) sum_e t_i^e <ab||ej> - P(ab) sum_m t_m^a <mb||ij>
                #pragma unroll 4
                for (int e = 0; e < v; ++e)
                    x += t1(i, e) * asy(V0 + a, V0 + b, V0 + e, j) - t1(j, e) * asy(V0 + a, V0 + b, V0 + e, i);
                #pragma unroll 4
                for (int m = 0; m < o; ++m)
                    x -= t1(m, a) * asy(m, V0 + b, i, j) - t1(m, b) * asy(m, V0 + a, i, j);
                Tn[k] = x / (f[i][i] + f[j][j] - f[V0 + a][V0 + a] - f[V0 + b][V0 + b]);
            }
        }
        gsync();
        // DIIS: store the update and its change, extrapolate
        const int slot = it % kCcDiis;
        double dmax = 0.0;
        for (int64_t k = gid; k < L; k += gst) {
            const double d = Tn[k] - T[k];
            Hist[slot * L + k] = Tn[k];
            Err[slot * L + k] = d;
            dmax = fmax(dmax, fabs(d));
        }
        dmax = grid_red(dmax, true);
        nh = nh < kCcDiis ? nh + 1 : kCcDiis;
        for (int q = 0; q < nh; ++q) {
            double d = 0.0;
            for (int64_t k = gid; k < L; k += gst) d += Err[slot * L + k] * Err[q * L + k];
            d = grid_red(d, false);
            if (tid == 0) {
                B[slot][q] = d;
                B[q][slot] = d;
            }
        }
        __syncthreads();
        if (tid == 0) {
            // (nh + 1) x (nh + 1) system [B -1; -1 0] c = [0; -1] by Gaussian elimination, partial pivoting
            double M[kCcDiis + 1][kCcDiis + 2];
            const int m = nh;
            double scale = 0.0;
            for (int i = 0; i < m; ++i) scale = fmax(scale, B[i][i]);
            scale = scale > 0.0 ? 1.0 / scale : 1.0;
            for (int i = 0; i <= m; ++i) {
                for (int j = 0; j <= m; ++j) M[i][j] = (i < m && j < m) ? B[i][j] * scale : (i == m && j == m ? 0.0 : -1.0);
                M[i][m + 1] = i < m ? 0.0 : -1.0;
            }
            bool ok = true;
            for (int c = 0; c <= m && ok; ++c) {
                int piv = c;
                for (int r = c + 1; r <= m; ++r)
                    if (fabs(M[r][c]) > fabs(M[piv][c])) piv = r;
                if (!(fabs(M[piv][c]) > 1e-300)) {
                    ok = false;
                    break;
                }
                if (piv != c)
                    for (int j = 0; j <= m + 1; ++j) {
                        const double x = M[c][j];
                        M[c][j] = M[piv][j];
                        M[piv][j] = x;
                    }
                for (int r = c + 1; r <= m; ++r) {
                    const double g = M[r][c] / M[c][c];
                    for (int j = c; j <= m + 1; ++j) M[r][j] -= g * M[c][j];
                }
            }
            if (ok) {
                double x[kCcDiis + 1];
                for (int r = m; r >= 0; --r) {
                    double s = M[r][m + 1];
                    for (int j = r + 1; j <= m; ++j) s -= M[r][j] * x[j];
                    x[r] = s / M[r][r];
                }
                for (int i = 0; i < m; ++i) coef[i] = x[i];
            } else {
                for (int i = 0; i < m; ++i) coef[i] = (i == slot) ? 1.0 : 0.0;
            }
        }
        __syncthreads();
        for (int64_t k = gid; k < L; k += gst) {
            double x = 0.0;
            for (int q = 0; q < nh; ++q) x += coef[q] * Hist[q * L + k];
            T[k] = x;
        }
        gsync();
        // correlation energy
        double e = 0.0;
        for (int64_t k = gid; k < o2v2; k += gst) {
            const int b = k % v, a = (k / v) % v, j = (k / v / v) % o, i = k / v / v / o;
            e += Ioovv[k] * (0.25 * T[ov + k] + 0.5 * t1(i, a) * t1(j, b));
        }
        for (int64_t k = gid; k < ov; k += gst) e += f[k / v][V0 + k % v] * T[k];
        e_cc = grid_red(e, false);
        __syncthreads();
        if (dmax < A.tol && fabs(e_cc - e_old) < 1e-2 * A.tol) {
            conv = 1;
            break;
        }
        e_old = e_cc;
    }
    if (L == 0) conv = 1;
    double e_t = 0.0;
    if (conv && A.triples) {
        // unique triples i<j<k, a<b<c, ranked by combination index
        const int64_t nocc3 = (int64_t)o * (o - 1) * (o - 2) / 6, nvir3 = (int64_t)v * (v - 1) * (v - 2) / 6;
        auto unrank3 = [](int64_t r, int m, int &x, int &y, int &z) {
            // lexicographic: x < y < z < m
            for (x = 0;; ++x) {
                const int64_t c = (int64_t)(m - x - 1) * (m - x - 2) / 2;
                if (r < c) break;
                r -= c;
            }
            for (y = x + 1;; ++y) {
                const int64_t c = m - y - 1;
                if (r < c) break;
                r -= c;
            }
            z = y + 1 + (int)r;
        };
        for (int64_t k = gid; k < nocc3 * nvir3; k += gst) {
            int i, j, kk, a, b, c;
            unrank3(k / nvir3, o, i, j, kk);
            unrank3(k % nvir3, v, a, b, c);
            if (so_spin[i] + so_spin[j] + so_spin[kk] != so_spin[V0 + a] + so_spin[V0 + b] + so_spin[V0 + c])
                continue;   // spin-forbidden: no amplitude
            const int I[3] = {i, j, kk}, Av[3] = {a, b, c};
            double x = 0.0, y = 0.0;
            // P(i/jk): (i,j,k) +, (j,i,k) -, (k,j,i) -; the same for (a/bc)
            for (int pi = 0; pi < 3; ++pi) {
                const int p1 = I[pi], p2 = I[pi == 1 ? 0 : 1], p3 = I[pi == 2 ? 0 : 2];
                const double si = pi == 0 ? 1.0 : -1.0;
                for (int pa = 0; pa < 3; ++pa) {
                    const int q1 = Av[pa], q2 = Av[pa == 1 ? 0 : 1], q3 = Av[pa == 2 ? 0 : 2];
                    const double s = si * (pa == 0 ? 1.0 : -1.0);
                    double u = 0.0;
                    for (int e = 0; e < v; ++e) u += t2(p2, p3, q1, e) * asy(V0 + e, p1, V0 + q2, V0 + q3);
                    for (int m = 0; m < o; ++m) u -= t2(p1, m, q2, q3) * asy(m, V0 + q1, p2, p3);
                    x += s * u;
                    y += s * t1(p1, q1) * iovv(p2, p3, q2, q3);
                }
            }
            const double D = f[i][i] + f[j][j] + f[kk][kk] - f[V0 + a][V0 + a] - f[V0 + b][V0 + b] - f[V0 + c][V0 + c];
            e_t += x * (x + y) / D;
        }
        e_t = grid_red(e_t, false);
    }
    if (tid == 0 && rk == 0) {
        A.out[t] = conv ? A.e_const + eref + e_cc + e_t : __builtin_nan("");
        A.status[t] = conv ? 0 : 2;
    }
}

hipError_t launch_ccsd(const double *h, const double *eri, int n, const int32_t *act, const int32_t *nact,
                       const int32_t *core, const int32_t *ncore, int stride, int nalpha, int nbeta, double e_const,
                       int ntup, double *work, int64_t slice, int triples, int max_iter, double tol, double *out,
                       int32_t *status, hipStream_t s) {
    if (ntup <= 0) return hipSuccess;
    CcArgs a{h, eri, n, act, nact, core, ncore, stride, nalpha, nbeta, e_const, work, slice, triples, max_iter, tol,
             out, status, 1, nullptr};
    hipLaunchKernelGGL(k_ccsd, dim3(ntup), dim3(kCcThreads), 0, s, a);
    return hipGetLastError();
}

// Workgroups that can run one tuple cooperatively (all resident at once).
int ccsd_coop_wgs() {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)k_ccsd, kCcThreads, 0) != hipSuccess) return 1;
    return std::max(1, std::min(cus * per, kCcMaxWgs));
}

// One tuple on wgs workgroups in a cooperative launch (grid barriers between
// the phases); part holds 2 wgs doubles.
hipError_t launch_ccsd_coop(const double *h, const double *eri, int n, const int32_t *act, const int32_t *nact,
                            const int32_t *core, const int32_t *ncore, int stride, int nalpha, int nbeta,
                            double e_const, double *work, int64_t slice, int triples, int max_iter, double tol,
                            double *out, int32_t *status, int wgs, double *part, hipStream_t s) {
    CcArgs a{h, eri, n, act, nact, core, ncore, stride, nalpha, nbeta, e_const, work, slice, triples, max_iter, tol,
             out, status, wgs, part};
    void *args[] = {&a};
    return hipLaunchCooperativeKernel((const void *)k_ccsd, dim3(wgs), dim3(kCcThreads), args, 0, s);
}

}  // namespace mbefci

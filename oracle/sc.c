/*
 * ORACLE (test infrastructure only) -- plain Slater-Condon determinant FCI.
 *
 * Only tests, the smoke check and the CPU-baseline leg of the benchmark load
 * this file.  It shares no code with the HIP path.
 *
 * What it computes: matrix elements <I|H|J> of the second-quantised
 * Hamiltonian (spin labels u, v)
 *     H = E_const + sum_{pq,u} h_pq a+_{pu} a_{qu}
 *               + 1/2 sum_{pqrs,u,v} (pq|rs) a+_{pu} a+_{rv} a_{sv} a_{qu}
 *       = E_const + sum h_pq E_pq + 1/2 sum (pq|rs) (E_pq E_rs - d_qr E_ps)
 * (the CASCI energy of the paper's Sec. 2 is the lowest eigenvalue of this H
 * restricted to determinants with a fixed core and a fixed virtual set), over
 * determinants given as full-orbital-space bit strings (orbital p <-> bit p,
 * n <= 64), using the Slater-Condon rules for zero, one and two differing
 * spin orbitals.  A determinant is
 *     |Ia Ib> = (prod_{p in Ia, ascending} a+_{p,alpha})
 *               (prod_{p in Ib, ascending} a+_{p,beta}) |vac>,
 * i.e. all alpha creators to the left of all beta creators.  Phases are found
 * by applying the annihilation/creation operators to the bit strings one at a
 * time, never from a precomputed table.
 *
 * Integrals: h is n*n row-major; eri is n^4 row-major, eri[((p*n+q)*n+r)*n+s]
 * = (pq|rs) in chemists' notation.
 *
 * Determinant lists: alpha strings alist[0..na-1] and beta strings
 * blist[0..nb-1], each sorted ascending; determinant index = ia*nb + ib.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ERI(p, q, r, s) eri[(((size_t)(p) * n + (q)) * n + (r)) * n + (s)]

static int popc(uint64_t x) { return __builtin_popcountll(x); }
static int lowest(uint64_t x) { return __builtin_ctzll(x); }
static uint64_t bit(int p) { return (uint64_t)1 << p; }

/* (-1)^(number of set bits of s strictly below p) */
static int phase_below(uint64_t s, int p) {
    return (popc(s & (bit(p) - 1)) & 1) ? -1 : 1;
}

/* a_p acting on a one-spin string; returns 0 if p is empty */
static int ann(uint64_t *s, int p) {
    if (!(*s & bit(p))) return 0;
    int ph = phase_below(*s, p);
    *s ^= bit(p);
    return ph;
}

/* a+_p acting on a one-spin string; returns 0 if p is occupied */
static int cre(uint64_t *s, int p) {
    if (*s & bit(p)) return 0;
    int ph = phase_below(*s, p);
    *s |= bit(p);
    return ph;
}

/* energy of a single determinant (zero differences) */
static double diag_elem(int n, const double *h, const double *eri, uint64_t a, uint64_t b) {
    double e = 0.0;
    for (uint64_t x = a; x; x &= x - 1) {
        int i = lowest(x);
        e += h[i * n + i];
        for (uint64_t y = a; y; y &= y - 1) {
            int j = lowest(y);
            e += 0.5 * (ERI(i, i, j, j) - ERI(i, j, j, i));
        }
        for (uint64_t y = b; y; y &= y - 1) {
            int j = lowest(y);
            e += ERI(i, i, j, j);
        }
    }
    for (uint64_t x = b; x; x &= x - 1) {
        int i = lowest(x);
        e += h[i * n + i];
        for (uint64_t y = b; y; y &= y - 1) {
            int j = lowest(y);
            e += 0.5 * (ERI(i, i, j, j) - ERI(i, j, j, i));
        }
    }
    return e;
}

/*
 * <J|H|I> without E_const.  (Ia, Ib) is the ket, (Ja, Jb) the bra.
 */
double sc_element(int n, const double *h, const double *eri,
                  uint64_t Ia, uint64_t Ib, uint64_t Ja, uint64_t Jb) {
    int da = popc(Ia ^ Ja) / 2, db = popc(Ib ^ Jb) / 2;
    if (popc(Ia) != popc(Ja) || popc(Ib) != popc(Jb)) return 0.0;
    if (da + db > 2) return 0.0;
    if (da + db == 0) return diag_elem(n, h, eri, Ia, Ib);

    if (da + db == 1) {
        /* one spin orbital differs: i -> a in spin "same"; "other" is spectator */
        uint64_t same = da ? Ia : Ib, other = da ? Ib : Ia;
        uint64_t tgt = da ? Ja : Jb;
        int i = lowest(same & ~tgt), a = lowest(tgt & ~same);
        uint64_t s = same;
        int ph = ann(&s, i);
        ph *= cre(&s, a);
        double v = h[a * n + i];
        for (uint64_t y = same; y; y &= y - 1) {
            int j = lowest(y);
            if (j == i) continue;
            v += ERI(a, i, j, j) - ERI(a, j, j, i);
        }
        for (uint64_t y = other; y; y &= y - 1) {
            int j = lowest(y);
            v += ERI(a, i, j, j);
        }
        return ph * v;
    }

    if (da == 1 && db == 1) {
        int i = lowest(Ia & ~Ja), a = lowest(Ja & ~Ia);
        int j = lowest(Ib & ~Jb), b = lowest(Jb & ~Ib);
        uint64_t sa = Ia, sb = Ib;
        int ph = ann(&sa, i);
        ph *= cre(&sa, a);
        ph *= ann(&sb, j);
        ph *= cre(&sb, b);
        return ph * ERI(a, i, b, j);
    }

    /* two spin orbitals of the same spin differ */
    uint64_t same = da ? Ia : Ib, tgt = da ? Ja : Jb;
    uint64_t rem = same & ~tgt, add = tgt & ~same;
    int i = lowest(rem), j = lowest(rem & (rem - 1));
    int a = lowest(add), b = lowest(add & (add - 1));
    uint64_t s = same;
    /* a+_a a+_b a_j a_i |same> */
    int ph = ann(&s, i);
    ph *= ann(&s, j);
    ph *= cre(&s, b);
    ph *= cre(&s, a);
    return ph * (ERI(a, i, b, j) - ERI(a, j, b, i));
}

/* Dense H over the determinant list (row-major ndet x ndet), E_const added on
 * the diagonal.  Every pair is evaluated by sc_element. */
void sc_hmat(int n, const double *h, const double *eri, double e_const,
             int64_t na, const uint64_t *alist, int64_t nb, const uint64_t *blist,
             double *H) {
    int64_t nd = na * nb;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t I = 0; I < nd; ++I) {
        uint64_t Ia = alist[I / nb], Ib = blist[I % nb];
        for (int64_t J = 0; J < nd; ++J) {
            uint64_t Ja = alist[J / nb], Jb = blist[J % nb];
            double v = sc_element(n, h, eri, Ja, Jb, Ia, Ib);
            if (I == J) v += e_const;
            H[I * nd + J] = v;
        }
    }
}

static int64_t find(const uint64_t *list, int64_t len, uint64_t key) {
    int64_t lo = 0, hi = len - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (list[mid] == key) return mid;
        if (list[mid] < key) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* Enumerate every single and double excitation of one spin string inside the
 * orbital set `act` into `out`.  Each distinct excited string is produced
 * exactly once. */
typedef struct {
    uint64_t *s;
    int64_t cnt;
} strlist;

static int64_t choose2(int64_t k) { return k * (k - 1) / 2; }

/* room for every single and double excitation of any string inside `nact`
 * orbitals */
static strlist *strlist_new(int nact) {
    int64_t best = 0;
    for (int o = 0; o <= nact; ++o) {
        int64_t v = nact - o, m = (int64_t)o * v + choose2(o) * choose2(v);
        if (m > best) best = m;
    }
    strlist *l = (strlist *)malloc(sizeof(strlist));
    l->s = (uint64_t *)malloc((size_t)(best + 1) * sizeof(uint64_t));
    l->cnt = 0;
    return l;
}

static void strlist_free(strlist *l) { free(l->s); free(l); }

static void excitations(uint64_t s, uint64_t act, int max_rank, strlist *out) {
    out->cnt = 0;
    uint64_t occ = s & act, vir = act & ~s;
    for (uint64_t x = occ; x; x &= x - 1) {
        int i = lowest(x);
        for (uint64_t y = vir; y; y &= y - 1) {
            int a = lowest(y);
            out->s[out->cnt++] = (s ^ bit(i)) | bit(a);
        }
    }
    if (max_rank < 2) return;
    for (uint64_t x = occ; x; x &= x - 1) {
        int i = lowest(x);
        for (uint64_t x2 = x & (x - 1); x2; x2 &= x2 - 1) {
            int j = lowest(x2);
            for (uint64_t y = vir; y; y &= y - 1) {
                int a = lowest(y);
                for (uint64_t y2 = y & (y - 1); y2; y2 &= y2 - 1) {
                    int b = lowest(y2);
                    out->s[out->cnt++] = (s ^ bit(i) ^ bit(j)) | bit(a) | bit(b);
                }
            }
        }
    }
}

/* y = H x (E_const included) over the determinant list, matrix-free.  The
 * determinants connected to row I are I itself, its alpha and beta single and
 * double excitations inside `act`, and the products of one alpha and one beta
 * single excitation; every element comes from sc_element. */
void sc_matvec(int n, const double *h, const double *eri, double e_const,
               int64_t na, const uint64_t *alist, int64_t nb, const uint64_t *blist,
               uint64_t act, const double *x, double *y) {
    int64_t nd = na * nb;
#pragma omp parallel
    {
        int nact = popc(act);
        strlist *ea = strlist_new(nact), *eb = strlist_new(nact);
        strlist *sa = strlist_new(nact), *sb = strlist_new(nact);
#pragma omp for schedule(dynamic, 64)
        for (int64_t I = 0; I < nd; ++I) {
            int64_t ia = I / nb, ib = I % nb;
            uint64_t Ia = alist[ia], Ib = blist[ib];
            double acc = (diag_elem(n, h, eri, Ia, Ib) + e_const) * x[I];
            excitations(Ia, act, 2, ea);
            excitations(Ib, act, 2, eb);
            for (int64_t k = 0; k < ea->cnt; ++k) {
                int64_t ja = find(alist, na, ea->s[k]);
                if (ja < 0) continue;
                int64_t J = ja * nb + ib;
                acc += sc_element(n, h, eri, ea->s[k], Ib, Ia, Ib) * x[J];
            }
            for (int64_t k = 0; k < eb->cnt; ++k) {
                int64_t jb = find(blist, nb, eb->s[k]);
                if (jb < 0) continue;
                int64_t J = ia * nb + jb;
                acc += sc_element(n, h, eri, Ia, eb->s[k], Ia, Ib) * x[J];
            }
            excitations(Ia, act, 1, sa);
            excitations(Ib, act, 1, sb);
            for (int64_t k = 0; k < sa->cnt; ++k) {
                int64_t ja = find(alist, na, sa->s[k]);
                if (ja < 0) continue;
                for (int64_t l = 0; l < sb->cnt; ++l) {
                    int64_t jb = find(blist, nb, sb->s[l]);
                    if (jb < 0) continue;
                    acc += sc_element(n, h, eri, sa->s[k], sb->s[l], Ia, Ib) * x[ja * nb + jb];
                }
            }
            y[I] = acc;
        }
        strlist_free(ea); strlist_free(eb); strlist_free(sa); strlist_free(sb);
    }
}

/* Apply a (spin, orbital) annihilator or creator to a determinant (a, b).
 * A beta operator passes all alpha creators: factor (-1)^{N_alpha}. */
static int op(uint64_t *a, uint64_t *b, int spin, int p, int create) {
    if (spin == 0) return create ? cre(a, p) : ann(a, p);
    int ph = (popc(*a) & 1) ? -1 : 1;
    int r = create ? cre(b, p) : ann(b, p);
    return r ? ph * r : 0;
}

/*
 * One- and two-particle density matrices of the normalised vector c over the
 * determinant list, by explicit operator action:
 *   gamma[p*n+q]            = sum_s  <c| a+_{ps} a_{qs} |c>
 *   Gamma[((p*n+q)*n+r)*n+s] = sum_{st} <c| a+_{ps} a+_{rt} a_{st} a_{qs} |c>
 * (spin labels s, t).  Determinants produced outside the list have zero
 * amplitude and are skipped.  Accumulation is per ket determinant into
 * thread-private arrays, reduced at the end.
 */
void sc_rdm12(int n, int64_t na, const uint64_t *alist, int64_t nb, const uint64_t *blist,
              const double *c, double *gamma, double *Gamma) {
    int64_t nd = na * nb;
    size_t n2 = (size_t)n * n, n4 = n2 * n2;
    memset(gamma, 0, n2 * sizeof(double));
    memset(Gamma, 0, n4 * sizeof(double));
#pragma omp parallel
    {
        double *g1 = (double *)calloc(n2, sizeof(double));
        double *g2 = (double *)calloc(n4, sizeof(double));
#pragma omp for schedule(dynamic, 16)
        for (int64_t J = 0; J < nd; ++J) {
            double cj = c[J];
            if (cj == 0.0) continue;
            uint64_t Ja = alist[J / nb], Jb = blist[J % nb];
            for (int s1 = 0; s1 < 2; ++s1)
                for (int q = 0; q < n; ++q) {
                    uint64_t a1 = Ja, b1 = Jb;
                    int f1 = op(&a1, &b1, s1, q, 0);
                    if (!f1) continue;
                    /* one-body: a+_p a_q */
                    for (int p = 0; p < n; ++p) {
                        uint64_t a2 = a1, b2 = b1;
                        int f2 = op(&a2, &b2, s1, p, 1);
                        if (!f2) continue;
                        int64_t ka = find(alist, na, a2), kb = find(blist, nb, b2);
                        if (ka < 0 || kb < 0) continue;
                        g1[p * n + q] += f1 * f2 * c[ka * nb + kb] * cj;
                    }
                    /* two-body: a+_p a+_r a_s a_q, applied right to left */
                    for (int s2 = 0; s2 < 2; ++s2)
                        for (int s = 0; s < n; ++s) {
                            uint64_t a2 = a1, b2 = b1;
                            int f2 = op(&a2, &b2, s2, s, 0);
                            if (!f2) continue;
                            for (int r = 0; r < n; ++r) {
                                uint64_t a3 = a2, b3 = b2;
                                int f3 = op(&a3, &b3, s2, r, 1);
                                if (!f3) continue;
                                for (int p = 0; p < n; ++p) {
                                    uint64_t a4 = a3, b4 = b3;
                                    int f4 = op(&a4, &b4, s1, p, 1);
                                    if (!f4) continue;
                                    int64_t ka = find(alist, na, a4), kb = find(blist, nb, b4);
                                    if (ka < 0 || kb < 0) continue;
                                    g2[(((size_t)p * n + q) * n + r) * n + s] +=
                                        f1 * f2 * f3 * f4 * c[ka * nb + kb] * cj;
                                }
                            }
                        }
                }
        }
#pragma omp critical
        {
            for (size_t k = 0; k < n2; ++k) gamma[k] += g1[k];
            for (size_t k = 0; k < n4; ++k) Gamma[k] += g2[k];
        }
        free(g1);
        free(g2);
    }
}

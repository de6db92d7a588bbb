/*
 * mbefci.h -- C ABI of the MI355X MBE-FCI library (libmbefci.so).
 *
 * What the library computes (Eriksen & Gauss, "Many-Body Expanded Full
 * Configuration Interaction. II. Strongly Correlated Regime"):
 *
 *   * Sec. 2, Eq. 3: for every tuple S of expansion orbitals, the CASCI energy
 *     eps(S) in the composite space A = [Pi] u S of the reference space [Pi] and
 *     the tuple, every other occupied orbital frozen doubly occupied; and the
 *     increment d_eps(S) = eps(S) - sum_{T proper subtuple of S} d_eps(T) with
 *     d_eps({}) = eps([Pi]).
 *   * Eq. 1: the order sums E^(k) = sum_{|S| = k} d_eps(S) and their total.
 *   * The screening threshold a (Sec. 4.1, "a = 5.0" / "a = 2.5"); the rule is
 *     a reading, stated at mbefci_options.a.
 *
 * Conventions that hold for every call:
 *   * Every function returns mbefci_status: 0 on success, < 0 on error; no C++
 *     exception crosses the ABI.  mbefci_last_error() gives a message.
 *   * Orbital indices are 0-based.  Occupied orbitals are chosen by index:
 *     alpha 0..nalpha-1, doubly occupied 0..nbeta-1 (nalpha >= nbeta).  The
 *     singly occupied orbitals nbeta..nalpha-1 must lie in [Pi] (the paper's
 *     open-shell case (b)).  Orbitals 0..nfrozen-1 are frozen (Sec. 3).
 *     Expansion space X = all orbitals outside the frozen set and [Pi].
 *   * For a tuple S: A = [Pi] u S (ascending), core C = frozen u (docc \ A),
 *     active electrons nalpha - |C| and nbeta - |C|.
 *   * Determinants of a CAS are ordered alpha-string-major: index
 *     ia * n_beta_strings + ib, strings ascending as bit masks over the
 *     positions of A, determinant = core creators, then active alpha creators
 *     (ascending), then active beta creators (ascending).  Against creators
 *     ordered over the whole orbital space a determinant differs by the sign
 *     (-1)^(pairs of an active electron below a core orbital, per spin); the
 *     spectrum is the same.
 *   * The caller owns every host array and the device workspace.  The library
 *     copies what it keeps (integrals, spaces, options).  All device work is
 *     enqueued on the stream given at creation; host outputs are complete
 *     (stream synchronised) when a call returns.
 *   * Energies are in hartree, FP64 end to end.
 */
#ifndef MBEFCI_H
#define MBEFCI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mbefci_ctx mbefci_ctx;         /* opaque; create/destroy below */
typedef struct mbefci_result mbefci_result;   /* opaque; owned until mbefci_result_free */

typedef enum {
    MBEFCI_OK = 0,
    MBEFCI_EINVAL = -1,     /* bad argument (non-finite or non-symmetric h, bad tuple, ...) */
    MBEFCI_ENOMEM = -2,     /* device workspace too small for even one tuple */
    MBEFCI_EDEVICE = -3,    /* a HIP runtime call failed */
    MBEFCI_ENOCONV = -4,    /* at least one tuple did not converge; per-tuple status filled */
    MBEFCI_ESTATE = -5,     /* call out of order (no Hamiltonian, host-only context, ...) */
    MBEFCI_ETOOLARGE = -6   /* a CAS exceeds the kernels' limits (more than 13 active orbitals) */
} mbefci_status;

/* per-tuple solve status */
enum {
    MBEFCI_TUPLE_OK = 0,        /* converged */
    MBEFCI_TUPLE_MAXITER = 1,   /* iteration limit reached */
    MBEFCI_TUPLE_NONFINITE = 2, /* NaN/Inf met in the iteration */
    MBEFCI_TUPLE_STALLED = 3,   /* correction vector fell inside the subspace before convergence */
    MBEFCI_TUPLE_PENDING = 4    /* listed in an open (streamed) order, not solved yet */
};

typedef enum {
    MBEFCI_ERI_FULL = 0,        /* n^4 row-major, eri[((p*n+q)*n+r)*n+s] = (pq|rs) */
    MBEFCI_ERI_PACKED8 = 1      /* unique elements: P = p(p+1)/2+q (p>=q), R likewise,
                                   element [P(P+1)/2 + R] for P >= R */
} mbefci_eri_layout;

typedef struct {
    /* Screening (a reading: the paper names the threshold a, larger a = more
     * aggressive).  tau_k = 1e-10 * a^(k-1) for increments of order k; an
     * order-(k+1) tuple is computed iff at least one of its k-subtuples was
     * computed at order k with |d_eps| >= tau_k.  Order 1 is never screened.
     * a <= 0 disables screening. */
    double a;
    int32_t max_order;      /* highest order; <= 0 means |X| (full order) */
    double e_tol;           /* Davidson: |theta - theta_prev| bound (default 1e-11) */
    double r_tol;           /* Davidson: residual 2-norm bound (default 1e-6; the Ritz value
                               then lies within about r_tol^2 / gap of the eigenvalue) */
    int32_t max_iter;       /* Davidson iterations per tuple in the first pass (default 300); a
                               tuple that does not converge (iteration limit or stalled) is
                               solved again in a second pass with a subspace of 32, no P space
                               and max(10 max_iter, 3000) iterations, and a shape class whose
                               first batch sends a quarter or more of its tuples there runs its
                               remaining batches with those settings.  The status is that of the
                               second pass. */
    int32_t max_space;      /* subspace vectors before restart, 2..32 (default 12) */
    int32_t batched;        /* 1: every tuple of a shape class in one batch of launches;
                               0: one tuple per launch sequence (the per-solve path) */
    int32_t gradient;       /* 1: mbefci_run also forms the gradient of the total with respect to
                               h1 and (pq|rs) (density matrices of every tuple at convergence,
                               weighted as at mbefci_backward, the last order's on the device as
                               it converges), kept in the result, so that mbefci_backward solves
                               nothing again.  Such a run, every backward pass and
                               mbefci_tuple_rdm converge each tuple to r_tol <= 1e-9 and
                               e_tol <= 1e-12 whatever the options say:
                               density matrices are first order in the residual.  Needs n^2 + n^4
                               doubles of workspace beyond the batches. (default 0) */
    int32_t profile;        /* 1: time every sigma launch with HIP events (mbefci_get_stats) */
    int32_t sigma_variant;  /* 0: automatic; 1: column strip (W kept in LDS, beta-beta part as a
                               GEMM with the dense beta-string Hamiltonian); 2: W materialised
                               in the workspace and gathered back.  1 falls back to 2 when the
                               strip does not fit in LDS (more than ~1100 alpha strings). */
    int32_t pspace;         /* Davidson preconditioner: the exact inverse of (theta - H) on the
                               pspace determinants of lowest diagonal energy, (theta - H_II)^-1
                               elsewhere; 0..128, 0 = diagonal only (default 128).  Only for
                               column-strip classes; the result does not depend on it beyond
                               the convergence tolerances. */
    int32_t linked_rows;    /* column-strip alpha-beta term: 0 forms all P_A pair rows of W; 1
                               (default) forms only the pair rows that link each alpha string
                               to another (1 + n_a (n_A - n_a) rows, at most 32; the diagonal
                               pairs summed first) where n_A >= 9 and they fit, with the A rows
                               resident in LDS where that fits and there are at least as many
                               alpha strings as pair rows, else gathered per string; where the
                               n_a (n_A - n_a) off-diagonal rows alone fill the 32 slots (n_A =
                               12 with 4 or 8 alpha electrons) the diagonal row goes to the
                               vector ALU (A rows resident, two halves of four waves); 2 and 3
                               use linked rows wherever they fit (n_A >= 4), 2 with the A rows
                               gathered, 3 resident (each where it fits, else the other); 4 the
                               vector-ALU diagonal form wherever it fits.  Where neither LDS form
                               fits (n_A = 12 at 5 or 6 electrons of the spin, whose sigma strips
                               fill the LDS) the linked rows, up to 48, are written to the
                               workspace and gathered back per target string; 5 uses that form
                               wherever it fits.  Same result up to rounding. */
    int32_t stream_last;    /* 1: mbefci_run solves orders 0 .. K-1 and only lists the last order K
                               (its tuples generated, status MBEFCI_TUPLE_PENDING), which the
                               caller then solves in slices with mbefci_order_solve and ends with
                               mbefci_order_close: the same result as one call, for orders too
                               large to solve in one go (default 0) */
    int32_t graph;          /* with profile = 0 the Davidson iterations of a batch run in blocks of
                               4-8 launched back to back (the running count is read once per
                               block; finished tuples are skipped by every kernel), and with
                               graph = 1 (default) one iteration's launches are captured once per
                               batch in a hipGraph on a private stream and replayed on the
                               context's stream.  profile = 1 keeps one host round trip per
                               iteration (every sigma launch timed).  Same results. */
    int32_t autotune;       /* 1 (default): with the automatic settings (linked_rows 1,
                               sigma_variant 0) the alpha-beta sigma form and the GEMM tile of
                               every shape class of at least 10^4 determinants are chosen by
                               timing one sigma of each candidate on up to 16 of its tuples, once
                               per process and device (the choice is kept, so repeated runs are
                               bitwise identical; processes can differ in the last bits) */
    int32_t restart_keep;   /* vectors a Davidson restart keeps: 1 the Ritz vector alone; 2
                               (default) also the previous iteration's Ritz vector made
                               orthogonal to it (where that direction is not negligible), as in
                               the locally optimal restarts of Murray, Racine and Davidson and of
                               Stathopoulos, Saad and Wu.  Same eigenvalue within the tolerances;
                               fewer iterations where restarts are frequent. */
    double spin_shift;      /* lambda >= 0 (default 0: off).  Spin-targeted CASCI: every tuple takes
                               the lowest eigenvalue of H + lambda S_- S_+ over its CAS instead of
                               H's, i.e. of its lowest state of total spin S = (n_alpha - n_beta) / 2
                               (the lowest singlet for closed shells).  S_- S_+ = N_beta -
                               sum_pq E^alpha_qp E^beta_pq is zero on the states of that spin and at
                               least lambda (S'(S'+1) - S(S+1)) on a state of spin S', so lambda must
                               exceed the energy by which the lowest state of any higher spin lies
                               below the target, divided by that factor; the energy returned is the
                               state's own (the shift vanishes on it).  The paper's energies are those
                               of singlet ground states (Sec. 4); the diagonal and the P space include
                               the shift. */
    int32_t whole_dim;      /* whole-tuple mode: with profile = 0, shape classes of at most this many
                               determinants (0..4900, default 1225; 0: off) and at most 10 active
                               orbitals run each tuple's whole Davidson solve in one workgroup of a
                               single launch (the batched path launches a dozen kernels per
                               iteration); their P space is at most 32 determinants unless it holds
                               the whole CAS.  Above about 1225 determinants the batched path's
                               MFMA sigma is faster.  Same energies within the tolerances. */
    int32_t base_model;     /* 0 (default): none.  1: the expansion of eps(S) - eps_base(S) with a
                               second-order base (MBE-FCI-b, Sec. 4.2.1 and Table 3, where the base
                               is CCSD(T)): eps_base(S) = <Phi|H|Phi> minus the second-order
                               Rayleigh-Schroedinger sum over the single and double excitations of
                               Phi within the tuple's CAS, Phi the determinant with the core doubly
                               occupied and the active orbitals of index below n_alpha (n_beta)
                               occupied by alpha (beta) electrons, H0 the diagonal of Phi's
                               spin-orbital Fock operator.  The orders' eps are then eps - eps_base,
                               screening acts on their increments, and the total adds the base
                               energy of the whole space (mbefci_result_base).  EINVAL with
                               options.gradient, and when an excitation does not raise the
                               zeroth-order energy (an intruder: the orbitals must be ordered like
                               canonical ones).  2: the same expansion with a CCSD base, 3: with the
                               paper's CCSD(T) base: spin-orbital CCSD on the same Phi within the
                               tuple's CAS (any orbitals; at most 32 active orbitals per tuple), the
                               amplitudes converged to a largest change of 1e-11 (ENOCONV after 300
                               iterations; EINVAL when an orbital energy difference of Phi is not
                               negative), and for 3 the (T) correction, which needs canonical
                               orbitals (EINVAL unless the Fock operator of Phi is diagonal to
                               1e-10 on the reference and expansion orbitals). */
    double sym_shift;       /* lambda >= 0 of a level shift toward spatial symmetry irrep (0: none):
                               sigma += lambda [irrep(I) != irrep] c(I), the irrep of a determinant
                               the XOR of the labels (mbefci_set_orbital_irreps) of its occupied
                               spin-orbitals; every CASCI energy is then that of the lowest state of
                               that irrep (the paper's states of given symmetry, Sec. 4.1) when
                               lambda exceeds its distance to the lowest state of the CAS.  Needs
                               labels that the Hamiltonian respects (EINVAL otherwise, checked to
                               1e-12 when a solve starts) and a determinant of the irrep in every
                               tuple's CAS (EINVAL otherwise). */
    int32_t irrep;          /* target irrep label 0..7 (with sym_shift > 0) */
} mbefci_options;

typedef struct {
    int64_t ntuples;            /* tuples solved by the last solve/run call */
    int64_t sigma_calls;        /* sigma applications (one per tuple per iteration) */
    int64_t sigma_launches;     /* launches of the dominant sigma kernel */
    double sigma_flops;         /* algorithmic FLOPs, 2 * R * P_A * dim per application: R = P_A pair
                                   rows, or 1 + n_a (n_A - n_a) with linked rows */
    double sigma_bytes;         /* algorithmic bytes, 16 * dim + 8 * P_A^2 per application */
    double sigma_ms;            /* HIP-event time of the dominant sigma kernel (profile = 1) */
    double sigma_total_ms;      /* HIP-event time of all sigma kernels (profile = 1) */
    int64_t iterations_total;   /* Davidson iterations summed over tuples */
    int64_t iterations_max;
    double solve_ms;            /* host wall time inside solve/run */
    int64_t gs_second_pass;     /* Davidson corrections that took two explicit Gram-Schmidt passes (the
                                   rest join the subspace unchanged: it keeps V = Q U, U triangular) */
    int64_t second_pass;        /* tuples solved again in the second pass (see max_iter) */
    double gather_ms;           /* HIP-event time of the gather of the W-in-HBM linked form (profile = 1;
                                   sigma_ms holds that form's MFMA kernel alone) */
    int64_t graph_batches;      /* batches whose iteration ran as a captured hipGraph */
    int64_t tuned_classes;      /* shape classes timed by the autotuner in this call */
    int64_t whole_batches;      /* batches solved in whole-tuple mode (options.whole_dim) */
} mbefci_stats;

/* Counters of one shape class (active orbitals, active alpha and beta
 * electrons) in the last solve/run call; times need profile = 1. */
typedef struct {
    int32_t n_active, n_alpha, n_beta;
    int32_t kernel;             /* alpha-beta sigma kernel: 0 k_sigma_strip (all pair rows),
                                   1 k_sigma_linked_gat, 2 k_sigma_linked_res, 3 k_sigma_linked_dv,
                                   4 k_sigma_w + k_sigma_g (W materialised), 5 k_linked_wr +
                                   k_linked_gw (linked rows through W in the workspace), 6 whole-
                                   tuple mode (k_whole: sigma by link pairs inside the solve) */
    int64_t dim;                /* determinants per tuple */
    int64_t tuples, iterations, sigma_calls, sigma_launches;
    double sigma_flops;         /* as mbefci_stats.sigma_flops */
    double sigma_ms;            /* HIP-event time of the alpha-beta kernel (the MFMA kernel of kernel 5) */
    double gather_ms;           /* of the gather of kernel 5 */
    double sigma_total_ms;      /* of all sigma kernels (with the string-Hamiltonian GEMMs) */
    double wall_ms;             /* host wall time of the class's batches */
} mbefci_class_stats;

/* Library version string. */
const char *mbefci_version(void);

/* Fill `opt` with the defaults listed at mbefci_options. */
void mbefci_default_options(mbefci_options *opt);

/* Create a context on HIP device `hip_device` (>= 0) using `hip_stream`
 * (a hipStream_t, NULL = the default stream).  hip_device = -1 creates a
 * host-only context: the planner (mbefci_run_host) works, device calls return
 * MBEFCI_ESTATE. */
mbefci_status mbefci_create(mbefci_ctx **ctx, int32_t hip_device, void *hip_stream);
void mbefci_destroy(mbefci_ctx *ctx);

/* Message of the last failing call on `ctx` (valid until the next call). */
const char *mbefci_last_error(const mbefci_ctx *ctx);

/* Hamiltonian in an orthonormal MO basis: h1 (norb*norb, symmetric within
 * 1e-12, finite), eri in `layout` (8-fold symmetric), constant e_const.
 * Copied; on a device context the integrals are kept resident on the device
 * (n^4 doubles, allocated by the library).  EINVAL on norb < 1 or > 64,
 * non-finite or non-symmetric input. */
mbefci_status mbefci_set_hamiltonian(mbefci_ctx *ctx, int32_t norb, const double *h1,
                                     const double *eri, mbefci_eri_layout layout,
                                     double e_const);

/* Electrons (totals, frozen core included), frozen orbitals 0..nfrozen-1 and
 * the reference space [Pi] (ref_orbs[0..nref-1], any order, no duplicates,
 * disjoint from the frozen set; nref may be 0).  EINVAL when a singly occupied
 * orbital is outside [Pi] or a frozen orbital is not doubly occupied. */
mbefci_status mbefci_set_spaces(mbefci_ctx *ctx, int32_t nalpha, int32_t nbeta, int32_t nfrozen,
                                const int32_t *ref_orbs, int32_t nref);

/* Pi-pruning (Sec. 3; Sec. 4.1.2, Table 2): npairs pairs of expansion
 * orbitals orbs[2i], orbs[2i+1] (the x and y components of a degenerate pi
 * pair; no orbital twice); increments are then computed only for tuples that
 * hold both components of every pair or neither.  Under screening an order-k
 * tuple is computed iff it adds one unpaired orbital to an order-(k-1) tuple
 * with |d_eps| >= tau_{k-1}, or one whole pair to an order-(k-2) tuple with
 * |d_eps| >= tau_{k-2} (the empty tuple always counts; a reading, as the rule
 * at mbefci_options.a); without screening every such tuple is computed.  An
 * order without tuples then ends the expansion only if the order before it
 * had none either.  npairs = 0 clears; mbefci_set_spaces clears too.  EINVAL
 * for an orbital outside X or in two pairs; ESTATE before mbefci_set_spaces. */
mbefci_status mbefci_set_pi_pairs(mbefci_ctx *ctx, const int32_t *orbs, int32_t npairs);

mbefci_status mbefci_set_options(mbefci_ctx *ctx, const mbefci_options *opt);

/* Device bytes needed to solve the given tuples: *min_bytes holds the
 * largest single tuple (one at a time), *want_bytes every tuple of the largest
 * shape class in one batch.  tuples: host int16, ntup rows of `order`
 * ascending expansion orbitals. */
mbefci_status mbefci_workspace_query(mbefci_ctx *ctx, int32_t order, int64_t ntup,
                                     const int16_t *tuples, size_t *min_bytes,
                                     size_t *want_bytes);

/* CASCI energies eps(S) (Sec. 2) of `ntup` tuples of one order.  d_workspace
 * is device memory of ws_bytes (e.g. a torch uint8 tensor) that must outlive
 * the call; tuples are split into batches that fit it.  energies/status are
 * host outputs of length ntup.  EINVAL for an unsorted or duplicated tuple, an
 * orbital outside X; ENOMEM if one tuple does not fit; ENOCONV if a tuple
 * failed (its status says why; its energy is the last Ritz value). */
mbefci_status mbefci_solve_tuples(mbefci_ctx *ctx, int32_t order, int64_t ntup,
                                  const int16_t *tuples, void *d_workspace, size_t ws_bytes,
                                  double *energies, int32_t *status);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * mbefci_solve_tuples with the workspace taken from a static device array of
 * 128 MiB that the library holds on every GPU it runs on until the process
 * ends (allocated with the code object, never by this call; the call itself
 * makes no hipMalloc, hipFree or other allocating device call).  Same
 * arguments, results and errors as mbefci_solve_tuples, plus ENOMEM when one
 * tuple needs more than 128 MiB (see mbefci_workspace_query); batches are cut
 * to fit.  Every call on one GPU shares that GPU's array, and the array keeps
 * the last call's contents (nothing in it is read before it is written):
 * calls that overlap on one GPU -- two contexts on one device, or two host
 * threads -- race and must be serialised by the caller. */
mbefci_status mbefci_solve_tuples_noalloc(mbefci_ctx *ctx, int32_t order, int64_t ntup,
                                          const int16_t *tuples, double *energies, int32_t *status);

/* The whole expansion (Eq. 1-3): order 0 ([Pi] alone), then orders 1.. up to
 * max_order, |X| or until screening leaves no tuple.  *out receives a result
 * owned by the caller (mbefci_result_free).  ENOCONV leaves *out valid. */
mbefci_status mbefci_run(mbefci_ctx *ctx, void *d_workspace, size_t ws_bytes,
                         mbefci_result **out);

/* Host-only variant of mbefci_run: the same tuple generation, screening and
 * increment assembly, with tuple energies supplied by `energy` (called once per
 * order with that order's tuple list; return 0 on success).  Works on a
 * host-only context. */
typedef int (*mbefci_energy_fn)(void *user, int32_t order, int64_t ntup,
                                const int16_t *tuples, double *energies);
mbefci_status mbefci_run_host(mbefci_ctx *ctx, mbefci_energy_fn energy, void *user,
                              mbefci_result **out);

/* Streamed last order (options.stream_last = 1; the paper's task farm over one
 * order, Sec. 4.2.3).  mbefci_order_solve solves the tuples first + i * stride,
 * i < count, of the open order of `res` (indices into its lexicographic list):
 * CASCI energies, increments against the completed lower orders (Eq. 3), and
 * with options.gradient their density matrices, weight 1 (no computed
 * superset), added to the result's gradient (n^2 + n^4 doubles of the
 * workspace used on the way).  Each tuple is solved once: EINVAL for a slice
 * outside the order or a tuple already solved; ESTATE without an open order;
 * ENOCONV as at mbefci_solve_tuples.  mbefci_order_close checks that every
 * tuple is solved (else ESTATE), forms the order sum and the total, and
 * closes the order; mbefci_backward refuses a result with an open order. */
mbefci_status mbefci_order_solve(mbefci_ctx *ctx, mbefci_result *res, int64_t first, int64_t stride,
                                 int64_t count, void *d_workspace, size_t ws_bytes);
mbefci_status mbefci_order_close(mbefci_ctx *ctx, mbefci_result *res);

int32_t mbefci_result_norders(const mbefci_result *res);     /* orders 0..norders-1 */
/* Views of order k (valid until mbefci_result_free): tuples [ntup*k] int16
 * lexicographic, eps, d_eps and status [ntup], order sum E^(k), and the host
 * wall time of the order in ms (tuple list ready -> increments assembled). */
mbefci_status mbefci_result_order(const mbefci_result *res, int32_t k, int64_t *ntup,
                                  const int16_t **tuples, const double **eps,
                                  const double **dinc, const int32_t **status,
                                  double *order_sum, double *wall_ms);
double mbefci_result_total(const mbefci_result *res);       /* sum of the order sums (plus the base
                                                               energy of the whole space with a base model) */
double mbefci_result_base(const mbefci_result *res);        /* base energy of the whole space (0: no base model) */
void mbefci_result_free(mbefci_result *res);

/* sigma = H c for the CAS of one tuple (E_core and E_const included, so H is
 * the projected full Hamiltonian), for `nvec` vectors stored one after the
 * other (dim doubles each) at device pointers d_c / d_sigma (non-overlapping).
 * The kernels are the ones the Davidson solver uses. */
mbefci_status mbefci_tuple_sigma(mbefci_ctx *ctx, int32_t order, const int16_t *tuple,
                                 void *d_workspace, size_t ws_bytes, const double *d_c,
                                 double *d_sigma, int32_t nvec);

/* Diagonal H_II (E_core included) of the CAS of one tuple into d_hdiag [dim]. */
mbefci_status mbefci_tuple_hdiag(mbefci_ctx *ctx, int32_t order, const int16_t *tuple,
                                 void *d_workspace, size_t ws_bytes, double *d_hdiag);

/* Host query of one tuple's CAS: number of alpha and beta strings (dim is
 * their product), active orbitals and active electrons. */
mbefci_status mbefci_tuple_shape(mbefci_ctx *ctx, int32_t order, const int16_t *tuple,
                                 int64_t *n_alpha_strings, int64_t *n_beta_strings,
                                 int32_t *n_active, int32_t *n_alpha_active,
                                 int32_t *n_beta_active);

/* String and single-excitation tables of one shape (host only, no context):
 * the C(norb_active, nel) strings as ascending bit masks, and for every string
 * I its n_entries = nel*(norb_active-nel) + nel entries (p, q) with q in I and
 * p not in I or p = q, encoding E_pq|I> = sign |J>: bits 0-19 = J, bits 20-29
 * = pair index P = max(p,q)(max(p,q)+1)/2 + min(p,q), bit 31 = 1 for sign -1.
 * Pass NULL arrays to query n_strings / n_entries only. */
mbefci_status mbefci_string_tables(int32_t norb_active, int32_t nel, int64_t *n_strings,
                                   int32_t *n_entries, uint32_t *strings, uint32_t *links);

/* Gradient of the summed MBE energy of `res` (Eq. 1-3, tuple set held fixed)
 * with respect to every entry of h1 and of (pq|rs), each treated as an
 * independent variable, times gE:
 *   grad_h1[p*n+q]            = gE * sum_S w_S gamma_pq(S)
 *   full layout: grad_eri[((p*n+q)*n+r)*n+s] = gE * 1/2 sum_S w_S Gamma_pqrs(S)
 *   packed layout (the integrals were set as MBEFCI_ERI_PACKED8): grad_eri[k]
 *     for packed element k = the sum of the full-layout entries over the
 *     distinct index quadruples of its orbit (the derivative with respect to
 *     that one stored number); n(n+1)/2 (n(n+1)/2 + 1)/2 doubles
 * where w = (I + L^T)^-1 1 are the integer adjoint weights of the increment
 * recursion (L_ST = 1 iff T is a proper subtuple of S), and gamma(S), Gamma(S)
 * are the full-space one- and two-particle density matrices of tuple S's
 * CASCI ground state (gamma_pq = <E_pq>, Gamma_pqrs = <E_pq E_rs> - d_qr
 * gamma_ps, frozen core included).  If `res` was computed with
 * options.gradient = 1 the stored gradient is returned and the workspace is
 * not used; otherwise the tuples with w_S != 0 are solved again (|r| <= 1e-9)
 * and their density matrices come from a device Gram contraction of
 * <I|E_pq|c>, embedded into the gradient on the device (n^2 + n^4 doubles of
 * the workspace).  Host outputs: n*n doubles and grad_eri in the layout of
 * the integrals.  ETOOLARGE for a CAS of more than 12 active orbitals.  The
 * ground states must be non-degenerate for the derivative to exist. */
mbefci_status mbefci_backward(mbefci_ctx *ctx, const mbefci_result *res, double gE, void *d_workspace,
                              size_t ws_bytes, double *grad_h1, double *grad_eri);

/* CASSCF expansion reference (Sec. 2: the orbitals of the reference space
 * chosen to minimise its CASCI energy; the paper's best results use them,
 * Sec. 4.1.3 and 4.2.2).  Minimises the reference-space CASCI energy (the
 * state of epsilon(()) of the expansion, options.spin_shift included) over
 * the rotations phi'_j = sum_i phi_i U_ij between the core (doubly occupied
 * orbitals outside [Pi] that are not frozen), the active ([Pi]) and the
 * virtual orbitals; frozen orbitals are not rotated.  Then the orbitals are
 * made canonical: eigenvectors of the Fock matrix f_pq = h_pq + sum_rs
 * gamma_rs [(pq|rs) - 1/2 (pr|sq)] in the core and the virtual blocks
 * (ascending), natural orbitals in the active block (descending occupation),
 * each space keeping its orbital positions, every column of U signed so that
 * its largest entry is positive.  On return the context's Hamiltonian is the
 * one in these orbitals (h' = U^T h U and the four-index transformation of
 * (pq|rs), on the device and in mbefci_get_hamiltonian), so that mbefci_run
 * expands in them.  The orbital gradient is 2 (F_qp - F_pq) with the
 * generalised Fock matrix F_pq = sum_r gamma_pr h_qr + sum_rst Gamma_prst
 * (qr|st); the steps are limited-memory BFGS in the frame of the current
 * orbitals on a diagonal Hessian estimate, with energy backtracking; each
 * energy is a device CASCI of [Pi] converged to |r| < 1e-11.
 * Arguments: d_workspace of at least 2 n^4 + n^2 + n^4 doubles plus what the
 * reference CASCI needs (the gradient accumulators and one batch); max_iter
 * >= 1 optimisation steps; g_tol > 0 on the largest gradient entry (the
 * tuples' energies are not stationary in the orbitals, so they follow its
 * accuracy: 1e-10 gives them to about 1e-9).  Host outputs (each may be
 * null): U [n*n] row-major (column j = new orbital j in the orbitals the
 * Hamiltonian had on entry), the CASSCF energy, the steps taken.  ENOCONV if
 * g_tol is not reached in max_iter steps (the Hamiltonian is then replaced
 * by the canonical form of the last orbitals); ETOOLARGE for a reference space
 * of more than 12 orbitals; ENOMEM if the workspace is too small. */
mbefci_status mbefci_casscf(mbefci_ctx *ctx, void *d_workspace, size_t ws_bytes, int32_t max_iter, double g_tol,
                            double *U, double *energy, int32_t *iterations);

/* Restricted closed-shell Hartree-Fock orbitals (the paper's expansion
 * orbitals, Sec. 1 and 2; the reference of its CCSD(T) base, Sec. 4.2.1):
 * the n_alpha = n_beta lowest-energy doubly occupied orbitals minimising
 * <Phi|H|Phi> over orthonormal rotations of the context's orbitals, found by
 * energy descent over the occupied-virtual rotations until the largest
 * element of the orbital gradient 4 f_ai is below g_tol; then made canonical
 * (the Fock matrix diagonal, ascending within the occupied and within the
 * virtual block, occupied orbitals first, each column signed so that its
 * largest entry is positive) and the context's Hamiltonian replaced by the
 * one in them (frozen orbitals are rotated too: afterwards they are the
 * lowest occupied HF orbitals; the reference space keeps its positions).
 * Host outputs, each may be null: U [n*n] (row p, column j: coefficient of
 * the entry orbital p in HF orbital j), the HF energy, the steps taken.
 * EINVAL for an open shell, ENOCONV if g_tol is not reached in max_iter steps
 * (the Hamiltonian is then replaced by the canonical form of the last
 * orbitals), ENOMEM if the workspace cannot hold two n^4 arrays. */
mbefci_status mbefci_hf(mbefci_ctx *ctx, void *d_workspace, size_t ws_bytes, int32_t max_iter, double g_tol,
                        double *U, double *energy, int32_t *iterations);

/* Abelian point-group irrep labels of the n orbitals (host array [n], each
 * 0..7; the product of two irreps is the XOR of their labels), for
 * options.sym_shift (Sec. 4.1: states of a given symmetry).  EINVAL for a label
 * out of range; the Hamiltonian is checked against them when a solve with
 * sym_shift > 0 starts. */
mbefci_status mbefci_set_orbital_irreps(mbefci_ctx *ctx, const int32_t *labels);

/* Base-model energies eps_base(S) of ntup tuples of one order, of the model
 * options.base_model names (the second-order one when it is 0).  Host tuples
 * as at mbefci_solve_tuples, host output energies [ntup].  Errors as listed at
 * options.base_model.  Order |X| with the tuple of every expansion orbital
 * gives the whole space. */
mbefci_status mbefci_tuple_base(mbefci_ctx *ctx, int32_t order, int64_t ntup, const int16_t *tuples,
                                void *d_workspace, size_t ws_bytes, double *energies);

/* The context's current Hamiltonian (host outputs, each may be null): h1
 * [n*n], (pq|rs) [n^4] in the full layout, the constant. */
mbefci_status mbefci_get_hamiltonian(const mbefci_ctx *ctx, double *h1, double *eri, double *e_const);

/* CASCI energy and full-space density matrices of one tuple (host outputs:
 * *energy, gamma [n*n], Gamma [n^4], conventions as at mbefci_backward). */
mbefci_status mbefci_tuple_rdm(mbefci_ctx *ctx, int32_t order, const int16_t *tuple, void *d_workspace,
                               size_t ws_bytes, double *energy, double *gamma, double *Gamma);

/* Counters of the last solve/run call. */
mbefci_status mbefci_get_stats(const mbefci_ctx *ctx, mbefci_stats *stats);

/* Per-class counters of the last solve/run call: *nclass receives the number
 * of classes; with out != NULL the first min(*nclass on entry, count) entries
 * are written (ordered by n_active, n_alpha, n_beta). */
mbefci_status mbefci_get_class_stats(const mbefci_ctx *ctx, int32_t *nclass, mbefci_class_stats *out);

#ifdef __cplusplus
}
#endif

#endif /* MBEFCI_H */

/*
 * qi_oracle.c -- plain FP64 CPU oracle for the synchronous quantum-inspired
 * (QI) low-energy search (Ueda, Otsuka, Yunoki, arXiv:2010.00180).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call this code:
 * only the tests, the smoke check and the benchmark's CPU-baseline leg use it.
 * It shares no code, header, table or helper with the HIP library.
 *
 * What it computes, in the paper's terms:
 *   - energy  E(x) = sum_{i<j} J_ij s_i s_j + sum_i h_i s_i          (Eq. 1)
 *     with s_i = +1 for sigma_i = 0 and s_i = -1 for sigma_i = 1, and the
 *     state integer psi = sum_i 2^i sigma_i                             (Eq. 15)
 *   - spin flips by XOR of the state integer with sum_k 2^{i_k}         (Alg. 1)
 *   - the neighbourhood of x: x itself, all N single flips and all
 *     N(N-1)/2 pair flips (i<j), i.e. the states reached by H_tot with the
 *     one- and two-body sigma^x terms of H1                              (Eq. 9, Eq. 16)
 *   - the energy of a flipped state from its parent's energy in O(N), using
 *     only the couplings of the flipped sites                            (Sec. III, cost paragraph)
 *   - one synchronous step: keep the M lowest distinct states of the union
 *     of the neighbourhoods of the kept states; in the infinitesimal-lambda
 *     limit the p_{M',k} selection reduces to this energy order       (Sec. II, Eqs. 9-14)
 *   - repeat until the kept set no longer changes                        (Sec. II)
 *   - independent searches from L initial states merged into the M lowest
 *     distinct states of the union of their kept sets                    (Alg. 4)
 *
 * Readings where the paper leaves a choice open:
 *   - ties in energy are broken by the state integer psi (smaller first), so
 *     the kept set is unique; the paper keeps arrival order;
 *   - a state already in the kept set never enters twice (distinctness);
 *   - "literal" mode expands every kept state each step; "frontier" mode
 *     expands only states that entered in the previous step.  Both give the
 *     same sets (children of an old member were already offered one step
 *     earlier and either entered or ranked behind the whole kept set).
 *
 * Two ways to get a flipped state's energy, both from the parent's energy:
 *   - qo_flip_change: the terms of Eq. 1 that touch the flipped sites, summed
 *     afresh, O(N) per flipped state (the cost paragraph of Sec. III);
 *   - the *_fields entry points: the parent's local fields
 *     F_k = h_k + sum_l J_kl s_l are summed once per parent (O(N^2)), and a
 *     flip of i changes E by -2 s_i F_i, a flip of i and j by
 *     -2 s_i F_i - 2 s_j F_j + 4 J_ij s_i s_j (the coupling of the pair keeps its
 *     sign, and F_i, F_j each counted it once with the wrong sign).  O(1) per
 *     flipped state, which makes N = 600 and N = 1000 steps affordable.
 * The two are pinned against each other and against Eq. 1 by the tests.
 *
 * The perturbation H1 decides the neighbourhood (Sec. VI names two others
 * besides the one- and two-spin flips of Eq. 16):
 *   h1 = 0  sigma^x_i and sigma^x_i sigma^x_j: all single and pair flips;
 *   h1 = 1  sigma^x_i only (the J = 1 case): the N single flips;
 *   h1 = 2  the XX interaction sum_{i<j} (sigma^x_i sigma^x_j + sigma^y_i sigma^y_j):
 *           it exchanges the spins of sites i and j, which changes the state only
 *           when they differ, and then it is the pair flip of i and j; the number
 *           of down spins (the total sigma^z) is conserved.
 *
 * Exactness: inputs on the 2^-24 grid with modest magnitudes make every sum
 * here exact in FP64, so the result does not depend on summation order.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int words_of(int N) { return (N + 63) / 64; }

static int spin_of(const uint64_t *x, int i)
{
    return ((x[i >> 6] >> (i & 63)) & 1u) ? -1 : +1;
}

/* Eq. 1 written out: pairs i<j, then the field term. */
double qo_energy(int N, const double *J, const double *h, const uint64_t *x)
{
    double e = 0.0;
    for (int i = 0; i < N; ++i) {
        int si = spin_of(x, i);
        for (int j = i + 1; j < N; ++j)
            e += J[(size_t)i * N + j] * (double)(si * spin_of(x, j));
    }
    for (int i = 0; i < N; ++i)
        e += h[i] * (double)spin_of(x, i);
    return e;
}

static int in_sites(int l, int nflip, const int *sites)
{
    for (int a = 0; a < nflip; ++a)
        if (sites[a] == l) return 1;
    return 0;
}

/*
 * E(x') - E(x) for x' = x with the spins in `sites` flipped (distinct sites).
 * Only the terms of Eq. 1 that touch a flipped site change: h_k s_k for a
 * flipped k, and J_kl s_k s_l with exactly one of k, l flipped (a pair with
 * both flipped keeps its sign).  Each such term changes by -2 times itself.
 */
double qo_flip_change(int N, const double *J, const double *h, const uint64_t *x,
                      int nflip, const int *sites)
{
    double d = 0.0;
    for (int a = 0; a < nflip; ++a) {
        int k = sites[a];
        double sk = (double)spin_of(x, k);
        double field = h[k];
        for (int l = 0; l < N; ++l) {
            if (in_sites(l, nflip, sites)) continue;
            field += J[(size_t)k * N + l] * (double)spin_of(x, l);
        }
        d += -2.0 * sk * field;
    }
    return d;
}

/* Local fields of state x by a direct sum: F_k = h_k + sum_l J_kl s_l. */
static void local_fields(int N, const double *J, const double *h, const uint64_t *x, double *F)
{
    for (int k = 0; k < N; ++k) {
        double f = h[k];
        for (int l = 0; l < N; ++l)
            f += J[(size_t)k * N + l] * (double)spin_of(x, l);
        F[k] = f;
    }
}

/* E(x') - E(x) for one or two distinct flipped sites, from the fields F of x. */
static double field_change(int N, const double *J, const uint64_t *x, const double *F,
                           int nflip, const int *sites)
{
    int i = sites[0];
    double si = (double)spin_of(x, i);
    double d = -2.0 * si * F[i];
    if (nflip == 2) {
        int j = sites[1];
        double sj = (double)spin_of(x, j);
        d += -2.0 * sj * F[j] + 4.0 * J[(size_t)i * N + j] * si * sj;
    }
    return d;
}

/* The same change through the local fields (one or two sites); a pin compares it with qo_flip_change. */
double qo_field_change(int N, const double *J, const double *h, const uint64_t *x, int nflip, const int *sites)
{
    if (nflip < 1 || nflip > 2) return NAN;
    double *F = (double *)malloc(sizeof(double) * (size_t)N);
    if (!F) return NAN;
    local_fields(N, J, h, x, F);
    double d = field_change(N, J, x, F, nflip, sites);
    free(F);
    return d;
}

/* Total order: energy first, then the state integer psi (highest word first). */
static int order_cmp(double Ea, const uint64_t *a, double Eb, const uint64_t *b, int W)
{
    if (Ea < Eb) return -1;
    if (Ea > Eb) return 1;
    for (int w = W - 1; w >= 0; --w) {
        if (a[w] < b[w]) return -1;
        if (a[w] > b[w]) return 1;
    }
    return 0;
}

/* A list of at most `cap` distinct states sorted by the total order. */
typedef struct {
    int cap, n, W;
    double *E;
    uint64_t *bits;
    uint8_t *flag;
} klist;

static int klist_init(klist *L, int cap, int W)
{
    L->cap = cap; L->n = 0; L->W = W;
    L->E = (double *)malloc(sizeof(double) * (size_t)(cap + 1));
    L->bits = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(cap + 1) * W);
    L->flag = (uint8_t *)malloc((size_t)(cap + 1));
    return (L->E && L->bits && L->flag) ? 0 : -1;
}

static void klist_free(klist *L)
{
    free(L->E); free(L->bits); free(L->flag);
    L->E = NULL; L->bits = NULL; L->flag = NULL;
}

/* Offer one state; it enters if it is new and ranks among the `cap` best. */
static int klist_offer(klist *L, double E, const uint64_t *x, uint8_t flag)
{
    int W = L->W;
    if (L->n == L->cap && order_cmp(E, x, L->E[L->n - 1], L->bits + (size_t)(L->n - 1) * W, W) >= 0)
        return 0;
    for (int k = 0; k < L->n; ++k)
        if (memcmp(L->bits + (size_t)k * W, x, sizeof(uint64_t) * W) == 0)
            return 0;
    int pos = L->n;
    while (pos > 0 && order_cmp(E, x, L->E[pos - 1], L->bits + (size_t)(pos - 1) * W, W) < 0)
        --pos;
    for (int k = L->n; k > pos; --k) {
        L->E[k] = L->E[k - 1];
        L->flag[k] = L->flag[k - 1];
        memcpy(L->bits + (size_t)k * W, L->bits + (size_t)(k - 1) * W, sizeof(uint64_t) * W);
    }
    L->E[pos] = E;
    L->flag[pos] = flag;
    memcpy(L->bits + (size_t)pos * W, x, sizeof(uint64_t) * W);
    if (L->n < L->cap) L->n++;
    return 1;
}

/* Energy change of a flip of x: from the fields F of x, or (F == NULL) afresh. */
static double change_of(int N, const double *J, const double *h, const uint64_t *x, const double *F,
                        int nflip, const int *sites)
{
    return F ? field_change(N, J, x, F, nflip, sites) : qo_flip_change(N, J, h, x, nflip, sites);
}

/* Offer the neighbourhood of parent x (energy Ex) under H1 mode h1: single
   flips, then pairs i<j.  F: the local fields of x, or NULL to evaluate each
   change afresh. */
static void offer_children(klist *L, int N, const double *J, const double *h, int h1,
                           const uint64_t *x, double Ex, uint64_t *child, const double *F)
{
    int W = words_of(N);
    int sites[2];
    for (int i = 0; i < N && h1 != 2; ++i) {
        memcpy(child, x, sizeof(uint64_t) * W);
        child[i >> 6] ^= (uint64_t)1 << (i & 63);
        sites[0] = i;
        klist_offer(L, Ex + change_of(N, J, h, x, F, 1, sites), child, 1);
    }
    for (int i = 0; i < N && h1 != 1; ++i) {
        for (int j = i + 1; j < N; ++j) {
            if (h1 == 2 && spin_of(x, i) == spin_of(x, j)) continue;   /* the exchange leaves x as it is */
            memcpy(child, x, sizeof(uint64_t) * W);
            child[i >> 6] ^= (uint64_t)1 << (i & 63);
            child[j >> 6] ^= (uint64_t)1 << (j & 63);
            sites[0] = i; sites[1] = j;
            klist_offer(L, Ex + change_of(N, J, h, x, F, 2, sites), child, 1);
        }
    }
}

/*
 * One synchronous step.  Input: the kept set S_t (n_in states, energies in_E
 * or NULL to evaluate Eq. 1, and in_front = 1 for states that entered in the
 * previous step).  Output: S_{t+1}, the M lowest distinct states of
 * S_t united with the neighbourhoods of the expanded states, sorted, with
 * out_front = 1 for states not in S_t.  literal != 0 expands every state of
 * S_t; otherwise only those with in_front set.  Returns the number of new
 * states (0 means the set is stable), or -1 on allocation failure.
 */
static int step_impl(int N, const double *J, const double *h, int M, int literal, int use_fields, int h1,
                     int n_in, const uint64_t *in_bits, const double *in_E, const uint8_t *in_front,
                     uint64_t *out_bits, double *out_E, uint8_t *out_front, int *n_out)
{
    int W = words_of(N);
    double *E_in = (double *)malloc(sizeof(double) * (size_t)(n_in > 0 ? n_in : 1));
    if (!E_in) return -1;
    for (int k = 0; k < n_in; ++k)
        E_in[k] = in_E ? in_E[k] : qo_energy(N, J, h, in_bits + (size_t)k * W);

    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    klist *part = (klist *)calloc((size_t)nthreads, sizeof(klist));
    int fail = (part == NULL);
    for (int t = 0; t < nthreads && !fail; ++t)
        fail |= klist_init(&part[t], M, W);

    if (!fail) {
#pragma omp parallel num_threads(nthreads)
        {
            int tid = 0;
#ifdef _OPENMP
            tid = omp_get_thread_num();
#endif
            uint64_t *child = (uint64_t *)malloc(sizeof(uint64_t) * W);
            double *F = use_fields ? (double *)malloc(sizeof(double) * (size_t)N) : NULL;
#pragma omp for schedule(dynamic, 1)
            for (int k = 0; k < n_in; ++k) {
                if (!literal && !in_front[k]) continue;
                const uint64_t *x = in_bits + (size_t)k * W;
                if (F) local_fields(N, J, h, x, F);
                offer_children(&part[tid], N, J, h, h1, x, E_in[k], child, F);
            }
            free(F);
            free(child);
        }
    }

    int n_new = -1;
    klist R;
    if (!fail && klist_init(&R, M, W) == 0) {
        /* S_t first, so a child equal to a kept state keeps the kept flag. */
        for (int k = 0; k < n_in; ++k)
            klist_offer(&R, E_in[k], in_bits + (size_t)k * W, 0);
        for (int t = 0; t < nthreads; ++t)
            for (int k = 0; k < part[t].n; ++k)
                klist_offer(&R, part[t].E[k], part[t].bits + (size_t)k * W, 1);
        n_new = 0;
        for (int k = 0; k < R.n; ++k) {
            out_E[k] = R.E[k];
            out_front[k] = R.flag[k];
            memcpy(out_bits + (size_t)k * W, R.bits + (size_t)k * W, sizeof(uint64_t) * W);
            n_new += R.flag[k];
        }
        *n_out = R.n;
        klist_free(&R);
    }
    if (part) {
        for (int t = 0; t < nthreads; ++t) klist_free(&part[t]);
        free(part);
    }
    free(E_in);
    return n_new;
}

int qo_step(int N, const double *J, const double *h, int M, int literal,
            int n_in, const uint64_t *in_bits, const double *in_E, const uint8_t *in_front,
            uint64_t *out_bits, double *out_E, uint8_t *out_front, int *n_out)
{
    return step_impl(N, J, h, M, literal, 0, 0, n_in, in_bits, in_E, in_front, out_bits, out_E, out_front, n_out);
}

/* qo_step with every energy change taken from the parent's local fields. */
int qo_step_fields(int N, const double *J, const double *h, int M, int literal,
                   int n_in, const uint64_t *in_bits, const double *in_E, const uint8_t *in_front,
                   uint64_t *out_bits, double *out_E, uint8_t *out_front, int *n_out)
{
    return step_impl(N, J, h, M, literal, 1, 0, n_in, in_bits, in_E, in_front, out_bits, out_E, out_front, n_out);
}

/* qo_step (use_fields = 0) or qo_step_fields (1) under H1 mode h1 (0, 1, 2, see the top of this file). */
int qo_step_h1(int N, const double *J, const double *h, int M, int literal, int use_fields, int h1,
               int n_in, const uint64_t *in_bits, const double *in_E, const uint8_t *in_front,
               uint64_t *out_bits, double *out_E, uint8_t *out_front, int *n_out)
{
    if (h1 < 0 || h1 > 2) return -1;
    return step_impl(N, J, h, M, literal, use_fields, h1, n_in, in_bits, in_E, in_front, out_bits, out_E,
                     out_front, n_out);
}

/*
 * One search from initial state x0 (S_0 = {x0}); steps until the set is
 * stable or max_iters steps were taken.  *iters counts the steps evaluated,
 * including the last one that found no new state.  Returns 1 if stable, 0 if
 * the cap was reached first, -1 on failure.
 */
/*
 * One step of the learned-proposal form (not in the paper; the proposal ranks
 * pair flips and only the ranked-in pairs are offered).  The candidates are
 * S_t itself, the N single flips of every expanded parent, and for parent p
 * only the pair flips listed for it: pairs[off_p .. off_p + npairs[p]), each
 * encoded i | j << 16 with i < j.  parent[p] indexes S_t.  The kept set is the
 * M lowest distinct candidates, as in qo_step.  Returns the number of new
 * states, or -1 on allocation failure or a malformed pair.
 */
static int step_proposed_impl(int N, const double *J, const double *h, int M, int use_fields,
                              int n_in, const uint64_t *in_bits, const double *in_E,
                              int n_par, const int *parent, const int *npairs, const uint32_t *pairs,
                              uint64_t *out_bits, double *out_E, uint8_t *out_front, int *n_out)
{
    int W = words_of(N);
    klist R;
    if (klist_init(&R, M, W) != 0) return -1;
    uint64_t *child = (uint64_t *)malloc(sizeof(uint64_t) * W);
    double *F = use_fields ? (double *)malloc(sizeof(double) * (size_t)N) : NULL;
    if (!child || (use_fields && !F)) { free(child); free(F); klist_free(&R); return -1; }
    for (int k = 0; k < n_in; ++k)
        klist_offer(&R, in_E[k], in_bits + (size_t)k * W, 0);
    size_t off = 0;
    int bad = 0;
    for (int p = 0; p < n_par && !bad; ++p) {
        const uint64_t *x = in_bits + (size_t)parent[p] * W;
        double Ex = in_E[parent[p]];
        int sites[2];
        if (F) local_fields(N, J, h, x, F);
        for (int i = 0; i < N; ++i) {
            memcpy(child, x, sizeof(uint64_t) * W);
            child[i >> 6] ^= (uint64_t)1 << (i & 63);
            sites[0] = i;
            klist_offer(&R, Ex + change_of(N, J, h, x, F, 1, sites), child, 1);
        }
        for (int q = 0; q < npairs[p]; ++q) {
            uint32_t code = pairs[off + q];
            int i = (int)(code & 0xFFFFu), j = (int)(code >> 16);
            if (!(0 <= i && i < j && j < N)) { bad = 1; break; }
            memcpy(child, x, sizeof(uint64_t) * W);
            child[i >> 6] ^= (uint64_t)1 << (i & 63);
            child[j >> 6] ^= (uint64_t)1 << (j & 63);
            sites[0] = i; sites[1] = j;
            klist_offer(&R, Ex + change_of(N, J, h, x, F, 2, sites), child, 1);
        }
        off += (size_t)npairs[p];
    }
    int n_new = -1;
    if (!bad) {
        n_new = 0;
        for (int k = 0; k < R.n; ++k) {
            out_E[k] = R.E[k];
            out_front[k] = R.flag[k];
            memcpy(out_bits + (size_t)k * W, R.bits + (size_t)k * W, sizeof(uint64_t) * W);
            n_new += R.flag[k];
        }
        *n_out = R.n;
    }
    free(child);
    free(F);
    klist_free(&R);
    return n_new;
}

int qo_step_proposed(int N, const double *J, const double *h, int M,
                     int n_in, const uint64_t *in_bits, const double *in_E,
                     int n_par, const int *parent, const int *npairs, const uint32_t *pairs,
                     uint64_t *out_bits, double *out_E, uint8_t *out_front, int *n_out)
{
    return step_proposed_impl(N, J, h, M, 0, n_in, in_bits, in_E, n_par, parent, npairs, pairs,
                              out_bits, out_E, out_front, n_out);
}

/* qo_step_proposed with every energy change taken from the parent's local fields. */
int qo_step_proposed_fields(int N, const double *J, const double *h, int M,
                            int n_in, const uint64_t *in_bits, const double *in_E,
                            int n_par, const int *parent, const int *npairs, const uint32_t *pairs,
                            uint64_t *out_bits, double *out_E, uint8_t *out_front, int *n_out)
{
    return step_proposed_impl(N, J, h, M, 1, n_in, in_bits, in_E, n_par, parent, npairs, pairs,
                              out_bits, out_E, out_front, n_out);
}

static int search_impl(int N, const double *J, const double *h, int M, int max_iters, int literal,
                       int use_fields, int h1, const uint64_t *x0, uint64_t *out_bits, double *out_E,
                       int *n_out, int *iters)
{
    int W = words_of(N);
    size_t cap = (size_t)M;
    uint64_t *cb = (uint64_t *)malloc(sizeof(uint64_t) * cap * W);
    uint64_t *nb = (uint64_t *)malloc(sizeof(uint64_t) * cap * W);
    double *cE = (double *)malloc(sizeof(double) * cap);
    double *nE = (double *)malloc(sizeof(double) * cap);
    uint8_t *cf = (uint8_t *)malloc(cap);
    uint8_t *nf = (uint8_t *)malloc(cap);
    int rc = -1;
    if (cb && nb && cE && nE && cf && nf) {
        int n = 1;
        memcpy(cb, x0, sizeof(uint64_t) * W);
        cE[0] = qo_energy(N, J, h, x0);
        cf[0] = 1;
        int t = 0, stable = 0;
        while (t < max_iters) {
            int nn = 0;
            int n_new = step_impl(N, J, h, M, literal, use_fields, h1, n, cb, cE, cf, nb, nE, nf, &nn);
            if (n_new < 0) { t = -1; break; }
            ++t;
            if (n_new == 0) { stable = 1; break; }
            uint64_t *tb = cb; cb = nb; nb = tb;
            double *tE = cE; cE = nE; nE = tE;
            uint8_t *tf = cf; cf = nf; nf = tf;
            n = nn;
        }
        if (t >= 0) {
            memcpy(out_bits, cb, sizeof(uint64_t) * (size_t)n * W);
            memcpy(out_E, cE, sizeof(double) * (size_t)n);
            *n_out = n;
            *iters = t;
            rc = stable;
        }
    }
    free(cb); free(nb); free(cE); free(nE); free(cf); free(nf);
    return rc;
}

int qo_search(int N, const double *J, const double *h, int M, int max_iters, int literal,
              const uint64_t *x0, uint64_t *out_bits, double *out_E, int *n_out, int *iters)
{
    return search_impl(N, J, h, M, max_iters, literal, 0, 0, x0, out_bits, out_E, n_out, iters);
}

/* qo_search under H1 mode h1, with the field (1) or afresh (0) energy changes. */
int qo_search_h1(int N, const double *J, const double *h, int M, int max_iters, int literal, int use_fields,
                 int h1, const uint64_t *x0, uint64_t *out_bits, double *out_E, int *n_out, int *iters)
{
    if (h1 < 0 || h1 > 2) return -1;
    return search_impl(N, J, h, M, max_iters, literal, use_fields, h1, x0, out_bits, out_E, n_out, iters);
}

/* Alg. 4 merge: the M lowest distinct states of the union of several lists. */
int qo_merge(int N, int M, int n_lists, const int *counts, const uint64_t *bits, const double *E,
             uint64_t *out_bits, double *out_E, int *n_out)
{
    int W = words_of(N);
    klist R;
    if (klist_init(&R, M, W) != 0) return -1;
    size_t off = 0;
    for (int l = 0; l < n_lists; ++l) {
        for (int k = 0; k < counts[l]; ++k, ++off)
            klist_offer(&R, E[off], bits + off * W, 0);
    }
    for (int k = 0; k < R.n; ++k) {
        out_E[k] = R.E[k];
        memcpy(out_bits + (size_t)k * W, R.bits + (size_t)k * W, sizeof(uint64_t) * W);
    }
    *n_out = R.n;
    klist_free(&R);
    return 0;
}

/*
 * Exhaustive search over all 2^N states (the paper's brute-force reference,
 * N small): the K lowest states under the total order.  States are visited
 * in Gray-code order; flipping spin i changes E by -2 s_i f_i with
 * f_i = h_i + sum_l J_il s_l, and then every f_k moves by -2 s_i J_ki.
 */
int qo_brute_lowest(int N, const double *J, const double *h, int K,
                    uint64_t *out_bits, double *out_E, int *n_out)
{
    if (N < 1 || N > 40) return -1;
    int W = words_of(N);
    klist R;
    if (klist_init(&R, K, W) != 0) return -1;
    double *f = (double *)malloc(sizeof(double) * N);
    int *s = (int *)malloc(sizeof(int) * N);
    uint64_t *x = (uint64_t *)calloc((size_t)W, sizeof(uint64_t));
    if (!f || !s || !x) { free(f); free(s); free(x); klist_free(&R); return -1; }
    for (int i = 0; i < N; ++i) s[i] = 1;
    for (int i = 0; i < N; ++i) {
        f[i] = h[i];
        for (int l = 0; l < N; ++l) f[i] += J[(size_t)i * N + l];
    }
    double E = qo_energy(N, J, h, x);
    klist_offer(&R, E, x, 0);
    uint64_t total = (uint64_t)1 << N;
    for (uint64_t g = 1; g < total; ++g) {
        int i = __builtin_ctzll(g);
        E += -2.0 * s[i] * f[i];
        for (int k = 0; k < N; ++k)
            f[k] += -2.0 * s[i] * J[(size_t)k * N + i];
        s[i] = -s[i];
        x[i >> 6] ^= (uint64_t)1 << (i & 63);
        if (R.n < R.cap || E <= R.E[R.n - 1])
            klist_offer(&R, E, x, 0);
    }
    for (int k = 0; k < R.n; ++k) {
        out_E[k] = R.E[k];
        memcpy(out_bits + (size_t)k * W, R.bits + (size_t)k * W, sizeof(uint64_t) * W);
    }
    *n_out = R.n;
    free(f); free(s); free(x);
    klist_free(&R);
    return 0;
}

int qo_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * ------------------------------------------------------------------ best-first search (Sec. III)
 * The paper's own sequential form of the method: Alg. 3 (QI single search)
 * with the list update of Alg. 2, and Alg. 4 (QI multi search).
 *
 * The list holds K + 1 entries in energy order; equal energies keep their
 * order of arrival, because a new entry goes after every entry of equal
 * energy.  Entries start as placeholders (the largest integer and the largest
 * real number); each real entry carries a flag telling whether it has been
 * expanded.  A flipped state enters when it is not in the list and its energy
 * is below the last entry's, which it then replaces.
 *
 * Alg. 3: for each of I iterations, the first entry in energy order that has
 * not been expanded is marked and expanded: its single flips (sites 0 .. N-1)
 * and then its pair flips ((0,1), (0,2), .., (N-2,N-1)) are offered to the
 * list one after the other, each with its energy from the parent's in O(N).
 * Readings: a placeholder is never expanded (when every real entry has been
 * expanded the iteration does nothing); h1 selects the flips offered as in
 * offer_children (1: single flips only; 2: exchanges of unequal spins, the
 * exchange of two equal spins giving back the parent, which the list already
 * holds).
 *
 * Alg. 4: L single searches; the first one's list is the result list, and the
 * entries of every later list, in that list's energy order, are offered to it
 * with the same rule (each state with its own energy and flag).
 */
typedef struct {
    int cap;            /* K + 1 */
    int W;
    double *E;          /* energy order; +INFINITY for a placeholder */
    uint64_t *x;        /* words of each entry */
    uint8_t *real;      /* 0 for a placeholder */
    uint8_t *used;      /* expanded */
    int *born;          /* iteration at which the entry arrived (0 = initial) */
} bflist;

static int bflist_init(bflist *B, int cap, int W)
{
    B->cap = cap; B->W = W;
    B->E = (double *)malloc(sizeof(double) * (size_t)cap);
    B->x = (uint64_t *)calloc((size_t)cap * W, sizeof(uint64_t));
    B->real = (uint8_t *)calloc((size_t)cap, 1);
    B->used = (uint8_t *)calloc((size_t)cap, 1);
    B->born = (int *)calloc((size_t)cap, sizeof(int));
    if (!B->E || !B->x || !B->real || !B->used || !B->born) return -1;
    for (int k = 0; k < cap; ++k) B->E[k] = INFINITY;
    return 0;
}

static void bflist_free(bflist *B)
{
    free(B->E); free(B->x); free(B->real); free(B->used); free(B->born);
}

static int bflist_has(const bflist *B, const uint64_t *x)
{
    for (int k = 0; k < B->cap; ++k)
        if (B->real[k] && memcmp(B->x + (size_t)k * B->W, x, sizeof(uint64_t) * B->W) == 0) return 1;
    return 0;
}

/* Offer a state that is not in the list: it enters if E is below the last
   entry's energy, after every entry of equal or lower energy. */
static void bflist_offer(bflist *B, const uint64_t *x, double E, uint8_t used, int born)
{
    int last = B->cap - 1;
    if (!(E < B->E[last])) return;
    int pos = 0;
    while (pos < last && B->E[pos] <= E) ++pos;
    for (int k = last; k > pos; --k) {
        B->E[k] = B->E[k - 1];
        B->real[k] = B->real[k - 1];
        B->used[k] = B->used[k - 1];
        B->born[k] = B->born[k - 1];
        memcpy(B->x + (size_t)k * B->W, B->x + (size_t)(k - 1) * B->W, sizeof(uint64_t) * B->W);
    }
    B->E[pos] = E;
    B->real[pos] = 1;
    B->used[pos] = used;
    B->born[pos] = born;
    memcpy(B->x + (size_t)pos * B->W, x, sizeof(uint64_t) * B->W);
}

static void bf_single(int N, const double *J, const double *h, int h1, int I, const uint64_t *x0,
                      bflist *B, uint64_t *child, int *expanded)
{
    int W = words_of(N);
    bflist_offer(B, x0, qo_energy(N, J, h, x0), 0, 0);
    int done = 0;
    for (int it = 1; it <= I; ++it) {
        int k = 0;
        while (k < B->cap && !(B->real[k] && !B->used[k])) ++k;
        if (k == B->cap) continue;
        B->used[k] = 1;
        ++done;
        uint64_t *x = child + W;   /* the parent, kept apart from the list (its entry may move) */
        memcpy(x, B->x + (size_t)k * W, sizeof(uint64_t) * W);
        double Ex = B->E[k];
        int sites[2];
        for (int i = 0; i < N && h1 != 2; ++i) {
            memcpy(child, x, sizeof(uint64_t) * W);
            child[i >> 6] ^= (uint64_t)1 << (i & 63);
            if (bflist_has(B, child)) continue;
            sites[0] = i;
            bflist_offer(B, child, Ex + qo_flip_change(N, J, h, x, 1, sites), 0, it);
        }
        for (int i = 0; i < N && h1 != 1; ++i) {
            for (int j = i + 1; j < N; ++j) {
                if (h1 == 2 && spin_of(x, i) == spin_of(x, j)) continue;
                memcpy(child, x, sizeof(uint64_t) * W);
                child[i >> 6] ^= (uint64_t)1 << (i & 63);
                child[j >> 6] ^= (uint64_t)1 << (j & 63);
                if (bflist_has(B, child)) continue;
                sites[0] = i; sites[1] = j;
                bflist_offer(B, child, Ex + qo_flip_change(N, J, h, x, 2, sites), 0, it);
            }
        }
    }
    *expanded = done;
}

static void bf_copy_out(const bflist *B, uint64_t *out_x, double *out_E, uint8_t *out_used, int *out_born,
                        int *n_out)
{
    int n = 0;
    for (int k = 0; k < B->cap; ++k) {
        if (!B->real[k]) continue;
        memcpy(out_x + (size_t)n * B->W, B->x + (size_t)k * B->W, sizeof(uint64_t) * B->W);
        out_E[n] = B->E[k];
        if (out_used) out_used[n] = B->used[k];
        if (out_born) out_born[n] = B->born[k];
        ++n;
    }
    *n_out = n;
}

/*
 * Alg. 3 from x0 with a list of K + 1 entries and I iterations.  Output: the
 * real entries in list order (at most K + 1): words, energies, expanded flags,
 * arrival iterations; *expanded = iterations that expanded a state.  Returns
 * 0, or -1 on allocation failure.
 */
int qo_bf_search(int N, const double *J, const double *h, int h1, int K, int I, const uint64_t *x0,
                 uint64_t *out_x, double *out_E, uint8_t *out_used, int *out_born, int *n_out, int *expanded)
{
    int W = words_of(N);
    bflist B = {0};
    uint64_t *child = (uint64_t *)malloc(sizeof(uint64_t) * 2 * W);
    if (!child || bflist_init(&B, K + 1, W) != 0) { free(child); bflist_free(&B); return -1; }
    bf_single(N, J, h, h1, I, x0, &B, child, expanded);
    bf_copy_out(&B, out_x, out_E, out_used, out_born, n_out);
    free(child);
    bflist_free(&B);
    return 0;
}

/*
 * Alg. 4: L searches from x0[l] (L*W words), merged.  Output as qo_bf_search
 * (the merged list); expanded[l] per search.  Returns 0 or -1.
 */
int qo_bf_multi(int N, const double *J, const double *h, int h1, int K, int I, int L, const uint64_t *x0,
                uint64_t *out_x, double *out_E, int *n_out, int *expanded)
{
    int W = words_of(N);
    bflist R = {0}, B = {0};
    uint64_t *child = (uint64_t *)malloc(sizeof(uint64_t) * 2 * W);
    int rc = -1;
    if (child && bflist_init(&R, K + 1, W) == 0 && bflist_init(&B, K + 1, W) == 0) {
        bf_single(N, J, h, h1, I, x0, &R, child, &expanded[0]);
        for (int l = 1; l < L; ++l) {
            for (int k = 0; k < B.cap; ++k) { B.E[k] = INFINITY; B.real[k] = 0; B.used[k] = 0; B.born[k] = 0; }
            bf_single(N, J, h, h1, I, x0 + (size_t)l * W, &B, child, &expanded[l]);
            for (int k = 0; k < B.cap; ++k)
                if (B.real[k] && !bflist_has(&R, B.x + (size_t)k * W))
                    bflist_offer(&R, B.x + (size_t)k * W, B.E[k], B.used[k], B.born[k]);
        }
        bf_copy_out(&R, out_x, out_E, NULL, NULL, n_out);
        rc = 0;
    }
    free(child);
    bflist_free(&R);
    bflist_free(&B);
    return rc;
}

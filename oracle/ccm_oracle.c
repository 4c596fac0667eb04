/*
 * ccm_oracle.c -- plain, slow CPU reference for the simplex cross-map that is
 * the hot path of convergent cross mapping (CCM).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * constant generator with the HIP library, and the HIP library never calls it.
 *
 * What is computed, in the order the method states it:
 *   - lagged-coordinate embedding (shadow manifold) of the library series
 *     (paper, Introduction: parameters tau and E; Section 3.2: "lagged-
 *     coordinate vector" in the shadow manifold);
 *   - r random library subsamples of size L per (E, tau, L)  (Introduction;
 *     Section 3.1: the input record holds subsamples of length L and (tau, E));
 *   - for every query point, its E+1 nearest library vectors, found by
 *     computing all distances and taking the first E+1 in sorted order
 *     (Section 3.2);
 *   - simplex-projection prediction of the other series from those
 *     neighbours (Section 2.1), with the usual CCM weights exp(-d_m / d_1);
 *   - Pearson correlation of observed against predicted values as the
 *     prediction skill (Section 2.1), in both directions (Introduction).
 *
 * Readings where the paper is silent (each one is also listed in the design
 * notes of the repository):
 *   - embedded point i (0-based) sits at time t_i = i + (E-1) tau and has
 *     coordinates v_i[k] = S[t_i - k tau], k = 0..E-1 (backward lags); the
 *     predicted target value is T[t_i];
 *   - squared distances are evaluated in IEEE binary32: the series are
 *     rounded to float (round to nearest even), then
 *     acc = fmaf(diff_k, diff_k, acc) for k = 0..E-1 from acc = +0 with
 *     diff_k = v_i[k] - v_j[k] rounded to float;
 *   - neighbours are the first E+1 candidates in ascending (d2, j) order, so
 *     distance ties go to the lower time index;
 *   - d_m = sqrt((double) d2_m); if d_1 > 0 then u_m = exp(-d_m / d_1), else
 *     u_m = 1 for d_m == 0 and 0 otherwise; w_m = u_m / sum(u); no weight floor;
 *   - the query point itself is excluded (exclusion radius 0); radius -1
 *     keeps it, radius w > 0 drops every candidate with |j - i| <= w;
 *   - L above the embedded count is clamped to it (L_eff);
 *   - Pearson is two-pass (means, then centred sums) in double; it is NaN when
 *     either input is constant;
 *   - library subsamples are drawn without replacement by Knuth's selection
 *     sampling (TAOCP Vol. 2, Sec. 3.4.2, Algorithm S) driven by SplitMix64
 *     (Steele, Lea & Flood, OOPSLA 2014); the stream for a realization is
 *     keyed by (seed, E, tau, L_eff, r_index) folded one field at a time
 *     through the SplitMix64 output mix, starting from state 0.
 *
 * Option of the build (not of the paper): nested libraries.  For each
 * (E, tau, r_index) one uniformly random ordering of the embedded points is
 * drawn and the library of size L_eff is its first L_eff points, so the
 * libraries of one r_index grow by inclusion with L.  The ordering is the
 * forward Fisher-Yates shuffle (Durstenfeld, CACM 7(7), 1964; Knuth's
 * Algorithm P, TAOCP Vol. 2, Sec. 3.4.2) of 0..N_e-1, stopped after the
 * positions needed: step k swaps position k with position
 * k + floor(z_k (N_e - k) / 2^64), z_k the k-th output of the SplitMix64
 * stream keyed by (seed, E, tau, r_index), folded as above.
 *
 * Option of the build: E-sweep sharing.  For a list of E with maximum
 * E_max, every E uses the same points, the times t >= (E_max - 1) tau
 * (N_c = N - (E_max - 1) tau of them, point c at time c + (E_max - 1) tau,
 * coordinates S[t - k tau] for k < E), the same queries (all N_c points)
 * and, per (tau, L, r), the same library: selection sampling over N_c
 * points with the stream keyed by (seed, 0, tau, L_eff, r_index) (the
 * embedding dimension replaced by 0).  Exclusion is in time steps as usual.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)

/* ------------------------------------------------------------------------ */
/* SplitMix64                                                                */
/* ------------------------------------------------------------------------ */

/* Output mix of SplitMix64 (two xor-shift-multiply rounds, final xor-shift). */
uint64_t oracle_sm64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* One SplitMix64 draw: advance the state by the golden-ratio gamma, mix it. */
uint64_t oracle_sm64_next(uint64_t *state)
{
    *state += 0x9e3779b97f4a7c15ULL;
    return oracle_sm64_mix(*state);
}

/* Stream state of one realization: fold each key field into the state. */
uint64_t oracle_library_state(uint64_t seed, int32_t E, int32_t tau,
                              int64_t L_eff, int32_t r_index)
{
    uint64_t s = 0;
    s = oracle_sm64_mix(s ^ seed);
    s = oracle_sm64_mix(s ^ (uint64_t)(int64_t)E);
    s = oracle_sm64_mix(s ^ (uint64_t)(int64_t)tau);
    s = oracle_sm64_mix(s ^ (uint64_t)L_eff);
    s = oracle_sm64_mix(s ^ (uint64_t)(int64_t)r_index);
    return s;
}

/*
 * Selection sampling (Algorithm S): walk the candidates 0..N_e-1 in order;
 * with s already chosen, candidate j is chosen with probability
 * (L_eff - s) / (N_e - j).  The uniform integer in [0, N_e - j) is the high
 * 64 bits of the 128-bit product of one draw with (N_e - j).
 * Writes L_eff ascending indices; returns how many were written.
 */
int64_t oracle_sample_library(uint64_t seed, int32_t E, int32_t tau,
                              int64_t L_eff, int32_t r_index, int64_t N_e,
                              int32_t *idx_out)
{
    uint64_t st = oracle_library_state(seed, E, tau, L_eff, r_index);
    int64_t s = 0;
    for (int64_t j = 0; j < N_e && s < L_eff; ++j) {
        uint64_t z = oracle_sm64_next(&st);
        unsigned __int128 prod = (unsigned __int128)z * (uint64_t)(N_e - j);
        uint64_t u = (uint64_t)(prod >> 64);
        if (u < (uint64_t)(L_eff - s))
            idx_out[s++] = (int32_t)j;
    }
    return s;
}

/* ------------------------------------------------------------------------ */
/* Distances and neighbours                                                  */
/* ------------------------------------------------------------------------ */

/* Squared distance between embedded points at times ti and tj, in binary32. */
static float sqdist_f32(const float *Sf, int64_t ti, int64_t tj, int E, int tau)
{
    float acc = 0.0f;
    for (int k = 0; k < E; ++k) {
        float diff = Sf[ti - (int64_t)k * tau] - Sf[tj - (int64_t)k * tau];
        acc = fmaf(diff, diff, acc);
    }
    return acc;
}

typedef struct { float d2; int32_t j; } cand_t;

static int cand_less(cand_t a, cand_t b)
{
    return a.d2 < b.d2 || (a.d2 == b.d2 && a.j < b.j);
}

/* Keep the k smallest candidates (lexicographic (d2, j)) in best[0..*n-1],
 * sorted ascending. */
static void keep_smallest(cand_t *best, int *n, int k, cand_t c)
{
    if (*n == k && !cand_less(c, best[k - 1]))
        return;
    int pos = (*n < k) ? *n : k - 1;
    while (pos > 0 && cand_less(c, best[pos - 1])) {
        best[pos] = best[pos - 1];
        --pos;
    }
    best[pos] = c;
    if (*n < k)
        ++*n;
}

/* Simplex-projection prediction from k neighbours sorted by distance. */
static double simplex_predict(const cand_t *best, int k, const double *T,
                              int64_t off)
{
    double d[11], u[11];
    for (int m = 0; m < k; ++m)
        d[m] = sqrt((double)best[m].d2);
    for (int m = 0; m < k; ++m) {
        if (d[0] > 0.0)
            u[m] = exp(-d[m] / d[0]);
        else
            u[m] = (d[m] == 0.0) ? 1.0 : 0.0;
    }
    double su = 0.0;
    for (int m = 0; m < k; ++m)
        su += u[m];
    double p = 0.0;
    for (int m = 0; m < k; ++m)
        p += (u[m] / su) * T[best[m].j + off];
    return p;
}

/* Pearson correlation, two-pass; NaN when either input is constant. */
double oracle_pearson(const double *a, const double *b, int64_t n)
{
    if (n < 2)
        return NAN;
    int a_const = 1, b_const = 1;
    for (int64_t i = 1; i < n; ++i) {
        if (a[i] != a[0]) a_const = 0;
        if (b[i] != b[0]) b_const = 0;
    }
    if (a_const || b_const)
        return NAN;
    double ma = 0.0, mb = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        ma += a[i];
        mb += b[i];
    }
    ma /= (double)n;
    mb /= (double)n;
    double sab = 0.0, saa = 0.0, sbb = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double da = a[i] - ma, db = b[i] - mb;
        sab += da * db;
        saa += da * da;
        sbb += db * db;
    }
    return sab / sqrt(saa * sbb);
}

static int excluded(int64_t i, int64_t j, int32_t excl)
{
    if (excl < 0)
        return 0;
    int64_t d = i > j ? i - j : j - i;
    return d <= excl;
}

/*
 * Neighbours and prediction of one query i: scan every library candidate,
 * keep the first k = E+1 in (d2, j) order, predict T at t_i.
 * Returns 0, or OR_EINVAL if fewer than k candidates remain.
 */
static int one_query(const float *Sf, const double *T, int32_t E, int32_t tau,
                     int64_t off, const int32_t *lib, int64_t L_eff, int32_t excl,
                     int64_t i, cand_t *best, double *pred)
{
    const int k = E + 1;
    int n = 0;
    for (int64_t c = 0; c < L_eff; ++c) {
        const int64_t j = lib[c];
        if (excluded(i, j, excl))
            continue;
        cand_t cd;
        cd.d2 = sqdist_f32(Sf, i + off, j + off, E, tau);
        cd.j = (int32_t)j;
        keep_smallest(best, &n, k, cd);
    }
    if (n < k)
        return OR_EINVAL;
    *pred = simplex_predict(best, k, T, off);
    return OR_OK;
}

/*
 * One realization: library series S (manifold), target T, library indices
 * lib[0..L_eff-1] (embedded-point indices).  Queries are every embedded point
 * (query_set 0) or the library points themselves (query_set 1).  For each
 * query q the k = E+1 neighbours, their squared distances and the prediction
 * are written (any output pointer may be NULL); *rho gets the skill.
 * Returns OR_EINVAL if some query has fewer than E+1 candidates.
 */
int oracle_neighbors(const double *S, const double *T, int64_t N, int32_t E,
                     int32_t tau, const int32_t *lib, int64_t L_eff,
                     int32_t excl, int32_t query_set, int32_t *nbr, float *d2,
                     double *pred, double *rho)
{
    if (!S || !T || !lib || N < 2 || E < 1 || E > 10 || tau < 1)
        return OR_EINVAL;
    const int64_t off = (int64_t)(E - 1) * tau; /* t_i = i + off */
    const int64_t Ne = N - off;
    if (Ne < 2 || L_eff < 1 || L_eff > Ne)
        return OR_EINVAL;
    const int k = E + 1;
    const int64_t Nq = query_set ? L_eff : Ne;

    float *Sf = (float *)malloc(sizeof(float) * (size_t)N);
    double *P = (double *)malloc(sizeof(double) * (size_t)Nq);
    double *O = (double *)malloc(sizeof(double) * (size_t)Nq);
    if (!Sf || !P || !O) {
        free(Sf); free(P); free(O);
        return OR_ENOMEM;
    }
    for (int64_t t = 0; t < N; ++t)
        Sf[t] = (float)S[t];

    int status = OR_OK;
    for (int64_t q = 0; q < Nq; ++q) {
        const int64_t i = query_set ? lib[q] : q;
        cand_t best[11];
        status = one_query(Sf, T, E, tau, off, lib, L_eff, excl, i, best, &P[q]);
        if (status != OR_OK)
            break;
        for (int m = 0; m < k; ++m) {
            if (nbr) nbr[q * k + m] = best[m].j;
            if (d2) d2[q * k + m] = best[m].d2;
        }
        O[q] = T[i + off];
        if (pred) pred[q] = P[q];
    }
    if (status == OR_OK && rho)
        *rho = oracle_pearson(O, P, Nq);
    free(Sf); free(P); free(O);
    return status;
}

/*
 * The same per-query results for an explicit list of queries (embedded
 * indices), without the skill: lets a large realization be checked at sampled
 * queries.  Outputs are [nq][E+1] and [nq].
 */
int oracle_neighbors_at(const double *S, const double *T, int64_t N, int32_t E,
                        int32_t tau, const int32_t *lib, int64_t L_eff,
                        int32_t excl, const int64_t *queries, int64_t nq,
                        int32_t *nbr, float *d2, double *pred)
{
    if (!S || !T || !lib || !queries || N < 2 || E < 1 || E > 10 || tau < 1)
        return OR_EINVAL;
    const int64_t off = (int64_t)(E - 1) * tau;
    const int64_t Ne = N - off;
    if (Ne < 2 || L_eff < 1 || L_eff > Ne)
        return OR_EINVAL;
    const int k = E + 1;
    float *Sf = (float *)malloc(sizeof(float) * (size_t)N);
    if (!Sf)
        return OR_ENOMEM;
    for (int64_t t = 0; t < N; ++t)
        Sf[t] = (float)S[t];
    int status = OR_OK;
    for (int64_t q = 0; q < nq; ++q) {
        const int64_t i = queries[q];
        if (i < 0 || i >= Ne) {
            status = OR_EINVAL;
            break;
        }
        cand_t best[11];
        double p = 0.0;
        status = one_query(Sf, T, E, tau, off, lib, L_eff, excl, i, best, &p);
        if (status != OR_OK)
            break;
        for (int m = 0; m < k; ++m) {
            if (nbr) nbr[q * k + m] = best[m].j;
            if (d2) d2[q * k + m] = best[m].d2;
        }
        if (pred) pred[q] = p;
    }
    free(Sf);
    return status;
}

/* Input rules shared by every entry point. */
static int valid_series(const double *s, int64_t n)
{
    for (int64_t t = 0; t < n; ++t)
        if (!isfinite(s[t]))
            return 0;
    return 1;
}

static int64_t min_library(int32_t E, int32_t excl)
{
    /* enough candidates for E+1 neighbours after the exclusion window */
    int64_t w = excl < 0 ? 0 : 2 * (int64_t)excl + 1;
    return (int64_t)E + 1 + w;
}

/*
 * One realization drawn from the sampler: library of size
 * L_eff = min(L, N_e) for r_index under seed, then oracle_neighbors.
 */
int oracle_realization(const double *S, const double *T, int64_t N, int32_t E,
                       int32_t tau, int64_t L, int32_t r_index, uint64_t seed,
                       int32_t excl, int32_t query_set, int64_t *L_eff_out,
                       double *rho)
{
    if (!S || !T || N < 2 || E < 1 || E > 10 || tau < 1)
        return OR_EINVAL;
    const int64_t Ne = N - (int64_t)(E - 1) * tau;
    const int64_t Le = L < Ne ? L : Ne;
    if (Ne < E + 2 || L < E + 2 || Le < min_library(E, excl))
        return OR_EINVAL;
    int32_t *lib = (int32_t *)malloc(sizeof(int32_t) * (size_t)Le);
    if (!lib)
        return OR_ENOMEM;
    oracle_sample_library(seed, E, tau, Le, r_index, Ne, lib);
    if (L_eff_out)
        *L_eff_out = Le;
    int st = oracle_neighbors(S, T, N, E, tau, lib, Le, excl, query_set,
                              NULL, NULL, NULL, rho);
    free(lib);
    return st;
}

/* Stream of the nested ordering of (E, tau, r_index) under seed. */
uint64_t oracle_nested_state(uint64_t seed, int32_t E, int32_t tau, int32_t r_index)
{
    uint64_t s = 0;
    s = oracle_sm64_mix(s ^ seed);
    s = oracle_sm64_mix(s ^ (uint64_t)(int64_t)E);
    s = oracle_sm64_mix(s ^ (uint64_t)(int64_t)tau);
    s = oracle_sm64_mix(s ^ (uint64_t)(int64_t)r_index);
    return s;
}

/*
 * First n_out points of the nested ordering of 0..N_e-1 (see the header):
 * idx_out[k] for k < n_out, n_out <= N_e.
 */
int oracle_sample_nested(uint64_t seed, int32_t E, int32_t tau, int32_t r_index,
                         int64_t N_e, int64_t n_out, int32_t *idx_out)
{
    if (!idx_out || N_e < 1 || n_out < 0 || n_out > N_e)
        return OR_EINVAL;
    int32_t *a = (int32_t *)malloc(sizeof(int32_t) * (size_t)N_e);
    if (!a)
        return OR_ENOMEM;
    for (int64_t i = 0; i < N_e; ++i)
        a[i] = (int32_t)i;
    uint64_t st = oracle_nested_state(seed, E, tau, r_index);
    for (int64_t k = 0; k < n_out; ++k) {
        uint64_t z = oracle_sm64_next(&st);
        unsigned __int128 prod = (unsigned __int128)z * (uint64_t)(N_e - k);
        int64_t j = k + (int64_t)(prod >> 64);
        int32_t t = a[k];
        a[k] = a[j];
        a[j] = t;
        idx_out[k] = a[k];
    }
    free(a);
    return OR_OK;
}

/*
 * Cross-map over nested libraries for one (E, tau): as oracle_ccm, but the
 * library of (L, r) is the first L_eff points of the nested ordering of r.
 * Queries are every embedded point.
 */
int oracle_ccm_nested(const double *X, const double *Y, int64_t N, int32_t E,
                      int32_t tau, const int64_t *L, int32_t nL, int32_t r,
                      uint64_t seed, int32_t excl, double *rho_xy, double *rho_yx,
                      int64_t *L_eff)
{
    if (!X || !Y || !L || !rho_xy || !rho_yx || N < 2 || E < 1 || E > 10 ||
        tau < 1 || nL < 1 || r < 1)
        return OR_EINVAL;
    if (!valid_series(X, N) || !valid_series(Y, N))
        return OR_EINVAL;
    const int64_t Ne = N - (int64_t)(E - 1) * tau;
    if (Ne < E + 2)
        return OR_EINVAL;
    int64_t Lmax = 0;
    for (int32_t l = 0; l < nL; ++l) {
        const int64_t le = L[l] < Ne ? L[l] : Ne;
        if (L[l] < E + 2 || le < min_library(E, excl))
            return OR_EINVAL;
        if (le > Lmax)
            Lmax = le;
        if (L_eff)
            L_eff[l] = le;
    }
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)Lmax);
    if (!perm)
        return OR_ENOMEM;
    int st = OR_OK;
    for (int32_t q = 0; q < r && st == OR_OK; ++q) {
        st = oracle_sample_nested(seed, E, tau, q, Ne, Lmax, perm);
        for (int32_t l = 0; l < nL && st == OR_OK; ++l) {
            const int64_t le = L[l] < Ne ? L[l] : Ne;
            st = oracle_neighbors(Y, X, N, E, tau, perm, le, excl, 0, NULL, NULL, NULL,
                                  &rho_xy[(int64_t)l * r + q]);
            if (st == OR_OK)
                st = oracle_neighbors(X, Y, N, E, tau, perm, le, excl, 0, NULL, NULL, NULL,
                                      &rho_yx[(int64_t)l * r + q]);
        }
    }
    free(perm);
    return st;
}

/*
 * Cross-map with E-sweep sharing (see the header) for one tau:
 * rho_xy[e][l][r] and rho_yx[e][l][r] for E = Es[e].  Point c of the common
 * range is embedded point c of E in the series shifted by
 * (E_max - E) tau, so each E runs the plain realization on shifted series.
 */
int oracle_ccm_shared_e(const double *X, const double *Y, int64_t N, const int32_t *Es,
                        int32_t nE, int32_t tau, const int64_t *L, int32_t nL, int32_t r,
                        uint64_t seed, int32_t excl, double *rho_xy, double *rho_yx,
                        int64_t *L_eff)
{
    if (!X || !Y || !Es || !L || !rho_xy || !rho_yx || N < 2 || nE < 1 || tau < 1 ||
        nL < 1 || r < 1)
        return OR_EINVAL;
    if (!valid_series(X, N) || !valid_series(Y, N))
        return OR_EINVAL;
    int32_t Emax = 0;
    for (int32_t e = 0; e < nE; ++e) {
        if (Es[e] < 1 || Es[e] > 10)
            return OR_EINVAL;
        if (Es[e] > Emax)
            Emax = Es[e];
    }
    const int64_t Nc = N - (int64_t)(Emax - 1) * tau;
    if (Nc < Emax + 2)
        return OR_EINVAL;
    for (int32_t l = 0; l < nL; ++l) {
        const int64_t le = L[l] < Nc ? L[l] : Nc;
        if (L[l] < Emax + 2 || le < min_library(Emax, excl))
            return OR_EINVAL;
        if (L_eff)
            L_eff[l] = le;
    }
    int32_t *lib = (int32_t *)malloc(sizeof(int32_t) * (size_t)Nc);
    if (!lib)
        return OR_ENOMEM;
    int st = OR_OK;
    for (int32_t l = 0; l < nL && st == OR_OK; ++l) {
        const int64_t le = L[l] < Nc ? L[l] : Nc;
        for (int32_t q = 0; q < r && st == OR_OK; ++q) {
            oracle_sample_library(seed, 0, tau, le, q, Nc, lib);
            for (int32_t e = 0; e < nE && st == OR_OK; ++e) {
                const int64_t d = (int64_t)(Emax - Es[e]) * tau;
                const int64_t at = ((int64_t)e * nL + l) * r + q;
                st = oracle_neighbors(Y + d, X + d, N - d, Es[e], tau, lib, le, excl, 0,
                                      NULL, NULL, NULL, &rho_xy[at]);
                if (st == OR_OK)
                    st = oracle_neighbors(X + d, Y + d, N - d, Es[e], tau, lib, le, excl, 0,
                                          NULL, NULL, NULL, &rho_yx[at]);
            }
        }
    }
    free(lib);
    return st;
}

/*
 * The whole cross-map for one (E, tau): rho_xy[l][r] is the skill of
 * predicting X from Y's manifold, rho_yx[l][r] that of Y from X's manifold.
 */
int oracle_ccm(const double *X, const double *Y, int64_t N, int32_t E,
               int32_t tau, const int64_t *L, int32_t nL, int32_t r,
               uint64_t seed, int32_t excl, int32_t query_set,
               double *rho_xy, double *rho_yx, int64_t *L_eff)
{
    if (!X || !Y || !L || !rho_xy || !rho_yx || N < 2 || E < 1 || E > 10 ||
        tau < 1 || nL < 1 || r < 1)
        return OR_EINVAL;
    if (!valid_series(X, N) || !valid_series(Y, N))
        return OR_EINVAL;
    const int64_t Ne = N - (int64_t)(E - 1) * tau;
    if (Ne < E + 2)
        return OR_EINVAL;
    for (int32_t l = 0; l < nL; ++l) {
        const int64_t le = L[l] < Ne ? L[l] : Ne;
        if (L[l] < E + 2 || le < min_library(E, excl))
            return OR_EINVAL;
    }
    for (int32_t l = 0; l < nL; ++l) {
        int64_t le = 0;
        for (int32_t q = 0; q < r; ++q) {
            int st = oracle_realization(Y, X, N, E, tau, L[l], q, seed, excl,
                                        query_set, &le, &rho_xy[(int64_t)l * r + q]);
            if (st != OR_OK)
                return st;
            st = oracle_realization(X, Y, N, E, tau, L[l], q, seed, excl,
                                    query_set, &le, &rho_yx[(int64_t)l * r + q]);
            if (st != OR_OK)
                return st;
        }
        if (L_eff)
            L_eff[l] = le;
    }
    return OR_OK;
}

/*
 * gm_oracle.c -- CPU oracle for the k-register Gumbel-Max sketch.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header, table or constant
 * generator with the HIP kernels; both sides implement the same written
 * specification (the "draw specification" below) independently.
 *
 * Paper: "Fast Gumbel-Max Sketch and its Applications" (Zhang, Qi, Wang et
 * al., arXiv:2302.05176).  What each function follows:
 *
 *   gmo_sketch(form = PLAIN)          -- Eq. (1) and Eq. (2): the sketch by
 *       its definition, s_j = argmin_i -ln(a_ij)/v_i, y_j = min_i ..., over
 *       every (positive entry, register) pair (Sec. 1, "the straightforward
 *       method", with a_ij generated on the fly from a seeded hash).
 *   gmo_sketch(form = FASTGM_FULL)    -- the FastGM form by its definition:
 *       every positive element emits all k ascending exponential arrivals
 *       (Eq. (7)-(8), Renyi's representation), each routed to the server
 *       named by a Fisher-Yates permutation (Sec. 2.2), and each register
 *       keeps the first arrival it receives.  No pruning.
 *   gmo_sketch(form = FASTGM_ALG1)    -- Algorithm 1 (FastSearch then
 *       FastPrune, Sec. 2.2), with the control-flow fixes listed at the
 *       function.
 *   gmo_sketch(form = FASTGM_STREAM)  -- Algorithm 2 (Stream-FastGM, Sec. 3).
 *   gmo_jaccard / gmo_wcard           -- the estimators of Sec. 1
 *       (probability-Jaccard from matching registers; weighted cardinality
 *       (k-1)/sum_j y_j).
 *   gmo_jp_brute                      -- the probability Jaccard similarity
 *       J_P by its closed form (Sec. 1), O(n^2).
 *   gmo_merge                         -- the sketch of a union from the
 *       sketches of its parts (Sec. 2.3, mergeability).
 *   gmo_setops                        -- union, intersection, relative
 *       complements and weighted Jaccard similarity of two sets from their
 *       sketches (the Lemiesz algebra the paper uses in Sec. 4.5; reading
 *       stated at the function).
 *
 * Parity pins: every function above is checked by the Python suite against
 * values fixed outside this file (splitmix64 known answers, the worked
 * example of Sec. 2.1, closed-form distributions of Sec. 1 and Sec. 2.4-2.5,
 * equality of the three FastGM forms, invariances).  The concrete register
 * values of a sketch are fixed only by the draw specification, so they are
 * pinned by the agreement of the independent implementations plus the
 * statistical checks; the paper prints none.
 *
 * Draw specification (the paper fixes the sketch only in distribution; the
 * readings below make it a deterministic function of (entries, k, seed)):
 *   sm(z)      splitmix64 output function: z += 0x9E3779B97F4A7C15;
 *              z = (z ^ z>>30) * 0xBF58476D1CE4E5B9;
 *              z = (z ^ z>>27) * 0x94D049BB133111EB; return z ^ z>>31.
 *   P_i        sm(sm(seed) ^ (u64)(u32)i)           per element index i
 *   x(tag,j)   sm(P_i ^ ((u64)tag << 32 | (u32)j))   tag 1 = plain register j
 *              (0-based), 2 = arrival uniform, 3 = shuffle draw (step z,
 *              1-based)
 *   U(x)       ((double)(x >> 11) + 0.5) * 2^-53     in [2^-54, 1]
 *   E(x)       neglog(U(x))                          an Exp(1) variate
 *   r_i        1.0 / (double)v_i
 *   plain key  E(x(1,j)) * r_i
 *   FastGM     O_0 = +0; O_z = fma(E(x(2,z)), 1.0/(double)(k-z+1), O_{z-1});
 *              t_z = O_z * r_i;
 *              j_z = z + (((x(3,z) >> 32) * (u64)(k-z+1)) >> 32)  in [z,k];
 *              swap(pi[z], pi[j_z]); server = pi[z] - 1 (0-based).
 *   order      registers keep the lexicographic minimum of (key, index).
 *   empty      register (index -1, value +inf); poisoned vector (index -2,
 *              value NaN) when an entry has a negative, NaN or infinite
 *              weight or a negative index.  Zero weights are skipped.
 *
 * Compile with -ffp-contract=off so no multiply-add is fused behind our back.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* draw specification                                                   */
/* ------------------------------------------------------------------ */

uint64_t gmo_sm64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double gmo_unif(uint64_t x)
{
    return ((double)(x >> 11) + 0.5) * 0x1p-53;
}

/*
 * neglog(u) = -ln(u) for u in (0, 1].
 * Method: the argument reduction of Sun's fdlibm logarithm
 * (u = 2^e * m, m in [sqrt(1/2), sqrt(2)), f = m - 1, s = f / (2 + f)),
 * with ln(1+f) = 2 atanh(s) = 2s + sum_{n>=1} 2 s^(2n+1)/(2n+1) evaluated
 * through the identity 2s = f - f^2/2 + s f^2/2, so that
 *   ln(1+f) = f - (h - s (h + R)),  h = f*f/2,  R = sum_{n=1}^{10} 2 z^n/(2n+1),
 * z = s^2 (Taylor coefficients of atanh; the first omitted term is below
 * 2^-60 relative for |s| <= 0.1716).  ln 2 is split as LN2_HI (exact in
 * e * LN2_HI for |e| < 2^11) plus LN2_LO.  Every operation is an IEEE
 * double +, -, *, / or fma, in the fixed order written here.
 */
static const double LN2_HI = 0x1.62e42fee00000p-1;   /* 6.93147180369123816490e-01 */
static const double LN2_LO = 0x1.a39ef35793c76p-33;  /* ln 2 - LN2_HI, rounded      */

double gmo_neglog(double u)
{
    uint64_t b;
    memcpy(&b, &u, 8);
    int e = (int)(b >> 52) - 1023;
    uint64_t mb = (b & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull;
    double m;
    memcpy(&m, &mb, 8);
    if (m > 0x1.6a09e667f3bcdp+0) { /* m > sqrt(2): move to [sqrt(1/2), 1) */
        m = m * 0.5;
        e = e + 1;
    }
    double f = m - 1.0;
    double s = f / (2.0 + f);
    double z = s * s;
    double R = 2.0 / 21.0;
    R = fma(R, z, 2.0 / 19.0);
    R = fma(R, z, 2.0 / 17.0);
    R = fma(R, z, 2.0 / 15.0);
    R = fma(R, z, 2.0 / 13.0);
    R = fma(R, z, 2.0 / 11.0);
    R = fma(R, z, 2.0 / 9.0);
    R = fma(R, z, 2.0 / 7.0);
    R = fma(R, z, 2.0 / 5.0);
    R = fma(R, z, 2.0 / 3.0);
    R = R * z;
    double h = 0.5 * f * f;
    double de = (double)e;
    double a = h + R;
    double bb = fma(s, a, de * LN2_LO);
    double c = h - bb;
    double d = c - f;              /* d = -(ln m) - e*LN2_LO */
    return d - de * LN2_HI;        /* -(ln u)                */
}

static inline uint64_t elem_prefix(uint64_t seed_mix, int32_t index)
{
    return gmo_sm64(seed_mix ^ (uint64_t)(uint32_t)index);
}

static inline uint64_t draw(uint64_t prefix, uint32_t tag, uint32_t j)
{
    return gmo_sm64(prefix ^ (((uint64_t)tag << 32) | (uint64_t)j));
}

int32_t gmo_randint(uint64_t x, int32_t z, int32_t k)
{
    uint64_t span = (uint64_t)(k - z + 1);
    return z + (int32_t)(((x >> 32) * span) >> 32);
}

uint64_t gmo_prefix(uint64_t seed, int32_t index)
{
    return elem_prefix(gmo_sm64(seed), index);
}

/* E(x): the Exp(1) variate of a draw (+0 when U(x) = 1). */
double gmo_exp1(uint64_t x)
{
    return gmo_neglog(gmo_unif(x));
}

/* ------------------------------------------------------------------ */
/* registers                                                            */
/* ------------------------------------------------------------------ */

/* (t, i) < (y, s) in the lexicographic order that fixes ties. */
static inline int lexless(double t, int32_t i, double y, int32_t s)
{
    return t < y || (t == y && i < s);
}

static void regs_empty(int32_t k, int32_t *s, double *y)
{
    for (int32_t j = 0; j < k; ++j) {
        s[j] = -1;
        y[j] = INFINITY;
    }
}

static void regs_poison(int32_t k, int32_t *s, double *y)
{
    for (int32_t j = 0; j < k; ++j) {
        s[j] = -2;
        y[j] = NAN;
    }
}

/* Entries of one vector: returns 1 if any entry is invalid. */
static int vector_invalid(const int32_t *idx, const float *w, int64_t a, int64_t b)
{
    for (int64_t e = a; e < b; ++e) {
        float v = w[e];
        if (idx[e] < 0 || isnan(v) || isinf(v) || v < 0.0f)
            return 1;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* one element's arrival sequence (the queue Q_i of Sec. 2.2)            */
/* ------------------------------------------------------------------ */

typedef struct {
    int32_t index;
    double r;          /* 1 / v_i               */
    uint64_t prefix;   /* P_i                   */
    int32_t z;         /* arrivals emitted      */
    double O;          /* unscaled order stat   */
    int32_t *pi;       /* pi[1..k], 1-based     */
    int32_t *touched;  /* positions written     */
    int32_t ntouched;
} queue_t;

static void queue_start(queue_t *q, uint64_t seed_mix, int32_t index, float w,
                        int32_t *pi, int32_t *touched)
{
    q->index = index;
    q->r = 1.0 / (double)w;
    q->prefix = elem_prefix(seed_mix, index);
    q->z = 0;
    q->O = 0.0;
    q->pi = pi;
    q->touched = touched;
    q->ntouched = 0;
}

/* pi must hold the identity on entry; restore it for the next element. */
static void queue_finish(queue_t *q)
{
    for (int32_t n = 0; n < q->ntouched; ++n)
        q->pi[q->touched[n]] = q->touched[n];
    q->ntouched = 0;
}

/* Next arrival of the queue: its time t and its 0-based server. */
static void queue_next(queue_t *q, int32_t k, double *t, int32_t *server)
{
    int32_t z = ++q->z;
    double E = gmo_neglog(gmo_unif(draw(q->prefix, 2u, (uint32_t)z)));
    q->O = fma(E, 1.0 / (double)(k - z + 1), q->O);
    *t = q->O * q->r;
    int32_t j = gmo_randint(draw(q->prefix, 3u, (uint32_t)z), z, k);
    int32_t pz = q->pi[z], pj = q->pi[j];
    q->pi[z] = pj;
    q->pi[j] = pz;
    q->touched[q->ntouched++] = z;
    if (j != z)
        q->touched[q->ntouched++] = j;
    *server = pj - 1;
}

/* All k arrivals of one element, for tests (t[z-1], server[z-1]). */
void gmo_element_arrivals(uint64_t seed, int32_t index, float weight, int32_t k,
                          double *t_out, int32_t *server_out)
{
    int32_t *pi = (int32_t *)malloc(sizeof(int32_t) * (size_t)(k + 1));
    int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * k + 2));
    for (int32_t p = 0; p <= k; ++p)
        pi[p] = p;
    queue_t q;
    queue_start(&q, gmo_sm64(seed), index, weight, pi, touched);
    for (int32_t z = 1; z <= k; ++z)
        queue_next(&q, k, &t_out[z - 1], &server_out[z - 1]);
    free(pi);
    free(touched);
}

/* ------------------------------------------------------------------ */
/* per-vector sketch forms                                              */
/* ------------------------------------------------------------------ */

enum { FORM_PLAIN = 0, FORM_FULL = 1, FORM_ALG1 = 2, FORM_STREAM = 3 };

typedef struct {
    int32_t *pi;
    int32_t *touched;
    /* Algorithm 1 per-element state */
    int64_t cap;
    int32_t *eidx;
    double *ev;
    queue_t *qs;
    int32_t *pis;      /* cap * (k+1) */
    int32_t *touch;    /* cap * (2k+2) */
    int64_t *alive;
} scratch_t;

/* Eq. (1)/(2) by definition: every (entry, register) key. */
static int64_t vec_plain(const int32_t *idx, const float *w, int64_t a, int64_t b,
                         int32_t k, uint64_t seed_mix, int32_t *s, double *y)
{
    int64_t keys = 0;
    regs_empty(k, s, y);
    for (int64_t e = a; e < b; ++e) {
        if (!(w[e] > 0.0f))
            continue;
        double r = 1.0 / (double)w[e];
        uint64_t P = elem_prefix(seed_mix, idx[e]);
        for (int32_t j = 0; j < k; ++j) {
            double key = gmo_neglog(gmo_unif(draw(P, 1u, (uint32_t)j))) * r;
            if (lexless(key, idx[e], y[j], s[j])) {
                y[j] = key;
                s[j] = idx[e];
            }
        }
        keys += k;
    }
    return keys;
}

/* FastGM form by definition: all k arrivals of every element, no pruning. */
static int64_t vec_full(const int32_t *idx, const float *w, int64_t a, int64_t b,
                        int32_t k, uint64_t seed_mix, int32_t *s, double *y, scratch_t *sc)
{
    int64_t arrivals = 0;
    regs_empty(k, s, y);
    for (int64_t e = a; e < b; ++e) {
        if (!(w[e] > 0.0f))
            continue;
        queue_t q;
        queue_start(&q, seed_mix, idx[e], w[e], sc->pi, sc->touched);
        for (int32_t z = 1; z <= k; ++z) {
            double t;
            int32_t c;
            queue_next(&q, k, &t, &c);
            if (lexless(t, idx[e], y[c], s[c])) {
                y[c] = t;
                s[c] = idx[e];
            }
        }
        queue_finish(&q);
        arrivals += k;
    }
    return arrivals;
}

static int32_t argmax_reg(int32_t k, const double *y)
{
    int32_t jm = 0;
    for (int32_t j = 1; j < k; ++j)
        if (y[j] > y[jm])
            jm = j;
    return jm;
}

/*
 * The k registers of one sketch with what pruning needs to know about them:
 * how many are still empty, and (once none is) which one holds the largest
 * value y* = max_j y_j.  The largest register can only change when it is
 * itself replaced, so its position is recomputed only then.
 */
typedef struct {
    int32_t k;
    int32_t *s;
    double *y;
    int32_t empty;
    int32_t jstar;
} regset_t;

static void regset_init(regset_t *R, int32_t k, int32_t *s, double *y)
{
    R->k = k;
    R->s = s;
    R->y = y;
    R->empty = k;
    R->jstar = 0;
    regs_empty(k, s, y);
}

/* y* once every register holds an arrival; +inf before (nothing prunes). */
static double regset_ystar(const regset_t *R)
{
    return R->empty > 0 ? INFINITY : R->y[R->jstar];
}

/* Arrival (t, index) at server c: the register keeps the lexicographically
 * smaller (key, index) pair. */
static void regset_offer(regset_t *R, double t, int32_t index, int32_t c)
{
    if (R->s[c] < 0) {
        R->y[c] = t;
        R->s[c] = index;
        if (--R->empty == 0)
            R->jstar = argmax_reg(R->k, R->y);
    } else if (lexless(t, index, R->y[c], R->s[c])) {
        R->y[c] = t;
        R->s[c] = index;
        if (R->empty == 0 && c == R->jstar)
            R->jstar = argmax_reg(R->k, R->y);
    }
}

/*
 * Emit queue q's arrivals until it has emitted `upto` of them (at most k),
 * offering each to its server.  With `prune`, the queue closes at its first
 * arrival later than y* (FastPrune, Sec. 2.2: its later arrivals are larger
 * still, so none of them can replace a register; an arrival equal to y* is
 * still offered).  Returns 1 when the queue is closed: pruned, or all of
 * its k customers emitted.
 */
static int queue_release(queue_t *q, int32_t upto, int prune, regset_t *R, double *last,
                         int64_t *arrivals)
{
    while (q->z < upto) {
        double t;
        int32_t c;
        queue_next(q, R->k, &t, &c);
        ++*arrivals;
        *last = t;
        if (prune && t > regset_ystar(R))
            return 1;
        regset_offer(R, t, q->index, c);
    }
    return q->z >= R->k;
}

static void scratch_grow_alg1(scratch_t *sc, int64_t n, int32_t k)
{
    if (n <= sc->cap)
        return;
    free(sc->eidx);
    free(sc->ev);
    free(sc->qs);
    free(sc->pis);
    free(sc->touch);
    free(sc->alive);
    sc->cap = n;
    sc->eidx = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    sc->ev = (double *)malloc(sizeof(double) * (size_t)n);
    sc->qs = (queue_t *)malloc(sizeof(queue_t) * (size_t)n);
    sc->pis = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * (size_t)(k + 1));
    sc->touch = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * (size_t)(2 * k + 2));
    sc->alive = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
}

/* Release budget of queue i after a total budget R (Sec. 2.1): its share
 * R v_i / S of the arrivals, rounded up, at most k. */
static int32_t release_budget(double R, double v, double S, int32_t k)
{
    double Ri = ceil(R * (v / S));
    return Ri >= (double)k ? k : (int32_t)Ri;
}

/*
 * Algorithm 1 (FastGM, Sec. 2.2).  Every queue releases its share of a
 * growing total budget (k more arrivals per round).  FastSearch: rounds run
 * without pruning until every register holds an arrival.  FastPrune: the
 * rounds go on, and a queue closes at its first arrival later than y*.
 * Readings applied where the printed pseudocode cannot run as written:
 *  - a queue's budget is capped at k (it has only k customers);
 *  - the budget is recomputed in every FastPrune round, and a queue closes
 *    once all of its k customers are out or its latest arrival already lies
 *    above y* (with the budget of an earlier round, a queue that has caught
 *    up would never be removed and the rounds would not end);
 *  - a vector without positive weight returns empty registers (FastSearch
 *    would never end);
 *  - "b_i < y_c" is the lexicographic (key, index) order; the prune test
 *    stays strict.
 */
static int64_t vec_alg1(const int32_t *idx, const float *w, int64_t a, int64_t b,
                        int32_t k, uint64_t seed_mix, int32_t *s, double *y, scratch_t *sc)
{
    regset_t R;
    regset_init(&R, k, s, y);
    int64_t n = 0;
    for (int64_t e = a; e < b; ++e)
        if (w[e] > 0.0f)
            ++n;
    if (n == 0)
        return 0;
    scratch_grow_alg1(sc, n, k);
    double S = 0.0;
    n = 0;
    for (int64_t e = a; e < b; ++e) {
        if (!(w[e] > 0.0f))
            continue;
        sc->eidx[n] = idx[e];
        sc->ev[n] = (double)w[e];
        S += (double)w[e];
        int32_t *pi = sc->pis + n * (int64_t)(k + 1);
        for (int32_t p = 0; p <= k; ++p)
            pi[p] = p;
        queue_start(&sc->qs[n], seed_mix, idx[e], w[e], pi,
                    sc->touch + n * (int64_t)(2 * k + 2));
        ++n;
    }
    int64_t arrivals = 0;
    double budget = 0.0;
    /* latest arrival of each queue (+0 before its first) */
    double *last = (double *)calloc((size_t)n, sizeof(double));
    /* FastSearch */
    while (R.empty > 0) {
        budget += (double)k;
        for (int64_t i = 0; i < n; ++i)
            (void)queue_release(&sc->qs[i], release_budget(budget, sc->ev[i], S, k), 0, &R,
                                &last[i], &arrivals);
    }
    /* FastPrune */
    int64_t nalive = 0;
    for (int64_t i = 0; i < n; ++i)
        sc->alive[nalive++] = i;
    while (nalive > 0) {
        budget += (double)k;
        int64_t keep = 0;
        for (int64_t m = 0; m < nalive; ++m) {
            int64_t i = sc->alive[m];
            queue_t *q = &sc->qs[i];
            int closed = q->z >= k || last[i] > regset_ystar(&R);
            if (!closed)
                closed = queue_release(q, release_budget(budget, sc->ev[i], S, k), 1, &R,
                                       &last[i], &arrivals);
            if (!closed)
                sc->alive[keep++] = i;
        }
        nalive = keep;
    }
    free(last);
    return arrivals;
}

/*
 * Algorithm 2 (Stream-FastGM, Sec. 3): the elements arrive one at a time;
 * each emits its arrivals in ascending order, offering each to its server,
 * and stops at its first arrival later than y* once every register holds an
 * arrival (the prune of Sec. 2.2 against the registers as they stand).
 * Reading: the printed "if k == 0" tests the count of registers still empty.
 */
static int64_t vec_stream(const int32_t *idx, const float *w, int64_t a, int64_t b,
                          int32_t k, uint64_t seed_mix, int32_t *s, double *y, scratch_t *sc)
{
    regset_t R;
    regset_init(&R, k, s, y);
    int64_t arrivals = 0;
    for (int64_t e = a; e < b; ++e) {
        if (!(w[e] > 0.0f))
            continue;
        queue_t q;
        double last = 0.0;
        queue_start(&q, seed_mix, idx[e], w[e], sc->pi, sc->touched);
        (void)queue_release(&q, k, 1, &R, &last, &arrivals);
        queue_finish(&q);
    }
    return arrivals;
}

static int g_threads = 1;

void gmo_set_threads(int n)
{
    g_threads = n < 1 ? 1 : n;
}

int gmo_get_threads(void)
{
    return g_threads;
}

/*
 * Sketch nvec vectors given in CSR form.  Vector v owns entries
 * [off[v], off[v+1]); registers of vector v go to out_*[v*k .. v*k+k).
 * work_out (optional) receives, per vector, the keys (plain) or arrivals
 * (FastGM forms) generated.  Returns 0, or -1 on bad arguments.
 */
int gmo_sketch(int form, const int32_t *idx, const float *w, const int64_t *off,
               int64_t nvec, int32_t k, uint64_t seed,
               int32_t *out_idx, double *out_val, int64_t *work_out)
{
    if (k < 1 || nvec < 0 || form < 0 || form > 3)
        return -1;
    uint64_t seed_mix = gmo_sm64(seed);
    int bad = 0;
#pragma omp parallel num_threads(g_threads)
    {
        scratch_t sc;
        memset(&sc, 0, sizeof(sc));
        sc.pi = (int32_t *)malloc(sizeof(int32_t) * (size_t)(k + 1));
        sc.touched = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * k + 2));
        for (int32_t p = 0; p <= k; ++p)
            sc.pi[p] = p;
#pragma omp for schedule(dynamic, 4)
        for (int64_t v = 0; v < nvec; ++v) {
            int64_t a = off[v], b = off[v + 1];
            int32_t *s = out_idx + v * (int64_t)k;
            double *y = out_val + v * (int64_t)k;
            int64_t work = 0;
            if (b < a) {
                regs_poison(k, s, y);
#pragma omp atomic write
                bad = 1;
            } else if (vector_invalid(idx, w, a, b)) {
                regs_poison(k, s, y);
            } else if (form == FORM_PLAIN) {
                work = vec_plain(idx, w, a, b, k, seed_mix, s, y);
            } else if (form == FORM_FULL) {
                work = vec_full(idx, w, a, b, k, seed_mix, s, y, &sc);
            } else if (form == FORM_ALG1) {
                work = vec_alg1(idx, w, a, b, k, seed_mix, s, y, &sc);
            } else {
                work = vec_stream(idx, w, a, b, k, seed_mix, s, y, &sc);
            }
            if (work_out)
                work_out[v] = work;
        }
        free(sc.pi);
        free(sc.touched);
        free(sc.eidx);
        free(sc.ev);
        free(sc.qs);
        free(sc.pis);
        free(sc.touch);
        free(sc.alive);
    }
    (void)bad;
    return 0;
}

/*
 * Arrivals any exact pruned FastGM run must generate for each vector:
 * sum over positive elements of min(k, #{z : t_z <= y*} + 1), where y* is
 * the largest register of the final sketch (the element must emit its first
 * arrival beyond y* to learn that it can stop; Sec. 2.5).  `y` holds the
 * final FastGM-form sketch values (nvec x k).
 */
void gmo_needed_arrivals(const int32_t *idx, const float *w, const int64_t *off,
                         int64_t nvec, int32_t k, uint64_t seed,
                         const double *y, int64_t *out)
{
    uint64_t seed_mix = gmo_sm64(seed);
#pragma omp parallel num_threads(g_threads)
    {
        int32_t *pi = (int32_t *)malloc(sizeof(int32_t) * (size_t)(k + 1));
        int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * k + 2));
        for (int32_t p = 0; p <= k; ++p)
            pi[p] = p;
#pragma omp for schedule(dynamic, 4)
        for (int64_t v = 0; v < nvec; ++v) {
            const double *yv = y + v * (int64_t)k;
            double ystar = yv[0];
            for (int32_t j = 1; j < k; ++j)
                if (yv[j] > ystar)
                    ystar = yv[j];
            int64_t cnt = 0;
            if (!vector_invalid(idx, w, off[v], off[v + 1])) {
                for (int64_t e = off[v]; e < off[v + 1]; ++e) {
                    if (!(w[e] > 0.0f))
                        continue;
                    queue_t q;
                    queue_start(&q, seed_mix, idx[e], w[e], pi, touched);
                    int32_t z = 0;
                    while (z < k) {
                        double t;
                        int32_t c;
                        queue_next(&q, k, &t, &c);
                        ++z;
                        if (t > ystar)
                            break;
                    }
                    queue_finish(&q);
                    cnt += z;
                }
            }
            out[v] = cnt;
        }
        free(pi);
        free(touched);
    }
}

/* ------------------------------------------------------------------ */
/* release heuristic of the worked example (Sec. 2.1)                   */
/* ------------------------------------------------------------------ */

/* R_i = ceil(R * v_i / sum(v)) for each element. */
void gmo_release_counts(const double *v, int64_t n, double R, int64_t *out)
{
    double S = 0.0;
    for (int64_t i = 0; i < n; ++i)
        S += v[i];
    for (int64_t i = 0; i < n; ++i)
        out[i] = (int64_t)ceil(R * (v[i] / S));
}

/* ------------------------------------------------------------------ */
/* estimators (Sec. 1)                                                  */
/* ------------------------------------------------------------------ */

/* (1/k) #{ j : s_j(a) = s_j(b) }, counting only filled registers. */
double gmo_jaccard(const int32_t *a, const int32_t *b, int32_t k)
{
    int64_t m = 0;
    for (int32_t j = 0; j < k; ++j)
        if (a[j] == b[j] && a[j] >= 0)
            ++m;
    return (double)m / (double)k;
}

/* (k-1) / sum_j y_j, the sum taken left to right. */
double gmo_wcard(const double *y, int32_t k)
{
    double sum = 0.0;
    for (int32_t j = 0; j < k; ++j)
        sum = sum + y[j];
    return (double)(k - 1) / sum;
}

/* ------------------------------------------------------------------ */
/* mergeability (Sec. 2.3) and the weighted-cardinality algebra of two  */
/* sets                                                                 */
/* ------------------------------------------------------------------ */

/*
 * Sketch of the union of r parts from the parts' sketches (Sec. 2.3):
 * y_j is the smallest y_j over the parts and s_j the index that came with
 * it; equal values are ordered by index, the order every register of this
 * oracle keeps.  Empty registers (-1, +inf) take part in nothing; a
 * register that is poisoned (-2, NaN) in any part is poisoned.
 * s_in/y_in: r row-major sketches of k registers.
 */
void gmo_merge(const int32_t *s_in, const double *y_in, int64_t r, int32_t k,
               int32_t *s_out, double *y_out)
{
    for (int32_t j = 0; j < k; ++j) {
        int32_t bs = -1;
        double by = INFINITY;
        int poison = 0;
        for (int64_t q = 0; q < r; ++q) {
            int32_t s = s_in[q * (int64_t)k + j];
            double y = y_in[q * (int64_t)k + j];
            if (s == -2 || isnan(y)) {
                poison = 1;
                continue;
            }
            if (s >= 0 && lexless(y, s, by, bs)) {
                by = y;
                bs = s;
            }
        }
        s_out[j] = poison ? -2 : bs;
        y_out[j] = poison ? NAN : by;
    }
}

/*
 * Weighted cardinalities of two sets A and B (each object with a fixed
 * positive weight, Sec. 1) from their sketches.  The paper names Lemiesz's
 * estimators of the union, intersection, relative complement and weighted
 * Jaccard similarity (Sec. 4.5) without stating them; this is the reading
 * used here:
 *  - the union's sketch is the merge of the two (Sec. 2.3), so its weighted
 *    cardinality is the Sec. 1 estimator (k-1)/sum_j y_j of the merge
 *    (unbiased by Theorem 2);
 *  - register j of the union is won by one object with probability
 *    proportional to its weight (the Gumbel-Max property of Sec. 1 applied
 *    to the union vector).  The winner lies in A and B exactly when both
 *    sketches hold the same (y_j, s_j); in A only when A's register is the
 *    lexicographically smaller; in B only when B's is.  The three counts over
 *    k registers estimate |A&B|_w, |A\B|_w and |B\A|_w as fractions of the
 *    union, and the first one is the weighted Jaccard similarity J_W (for
 *    sets J_W equals J_P of Sec. 1);
 *  - the winner's identity is independent of the union's register values,
 *    so each fraction times the union estimate is unbiased for its part.
 * out[0] = union, out[1] = intersection, out[2] = |A\B|_w, out[3] = |B\A|_w,
 * out[4] = J_W, computed as union = (k-1) / (sum of the merged values, left
 * to right), f = (double)count / (double)k, part = union * f.  Two empty
 * sketches give zeros; a poisoned register makes every output NaN.
 */
void gmo_setops(const int32_t *sa, const double *ya, const int32_t *sb, const double *yb,
                int32_t k, double *out)
{
    double sum = 0.0;
    int64_t neq = 0, nlt = 0, ngt = 0;
    int poison = 0;
    for (int32_t j = 0; j < k; ++j) {
        if (sa[j] == -2 || sb[j] == -2 || isnan(ya[j]) || isnan(yb[j])) {
            poison = 1;
            continue;
        }
        double m;
        if (lexless(ya[j], sa[j], yb[j], sb[j])) {
            m = ya[j];
            if (sa[j] >= 0)
                ++nlt;
        } else if (lexless(yb[j], sb[j], ya[j], sa[j])) {
            m = yb[j];
            if (sb[j] >= 0)
                ++ngt;
        } else {
            m = ya[j];
            if (sa[j] >= 0)
                ++neq;
        }
        sum = sum + m;
    }
    if (poison) {
        for (int q = 0; q < 5; ++q)
            out[q] = NAN;
        return;
    }
    double uni = (double)(k - 1) / sum;
    out[0] = uni;
    out[1] = uni * ((double)neq / (double)k);
    out[2] = uni * ((double)nlt / (double)k);
    out[3] = uni * ((double)ngt / (double)k);
    out[4] = (double)neq / (double)k;
}

/*
 * J_P(u, v) = sum_{i in N+(u) & N+(v)} 1 / sum_l max(u_l/u_i, v_l/v_i),
 * l over the union of the supports (other l contribute 0).  Indices of each
 * side must be distinct.
 */
double gmo_jp_brute(const int32_t *ia, const double *wa, int64_t na,
                    const int32_t *ib, const double *wb, int64_t nb)
{
    /* union support as parallel arrays */
    int64_t nu = 0;
    int32_t *ui = (int32_t *)malloc(sizeof(int32_t) * (size_t)(na + nb + 1));
    double *ua = (double *)malloc(sizeof(double) * (size_t)(na + nb + 1));
    double *ub = (double *)malloc(sizeof(double) * (size_t)(na + nb + 1));
    for (int64_t p = 0; p < na; ++p) {
        if (!(wa[p] > 0.0))
            continue;
        ui[nu] = ia[p];
        ua[nu] = wa[p];
        ub[nu] = 0.0;
        ++nu;
    }
    for (int64_t q = 0; q < nb; ++q) {
        if (!(wb[q] > 0.0))
            continue;
        int64_t p;
        for (p = 0; p < nu; ++p)
            if (ui[p] == ib[q])
                break;
        if (p == nu) {
            ui[nu] = ib[q];
            ua[nu] = 0.0;
            ++nu;
        }
        ub[p] = wb[q];
    }
    double jp = 0.0;
    for (int64_t i = 0; i < nu; ++i) {
        if (!(ua[i] > 0.0 && ub[i] > 0.0))
            continue;
        double den = 0.0;
        for (int64_t l = 0; l < nu; ++l) {
            double x = ua[l] / ua[i], yv = ub[l] / ub[i];
            den += x > yv ? x : yv;
        }
        jp += 1.0 / den;
    }
    free(ui);
    free(ua);
    free(ub);
    return jp;
}

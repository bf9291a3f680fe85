/*
 * oracle.c -- plain, slow, single-threaded CPU reference for the per-edge
 * pattern counts.  TEST INFRASTRUCTURE ONLY: it is called by the tests, by the
 * smoke check and by the benchmark's CPU-baseline leg, never by the product
 * path.  It shares no code, header, table or helper with the HIP library.
 *
 * What it computes (the paper's Section 5 stage compositions, Algorithm 1's
 * nested-loop semantics, and the readings listed in the design notes where
 * the paper is silent):
 *
 *   edge i = (src_i -> dst_i, ts_i); self-loops (src == dst) take part in
 *   nothing and get all-zero rows (the "differentiate" primitive that removes
 *   self-connections, Section 6).  For anchor e = (u -> v, t), window
 *   W = [t - delta, t] (Find_Start(t - delta) then break once a timestamp
 *   exceeds t, Section 6 input specification and the scatter-gather example).
 *
 *   FAN_OUT(e) = #{out-edges of u with ts in W}
 *   FAN_IN(e)  = #{in-edges of v with ts in W}
 *   S(e)       = distinct senders s != v of an edge s -> u, ts in [t-delta, t)
 *                (scatter-gather example: for_all over N0.in_neigh, skip N2 == N1)
 *   M_e(s)     = distinct m with a: s -> m, b: m -> v,
 *                t - delta <= ts_a < ts_b <= t
 *                (the intersection N2.out_neigh with N1.in_neigh; Section 3's
 *                per-intermediate partial order t_i < t_{i+1})
 *   SG_k(e)    = #{s in S(e) : |M_e(s)| >= k}   (a threshold on the number of intermediates, Section 4)
 *   with OR_SG_UNORDERED, M_e(s) drops the order of the two legs:
 *                t - delta <= ts_a < t and t - delta <= ts_b <= t, the
 *                window-only checks of the compiled scatter-gather example
 *                (Section 6) and the optional per-step order of Section 4
 *   GS_k(e)    = |S(e)| if |S(e)| >= k and |D(e)| >= k, else 0, with
 *                tau = earliest ts of an edge into u from s != v in [t-delta, t)
 *                and D(e) = distinct d with u -> d, tau < ts <= t
 *                (the integration phase follows the placement phase, Section 4)
 *   with OR_SG_PHASE, the legs are ordered by phase instead: every scatter
 *                leg of the chosen intermediates (u's included) comes before
 *                every gather leg (the anchor is u's), i.e. SG_k counts the s
 *                for which some split time tau in (t - delta, t] has u's
 *                scatter leg before tau and at least k - 1 other m with a
 *                scatter leg in [t - delta, tau) and a gather leg in
 *                [tau, t] (integration after placement as a whole, Section 4)
 *   CYC_l(e)   = number of l-cycles containing e, 2 <= l <= L: l edges
 *                c_1..c_l with dst(c_i) = src(c_{i+1}) cyclically, strictly
 *                increasing timestamps, ts(c_l) - ts(c_1) <= delta and
 *                pairwise distinct vertices (the classical temporal motif
 *                special case, Section 6; cycle decomposition, Section 5)
 *   with OR_CYC_ANY_ORDER, the cycle's edges may occur in any order (the
 *                anticipatory / out-of-order edges of Section 4): l edges
 *                forming a directed cycle through l distinct vertices whose
 *                timestamps span at most delta; each cycle is counted once,
 *                from its edge of greatest (ts, edge id)
 *   DEG_OUT(e) = distinct destinations of u's out-edges with ts in W, and
 *   DEG_IN(e)  = distinct sources of v's in-edges with ts in W (the
 *                counterparty counts beside the transaction counts FAN_OUT
 *                and FAN_IN; Section 8's Degree features)
 *   with OR_PART, every edge also gets the number of scatter-gather and
 *                gather-scatter instances it belongs to (Table 2's features
 *                count, per transaction, the instances it takes part in):
 *                an instance is a pair (anchor e, sender s) that SG_k(e) or
 *                GS_k(e) counts, and an edge belongs to it when it is an
 *                edge of some realisation of it (one edge per leg, the
 *                legs' order and window conditions met):
 *     SG_PART    the anchor; every s -> u in [t-delta, t); for each
 *                m in M_e(s) other than u, every s -> m in [t-delta, t)
 *                earlier than m's latest gather leg into v (any, unordered)
 *                and every m -> v in [t-delta, t] later than m's first
 *                scatter leg from s (any, unordered); not with OR_SG_PHASE
 *     GS_PART    sender s's legs s -> u in [t-delta, t), and u's
 *                scatter legs u -> d with tau < ts <= t (the anchor among
 *                them), which belong to all |S(e)| instances of e
 *   with OR_SG_SIZES, the SG_k instances of e binned by their size (the
 *                streaming passage of Section 5 counts scatter-gathers of
 *                different sizes): the number of s in S(e) with
 *                |M_e(s)| = k, = k + 1, = k + 2 and >= k + 3 (four columns
 *                summing to SG_k(e)); not with OR_SG_PHASE
 *
 * Stage outputs are vertex sets (Algorithm 1: the output of a stage is nodes,
 * not edges), so S, M and D count distinct vertices; FAN counts edges; cycles
 * are edge sets, so parallel edges give distinct cycles.  Every count is
 * accumulated in 64 bits and saturates on output at a ceiling (2^32 - 1
 * unless the caller lowers it, which lets small graphs reach it).
 *
 * Algorithmic bytes (optional output, one 64-bit counter per anchor and
 * stage) follow a canonical procedure of the method: what an exact miner
 * must read and write for each anchor e = (u -> v, t) when nothing is reused
 * across anchors, an element being a neighbour id plus a time (8 bytes):
 *   B_io(e)    = 12 (src, dst, ts of the edge) + 4 per output column
 *   B_sg/gs(e) = 8 |IN(u) in [t-delta, t)|                    (sender scan)
 *              + 8 sum over s in S(e) of min(n_s, |IN(v) in [t-delta, t]|)
 *                n_s: elements of s's out-slice [t-delta, t) scanned in time
 *                order until k-1 intermediates other than u have qualified
 *                (all of them if fewer do): the set intersection of the
 *                compiled scatter-gather example, bounded by the smaller
 *                side as in Section 6's degree-ordered intersection and
 *                ended early as in Algorithm 1's break conditions
 *              + 8 (elements of OUT(u) in (tau, t] scanned until k distinct
 *                destinations are seen), only when GS is asked for and
 *                |S(e)| >= k
 *   B_cyc(e)   = 12 |OUT(h) in interval| for each partial path of depth
 *                0 .. L-3 (depth 0: head v, interval [t-delta, t); deeper:
 *                (time of the last path edge, t)), + 8 ceil(log2 indeg(u))
 *                for each partial path of depth L-2 whose head has an
 *                out-edge in its interval (the closing edge found by binary
 *                search, Section 6's 4-cycle example), + 8 l for every
 *                l-cycle found (its credits)
 * Only SG / GS and CYC stages that are asked for are charged.
 *
 * Columns, in this order, for the requested patterns only:
 *   FAN_OUT, FAN_IN, SG, GS, CYC_2 .. CYC_L, DEG_OUT, DEG_IN, SG_PART,
 *   GS_PART (with OR_PART, each when its pattern is asked for), then the
 *   four SG size bins.
 * Layout [ncols][n_edges].  DEG_OUT / DEG_IN charge 8 bytes per window
 * element to B_io; the phase-ordered SG scans each sender's out-slice until
 * its condition first holds (the same min with the gather side).  The
 * participation and size columns add only their 4 output bytes each to
 * B_io.
 */
#define _POSIX_C_SOURCE 199309L
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define OR_FAN_OUT 1u
#define OR_FAN_IN 2u
#define OR_SG 4u
#define OR_GS 8u
#define OR_CYC 16u
#define OR_SG_UNORDERED 32u /* modifies OR_SG; adds no column */
#define OR_DEG_OUT 64u
#define OR_DEG_IN 128u
#define OR_SG_PHASE 256u     /* modifies OR_SG; adds no column */
#define OR_CYC_ANY_ORDER 512u /* modifies OR_CYC; adds no column */
#define OR_PART 1024u        /* participation columns of SG and GS */
#define OR_SG_SIZES 2048u    /* SG instances binned by their number of intermediates */

typedef struct {
    uint64_t n;
    uint32_t nv;
    const uint32_t *src, *dst;
    const int64_t *ts;
    uint64_t *out_ptr, *in_ptr; /* nv + 1 */
    uint64_t *out_e, *in_e;     /* valid edge ids per row, sorted by (ts, id) */
} og_graph;

/* ---- sorting valid edge ids by (ts, id) ---------------------------------- */
static const int64_t *g_sort_ts;
static int cmp_ts_id(const void *a, const void *b) {
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    if (g_sort_ts[x] != g_sort_ts[y]) return g_sort_ts[x] < g_sort_ts[y] ? -1 : 1;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static int og_build(og_graph *g, uint64_t n, uint32_t nv, const uint32_t *src, const uint32_t *dst,
                    const int64_t *ts) {
    memset(g, 0, sizeof(*g));
    g->n = n; g->nv = nv; g->src = src; g->dst = dst; g->ts = ts;
    uint64_t nvalid = 0;
    for (uint64_t i = 0; i < n; i++) {
        if (src[i] >= nv || dst[i] >= nv) return 1;
        if (src[i] != dst[i]) nvalid++;
    }
    uint64_t *order = (uint64_t *)malloc(sizeof(uint64_t) * (nvalid ? nvalid : 1));
    g->out_ptr = (uint64_t *)calloc((size_t)nv + 1, sizeof(uint64_t));
    g->in_ptr = (uint64_t *)calloc((size_t)nv + 1, sizeof(uint64_t));
    g->out_e = (uint64_t *)malloc(sizeof(uint64_t) * (nvalid ? nvalid : 1));
    g->in_e = (uint64_t *)malloc(sizeof(uint64_t) * (nvalid ? nvalid : 1));
    uint64_t *fo = (uint64_t *)calloc((size_t)nv + 1, sizeof(uint64_t));
    uint64_t *fi = (uint64_t *)calloc((size_t)nv + 1, sizeof(uint64_t));
    if (!order || !g->out_ptr || !g->in_ptr || !g->out_e || !g->in_e || !fo || !fi) return 2;
    uint64_t m = 0;
    for (uint64_t i = 0; i < n; i++)
        if (src[i] != dst[i]) order[m++] = i;
    g_sort_ts = ts;
    qsort(order, nvalid, sizeof(uint64_t), cmp_ts_id);
    for (uint64_t j = 0; j < nvalid; j++) {
        g->out_ptr[src[order[j]] + 1]++;
        g->in_ptr[dst[order[j]] + 1]++;
    }
    for (uint32_t x = 0; x < nv; x++) {
        g->out_ptr[x + 1] += g->out_ptr[x];
        g->in_ptr[x + 1] += g->in_ptr[x];
    }
    /* appending in (ts, id) order keeps every row in (ts, id) order */
    for (uint64_t j = 0; j < nvalid; j++) {
        uint64_t i = order[j];
        g->out_e[g->out_ptr[src[i]] + fo[src[i]]++] = i;
        g->in_e[g->in_ptr[dst[i]] + fi[dst[i]]++] = i;
    }
    free(order); free(fo); free(fi);
    return 0;
}

static void og_free(og_graph *g) {
    free(g->out_ptr); free(g->in_ptr); free(g->out_e); free(g->in_e);
}

/* first position p in row [b, e) of edge ids with ts[id] >= x */
static uint64_t lower_ts(const og_graph *g, const uint64_t *row, uint64_t b, uint64_t e, int64_t x) {
    while (b < e) {
        uint64_t mid = b + (e - b) / 2;
        if (g->ts[row[mid]] < x) b = mid + 1; else e = mid;
    }
    return b;
}
/* first position p in row [b, e) with ts[id] > x */
static uint64_t upper_ts(const og_graph *g, const uint64_t *row, uint64_t b, uint64_t e, int64_t x) {
    while (b < e) {
        uint64_t mid = b + (e - b) / 2;
        if (g->ts[row[mid]] <= x) b = mid + 1; else e = mid;
    }
    return b;
}

/* saturation at the ceiling (2^32 - 1 by default) */
static uint32_t sat(uint64_t x, uint32_t ceiling) { return x > ceiling ? ceiling : (uint32_t)x; }

uint32_t oracle_num_columns(uint32_t patterns, uint32_t L) {
    uint32_t c = 0;
    if (patterns & OR_FAN_OUT) c++;
    if (patterns & OR_FAN_IN) c++;
    if (patterns & OR_SG) c++;
    if (patterns & OR_GS) c++;
    if (patterns & OR_CYC) c += L - 1;
    if (patterns & OR_DEG_OUT) c++;
    if (patterns & OR_DEG_IN) c++;
    if ((patterns & OR_PART) && (patterns & OR_SG)) c++;
    if ((patterns & OR_PART) && (patterns & OR_GS)) c++;
    if (patterns & OR_SG_SIZES) c += 4;
    return c;
}

/* scratch for the distinct-vertex sets (stamp arrays, one entry per vertex) */
typedef struct {
    uint64_t *stamp_s, *stamp_b, *stamp_m, *stamp_d;
    int64_t *maxb;
    uint64_t *slist;
    int64_t *iv_f, *iv_g;   /* phase order: (first scatter, last gather) per intermediate */
    int64_t *minf;          /* first scatter time from the current sender, per intermediate */
    uint64_t clock;
} og_scratch;

static int scratch_init(og_scratch *s, uint32_t nv) {
    size_t nn = (size_t)nv + 1;
    s->stamp_s = (uint64_t *)calloc(nn, 8); s->stamp_b = (uint64_t *)calloc(nn, 8);
    s->stamp_m = (uint64_t *)calloc(nn, 8); s->stamp_d = (uint64_t *)calloc(nn, 8);
    s->maxb = (int64_t *)calloc(nn, 8); s->slist = (uint64_t *)calloc(nn, 8);
    s->iv_f = (int64_t *)calloc(nn, 8); s->iv_g = (int64_t *)calloc(nn, 8);
    s->minf = (int64_t *)calloc(nn, 8);
    s->clock = 0;
    return (s->stamp_s && s->stamp_b && s->stamp_m && s->stamp_d && s->maxb && s->slist && s->iv_f && s->iv_g &&
            s->minf)
               ? 0 : 2;
}
static void scratch_free(og_scratch *s) {
    free(s->stamp_s); free(s->stamp_b); free(s->stamp_m); free(s->stamp_d); free(s->maxb); free(s->slist);
    free(s->iv_f); free(s->iv_g); free(s->minf);
}

/* Phase order: is there a split time tau with f_u < tau <= (every chosen
 * gather) and at least `need` of the intervals (f_i, g_i] containing tau?
 * The count only rises just after some f_i (or f_u), so those points are
 * the only candidates (the count is checked by brute force). */
static int phase_ok(const int64_t *f, const int64_t *g, uint64_t n, int64_t f_u, int64_t t, uint64_t need) {
    if (need == 0) return 1;
    for (uint64_t c = 0; c <= n; c++) {
        int64_t tau = (c == n ? f_u : f[c]) + 1;
        if (tau <= f_u || tau > t) continue;
        uint64_t cnt = 0;
        for (uint64_t i = 0; i < n; i++) cnt += f[i] < tau && tau <= g[i];
        if (cnt >= need) return 1;
    }
    return 0;
}

/* Anchored columns of edge e: FAN_OUT, FAN_IN, SG_k, GS_k, DEG_OUT, DEG_IN and
 * the four size bins of SG_k (written to out4[0..9]).
 * want_sg / want_gs: which of the scatter-gather columns are asked for (they
 * only decide what *work is charged).  work (may be NULL) receives B_sg/gs.
 * psg / pgs (may be NULL): per-edge participation counters, credited with
 * the edges of every SG / GS instance anchored at e. */
static void anchored(const og_graph *g, og_scratch *sc, uint64_t e, int64_t delta, uint32_t k, int unordered,
                     int phase, int want_sg, int want_gs, int want_deg, uint64_t out4[10], uint64_t *work,
                     uint64_t *psg, uint64_t *pgs) {
    uint32_t u = g->src[e], v = g->dst[e];
    int64_t t = g->ts[e], lo = t - delta;
    for (int i = 0; i < 10; i++) out4[i] = 0;
    if (work) *work = 0;
    if (u == v) return;

    /* FAN: sizes of the window slices (rows are sorted by timestamp) */
    uint64_t ob = g->out_ptr[u], oe = g->out_ptr[u + 1];
    uint64_t ib = g->in_ptr[v], ie = g->in_ptr[v + 1];
    out4[0] = upper_ts(g, g->out_e, ob, oe, t) - lower_ts(g, g->out_e, ob, oe, lo);
    out4[1] = upper_ts(g, g->in_e, ib, ie, t) - lower_ts(g, g->in_e, ib, ie, lo);

    /* DEG: distinct counterparties inside the same slices (only when asked:
       a hub's slices are long) */
    if (want_deg) {
        uint64_t cd = ++sc->clock, nd = 0;
        for (uint64_t p = lower_ts(g, g->out_e, ob, oe, lo); p < upper_ts(g, g->out_e, ob, oe, t); p++) {
            uint32_t d = g->dst[g->out_e[p]];
            if (sc->stamp_d[d] != cd) { sc->stamp_d[d] = cd; nd++; }
        }
        out4[4] = nd;
        cd = ++sc->clock;
        nd = 0;
        for (uint64_t p = lower_ts(g, g->in_e, ib, ie, lo); p < upper_ts(g, g->in_e, ib, ie, t); p++) {
            uint32_t m = g->src[g->in_e[p]];
            if (sc->stamp_d[m] != cd) { sc->stamp_d[m] = cd; nd++; }
        }
        out4[5] = nd;
    }

    /* S(e): distinct senders into u in [lo, t), excluding v */
    uint64_t ub_ = g->in_ptr[u], ue_ = g->in_ptr[u + 1];
    uint64_t p0 = lower_ts(g, g->in_e, ub_, ue_, lo), p1 = lower_ts(g, g->in_e, ub_, ue_, t);
    uint64_t cs = ++sc->clock, nS = 0;
    int have_tau = 0;
    int64_t tau = 0;
    for (uint64_t p = p0; p < p1; p++) {
        uint64_t a = g->in_e[p];
        uint32_t s = g->src[a];
        if (s == v) continue;
        if (!have_tau) { have_tau = 1; tau = g->ts[a]; } /* rows are time-sorted */
        if (sc->stamp_s[s] != cs) { sc->stamp_s[s] = cs; sc->slist[nS++] = s; }
    }
    uint64_t w = 0;
    if (want_sg || want_gs) w += 8 * (p1 - p0);

    /* SG_k: latest gather time into v per in-neighbour m, over [lo, t] */
    uint64_t cb = ++sc->clock;
    uint64_t q0 = lower_ts(g, g->in_e, ib, ie, lo), q1 = upper_ts(g, g->in_e, ib, ie, t);
    for (uint64_t p = q0; p < q1; p++) {
        uint64_t b = g->in_e[p];
        uint32_t m = g->src[b];
        if (sc->stamp_b[m] != cb) { sc->stamp_b[m] = cb; sc->maxb[m] = g->ts[b]; }
        else if (g->ts[b] > sc->maxb[m]) sc->maxb[m] = g->ts[b];
    }
    const uint64_t r_gather = q1 - q0; /* |IN(v) in [lo, t]| */
    uint64_t sg = 0;
    for (uint64_t i = 0; i < nS; i++) {
        uint32_t s = (uint32_t)sc->slist[i];
        uint64_t cm = ++sc->clock, nm = 0;
        uint64_t sb = g->out_ptr[s], se = g->out_ptr[s + 1];
        uint64_t r0 = lower_ts(g, g->out_e, sb, se, lo), r1 = lower_ts(g, g->out_e, sb, se, t);
        /* canonical scan length: elements up to the (k-1)-th qualifying
           intermediate other than u, or the whole slice */
        uint64_t n_s = k >= 2 ? r1 - r0 : 0, found = 0;
        if (phase) {
            /* first scatter leg to u, then the intervals of the other
               intermediates in scan (time) order */
            int64_t f_u = t;
            for (uint64_t p = r0; p < r1; p++)
                if (g->dst[g->out_e[p]] == u) { f_u = g->ts[g->out_e[p]]; break; }
            uint64_t ni = 0;
            int ok = k <= 1;
            for (uint64_t p = r0; p < r1 && !ok; p++) {
                uint64_t a = g->out_e[p];
                uint32_t m = g->dst[a];
                if (m == u || sc->stamp_m[m] == cm) continue;
                sc->stamp_m[m] = cm;           /* first s -> m edge in the window */
                if (sc->stamp_b[m] != cb || g->ts[a] >= sc->maxb[m]) continue;
                sc->iv_f[ni] = g->ts[a];
                sc->iv_g[ni] = sc->maxb[m];
                ni++;
                if (phase_ok(sc->iv_f, sc->iv_g, ni, f_u, t, k - 1)) {
                    ok = 1;
                    n_s = p - r0 + 1;
                }
            }
            if (ok) sg++;
            if (want_sg) w += 8 * (n_s < r_gather ? n_s : r_gather);
            continue;
        }
        for (uint64_t p = r0; p < r1; p++) {
            uint64_t a = g->out_e[p];
            uint32_t m = g->dst[a];
            /* maxb >= lo always: it is a gather time inside the window */
            if (sc->stamp_b[m] == cb && (unordered || g->ts[a] < sc->maxb[m]) && sc->stamp_m[m] != cm) {
                sc->stamp_m[m] = cm;
                sc->minf[m] = g->ts[a]; /* slices run in time order: m's first leg from s */
                nm++;
                if (m != u && k >= 2 && ++found == k - 1) n_s = p - r0 + 1;
            }
        }
        if (nm >= k) {
            sg++;
            /* size bins: exactly k, k + 1, k + 2, at least k + 3 */
            out4[6 + (nm - k < 3 ? nm - k : 3)]++;
            if (psg) {
                /* the edges of the instance (e, s): the anchor, the sender
                   legs, and for every other intermediate m each scatter leg
                   with a later gather leg and each gather leg with an
                   earlier scatter leg (any, unordered) */
                psg[e]++;
                for (uint64_t p = p0; p < p1; p++)
                    if (g->src[g->in_e[p]] == s) psg[g->in_e[p]]++;
                for (uint64_t p = r0; p < r1; p++) {
                    uint64_t a = g->out_e[p];
                    uint32_t m = g->dst[a];
                    if (m != u && sc->stamp_m[m] == cm && (unordered || g->ts[a] < sc->maxb[m])) psg[a]++;
                }
                for (uint64_t p = q0; p < q1; p++) {
                    uint64_t b = g->in_e[p];
                    uint32_t m = g->src[b];
                    if (m != u && sc->stamp_m[m] == cm && (unordered || g->ts[b] > sc->minf[m])) psg[b]++;
                }
            }
        }
        if (want_sg) w += 8 * (n_s < r_gather ? n_s : r_gather);
    }
    out4[2] = sg;

    /* GS_k: distinct destinations of u strictly after tau, up to t */
    if (nS >= k && have_tau) {
        uint64_t cd = ++sc->clock, nd = 0;
        uint64_t d0 = upper_ts(g, g->out_e, ob, oe, tau), d1 = upper_ts(g, g->out_e, ob, oe, t);
        uint64_t scanned = d1 - d0;
        for (uint64_t p = d0; p < d1; p++) {
            uint32_t d = g->dst[g->out_e[p]];
            if (sc->stamp_d[d] != cd) {
                sc->stamp_d[d] = cd;
                if (++nd == k && scanned == d1 - d0) scanned = p - d0 + 1;
            }
        }
        if (nd >= k) {
            out4[3] = nS;
            if (pgs) {
                /* each of the nS instances holds all of u's scatter legs in
                   (tau, t] and its own sender's legs into u */
                for (uint64_t p = d0; p < d1; p++) pgs[g->out_e[p]] += nS;
                for (uint64_t p = p0; p < p1; p++)
                    if (g->src[g->in_e[p]] != v) pgs[g->in_e[p]]++;
            }
        }
        if (want_gs) w += 8 * scanned;
    }
    if (work) *work = w;
}

/* ---- cycles anchored on their last edge, credited to every member edge ---- */
typedef struct {
    const og_graph *g;
    int64_t t, lo;
    uint32_t u, L;
    uint64_t anchor;
    uint64_t path_e[16];
    uint32_t path_v[16];
    uint64_t *acc;      /* [L-1][n] accumulators, column l-2 */
    uint64_t work;      /* B_cyc of the current anchor */
    uint64_t close_b;   /* bytes of one closing search: 8 ceil(log2 indeg(u)) */
    int any_order;      /* edges in any order inside [lo, t], before the anchor by (ts, id) */
} cyc_ctx;

static uint64_t ceil_log2(uint64_t x) {
    uint64_t c = 0;
    while (((uint64_t)1 << c) < x) c++;
    return c;
}

static void cyc_dfs(cyc_ctx *c, uint32_t h, uint32_t d, int64_t tlast) {
    const og_graph *g = c->g;
    uint64_t rb = g->out_ptr[h], re = g->out_ptr[h + 1];
    /* first hop: [lo, t); later hops: (tlast, t); any order: [lo, t] */
    uint64_t p0 = d == 0 || c->any_order ? lower_ts(g, g->out_e, rb, re, c->lo) : upper_ts(g, g->out_e, rb, re, tlast);
    uint64_t p1 = c->any_order ? upper_ts(g, g->out_e, rb, re, c->t) : lower_ts(g, g->out_e, rb, re, c->t);
    /* canonical bytes: scan the slice at depths 0 .. L-3, one closing search
       at depth L-2 (the loop below still walks it, to count the cycles) */
    if (d + 3 <= c->L) c->work += 12 * (p1 - p0);
    else if (p1 > p0) c->work += c->close_b;
    for (uint64_t p = p0; p < p1; p++) {
        uint64_t j = g->out_e[p];
        uint32_t w = g->dst[j];
        /* any order: the anchor is the cycle's edge of greatest (ts, id) */
        if (c->any_order && g->ts[j] == c->t && j >= c->anchor) continue;
        if (w == c->u) {
            uint32_t l = d + 2; /* d path edges + closing edge j + anchor */
            uint64_t *col = c->acc + (uint64_t)(l - 2) * g->n;
            for (uint32_t q = 0; q < d; q++) col[c->path_e[q]]++;
            col[j]++;
            col[c->anchor]++;
            c->work += 8 * (uint64_t)l;
        } else if (d + 1 <= c->L - 2) {
            int seen = 0;
            for (uint32_t q = 0; q <= d; q++)
                if (c->path_v[q] == w) { seen = 1; break; }
            if (seen) continue;
            c->path_e[d] = j;
            c->path_v[d + 1] = w;
            cyc_dfs(c, w, d + 1, g->ts[j]);
        }
    }
}

static int check_params(uint32_t patterns, int64_t delta, uint32_t L, uint32_t k) {
    if (delta < 0) return 3;
    if ((patterns & (OR_SG | OR_GS)) && k == 0) return 3;
    if ((patterns & OR_CYC) && (L < 2 || L > 8)) return 3;
    if ((patterns & OR_SG_UNORDERED) && !(patterns & OR_SG)) return 3;
    if ((patterns & OR_SG_PHASE) && (!(patterns & OR_SG) || (patterns & OR_SG_UNORDERED))) return 3;
    if ((patterns & OR_CYC_ANY_ORDER) && !(patterns & OR_CYC)) return 3;
    if ((patterns & OR_PART) && (!(patterns & (OR_SG | OR_GS)) || (patterns & OR_SG_PHASE))) return 3;
    if ((patterns & OR_SG_SIZES) && (!(patterns & OR_SG) || (patterns & OR_SG_PHASE))) return 3;
    if (patterns & ~(OR_FAN_OUT | OR_FAN_IN | OR_SG | OR_GS | OR_CYC | OR_SG_UNORDERED | OR_DEG_OUT | OR_DEG_IN |
                     OR_SG_PHASE | OR_CYC_ANY_ORDER | OR_PART | OR_SG_SIZES))
        return 3;
    if (!(patterns & (OR_FAN_OUT | OR_FAN_IN | OR_SG | OR_GS | OR_CYC | OR_DEG_OUT | OR_DEG_IN))) return 3;
    return 0;
}

static double now_s(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/*
 * Mining with the anchors restricted to edge ids [a_lo, a_hi): the anchored
 * columns of those edges, and every cycle whose LAST edge is one of them,
 * credited to all of its edges.  Over disjoint ranges the results add up to
 * the full mining.  counts: [ncols][n] uint32 (caller-owned); every count
 * saturates at `ceiling` (0 means 2^32 - 1).  work (may be NULL): [3][n]
 * uint64, the algorithmic bytes B_io, B_sg/gs and B_cyc of each anchor in
 * the range (zero elsewhere).  seconds, if not NULL, receives the wall time
 * of the anchor loops (graph set-up excluded).  Returns 0 on success, 1 on
 * an out-of-range vertex id, 2 on allocation failure, 3 on invalid
 * parameters.
 */
int oracle_mine_ex(uint64_t n, uint32_t nv, const uint32_t *src, const uint32_t *dst, const int64_t *ts,
                   uint32_t patterns, int64_t delta, uint32_t L, uint32_t k, uint64_t a_lo, uint64_t a_hi,
                   uint32_t ceiling, uint32_t *counts, uint64_t *work, double *seconds) {
    int rc = check_params(patterns, delta, L, k);
    if (rc) return rc;
    if (ceiling == 0) ceiling = 0xffffffffu;
    if (a_hi > n) a_hi = n;
    if (a_lo > a_hi) a_lo = a_hi;
    og_graph g;
    og_scratch sc;
    if ((rc = og_build(&g, n, nv, src, dst, ts))) return rc;
    if ((rc = scratch_init(&sc, nv))) return rc;
    uint32_t ncols = oracle_num_columns(patterns, L);
    memset(counts, 0, sizeof(uint32_t) * (size_t)ncols * n);
    if (work) memset(work, 0, sizeof(uint64_t) * 3 * (size_t)n);
    uint32_t col = 0;
    int c_fo = -1, c_fi = -1, c_sg = -1, c_gs = -1, c_cy = -1, c_do = -1, c_di = -1;
    if (patterns & OR_FAN_OUT) c_fo = col++;
    if (patterns & OR_FAN_IN) c_fi = col++;
    if (patterns & OR_SG) c_sg = col++;
    if (patterns & OR_GS) c_gs = col++;
    if (patterns & OR_CYC) { c_cy = col; col += L - 1; }
    if (patterns & OR_DEG_OUT) c_do = col++;
    if (patterns & OR_DEG_IN) c_di = col++;
    int c_ps = -1, c_pg = -1;
    if ((patterns & OR_PART) && (patterns & OR_SG)) c_ps = col++;
    if ((patterns & OR_PART) && (patterns & OR_GS)) c_pg = col++;
    int c_sz = (patterns & OR_SG_SIZES) ? (int)col : -1;
    if (c_sz >= 0) col += 4;
    uint64_t *acc = NULL, *psg = NULL, *pgs = NULL;
    if (c_cy >= 0) {
        acc = (uint64_t *)calloc((size_t)(L - 1) * (n ? n : 1), sizeof(uint64_t));
        if (!acc) { og_free(&g); scratch_free(&sc); return 2; }
    }
    if (c_ps >= 0) psg = (uint64_t *)calloc(n ? n : 1, sizeof(uint64_t));
    if (c_pg >= 0) pgs = (uint64_t *)calloc(n ? n : 1, sizeof(uint64_t));
    if ((c_ps >= 0 && !psg) || (c_pg >= 0 && !pgs)) {
        free(acc); free(psg); free(pgs); og_free(&g); scratch_free(&sc);
        return 2;
    }
    double t0 = now_s();
    if (work)
        for (uint64_t e = a_lo; e < a_hi; e++) work[e] = 12 + 4 * (uint64_t)ncols;
    if (patterns & (OR_FAN_OUT | OR_FAN_IN | OR_SG | OR_GS | OR_DEG_OUT | OR_DEG_IN)) {
        for (uint64_t e = a_lo; e < a_hi; e++) {
            uint64_t r[10];
            anchored(&g, &sc, e, delta, k, (patterns & OR_SG_UNORDERED) != 0, (patterns & OR_SG_PHASE) != 0,
                     (patterns & OR_SG) != 0, (patterns & OR_GS) != 0, (patterns & (OR_DEG_OUT | OR_DEG_IN)) != 0, r,
                     work ? work + n + e : NULL, psg, pgs);
            if (c_fo >= 0) counts[(uint64_t)c_fo * n + e] = sat(r[0], ceiling);
            if (c_fi >= 0) counts[(uint64_t)c_fi * n + e] = sat(r[1], ceiling);
            if (c_sg >= 0) counts[(uint64_t)c_sg * n + e] = sat(r[2], ceiling);
            if (c_gs >= 0) counts[(uint64_t)c_gs * n + e] = sat(r[3], ceiling);
            if (c_do >= 0) counts[(uint64_t)c_do * n + e] = sat(r[4], ceiling);
            if (c_di >= 0) counts[(uint64_t)c_di * n + e] = sat(r[5], ceiling);
            for (int b = 0; b < 4 && c_sz >= 0; b++) counts[(uint64_t)(c_sz + b) * n + e] = sat(r[6 + b], ceiling);
            if (work && src[e] != dst[e]) {
                /* the distinct-counterparty scans read the FAN slices */
                if (c_do >= 0) work[e] += 8 * r[0];
                if (c_di >= 0) work[e] += 8 * r[1];
            }
        }
    }
    if (c_cy >= 0) {
        cyc_ctx c;
        memset(&c, 0, sizeof(c));
        c.g = &g; c.L = L; c.acc = acc; c.any_order = (patterns & OR_CYC_ANY_ORDER) != 0;
        for (uint64_t e = a_lo; e < a_hi; e++) {
            if (src[e] == dst[e]) continue;
            c.u = src[e]; c.t = ts[e]; c.lo = ts[e] - delta; c.anchor = e;
            c.path_v[0] = dst[e];
            c.work = 0;
            c.close_b = 8 * ceil_log2(g.in_ptr[src[e] + 1] - g.in_ptr[src[e]]);
            cyc_dfs(&c, dst[e], 0, 0);
            if (work) work[2 * n + e] = c.work;
        }
    }
    double t1 = now_s();
    if (c_cy >= 0) {
        for (uint32_t l = 0; l + 1 < L; l++)
            for (uint64_t e = 0; e < n; e++)
                counts[(uint64_t)(c_cy + l) * n + e] = sat(acc[(uint64_t)l * n + e], ceiling);
        free(acc);
    }
    /* participation counts: credited to any edge by the anchors in range */
    for (uint64_t e = 0; e < n && c_ps >= 0; e++) counts[(uint64_t)c_ps * n + e] = sat(psg[e], ceiling);
    for (uint64_t e = 0; e < n && c_pg >= 0; e++) counts[(uint64_t)c_pg * n + e] = sat(pgs[e], ceiling);
    free(psg);
    free(pgs);
    if (seconds) *seconds = t1 - t0;
    og_free(&g);
    scratch_free(&sc);
    return 0;
}

/* oracle_mine_ex at the default ceiling, without work counters */
int oracle_mine_range(uint64_t n, uint32_t nv, const uint32_t *src, const uint32_t *dst, const int64_t *ts,
                      uint32_t patterns, int64_t delta, uint32_t L, uint32_t k, uint64_t a_lo, uint64_t a_hi,
                      uint32_t *counts, double *seconds) {
    return oracle_mine_ex(n, nv, src, dst, ts, patterns, delta, L, k, a_lo, a_hi, 0, counts, NULL, seconds);
}

/* Full mining of every edge (see oracle_mine_ex). */
int oracle_mine(uint64_t n, uint32_t nv, const uint32_t *src, const uint32_t *dst, const int64_t *ts,
                uint32_t patterns, int64_t delta, uint32_t L, uint32_t k, uint32_t *counts) {
    return oracle_mine_range(n, nv, src, dst, ts, patterns, delta, L, k, 0, n, counts, NULL);
}

/* ---- cycles through one edge at any position (sampled checks) ----------- */
/*
 * Enumerate the cycle read from e onwards: e, f_1, ..., f_{l-1}, a simple path
 * v -> ... -> u.  In cycle order the timestamps rise everywhere except at the
 * single wrap from c_l back to c_1, so the path is a rising run of edges later
 * than t (they follow e), then a rising run earlier than t (they precede e).
 * The span condition is c_l - c_1 <= delta, c_l being the last edge of the
 * first run (or e) and c_1 the first edge of the second run (or e).
 */
typedef struct {
    const og_graph *g;
    uint64_t e;
    int64_t t, delta;
    uint32_t u, L;
    uint32_t path_v[16];
    uint64_t cnt[9];
} thr_ctx;

static void thr_dfs(thr_ctx *c, uint32_t h, uint32_t d, int phase, int64_t tprev, int64_t c_last,
                    int64_t c_first) {
    /* d edges taken after e; h = head; phase 0 = rising after t, 1 = rising before t */
    const og_graph *g = c->g;
    uint64_t rb = g->out_ptr[h], re = g->out_ptr[h + 1];
    /* every edge of a cycle through e lies within delta of t */
    uint64_t pb = lower_ts(g, g->out_e, rb, re, c->t - c->delta);
    uint64_t pe = upper_ts(g, g->out_e, rb, re, c->t + c->delta);
    for (uint64_t p = pb; p < pe; p++) {
        uint64_t j = g->out_e[p];
        int64_t tj = g->ts[j];
        uint32_t w = g->dst[j];
        int nphase;
        int64_t nlast = c_last, nfirst = c_first;
        if (phase == 0 && tj > tprev && tj > c->t) {
            nphase = 0;
            nlast = tj;
        } else if (tj < c->t && ((phase == 0) || tj > tprev)) {
            nphase = 1;
            if (phase == 0) nfirst = tj;
        } else {
            continue;
        }
        if (nlast - nfirst > c->delta) continue;
        if (w == c->u) {
            uint32_t l = d + 2;
            if (l <= c->L) c->cnt[l]++;
            continue;
        }
        if (d + 2 >= c->L) continue; /* a longer path could not close within L */
        int seen = 0;
        for (uint32_t q = 0; q <= d; q++)
            if (c->path_v[q] == w) { seen = 1; break; }
        if (seen) continue;
        c->path_v[d + 1] = w;
        thr_dfs(c, w, d + 1, nphase, tj, nlast, nfirst);
    }
}

/*
 * Sampled mining: the same columns as oracle_mine but only for the listed
 * edges (rows of out: [ncols][n_sel]).  Cycle columns are computed by the
 * through-edge enumeration above, independently of oracle_mine's
 * last-edge-anchored search.
 */
int oracle_mine_selected(uint64_t n, uint32_t nv, const uint32_t *src, const uint32_t *dst,
                         const int64_t *ts, uint32_t patterns, int64_t delta, uint32_t L, uint32_t k,
                         const uint64_t *sel, uint64_t n_sel, uint32_t *out) {
    int rc = check_params(patterns, delta, L, k);
    if (rc) return rc;
    /* the time-ordered patterns only (the through-edge enumeration is theirs) */
    if (patterns & (OR_SG_PHASE | OR_CYC_ANY_ORDER | OR_DEG_OUT | OR_DEG_IN | OR_PART | OR_SG_SIZES)) return 3;
    og_graph g;
    og_scratch sc;
    if ((rc = og_build(&g, n, nv, src, dst, ts))) return rc;
    if ((rc = scratch_init(&sc, nv))) return rc;
    uint32_t ncols = oracle_num_columns(patterns, L);
    memset(out, 0, sizeof(uint32_t) * (size_t)ncols * n_sel);
    for (uint64_t i = 0; i < n_sel; i++) {
        uint64_t e = sel[i];
        if (e >= n) { og_free(&g); scratch_free(&sc); return 3; }
        uint32_t col = 0;
        uint64_t r[10];
        anchored(&g, &sc, e, delta, k, (patterns & OR_SG_UNORDERED) != 0, 0, 0, 0, 0, r, NULL, NULL, NULL);
        if (patterns & OR_FAN_OUT) out[(uint64_t)(col++) * n_sel + i] = sat(r[0], 0xffffffffu);
        if (patterns & OR_FAN_IN) out[(uint64_t)(col++) * n_sel + i] = sat(r[1], 0xffffffffu);
        if (patterns & OR_SG) out[(uint64_t)(col++) * n_sel + i] = sat(r[2], 0xffffffffu);
        if (patterns & OR_GS) out[(uint64_t)(col++) * n_sel + i] = sat(r[3], 0xffffffffu);
        if ((patterns & OR_CYC) && src[e] != dst[e]) {
            thr_ctx c;
            memset(&c, 0, sizeof(c));
            c.g = &g; c.e = e; c.t = ts[e]; c.delta = delta; c.u = src[e]; c.L = L;
            c.path_v[0] = dst[e];
            thr_dfs(&c, dst[e], 0, 0, ts[e], ts[e], ts[e]);
            for (uint32_t l = 2; l <= L; l++) out[(uint64_t)(col + l - 2) * n_sel + i] = sat(c.cnt[l], 0xffffffffu);
        }
    }
    og_free(&g);
    scratch_free(&sc);
    return 0;
}

/*
 * Number of distinct l-cycles, each counted once from its FIRST edge c_1:
 * a forward search over strictly later edges with timestamps up to
 * ts(c_1) + delta that closes back at src(c_1).  Used for the identity
 * sum_e CYC_l(e) = l * C_l.  Output cnt[l] for l = 2..L (cnt has L+1 slots).
 */
typedef struct {
    const og_graph *g;
    int64_t t1, delta;
    uint32_t s0, L;
    uint32_t path_v[16];
    uint64_t *cnt;
} fwd_ctx;

/* m = edges on the path so far; path_v[0..m] = s0, ..., h */
static void fwd_dfs(fwd_ctx *c, uint32_t h, uint32_t m, int64_t tprev) {
    const og_graph *g = c->g;
    uint64_t rb = g->out_ptr[h], re = g->out_ptr[h + 1];
    uint64_t p0 = upper_ts(g, g->out_e, rb, re, tprev);
    uint64_t p1 = upper_ts(g, g->out_e, rb, re, c->t1 + c->delta);
    for (uint64_t p = p0; p < p1; p++) {
        uint64_t j = g->out_e[p];
        uint32_t w = g->dst[j];
        if (w == c->s0) {
            if (m + 1 <= c->L) c->cnt[m + 1]++;
            continue;
        }
        if (m + 2 > c->L) continue;
        int seen = 0;
        for (uint32_t q = 0; q <= m; q++)
            if (c->path_v[q] == w) { seen = 1; break; }
        if (seen) continue;
        c->path_v[m + 1] = w;
        fwd_dfs(c, w, m + 1, g->ts[j]);
    }
}

int oracle_count_cycles_first(uint64_t n, uint32_t nv, const uint32_t *src, const uint32_t *dst,
                              const int64_t *ts, int64_t delta, uint32_t L, uint64_t *cnt) {
    int rc = check_params(OR_CYC, delta, L, 1);
    if (rc) return rc;
    og_graph g;
    if ((rc = og_build(&g, n, nv, src, dst, ts))) return rc;
    memset(cnt, 0, sizeof(uint64_t) * (L + 1));
    fwd_ctx c;
    memset(&c, 0, sizeof(c));
    c.g = &g; c.delta = delta; c.L = L; c.cnt = cnt;
    for (uint64_t e = 0; e < n; e++) {
        if (src[e] == dst[e]) continue;
        c.s0 = src[e];
        c.t1 = ts[e];
        c.path_v[0] = src[e];
        c.path_v[1] = dst[e];
        fwd_dfs(&c, dst[e], 1, ts[e]);
    }
    og_free(&g);
    return 0;
}

/*
 * CPU oracle for round-synchronous peeling and IBLT listing.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path may link,
 * load or call this file; only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg do.  It shares no code, header, table or helper
 * with the HIP library: every routine below is written directly from the
 * paper's definitions, plainly and slowly, so that a reader can check it
 * against the paper by eye.
 *
 * Paper: J. Jiang, M. Mitzenmacher, J. Thaler, "Parallel Peeling Algorithms".
 *
 *   - k-core and the sequential peeling process: Section 1 (Introduction).
 *   - Round-synchronous parallel peeling (every vertex of degree < k removed
 *     at once, with its incident edges, each round): Section 1 and Section 3.
 *   - IBLT insert/delete, pure cells and recovery: Section 5, "Motivation".
 *   - One pure-cell thread per cell per round, stop when a round recovers
 *     nothing, never peel an item twice: Section 5, "Implementation Details".
 *
 * Conventions the paper leaves open (each is a stated reading):
 *   - Degree counts incidences with multiplicity (an edge listing a vertex
 *     twice adds two to its degree).
 *   - Rounds are numbered from 1; a vertex's round is the round that removed
 *     it, 0 means it is in the k-core; an edge's round is the round that
 *     removed it, 0 means it is in the core.  A vertex of degree 0 is removed
 *     in round 1.  The run's round count is the last round that removed a
 *     vertex; the empty round that detects termination is not counted.
 *   - Final degree: a core vertex keeps its degree within the core; a removed
 *     vertex ends at 0, because every edge that still held it died in its
 *     removal round.
 *   - IBLT cells carry an int32 count beside the key and checksum fields; a
 *     cell is pure when its count is 1 and its checksum field equals the
 *     checksum of its key field.  A cell with count 1 whose checksum does not
 *     match is not pure and flags the table as corrupt.
 *   - Hashing: the r cell hashes and the checksum are SplitMix64's finaliser
 *     applied to key XOR a per-function salt, the cell drawn from its
 *     subtable by multiply-shift; salts are draws 0..r-1 (cells) and 8
 *     (checksum) of the SplitMix64 stream of the table seed.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ERANGE (-2)
#define ORC_ENOSPC (-3)
#define ORC_EROUNDS (-4)
#define ORC_ECORRUPT (-5)
#define ORC_ENOMEM (-7)

/* ------------------------------------------------------------------------- */
/* SplitMix64 (Steele, Lea, Flood, OOPSLA 2014), written from its definition. */

static uint64_t orc_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

uint64_t orc_splitmix64(uint64_t seed, uint64_t i)
{
    return orc_mix64(seed + (i + 1) * 0x9e3779b97f4a7c15ULL);
}

static uint64_t orc_mulhi(uint64_t a, uint64_t b)
{
    return (uint64_t)(((unsigned __int128)a * (unsigned __int128)b) >> 64);
}

/* ------------------------------------------------------------------------- */
/* Vertex -> incident edge lists (one entry per incidence).                   */

typedef struct {
    uint64_t *start; /* n+1 */
    uint64_t *edge;  /* m*r */
} orc_incidence;

static int orc_incidence_build(uint32_t n, uint64_t m, uint32_t r,
                               const uint32_t *edges, orc_incidence *g)
{
    uint64_t i, nr = m * (uint64_t)r;
    uint64_t *fill;
    g->start = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    g->edge = (uint64_t *)malloc((size_t)(nr ? nr : 1) * sizeof(uint64_t));
    fill = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    if (!g->start || !g->edge || !fill) {
        free(g->start); free(g->edge); free(fill);
        return ORC_ENOMEM;
    }
    for (i = 0; i < nr; i++) {
        if (edges[i] >= n) { free(g->start); free(g->edge); free(fill); return ORC_ERANGE; }
        g->start[edges[i] + 1]++;
    }
    for (i = 0; i < n; i++) g->start[i + 1] += g->start[i];
    for (i = 0; i < nr; i++) {
        uint32_t v = edges[i];
        g->edge[g->start[v] + fill[v]] = i / r;
        fill[v]++;
    }
    free(fill);
    return ORC_OK;
}

static void orc_incidence_free(orc_incidence *g)
{
    free(g->start);
    free(g->edge);
}

/* ------------------------------------------------------------------------- */
/* Round-synchronous parallel peeling (Section 1; Section 3).                 */
/*
 * Round t = 1, 2, ...:
 *   F_t = { v alive : deg(v) < k }, degrees taken at the start of the round;
 *   stop when F_t is empty;
 *   every v in F_t is removed in round t;
 *   every alive edge with a vertex in F_t is removed in round t;
 *   each removed edge lowers the degree of each of its r slots by one.
 * V[t-1] = |F_t|, E[t-1] = number of edges removed in round t.
 * Returns ORC_EROUNDS, with the state after max_rounds rounds, if round
 * max_rounds+1 would still remove a vertex.
 */
int orc_peel_rounds(uint32_t n, uint64_t m, uint32_t r, uint32_t k,
                    const uint32_t *edges, uint32_t max_rounds,
                    uint32_t *vertex_round, uint32_t *edge_round,
                    uint32_t *deg_out, uint64_t *V, uint64_t *E,
                    uint32_t *rounds_out, uint32_t *edge_rounds_out)
{
    orc_incidence g;
    uint32_t *deg, *frontier;
    uint64_t *killed;
    uint64_t i, v;
    uint32_t t, last_v = 0, last_e = 0;
    int rc;

    if (n == 0 || r < 2 || r > 8 || k == 0) return ORC_EINVAL;
    rc = orc_incidence_build(n, m, r, edges, &g);
    if (rc) return rc;
    deg = (uint32_t *)calloc(n, sizeof(uint32_t));
    frontier = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    killed = (uint64_t *)malloc((size_t)(m ? m : 1) * sizeof(uint64_t));
    if (!deg || !frontier || !killed) {
        free(deg); free(frontier); free(killed); orc_incidence_free(&g);
        return ORC_ENOMEM;
    }
    for (i = 0; i < m * (uint64_t)r; i++) deg[edges[i]]++;
    memset(vertex_round, 0, (size_t)n * sizeof(uint32_t));
    memset(edge_round, 0, (size_t)m * sizeof(uint32_t));

    rc = ORC_OK;
    for (t = 1;; t++) {
        uint64_t nf = 0, ne = 0;
        /* F_t from the degrees at the start of round t. */
        for (v = 0; v < n; v++)
            if (vertex_round[v] == 0 && deg[v] < k) frontier[nf++] = (uint32_t)v;
        if (nf == 0) break;
        if (t > max_rounds) { rc = ORC_EROUNDS; break; }
        for (i = 0; i < nf; i++) vertex_round[frontier[i]] = t;
        /* Every alive edge touching F_t dies in round t (once). */
        for (i = 0; i < nf; i++) {
            uint32_t u = frontier[i];
            uint64_t p;
            for (p = g.start[u]; p < g.start[u + 1]; p++) {
                uint64_t e = g.edge[p];
                if (edge_round[e] == 0) {
                    edge_round[e] = t;
                    killed[ne++] = e;
                }
            }
        }
        /* Each removed edge lowers the degree of each of its slots. */
        for (i = 0; i < ne; i++) {
            uint32_t j;
            for (j = 0; j < r; j++) deg[edges[killed[i] * r + j]]--;
        }
        V[t - 1] = nf;
        E[t - 1] = ne;
        last_v = t;
        if (ne) last_e = t;
    }
    memcpy(deg_out, deg, (size_t)n * sizeof(uint32_t));
    *rounds_out = last_v;
    *edge_rounds_out = last_e;
    free(deg); free(frontier); free(killed);
    orc_incidence_free(&g);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Peeling with subtables (Appendix B): the vertex ids are split into r      */
/* consecutive subtables of near-equal size (the first n mod r one larger),  */
/* and each round is r subrounds; subround (i, j) removes, at once, every    */
/* alive vertex of subtable j whose degree is below k at the start of the    */
/* subround, with the edges it still holds.  Subrounds are numbered          */
/* s = (i-1) r + j from 1 and an empty subround still takes its number; the  */
/* run ends after r empty subrounds in a row (no subtable has a vertex to    */
/* remove).  Outputs as orc_peel_rounds, per subround; *rounds_out is the    */
/* last subround that removed a vertex.                                      */

int orc_peel_subrounds(uint32_t n, uint64_t m, uint32_t r, uint32_t k,
                       const uint32_t *edges, uint32_t max_rounds,
                       uint32_t *vertex_round, uint32_t *edge_round,
                       uint32_t *deg_out, uint64_t *V, uint64_t *E,
                       uint32_t *rounds_out, uint32_t *edge_rounds_out)
{
    orc_incidence g;
    uint32_t *deg, *frontier, *lo;
    uint64_t *killed;
    uint64_t i, v;
    uint32_t s, j, empty = 0, last_v = 0, last_e = 0;
    int rc;

    if (n == 0 || r < 2 || r > 8 || k == 0) return ORC_EINVAL;
    rc = orc_incidence_build(n, m, r, edges, &g);
    if (rc) return rc;
    deg = (uint32_t *)calloc(n, sizeof(uint32_t));
    frontier = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    killed = (uint64_t *)malloc((size_t)(m ? m : 1) * sizeof(uint64_t));
    lo = (uint32_t *)malloc((r + 1) * sizeof(uint32_t));
    if (!deg || !frontier || !killed || !lo) {
        free(deg); free(frontier); free(killed); free(lo); orc_incidence_free(&g);
        return ORC_ENOMEM;
    }
    /* subtable j holds ids lo[j] .. lo[j+1]-1 */
    lo[0] = 0;
    for (j = 0; j < r; j++) lo[j + 1] = lo[j] + n / r + (j < n % r ? 1u : 0u);
    for (i = 0; i < m * (uint64_t)r; i++) deg[edges[i]]++;
    memset(vertex_round, 0, (size_t)n * sizeof(uint32_t));
    memset(edge_round, 0, (size_t)m * sizeof(uint32_t));

    rc = ORC_OK;
    for (s = 1;; s++) {
        uint64_t nf = 0, ne = 0;
        j = (s - 1) % r;
        for (v = lo[j]; v < lo[j + 1]; v++)
            if (vertex_round[v] == 0 && deg[v] < k) frontier[nf++] = (uint32_t)v;
        if (nf == 0) {
            if (s <= max_rounds) { V[s - 1] = 0; E[s - 1] = 0; }
            if (++empty == r) break;
            continue;
        }
        empty = 0;
        if (s > max_rounds) { rc = ORC_EROUNDS; break; }
        for (i = 0; i < nf; i++) vertex_round[frontier[i]] = s;
        for (i = 0; i < nf; i++) {
            uint32_t u = frontier[i];
            uint64_t p;
            for (p = g.start[u]; p < g.start[u + 1]; p++) {
                uint64_t e = g.edge[p];
                if (edge_round[e] == 0) {
                    edge_round[e] = s;
                    killed[ne++] = e;
                }
            }
        }
        for (i = 0; i < ne; i++) {
            uint32_t q;
            for (q = 0; q < r; q++) deg[edges[killed[i] * r + q]]--;
        }
        V[s - 1] = nf;
        E[s - 1] = ne;
        last_v = s;
        if (ne) last_e = s;
    }
    memcpy(deg_out, deg, (size_t)n * sizeof(uint32_t));
    *rounds_out = last_v;
    *edge_rounds_out = last_e;
    free(deg); free(frontier); free(killed); free(lo);
    orc_incidence_free(&g);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Sequential peeling process (Section 1): repeatedly remove one vertex of   */
/* degree < k with its edges.  order_seed == 0 pops in FIFO order; any other */
/* value pops a uniformly chosen queued vertex (used to check that the core  */
/* does not depend on the order).  Outputs 0/1 core membership masks.        */

int orc_peel_queue(uint32_t n, uint64_t m, uint32_t r, uint32_t k,
                   const uint32_t *edges, uint64_t order_seed,
                   uint8_t *core_vertex, uint8_t *core_edge)
{
    orc_incidence g;
    uint32_t *deg, *queue;
    uint8_t *queued;
    uint64_t i, head = 0, tail = 0, draw = 0;
    int rc;

    if (n == 0 || r < 2 || r > 8 || k == 0) return ORC_EINVAL;
    rc = orc_incidence_build(n, m, r, edges, &g);
    if (rc) return rc;
    deg = (uint32_t *)calloc(n, sizeof(uint32_t));
    queue = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    queued = (uint8_t *)calloc(n, 1);
    if (!deg || !queue || !queued) {
        free(deg); free(queue); free(queued); orc_incidence_free(&g);
        return ORC_ENOMEM;
    }
    for (i = 0; i < m * (uint64_t)r; i++) deg[edges[i]]++;
    memset(core_vertex, 1, n);
    memset(core_edge, 1, (size_t)m);
    for (i = 0; i < n; i++)
        if (deg[i] < k) { queue[tail++] = (uint32_t)i; queued[i] = 1; }
    while (head < tail) {
        uint32_t v;
        uint64_t p;
        if (order_seed) {
            uint64_t pick = head + orc_mulhi(orc_splitmix64(order_seed, draw++), tail - head);
            uint32_t tmp = queue[pick];
            queue[pick] = queue[head];
            queue[head] = tmp;
        }
        v = queue[head++];
        core_vertex[v] = 0;
        for (p = g.start[v]; p < g.start[v + 1]; p++) {
            uint64_t e = g.edge[p];
            uint32_t j;
            if (!core_edge[e]) continue;
            core_edge[e] = 0;
            for (j = 0; j < r; j++) {
                uint32_t u = edges[e * r + j];
                deg[u]--;
                if (core_vertex[u] && !queued[u] && deg[u] < k) {
                    queue[tail++] = u;
                    queued[u] = 1;
                }
            }
        }
    }
    free(deg); free(queue); free(queued);
    orc_incidence_free(&g);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Brute force k-core for tiny hypergraphs (m <= 24).  The k-core is the      */
/* maximal sub-hypergraph in which every vertex has degree >= k (Section 1):  */
/* its edge set is the union of all edge sets S such that every vertex that  */
/* S touches has >= k incidences in S (such sets are closed under union).    */
/* Its vertex set is the set of vertices those edges touch.                  */

int orc_core_brute(uint32_t n, uint64_t m, uint32_t r, uint32_t k,
                   const uint32_t *edges, uint8_t *core_vertex, uint8_t *core_edge)
{
    uint64_t s, e;
    uint64_t best = 0;
    uint32_t *cnt;
    if (n == 0 || r < 2 || r > 8 || k == 0 || m > 24) return ORC_EINVAL;
    cnt = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    if (!cnt) return ORC_ENOMEM;
    for (s = 1; s < (1ULL << m); s++) {
        int ok = 1;
        memset(cnt, 0, (size_t)n * sizeof(uint32_t));
        for (e = 0; e < m; e++)
            if (s >> e & 1) {
                uint32_t j;
                for (j = 0; j < r; j++) cnt[edges[e * r + j]]++;
            }
        for (e = 0; e < m && ok; e++)
            if (s >> e & 1) {
                uint32_t j;
                for (j = 0; j < r; j++)
                    if (cnt[edges[e * r + j]] < k) ok = 0;
            }
        if (ok) best |= s;
    }
    memset(core_vertex, 0, n);
    for (e = 0; e < m; e++) {
        core_edge[e] = (uint8_t)(best >> e & 1);
        if (core_edge[e]) {
            uint32_t j;
            for (j = 0; j < r; j++) core_vertex[edges[e * r + j]] = 1;
        }
    }
    free(cnt);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* IBLT (Section 5).                                                          */

typedef struct {
    uint64_t ncells;
    uint32_t r;
    uint64_t base[8], size[8];
    uint64_t salt[8];
    uint64_t salt_chk;
} orc_iblt;

static int orc_iblt_setup(orc_iblt *t, uint64_t ncells, uint32_t r, uint64_t seed)
{
    uint32_t j;
    uint64_t acc = 0;
    if (r < 2 || r > 8 || ncells < r || ncells > 0xFFFFFFFFULL) return ORC_EINVAL;
    t->ncells = ncells;
    t->r = r;
    for (j = 0; j < r; j++) {
        t->size[j] = ncells / r + (j < ncells % r ? 1 : 0);
        t->base[j] = acc;
        acc += t->size[j];
        t->salt[j] = orc_splitmix64(seed, j);
    }
    t->salt_chk = orc_splitmix64(seed, 8);
    return ORC_OK;
}

/* Cell of key x in subtable j: one uniform cell of that subtable. */
static uint64_t orc_iblt_cell(const orc_iblt *t, uint32_t j, uint64_t x)
{
    return t->base[j] + orc_mulhi(orc_mix64(x ^ t->salt[j]), t->size[j]);
}

/* checkSum(x): the "simple pseudorandom function" of the checksum field. */
static uint64_t orc_iblt_check(const orc_iblt *t, uint64_t x)
{
    return orc_mix64(x ^ t->salt_chk);
}

int orc_iblt_cells_of(uint64_t ncells, uint32_t r, uint64_t seed,
                      const uint64_t *keys, uint64_t nkeys,
                      uint64_t *cells /* nkeys*r */, uint64_t *checks /* nkeys */)
{
    orc_iblt t;
    uint64_t i;
    uint32_t j;
    int rc = orc_iblt_setup(&t, ncells, r, seed);
    if (rc) return rc;
    for (i = 0; i < nkeys; i++) {
        for (j = 0; j < r; j++) cells[i * r + j] = orc_iblt_cell(&t, j, keys[i]);
        checks[i] = orc_iblt_check(&t, keys[i]);
    }
    return ORC_OK;
}

/* Insert (sign = +1) or delete (sign = -1) keys: XOR x into the key field and */
/* checkSum(x) into the checksum field of each of the key's r cells; the count */
/* moves by sign.  Insert and delete XOR the same values.                      */
int orc_iblt_update(uint64_t ncells, uint32_t r, uint64_t seed,
                    int32_t *count, uint64_t *key_sum, uint64_t *hash_sum,
                    const uint64_t *keys, uint64_t nkeys, int32_t sign)
{
    orc_iblt t;
    uint64_t i;
    uint32_t j;
    int rc = orc_iblt_setup(&t, ncells, r, seed);
    if (rc) return rc;
    for (i = 0; i < nkeys; i++) {
        uint64_t x = keys[i], h = orc_iblt_check(&t, x);
        for (j = 0; j < r; j++) {
            uint64_t c = orc_iblt_cell(&t, j, x);
            count[c] += sign;
            key_sum[c] ^= x;
            hash_sum[c] ^= h;
        }
    }
    return ORC_OK;
}

static int orc_cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : x > y;
}

/* Round-synchronous listing.  In round t every cell that is pure at the start */
/* of the round yields its key; K_t is that set of keys (a key pure in several */
/* cells counts once).  Stop when K_t is empty.  Every key of K_t is then      */
/* deleted from its r cells.  Keys are written to out_keys round after round,  */
/* ascending within a round.  K[t-1] = |K_t|.                                  */
int orc_iblt_list_rounds(uint64_t ncells, uint32_t r, uint64_t seed,
                         int32_t *count, uint64_t *key_sum, uint64_t *hash_sum,
                         uint64_t *out_keys, uint64_t out_cap,
                         uint64_t *K, uint32_t max_rounds,
                         uint64_t *n_listed_out, uint32_t *rounds_out,
                         int32_t *corrupt_out)
{
    orc_iblt t;
    uint64_t n_listed = 0, c, *got;
    uint32_t round;
    int32_t corrupt = 0;
    int rc = orc_iblt_setup(&t, ncells, r, seed);
    if (rc) return rc;
    got = (uint64_t *)malloc((size_t)ncells * sizeof(uint64_t));
    if (!got) return ORC_ENOMEM;
    *rounds_out = 0;
    for (round = 1;; round++) {
        uint64_t np = 0, nk = 0, i;
        /* Keys of the cells that are pure at the start of the round. */
        for (c = 0; c < ncells; c++) {
            if (count[c] != 1) continue;
            if (hash_sum[c] != orc_iblt_check(&t, key_sum[c])) { corrupt = 1; continue; }
            got[np++] = key_sum[c];
        }
        if (np == 0) break;
        if (round > max_rounds) { rc = ORC_EROUNDS; break; }
        /* As a set: each key once. */
        qsort(got, np, sizeof(uint64_t), orc_cmp_u64);
        for (i = 0; i < np; i++)
            if (i == 0 || got[i] != got[i - 1]) got[nk++] = got[i];
        if (n_listed + nk > out_cap) { rc = ORC_ENOSPC; break; }
        for (i = 0; i < nk; i++) {
            uint64_t x = got[i], h = orc_iblt_check(&t, x);
            uint32_t j;
            out_keys[n_listed + i] = x;
            for (j = 0; j < r; j++) {
                uint64_t cc = orc_iblt_cell(&t, j, x);
                count[cc] -= 1;
                key_sum[cc] ^= x;
                hash_sum[cc] ^= h;
            }
        }
        K[round - 1] = nk;
        n_listed += nk;
        *rounds_out = round;
    }
    free(got);
    *n_listed_out = n_listed;
    *corrupt_out = corrupt;
    return rc;
}

/* Sequential listing: keep a stack of cells that may be pure; pop one, and if */
/* it is pure output its key and delete the key from its r cells, pushing any  */
/* of those cells that become pure.  Keys are written in discovery order.      */
int orc_iblt_list_seq(uint64_t ncells, uint32_t r, uint64_t seed,
                      int32_t *count, uint64_t *key_sum, uint64_t *hash_sum,
                      uint64_t *out_keys, uint64_t out_cap, uint64_t *n_listed_out)
{
    orc_iblt t;
    uint64_t *stack, top = 0, n_listed = 0, c;
    int rc = orc_iblt_setup(&t, ncells, r, seed);
    if (rc) return rc;
    stack = (uint64_t *)malloc((size_t)ncells * sizeof(uint64_t) * (r + 1));
    if (!stack) return ORC_ENOMEM;
    for (c = 0; c < ncells; c++)
        if (count[c] == 1) stack[top++] = c;
    while (top) {
        uint64_t cell = stack[--top], x, h;
        uint32_t j;
        if (count[cell] != 1) continue;
        x = key_sum[cell];
        h = orc_iblt_check(&t, x);
        if (hash_sum[cell] != h) continue;
        if (n_listed >= out_cap) { rc = ORC_ENOSPC; break; }
        out_keys[n_listed++] = x;
        for (j = 0; j < r; j++) {
            uint64_t cc = orc_iblt_cell(&t, j, x);
            count[cc] -= 1;
            key_sum[cc] ^= x;
            hash_sum[cc] ^= h;
            if (count[cc] == 1) stack[top++] = cc;
        }
    }
    free(stack);
    *n_listed_out = n_listed;
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Listing with subtables (Section 5, "Implementation Details"; Appendix B):  */
/* the paper's GPU process.  Each round is r subrounds; subround (i, j)       */
/* lists the key of every cell of subtable j that is pure at the start of    */
/* the subround (a key has one cell per subtable, so each key once) and      */
/* deletes each of those keys from its r cells.  Subrounds are numbered      */
/* s = (i-1) r + j from 1, an empty one keeping its number; the run ends     */
/* after r empty subrounds in a row.  K[s-1] = keys listed in subround s;    */
/* *rounds_out = the last subround that listed a key.  Limits as for         */
/* orc_iblt_list_rounds.                                                     */

int orc_iblt_list_subrounds(uint64_t ncells, uint32_t r, uint64_t seed,
                            int32_t *count, uint64_t *key_sum, uint64_t *hash_sum,
                            uint64_t *out_keys, uint64_t out_cap,
                            uint64_t *K, uint32_t max_rounds,
                            uint64_t *n_listed_out, uint32_t *rounds_out,
                            int32_t *corrupt_out)
{
    orc_iblt t;
    uint64_t n_listed = 0, c, *got;
    uint32_t s, empty = 0;
    int32_t corrupt = 0;
    int rc = orc_iblt_setup(&t, ncells, r, seed);
    if (rc) return rc;
    got = (uint64_t *)malloc((size_t)ncells * sizeof(uint64_t));
    if (!got) return ORC_ENOMEM;
    *rounds_out = 0;
    for (s = 1;; s++) {
        uint32_t j = (s - 1) % r;
        uint64_t nk = 0, i;
        for (c = t.base[j]; c < t.base[j] + t.size[j]; c++) {
            if (count[c] != 1) continue;
            if (hash_sum[c] != orc_iblt_check(&t, key_sum[c])) { corrupt = 1; continue; }
            got[nk++] = key_sum[c];
        }
        if (nk == 0) {
            if (s <= max_rounds) K[s - 1] = 0;
            if (++empty == r) break;
            continue;
        }
        empty = 0;
        if (s > max_rounds) { rc = ORC_EROUNDS; break; }
        if (n_listed + nk > out_cap) { rc = ORC_ENOSPC; break; }
        qsort(got, nk, sizeof(uint64_t), orc_cmp_u64);
        for (i = 0; i < nk; i++) {
            uint64_t x = got[i], h = orc_iblt_check(&t, x);
            uint32_t q;
            out_keys[n_listed + i] = x;
            for (q = 0; q < r; q++) {
                uint64_t cc = orc_iblt_cell(&t, q, x);
                count[cc] -= 1;
                key_sum[cc] ^= x;
                hash_sum[cc] ^= h;
            }
        }
        K[s - 1] = nk;
        n_listed += nk;
        *rounds_out = s;
    }
    free(got);
    *n_listed_out = n_listed;
    *corrupt_out = corrupt;
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Listing a table that holds deletions too (Section 5, "Motivation": the    */
/* count field goes down on a deletion, and the table can hold the          */
/* difference of two sets).  A cell is pure when its count is +1 or -1 and    */
/* its checksum field is C(key_sum): it holds that one key, inserted (+1) or  */
/* deleted (-1) once more than the other way.  Round t takes the pure cells   */
/* at its start, lists each key once with its sign, and takes every listed    */
/* key back out of its r cells (count -= sign, XOR the fields).  A count of   */
/* +-1 with a wrong checksum is ordinary here (a cell holding several keys). */
/* signs[i] is the sign of out_keys[i]; *nonempty_out = cells left non-zero.  */

typedef struct { uint64_t key; int32_t sign; } orc_signed_key;

static int orc_cmp_signed(const void *a, const void *b)
{
    uint64_t x = ((const orc_signed_key *)a)->key, y = ((const orc_signed_key *)b)->key;
    return x < y ? -1 : x > y ? 1 : 0;
}

int orc_iblt_list_signed(uint64_t ncells, uint32_t r, uint64_t seed,
                         int32_t *count, uint64_t *key_sum, uint64_t *hash_sum,
                         uint64_t *out_keys, int8_t *signs, uint64_t out_cap,
                         uint64_t *K, uint32_t max_rounds,
                         uint64_t *n_listed_out, uint32_t *rounds_out,
                         uint64_t *nonempty_out)
{
    orc_iblt t;
    uint64_t n_listed = 0, c, ne = 0;
    orc_signed_key *got;
    uint32_t round;
    int rc = orc_iblt_setup(&t, ncells, r, seed);
    if (rc) return rc;
    got = (orc_signed_key *)malloc((size_t)ncells * sizeof(orc_signed_key));
    if (!got) return ORC_ENOMEM;
    *rounds_out = 0;
    for (round = 1;; round++) {
        uint64_t np = 0, nk = 0, i;
        for (c = 0; c < ncells; c++) {
            if (count[c] != 1 && count[c] != -1) continue;
            if (hash_sum[c] != orc_iblt_check(&t, key_sum[c])) continue;
            got[np].key = key_sum[c];
            got[np].sign = count[c];
            np++;
        }
        if (np == 0) break;
        if (round > max_rounds) { rc = ORC_EROUNDS; break; }
        qsort(got, np, sizeof(orc_signed_key), orc_cmp_signed);
        for (i = 0; i < np; i++)
            if (i == 0 || got[i].key != got[i - 1].key) got[nk++] = got[i];
        if (n_listed + nk > out_cap) { rc = ORC_ENOSPC; break; }
        for (i = 0; i < nk; i++) {
            uint64_t x = got[i].key, h = orc_iblt_check(&t, x);
            uint32_t j;
            out_keys[n_listed + i] = x;
            signs[n_listed + i] = (int8_t)got[i].sign;
            for (j = 0; j < r; j++) {
                uint64_t cc = orc_iblt_cell(&t, j, x);
                count[cc] -= got[i].sign;
                key_sum[cc] ^= x;
                hash_sum[cc] ^= h;
            }
        }
        K[round - 1] = nk;
        n_listed += nk;
        *rounds_out = round;
    }
    for (c = 0; c < ncells; c++)
        if (count[c] != 0 || key_sum[c] != 0 || hash_sum[c] != 0) ne++;
    free(got);
    *n_listed_out = n_listed;
    *nonempty_out = ne;
    return rc;
}

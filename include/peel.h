/*
 * peel.h -- C ABI of libpeel, round-synchronous parallel peeling on gfx950.
 *
 * Paper: J. Jiang, M. Mitzenmacher, J. Thaler, "Parallel Peeling Algorithms".
 *
 * Two forms of one process.  (1) k-core peeling of an r-uniform hypergraph:
 * in each round every vertex of degree < k is removed at once together with
 * its incident edges, until no vertex of degree < k is left (Section 1;
 * Section 3).  (2) Listing an Invertible Bloom Lookup Table: keys are edges,
 * cells are vertices, and in each round every pure cell gives up its key,
 * which is then deleted from its r cells (Section 5).  No edge or key is ever
 * peeled twice (Section 5, "Implementation Details").
 *
 * Conventions shared by every entry point:
 *   - Pointers marked (device) are device memory of the current HIP device;
 *     pointers marked (host) are host memory read before the call returns.
 *   - The caller owns every buffer.  The library never allocates, frees or
 *     copies to the host; scratch space is the caller's workspace, sized by
 *     the matching *_workspace() query, 256-byte aligned.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue
 *     work on it and return without waiting.  The returned status covers
 *     argument errors found on the host, and launch failures.  Errors found
 *     by the device (an id out of range, a round limit, a corrupt cell) are
 *     written as flags into the call's device summary, to be read after the
 *     stream is synchronised.
 *   - Rounds are numbered from 1.  Round numbers stored per vertex or edge
 *     use 0 for "still present at the end" (in the k-core / in the table).
 *   - Calls on different streams are independent when their buffers and
 *     workspaces are disjoint.
 */
#ifndef PEEL_H
#define PEEL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t peel_status;

#define PEEL_OK 0
#define PEEL_EINVAL (-1)   /* bad argument (size, null pointer, r, k)        */
#define PEEL_ERANGE (-2)   /* a vertex id >= n                               */
#define PEEL_ENOSPC (-3)   /* output or workspace too small                  */
#define PEEL_EROUNDS (-4)  /* round limit reached before the process ended   */
#define PEEL_ECORRUPT (-5) /* an IBLT cell with count 1 and a bad checksum   */
#define PEEL_EHIP (-6)     /* the HIP runtime reported an error              */

/* Device summary flag bits (summary status words). */
#define PEEL_FLAG_ERANGE 0x1u
#define PEEL_FLAG_EROUNDS 0x2u
#define PEEL_FLAG_ENOSPC 0x4u
#define PEEL_FLAG_ECORRUPT 0x8u
#define PEEL_FLAG_TIMEOUT 0x10u /* a device-wide barrier waited past its limit; */
                                /* the call's other outputs are then undefined  */
#define PEEL_FLAG_EINVAL 0x20u  /* a batch entry was rejected (r, size, or      */
                                /* alignment); that table was left untouched    */
#define PEEL_FLAG_ETEAM 0x40u   /* peel_k2_xor: the resident team that formed   */
                                /* was too small to hold n vertices in LDS;     */
                                /* nothing was peeled (peel_kcore has no limit) */

/* Human-readable name of a status code; never NULL. */
const char *peel_strerror(peel_status s);

/* ABI revision of this header; bumped on any incompatible change. */
int peel_abi_version(void);

/* ------------------------------------------------------------------------ */
/* Hypergraph incidence (CSR).                                              */
/*
 * The peeling process removes a vertex "together with its incident edges"
 * (Section 1), so peel_kcore needs, per vertex, the list of edges that hold
 * it.  hg_build makes it by counting sort.
 *
 *   edges   (device) m rows of r uint32 vertex ids, row-major (edge e holds
 *           edges[e*r .. e*r+r-1]).  An id may repeat inside a row; degree
 *           then counts it with multiplicity.
 *   m, r, n 2 <= r <= 8, n >= 1, m*r < 2^32.
 *   offsets (device, out) n+1 uint32: the incidences of vertex v are
 *           inc[offsets[v] .. offsets[v+1]-1]; offsets[n] = m*r.
 *   inc     (device, out) m*r uint32 edge ids.  Order within a vertex's list
 *           is unspecified.
 *   deg     (device, out) n uint32: offsets[v+1] - offsets[v].
 *   info    (device, out) 2 uint32: [0] status flags (PEEL_FLAG_ERANGE if an
 *           id >= n was seen; the other outputs are then undefined),
 *           [1] maximum degree.
 *   ws      (device) workspace of ws_bytes >= hg_build_workspace(n, m, r).
 */
size_t hg_build_workspace(uint32_t n, uint64_t m, uint32_t r);
peel_status hg_build(const uint32_t *edges, uint64_t m, uint32_t r, uint32_t n,
                     uint32_t *offsets, uint32_t *inc, uint32_t *deg, uint32_t *info,
                     void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Round-synchronous k-core peeling (Section 1; Section 3; Section 5).      */
/*
 * Round t removes F_t = { alive v : deg(v) < k }, degrees taken at the start
 * of round t, and every alive edge that holds a vertex of F_t; each removed
 * edge lowers the degree of each of its r slots by one.  The run stops at the
 * first empty F_t.  An edge hit by several peeled vertices in one round dies
 * once (its owning workgroup clears its alive bit in LDS; the fallback engine
 * claims it by compare-and-swap on its round word).
 *
 *   edges, m, r, n   as for hg_build;  k >= 1.
 *   offsets, inc     (device) the CSR from hg_build for these edges.
 *   deg              (device, in/out) n uint32.  In: the degrees from
 *                    hg_build.  Out: the core degree of each core vertex, 0
 *                    for every removed vertex.
 *   vertex_round     (device, out) n uint32: round that removed v, 0 = core.
 *   edge_round       (device, out) m uint32: round that removed e, 0 = core.
 *   round_stats      (device, out) 2*max_rounds uint64: for round t,
 *                    [2(t-1)] = vertices removed, [2(t-1)+1] = edges removed.
 *                    Entries past the last round are 0.
 *   max_rounds       >= 1.  If round max_rounds+1 would still remove a vertex,
 *                    the run stops and sets PEEL_FLAG_EROUNDS; the outputs
 *                    then hold the state after max_rounds rounds.
 *   summary          (device, out) 8 uint32: [0] rounds (last round that
 *                    removed a vertex), [1] last round that removed an edge,
 *                    [2] status flags, [3] number of core vertices, [4] the
 *                    workgroups that ran the rounds (diagnostic), [5..7] 0.
 *   ws               (device) ws_bytes >= peel_kcore_workspace(n, m, r).
 */
size_t peel_kcore_workspace(uint32_t n, uint64_t m, uint32_t r);
peel_status peel_kcore(const uint32_t *edges, uint64_t m, uint32_t r, uint32_t n, uint32_t k,
                       const uint32_t *offsets, const uint32_t *inc, uint32_t *deg,
                       uint32_t *vertex_round, uint32_t *edge_round, uint64_t *round_stats,
                       uint32_t max_rounds, uint32_t *summary, void *ws, size_t ws_bytes,
                       void *stream);

/*
 * Peeling with subtables (Appendix B): the process the paper's GPU code runs.
 * The vertex ids are split into r consecutive subtables of near-equal size
 * (the first n mod r one larger), and every round is r subrounds: subround
 * (i, j) removes, at once, each alive vertex of subtable j whose degree is
 * below k at the start of the subround, with every alive edge it holds.
 * Subrounds are numbered s = (i-1) r + j from 1, an empty subround keeping its
 * number; the run ends when no subtable has a vertex to remove.  It ends at
 * the same k-core as peel_kcore.
 *
 * Arguments, outputs and errors are those of peel_kcore, with "round" read as
 * "subround": vertex_round and edge_round hold subround numbers, round_stats
 * has one entry pair per subround (0 for an empty one), max_rounds bounds the
 * subrounds, and summary[0] is the last subround that removed a vertex.  The
 * workspace is peel_kcore_workspace(n, m, r).
 */
peel_status peel_kcore_subtables(const uint32_t *edges, uint64_t m, uint32_t r, uint32_t n,
                                 uint32_t k, const uint32_t *offsets, const uint32_t *inc,
                                 uint32_t *deg, uint32_t *vertex_round, uint32_t *edge_round,
                                 uint64_t *round_stats, uint32_t max_rounds, uint32_t *summary,
                                 void *ws, size_t ws_bytes, void *stream);

/*
 * Peeling to the 2-core without vertex -> edge lists (Section 5,
 * "Motivation": listing an IBLT is peeling its hypergraph, and a pure cell --
 * a vertex of degree one -- names its one item by its key sum).  Every vertex
 * keeps its degree and the XOR of the ids of its alive incident edges, so at
 * k = 2 a vertex of F_t that still holds an edge names it directly.  The same
 * rounds as peel_kcore with k = 2, and the same outputs, bit for bit; no
 * hg_build is needed.  An edge taken in round t is taken by its vertex of
 * F_t in the lowest slot of its row (F_t is published as a bitmap each
 * round), so it dies once with no compare-and-swap.
 *
 *   edges, m, r, n   as for hg_build (k is 2).
 *   deg              (device, out) n uint32: the core degree of each core
 *                    vertex, 0 for every removed vertex (the initial degrees
 *                    are computed here).
 *   vertex_round, edge_round, round_stats, max_rounds, summary
 *                    as for peel_kcore.  summary[2] also carries
 *                    PEEL_FLAG_ERANGE (an id >= n; such ids are ignored) and
 *                    PEEL_FLAG_ETEAM.
 *   ws               (device) ws_bytes >= peel_k2_xor_workspace(n, m, r):
 *                    the XORs (4n bytes), the round's messages (8 r m bytes
 *                    and about 8 (r-1) n of staging), the frontier (4n) and
 *                    its bitmap (n/8), and the degree build's scratch.
 * The vertices are held in LDS by a team of resident workgroups of at most
 * 98304 vertices each: with fewer than n / 98304 workgroups resident the call
 * peels nothing and sets PEEL_FLAG_ETEAM (peel_kcore has no such limit).
 */
size_t peel_k2_xor_workspace(uint32_t n, uint64_t m, uint32_t r);
peel_status peel_k2_xor(const uint32_t *edges, uint64_t m, uint32_t r, uint32_t n,
                        uint32_t *deg, uint32_t *vertex_round, uint32_t *edge_round,
                        uint64_t *round_stats, uint32_t max_rounds, uint32_t *summary,
                        void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Invertible Bloom Lookup Table (Section 5).                                */
/*
 * A table of `ncells` cells split into r near-equal subtables (subtable j
 * holds ncells/r cells, the first ncells%r subtables one more); a key has one
 * cell in each subtable (Section 5, "Implementation Details"; Appendix B).
 * Cell of key x in subtable j: base_j + floor(H_j(x) * size_j / 2^64) with
 * H_j(x) = mix64(x ^ salt_j); checksum C(x) = mix64(x ^ salt_c); mix64 is the
 * SplitMix64 output finaliser and salt_j (j < r), salt_c are draws j and 8 of
 * the SplitMix64 stream whose state starts at `seed`.
 *
 * A cell is pure when count == 1 and hash_sum == C(key_sum): it holds exactly
 * one key, key_sum.
 */
typedef struct iblt_cell {
    int32_t count;      /* keys inserted minus keys deleted */
    uint32_t reserved0; /* 0 */
    uint64_t key_sum;   /* XOR of the keys                  */
    uint64_t hash_sum;  /* XOR of C(key)                    */
    uint64_t reserved1; /* 0; pads the cell to 32 bytes     */
} iblt_cell;

typedef struct iblt_desc {
    uint64_t ncells;     /* r <= ncells < 2^32 */
    uint32_t r;          /* 2..8 */
    uint32_t workgroups; /* iblt_list only: persistent workgroups; 0 = one per
                            4096 cells, at most one per CU (more than one per CU
                            is taken as one per CU); callers that run several
                            listings at once give each a share */
    uint64_t seed;
} iblt_desc;

/*
 * Tables are 32-byte aligned (as torch and hipMalloc allocations are);
 * calls with a misaligned table return PEEL_EINVAL.
 *
 * Insert keys: for each key x and each subtable j, count += 1,
 * key_sum ^= x, hash_sum ^= C(x) in x's cell of subtable j (Section 5,
 * "Motivation").  Accumulates into `cells` (device, ncells entries), which
 * the caller zeroes before the first insert.  Keys (device) must be
 * distinct from each other and from keys already in the table: a repeated
 * key cancels in the XOR fields.
 *
 * Each key costs 3 r device atomics, which run at a fixed rate on this GPU
 * (about 27 G/s, about 370 GB/s of cell traffic): this is the call for small
 * tables and for callers without a workspace.  For a table larger than the
 * caches, iblt_update (below) gives the same cells bit for bit, 4-5 times
 * faster (2^24 cells, 10.3 M keys: 0.78 ms against 3.56 ms).
 */
peel_status iblt_insert(const iblt_desc *desc, iblt_cell *cells, const uint64_t *keys,
                        uint64_t nkeys, void *stream);

/*
 * Delete keys: for each key x and each subtable j, count -= 1, key_sum ^= x,
 * hash_sum ^= C(x) in x's cell of subtable j (Section 5, "Motivation": the
 * same update with the count going down).  A key deleted without having been
 * inserted stays in the table with count -1 in its cells: inserting a set A
 * and deleting a set B leaves the table of their difference.  Arguments as
 * for iblt_insert.
 */
peel_status iblt_delete(const iblt_desc *desc, iblt_cell *cells, const uint64_t *keys,
                        uint64_t nkeys, void *stream);

/*
 * iblt_insert (sign = +1) or iblt_delete (sign = -1) computed another way, for
 * large tables: the cells come out bit for bit as the per-key updates leave
 * them (Section 5: each key's r cells take count += sign, key_sum ^= x,
 * hash_sum ^= C(x), and these updates commute).  Instead of 3r device atomics
 * per key into a table far larger than the caches, the keys are counting-
 * sorted by block of cells and each block is updated once in LDS, so the
 * table is read and written once, in order.  The reserved words of each cell
 * are left as they were.
 *
 *   desc, cells, keys, nkeys   as for iblt_insert (cells 32-byte aligned).
 *   sign                       +1 or -1; anything else is PEEL_EINVAL.
 *   ws                         (device) ws_bytes >= iblt_update_workspace(desc,
 *                              nkeys): the sorted entries (10 r bytes per key)
 *                              and their counts.
 *
 * Tables of more than 2^24 cells, or r * nkeys >= 2^32, take the per-key
 * atomic path instead (same result; the workspace is then not used).
 */
size_t iblt_update_workspace(const iblt_desc *desc, uint64_t nkeys);
peel_status iblt_update(const iblt_desc *desc, iblt_cell *cells, const uint64_t *keys,
                        uint64_t nkeys, int32_t sign, void *ws, size_t ws_bytes, void *stream);

/*
 * List the table by round-synchronous pure-cell peeling, consuming `cells`
 * in place.  Round t takes K_t = the keys of the cells that are pure at the
 * start of the round (each key once, however many of its cells are pure);
 * the run stops at the first empty K_t; every key of K_t is then deleted
 * from its r cells.
 *
 *   out_keys     (device, out) keys, grouped by round in round order; the
 *                order inside a round is unspecified.
 *   out_cap      capacity of out_keys.  If a round would overflow it, the run
 *                stops before that round and sets PEEL_FLAG_ENOSPC.
 *   round_stats  (device, out) max_rounds uint64: K_t per round.
 *   max_rounds   >= 1; PEEL_FLAG_EROUNDS as for peel_kcore.
 *   summary      (device, out) 8 uint64: [0] keys listed, [1] rounds, [2]
 *                keys still in the table (sum of counts / r minus [0]; 0 means
 *                the table was emptied), [3] status flags (PEEL_FLAG_ECORRUPT
 *                if a count-1 cell failed its checksum; such a cell is not
 *                pure), [4] the workgroups that ran the rounds (diagnostic),
 *                [5..7] 0.
 *   ws           (device) ws_bytes >= iblt_list_workspace(desc): about
 *                (16 r + 32) bytes per cell.
 * The rounds run in one persistent kernel.  Each workgroup owns a piece of
 * every subtable and is the only writer of those cells: a listed key's
 * deletions from its other cells are sent to those cells' owners, which
 * combine them and update each cell with one plain read-modify-write (no
 * device atomics).  With
 * PEEL_LIST_ENGINE=atomic in the environment the deletions are device
 * atomics instead (the signed listing's engine); the results are the same.
 */
size_t iblt_list_workspace(const iblt_desc *desc);
peel_status iblt_list(const iblt_desc *desc, iblt_cell *cells, uint64_t *out_keys,
                      uint64_t out_cap, uint64_t *round_stats, uint32_t max_rounds,
                      uint64_t *summary, void *ws, size_t ws_bytes, void *stream);

/*
 * Signed listing, for tables that hold deletions too (Section 5): a cell is
 * pure when its count is +1 or -1 and hash_sum == C(key_sum); each round
 * lists the keys of the cells pure at its start, each once with its sign (the
 * pure cell's count: +1 for a key inserted, -1 for a key deleted), and takes
 * every listed key back out of its r cells (count -= sign, XOR the fields).
 * Listing the table of "insert A, delete B" gives A \ B with sign +1 and
 * B \ A with sign -1 once the difference is below the threshold.
 *
 *   out_signs   (device, out) out_cap int8: out_signs[i] is the sign of
 *               out_keys[i].
 * Other arguments and limits as for iblt_list, except: a count of +-1 with a
 * wrong checksum is an ordinary cell here (never PEEL_FLAG_ECORRUPT), and
 * summary[2] is the number of cells left non-zero (0 means the difference
 * was listed whole).  A cell's count can land on +-1 more than once in a
 * round, and each time the cell is queued for the next round's detect; if a
 * round queues more cells than the workspace's queues hold (more than about
 * 2 * ncells in all, far above what a table below the threshold does), the
 * cells past that are not examined and PEEL_FLAG_ENOSPC is set.
 */
peel_status iblt_list_signed(const iblt_desc *desc, iblt_cell *cells, uint64_t *out_keys,
                             int8_t *out_signs, uint64_t out_cap, uint64_t *round_stats,
                             uint32_t max_rounds, uint64_t *summary, void *ws, size_t ws_bytes,
                             void *stream);

/*
 * Listing with subtables (Section 5, "Implementation Details"; Appendix B):
 * the process the paper's GPU code runs.  Every round is r subrounds;
 * subround (i, j) lists the key of each cell of subtable j that is pure at the
 * start of the subround (a key has one cell per subtable, so it is listed
 * once) and deletes those keys from their r cells.  Subrounds are numbered
 * s = (i-1) r + j from 1, an empty subround keeping its number; the run ends
 * when no subtable has a pure cell.  It lists the same keys as iblt_list and
 * leaves the same table.
 *
 * Arguments, outputs and errors are those of iblt_list, with "round" read as
 * "subround": out_keys is grouped by subround, round_stats[s-1] = keys listed
 * in subround s (0 for an empty one), max_rounds bounds the subrounds and
 * summary[1] is the last subround that listed a key.  The workspace is
 * iblt_list_workspace(desc).
 */
peel_status iblt_list_subtables(const iblt_desc *desc, iblt_cell *cells, uint64_t *out_keys,
                                uint64_t out_cap, uint64_t *round_stats, uint32_t max_rounds,
                                uint64_t *summary, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Batched listing (many independent tables in one launch).                   */
/*
 * Not in the paper, which lists one table.  Each table is listed exactly as
 * iblt_list lists it (same rounds, same per-round key sets, same summary),
 * but all tables run in one kernel launch: workgroups take tables in the
 * order of `entries` from a shared counter and list each with workgroup-wide
 * barriers only.  Sorting `entries` by decreasing ncells balances the load.
 *
 * Three per-table schedules exist, chosen by size class:
 *   - a table of at most `lds_max_cells` cells that fits the workgroup's
 *     local memory (LDS) is read once into it, listed there with LDS
 *     atomics, and written back.  A workgroup of 1024 threads holds up to
 *     IBLT_LDS_MAX_CELLS = 5120 cells, one of 512 up to 3072, one of 256 up
 *     to 2048; a larger table is listed in place;
 *   - a table of at least `tile_min_cells` cells (with tile_workgroups >= 2)
 *     is listed by a team of tile_workgroups workgroups of the same launch:
 *     member g detects the g-th slice of the cells in round 1 and then the
 *     cells it pushed, keys leave the shared cells by device atomics, and a
 *     barrier among the members (with the time limit of iblt_list's) ends
 *     each half round;
 *   - any other table is listed in place in device memory by one workgroup,
 *     the table's only writer, with plain read-modify-writes of its cells.
 * All give the same results.  A team takes tile_workgroups consecutive work
 * units from the shared counter; members are only ever workgroups that are
 * running, and at least tile_workgroups of them are, so a team always forms.
 *
 *   entries       (device) ntables descriptors; every pointer in them is
 *                 device memory and every table is disjoint from the others.
 *   max_cells     >= the largest ncells among the tables.
 *   max_rounds    >= 1, for every table (round_stats hold max_rounds each).
 *   sched         (host) the schedule, or NULL for the defaults (512 threads,
 *                 lds_max_cells = IBLT_LDS_MAX_CELLS, no teams).
 *                 block_threads must be 256, 512 or 1024 (0 = 512),
 *                 lds_max_cells at most IBLT_LDS_MAX_CELLS and tile_workgroups
 *                 at most 64, else PEEL_EINVAL.
 *   ws            (device) ws_bytes >= iblt_list_batched_workspace(), which
 *                 covers every schedule.
 * Each table's summary is written as iblt_list's ([4] = the workgroups that
 * listed it; PEEL_FLAG_TIMEOUT if a team's barrier gave up).  An
 * entry with r outside 2..8, ncells < r, ncells > max_cells, or cells that are
 * null or not 32-byte aligned is not listed: its summary (if not null) gets
 * [3] = PEEL_FLAG_EINVAL and zeros elsewhere, and the other tables go on.
 */
#define IBLT_LDS_MAX_CELLS 5120u

typedef struct iblt_batch_schedule {
    uint32_t block_threads;   /* threads per workgroup: 256, 512, 1024; 0 = 512  */
    uint32_t lds_max_cells;   /* tables this small are listed in LDS; 0 = none   */
    uint32_t tile_min_cells;  /* tables at least this large are listed by a team */
    uint32_t tile_workgroups; /* of this many workgroups (2..64); 0 or 1 = none  */
} iblt_batch_schedule;

typedef struct iblt_batch_entry {
    iblt_desc desc;
    iblt_cell *cells;      /* ncells cells, 32-byte aligned, consumed in place */
    uint64_t *out_keys;    /* out_cap entries                                  */
    uint64_t out_cap;
    uint64_t *round_stats; /* max_rounds entries                               */
    uint64_t *summary;     /* 8 entries                                        */
} iblt_batch_entry;

size_t iblt_list_batched_workspace(uint32_t ntables, uint64_t max_cells);
peel_status iblt_list_batched(const iblt_batch_entry *entries, uint32_t ntables,
                              uint64_t max_cells, uint32_t max_rounds,
                              const iblt_batch_schedule *sched, void *ws, size_t ws_bytes,
                              void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the batched
 * listing of iblt_list_batched, same arguments, same per-table results, with
 * no workspace argument.  Its scratch (the batch's ticket counter and two
 * max_cells-entry cell lists per workgroup) is one static device array of
 * 64 MiB + 4 KiB that the library holds on each device it runs on until the
 * process ends; it calls no allocator.  Its address is looked up on the
 * device's first call.
 *
 *   max_cells     at most IBLT_NOALLOC_MAX_CELLS, else PEEL_ENOSPC (nothing
 *                 runs); tables beyond it go through iblt_list_batched.
 *   Other arguments as iblt_list_batched.  At most 512 workgroups run.
 * Every call on one device shares that device's array, and it keeps the last
 * call's contents (the ticket counter is cleared by a kernel at the start of
 * each call, so the call can be graph-captured).  Calls that overlap on one
 * device -- on different streams, or from different host threads -- race on
 * it and must be serialised by the caller.  PEEL_EHIP if the array's address
 * cannot be looked up.
 */
#define IBLT_NOALLOC_MAX_CELLS 16384u

peel_status iblt_list_batched_noalloc(const iblt_batch_entry *entries, uint32_t ntables,
                                      uint64_t max_cells, uint32_t max_rounds,
                                      const iblt_batch_schedule *sched, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PEEL_H */

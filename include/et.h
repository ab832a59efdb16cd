/*
 * et.h -- C ABI of the MI355X (gfx950) Euler-tour library.
 *
 * Implements the data-parallel path of "Euler Meets GPU: Practical Graph
 * Algorithms with Theoretical Guarantees" (Polak, Siwiec, Stobierski,
 * arXiv 2103.15217): Euler tour of a rooted tree, list ranking, depth /
 * preorder / subtree size, batched LCA queries with the Inlabel
 * (Schieber-Vishkin) scheme, and bridges with Tarjan-Vishkin.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers named d_* are DEVICE pointers owned by the caller (for example
 *    the data_ptr() of a tensor on the current device). h_* pointers are
 *    host pointers. Nothing is copied between host and device except where
 *    an entry point says so.
 *  - Every call is asynchronous and ordered on the HIP stream it is given.
 *    Outputs are valid once that stream has reached the call's end.
 *  - An et_ctx owns scratch memory (a caching pool), a device status word
 *    and the device it was created on. Calls that share a context must be
 *    ordered with respect to each other (one stream at a time per context),
 *    with two exceptions:
 *      . the query calls et_lca, et_lca_batch and et_lca_rmq take nothing
 *        from the pool and write nothing of the context but its status bits
 *        (an atomic OR), so they may run on any stream, concurrently with
 *        each other and with other calls of the context, as long as the
 *        tree they read is neither freed nor rebuilt meanwhile;
 *      . pool blocks are reused in stream order: blocks released on stream A
 *        (at the end of a call, or by et_tree_free on A) and taken by a call
 *        on stream B make B wait for an event recorded on A at that moment,
 *        so work still running on A is not overwritten. (While B is being
 *        captured into a graph the wait is skipped: capture starts from a
 *        synchronised device.)
 *  - Ids are 0-based int32. Half-edge ids of a tree with n nodes: 2c is the
 *    half-edge (parent(c) -> c) going down into c, 2c+1 is (c -> parent(c))
 *    going up out of c; the root r's ids 2r and 2r+1 are unused.
 *  - Children are visited in ascending id order and the tour starts with
 *    the half-edge into the root's smallest child. (The paper's DCEL visits
 *    children cyclically after the parent in sorted order and splits the
 *    cyclic tour at an arbitrary root edge, Section 2.1; the two agree
 *    whenever parent ids are smaller than child ids.)
 *  - Return codes: ET_OK, or a negative ET_E* code. Argument errors that
 *    the host can see are returned immediately and enqueue nothing.
 *    Malformed input found on the device (not a tree, a list that is not a
 *    set of simple paths, an id out of range, a CSR that is not symmetric)
 *    never faults and never hangs: kernels clamp every index they gather,
 *    bound every walk, and record the error in the context's status word,
 *    which et_ctx_status() reports. Outputs of such a call are unspecified.
 */
#ifndef ET_H
#define ET_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ET_OK 0
#define ET_EINVAL (-1)  /* bad argument: null pointer, negative or too large size */
#define ET_ENOMEM (-2)  /* device memory exhausted */
#define ET_EHIP (-3)    /* a HIP runtime call failed */
#define ET_EINPUT (-4)  /* malformed input detected on the device */
#define ET_ESIZE (-5)   /* input beyond a fixed-size limit of the entry point (its scratch or LDS) */

typedef struct et_ctx et_ctx;
typedef struct et_tree et_tree;

/* Library version as 10000*major + 100*minor + patch. */
int et_version(void);

/* Human-readable text for a return code. Never NULL. */
const char* et_strerror(int code);

/* Create a context on the current HIP device. *out receives the handle.
 * Allocates the device status word; scratch grows on demand. */
int et_ctx_create(et_ctx** out);

/* Release a context and all scratch it holds. Trees built with it must be
 * freed first. Waits for the device to finish work that uses the scratch. */
void et_ctx_destroy(et_ctx* ctx);

/* Wait for stream s, then return ET_OK if no kernel enqueued on this
 * context since the previous call flagged malformed input, else ET_EINPUT
 * (or ET_EHIP). Clears the flag. */
int et_ctx_status(et_ctx* ctx, hipStream_t s);

/* Raw device status bits accumulated since the last et_ctx_status (for
 * diagnostics; same waiting semantics). */
int et_ctx_status_bits(et_ctx* ctx, hipStream_t s, uint32_t* h_bits);

/* Tunable launch parameters of this context (used by later calls):
 *   "lr_k1_log2"    list ranking, level 1: one splitter per 2^v ids at most
 *                   (1..10, default 4); a list of L elements uses
 *                   min(v, max(2, (floor(log2 L) - 15) / 2))
 *   "lr_per_wave1"  level 1: sublists owned by one wavefront at most
 *                   (64..65536, default 256); fewer when that would leave
 *                   under 4096 wavefronts, never under 64
 *   "lr_kn_log2"    upper levels: one splitter per 2^v elements (1..10, default 3)
 *   "lr_per_waven"  upper levels: sublists per wavefront at most (64..65536,
 *                   default 128), reduced like lr_per_wave1
 *   "rmq_block_log2"  range-minimum blocks of 2^v positions for the bridge
 *                   low / high tables and et_tree_rmq_build (5 or 6, default 5)
 *   "query_block"   threads per workgroup of the LCA query kernels (a power
 *                   of two in 64..1024, default 256)
 * Results never depend on them. ET_EINVAL for an unknown name or value. */
int et_ctx_set_param(et_ctx* ctx, const char* name, int64_t value);

/* Kernel timing. With enable != 0 every kernel launch of later calls on
 * this context is bracketed by a pair of HIP events on its stream. */
int et_ctx_profile(et_ctx* ctx, int enable);

/* Restrict that timing to the launches of one kernel (its name as reported
 * by et_ctx_profile_read, copied); NULL or "" times every kernel again.
 * Timing few launches keeps the events' own cost out of the work measured. */
int et_ctx_profile_only(et_ctx* ctx, const char* kernel_name);

/* Wait for stream s, then write a JSON object into h_buf (NUL-terminated,
 * at most buflen bytes): {"kernel": [launches, total_ms, max_ms], ...} over
 * the launches timed since the previous read; clears the records. Returns
 * ET_EINVAL if the buffer is too small (records are kept). */
int et_ctx_profile_read(et_ctx* ctx, hipStream_t s, char* h_buf, int32_t buflen);

/*
 * List ranking (Section 2.2: the rank of an element is its distance from
 * the head of its list).
 *   d_succ[len]      successor of each element; -1 ends a list; -2 marks an
 *                    unused slot. Every used slot must lie on exactly one
 *                    of the lists that start at d_heads.
 *   d_heads[n_heads] first element of each list (device array).
 *   d_rank[len]      output: steps from the element's list head (head = 0);
 *                    -1 for unused slots.
 * Sublist ranking: pseudo-randomly placed splitters cut the lists into
 * short sublists that wavefront lanes walk independently, the list of
 * sublists is ranked the same way until it fits one workgroup's LDS, and
 * the offsets are pushed back down.
 * len < 2^31 - 2^20. Malformed lists set ET_EINPUT in the status word.
 */
int et_list_rank(et_ctx* ctx, const int32_t* d_succ, int32_t len, const int32_t* d_heads,
                 int32_t n_heads, int32_t* d_rank, hipStream_t s);

/*
 * List ranking without allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same operation, arguments and results as
 * et_list_rank, with the scratch taken from one fixed array of
 * ET_NOALLOC_SCRATCH_BYTES in the library's device memory instead of the
 * context's pool. Nothing is allocated or freed by this call (and no memset
 * is enqueued: counters are cleared by kernels).
 *   Limits: len <= ET_NOALLOC_MAX_LEN, n_heads <= ET_NOALLOC_MAX_HEADS;
 *   larger inputs return ET_ESIZE and enqueue nothing. Within these limits
 *   the scratch fits every launch shape et_ctx_set_param allows (the plan is
 *   still checked on every call, ET_ESIZE if it would not fit).
 *   The array is per GPU, created with the library's code on that GPU and
 *   held until the process ends; its device address is resolved when a
 *   context is created on the device. Every call on one GPU uses the same
 *   array and leaves the last call's contents in it (each call clears what
 *   it needs), so calls that overlap on one GPU -- concurrent streams, or
 *   several contexts -- race and give wrong ranks: order them.
 */
#define ET_NOALLOC_MAX_LEN (1 << 20)
#define ET_NOALLOC_MAX_HEADS (1 << 16)
#define ET_NOALLOC_SCRATCH_BYTES (40u << 20)
int et_list_rank_noalloc(et_ctx* ctx, const int32_t* d_succ, int32_t len, const int32_t* d_heads,
                         int32_t n_heads, int32_t* d_rank, hipStream_t s);

/*
 * Weighted list ranking: prefix sums along lists (Section 2.2: list ranking
 * with weights on the elements, the form that gives depth from +1 / -1
 * weights on a tour).
 *   d_succ[len], d_heads[n_heads]  as for et_list_rank
 *   d_weight[len]    weight of each element (int32)
 *   d_sum[len]       output: the sum of the weights from the element's list
 *                    head through the element itself, in 32-bit two's
 *                    complement (sums wrap); 0 for unused slots
 *   d_rank[len]      optional output (may be NULL): as for et_list_rank
 * Same sublist ranking, with the weight sums carried next to the lengths.
 * Scratch from the context's pool: {successor, weight} pairs (8 bytes per
 * element) that the walk reads with one load per step, and one record per
 * element of 8 bytes (16 with d_rank) holding its local sum. len < 2^31 -
 * 2^20. Malformed lists set ET_EINPUT in the status word.
 */
int et_list_scan(et_ctx* ctx, const int32_t* d_succ, const int32_t* d_weight, int32_t len,
                 const int32_t* d_heads, int32_t n_heads, int32_t* d_rank, int32_t* d_sum, hipStream_t s);

/*
 * Euler tour and node statistics of a rooted tree (Section 2, Section 2.2),
 * plus the Inlabel tables for LCA queries (Section 3.1).
 *   d_parent[n]  parent id of every node; exactly one node (the root) has
 *                parent -1. n >= 1, n < 2^30.
 * The tree keeps its own device tables (tour successor and rank arrays,
 * depth / preorder / size, inlabel / ascendant, path-head table); d_parent
 * may be released once stream s has passed this call. The caller frees the
 * tree with et_tree_free. A parent array that is not a tree (no root or
 * several, an id out of range, a cycle) sets ET_EINPUT in ctx's status.
 */
int et_tree_build(et_ctx* ctx, const int32_t* d_parent, int32_t n, hipStream_t s,
                  et_tree** out);

/*
 * Euler tour and tree tables from the unordered edge list of a tree, by the
 * DCEL construction of Section 2.1 (Fig. 2): both directions of each edge
 * as twin half-edges, the half-edges sorted lexicographically, next() inside
 * a node's sorted run (cyclic), succ = next(twin), the cycle cut before the
 * root's first half-edge.
 *   d_u[n-1], d_v[n-1]  edge i joins d_u[i] and d_v[i] (any order, any
 *                       orientation); half-edge 2i is (u_i -> v_i), 2i+1 its
 *                       twin. n >= 1, n < 2^30, 0 <= root < n.
 *   d_parent_out[n]     optional (NULL allowed): parent of every node in the
 *                       tree rooted at root (-1 at the root).
 * The tour visits the children of a node entered from p in cyclic id order
 * starting after p (at the root: ascending), so it differs from
 * et_tree_build's ascending order; depth, subtree size and LCA answers do
 * not depend on the order. et_tree_export's succ / rank are indexed by these
 * half-edge ids (2n - 2 used; the last two are -2 / -1). Edges that are not
 * one tree on n nodes (an id out of range, a self-loop, a repeated edge, a
 * cycle) set ET_EINPUT in ctx's status.
 */
int et_tree_build_edges(et_ctx* ctx, const int32_t* d_u, const int32_t* d_v, int32_t n, int32_t root,
                        int32_t* d_parent_out, hipStream_t s, et_tree** out);

/*
 * LCA by range minima over the Euler tour (the RMQ approach that Section 3
 * compares Inlabel with): et_tree_rmq_build adds to a tree built by
 * et_tree_build the tour's node sequence as {depth, node} keys, in-block
 * suffix-minimum masks over 32-position blocks and a sparse table over the
 * block minima (about 14 bytes per half-edge); et_lca_rmq answers queries
 * with them (same results as et_lca).
 *   d_parent[n]  the parent array the tree was built from (read during the
 *                call only).
 * ET_EINVAL for a batch, a tree built from an edge list, or et_lca_rmq on a
 * tree without the tables. The tables are freed with the tree.
 */
int et_tree_rmq_build(et_tree* tree, const int32_t* d_parent, hipStream_t s);
int et_lca_rmq(const et_tree* tree, const int32_t* d_qx, const int32_t* d_qy, int64_t q, int32_t* d_out,
               hipStream_t s);

/*
 * Batch of independent rooted trees, built in one pass (Section 3.3, batched
 * queries; the C4 workload of thousands of trees of uneven size).
 *   d_parent[n_total]        the trees' parent arrays concatenated; ids are
 *                            local to each tree (0-based), its root has -1
 *   d_offsets[n_trees + 1]   device int64: tree t is [offsets[t], offsets[t+1]);
 *                            offsets[0] = 0, offsets[n_trees] = n_total
 * All trees hang below one virtual root, so one tour, one list ranking and
 * one set of Inlabel tables serve the whole batch; the LCA of two nodes of
 * one tree is unchanged. n_total + 1 < 2^30. A tree without exactly one
 * root or with a bad id sets ET_EINPUT in ctx's status.
 * et_tree_export on a batch accepts only depth / pre / size (per-tree
 * values, n_total entries); et_lca on a batch is ET_EINVAL (use
 * et_lca_batch).
 */
int et_tree_build_batch(et_ctx* ctx, const int32_t* d_parent, const int64_t* d_offsets,
                        int32_t n_trees, int64_t n_total, hipStream_t s, et_tree** out);

/*
 * LCA queries on a batch: query i asks for the LCA of the local nodes
 * d_qx[i], d_qy[i] of tree d_qtree[i]; d_out[i] is a local id, or -1 for a
 * query with an id out of range (which also sets ET_EINPUT).
 */
int et_lca_batch(const et_tree* tree, const int32_t* d_qtree, const int32_t* d_qx,
                 const int32_t* d_qy, int64_t q, int32_t* d_out, hipStream_t s);

/*
 * Many small trees built and queried in one kernel launch (Section 3.3,
 * batched queries on preprocessed trees; Sections 2 and 3.1 for each
 * tree's path). Each tree is built entirely in one workgroup's LDS (stable
 * child grouping, successors, sublist list ranking of the tour, depth /
 * preorder / size, Inlabel tables) and its queries are answered from those
 * tables, so HBM sees only the parent arrays, the queries and the answers.
 * Workgroups take trees from a counter until none are left (a persistent
 * grid sized to the GPU). Nothing is kept: the call returns no et_tree.
 *   d_parent[n_total]        concatenated parent arrays, local ids, -1 at
 *                            each tree's root (as for et_tree_build_batch)
 *   d_offsets[n_trees + 1]   device int64 node offsets: tree t is
 *                            [offsets[t], offsets[t+1]); offsets[0] = 0,
 *                            offsets[n_trees] = n_total
 *   max_tree_nodes           an upper bound on every tree's size, 1 ..
 *                            ET_FUSED_MAX_NODES; it sets the LDS each
 *                            workgroup takes (a smaller bound lets more
 *                            workgroups share a compute unit)
 *   d_qoffsets[n_trees + 1]  device int64 query offsets: the queries of tree
 *                            t are [qoffsets[t], qoffsets[t+1]) (queries come
 *                            grouped by tree); qoffsets[n_trees] = q_total
 *   d_qx, d_qy[q_total]      local node ids of each query
 *   d_out[q_total]           output: the LCA as a local id; -1 for a query
 *                            with an id out of range or on a malformed tree
 *   d_depth, d_pre, d_size   optional outputs (NULL allowed), n_total
 *                            entries each: depth, 0-based preorder and
 *                            subtree size of every node within its tree
 *   d_order[n_trees]         optional (NULL = 0, 1, 2, ...): the order in
 *                            which workgroups take the trees, a permutation
 *                            of 0 .. n_trees-1; the data stays where it is.
 *                            Costly trees first shortens the launch's tail
 *                            (the last trees running on few compute units).
 *                            An entry out of range sets ET_EINPUT and is
 *                            skipped; a repeated entry leaves the tree it
 *                            displaces unanswered
 * Same results as et_tree_build_batch + et_lca_batch (and per tree as
 * et_tree_build + et_lca). ET_ESIZE if max_tree_nodes exceeds
 * ET_FUSED_MAX_NODES or the LDS it needs exceeds what one workgroup may
 * take on this GPU. A tree larger than max_tree_nodes, a parent array that
 * is not one tree, or inconsistent offsets set ET_EINPUT in ctx's status.
 * Uses a counter pair of ctx: calls sharing a context must be ordered on
 * one stream.
 */
#define ET_FUSED_MAX_NODES 4096
int et_lca_batch_fused(et_ctx* ctx, const int32_t* d_parent, const int64_t* d_offsets, int32_t n_trees,
                       int64_t n_total, int32_t max_tree_nodes, const int64_t* d_qoffsets, const int32_t* d_qx,
                       const int32_t* d_qy, int64_t q_total, int32_t* d_out, int32_t* d_depth, int32_t* d_pre,
                       int32_t* d_size, const int32_t* d_order, hipStream_t s);

/*
 * The tour itself as an array (Section 2: the Euler tour as the sequence of
 * its half-edges, the inverse of the rank): d_tour[r] = the half-edge id at
 * tour position r, for r in [0, 2(n-1)). Half-edge ids as for d_rank of
 * et_tree_export (2c / 2c+1 for a parent-array tree, 2i / 2i+1 for an
 * edge-list tree). ET_EINVAL for a batch.
 */
int et_tree_export_tour(const et_tree* tree, int32_t* d_tour, hipStream_t s);

/* Number of nodes of a built tree or batch (host value). */
int32_t et_tree_size(const et_tree* tree);

/* Number of trees of a batch (0 for a single tree). */
int32_t et_tree_batch_size(const et_tree* tree);

/*
 * Copy tables of a built tree into caller-owned device arrays; any output
 * may be NULL.
 *   d_succ[2n], d_rank[2n]   tour successor (-1 at the tail, -2 on the
 *                            root's two ids) and tour position (-1 there)
 *   d_depth[n]               distance from the root
 *   d_pre[n]                 0-based preorder number (root 0)
 *   d_size[n]                number of nodes in the subtree
 *   d_inlabel[n], d_asc[n]   Schieber-Vishkin inlabel and ascendant words
 */
int et_tree_export(const et_tree* tree, int32_t* d_succ, int32_t* d_rank, int32_t* d_depth,
                   int32_t* d_pre, int32_t* d_size, uint32_t* d_inlabel, uint32_t* d_asc,
                   hipStream_t s);

/* Release a tree's device tables to its context's pool, ordered on stream
 * s: work enqueued on s before this call may still read them, and a later
 * call on another stream that reuses the blocks first waits for s. */
void et_tree_free(et_tree* tree, hipStream_t s);

/*
 * Device-memory footprints, for admission control by callers that share a
 * GPU between jobs (host-only functions: no device call, no GPU needed).
 * Launch shapes are taken from ctx, or the library defaults when ctx is
 * NULL.
 *
 * et_tree_footprint: for et_tree_build on one tree of n_total nodes
 * (n_trees = 0) or et_tree_build_batch on n_trees trees of n_total nodes in
 * all: *h_table_bytes = the bytes of the tables the tree keeps until
 * et_tree_free (exact), *h_scratch_bytes = an upper bound on the scratch
 * the build takes from the context's pool (the sum of all its scratch
 * blocks, so a pool that caches nothing grows by at most table + scratch).
 * Either output may be NULL. ET_EINVAL for sizes the build rejects.
 */
int et_tree_footprint(const et_ctx* ctx, int64_t n_total, int32_t n_trees, int64_t* h_table_bytes,
                      int64_t* h_scratch_bytes);

/* The same bound for et_bridges on one graph (n_graphs = 0) or
 * et_bridges_batch on n_graphs graphs with n_total vertices and nnz_total
 * CSR slots in all. */
int et_bridges_footprint(const et_ctx* ctx, int32_t n_total, int32_t nnz_total, int32_t n_graphs,
                         int64_t* h_scratch_bytes);

/* Device bytes a built tree holds now (its pool blocks, RMQ tables included). */
int et_tree_bytes(const et_tree* tree, int64_t* h_bytes);

/* The context's pool: *h_held = bytes allocated from the device (cached
 * blocks included), *h_live = bytes handed out now (trees' tables, scratch
 * of calls in progress), *h_peak_live = the most live bytes since the last
 * reset; reset_peak != 0 then restarts the peak at the live bytes. Outputs
 * may be NULL. Host bookkeeping only: no device call. */
int et_ctx_pool_stats(et_ctx* ctx, int64_t* h_held, int64_t* h_live, int64_t* h_peak_live, int reset_peak);

/*
 * Batched LCA queries on a built tree (Section 3: for each pair (x_i, y_i)
 * the deepest node that is an ancestor of both). One lane per query,
 * constant work per query (Inlabel query of Schieber and Vishkin).
 *   d_qx[q], d_qy[q]  query endpoints (node ids)
 *   d_out[q]          output: LCA id; -1 for a query with an id out of
 *                     range (which also sets ET_EINPUT)
 */
int et_lca(const et_tree* tree, const int32_t* d_qx, const int32_t* d_qy, int64_t q,
           int32_t* d_out, hipStream_t s);

/*
 * Node levels (distance from the root) by pointer jumping: the
 * preprocessing of the naive LCA algorithm the paper compares against
 * (Section 3.1, "The Naive Algorithm"). Every node's ancestor pointer starts
 * at its parent and is doubled until it reaches a node of known level; five
 * jumps are made between global synchronisations.
 *   d_parent[n]  parent array as for et_tree_build (n >= 1, n < 2^30)
 *   d_level[n]   output (caller-owned device array)
 * A parent array that is not a tree sets ET_EINPUT in ctx's status (nodes
 * that never reach the root keep level -1).
 */
int et_levels(et_ctx* ctx, const int32_t* d_parent, int32_t n, int32_t* d_level, hipStream_t s);

/*
 * LCA queries by climbing (Section 3.1, "The Naive Algorithm"): one lane per
 * query moves the deeper of x, y up to the other's level, then both up
 * until they meet; time grows with the x-y distance.
 *   d_parent[n], d_level[n]  the tree and its levels from et_levels
 *   d_qx[q], d_qy[q]         query pairs; d_out[q] receives the LCA, or -1
 *                            for a query with an id out of range or levels
 *                            that do not match the parent array (both also
 *                            set ET_EINPUT).
 */
int et_lca_naive(et_ctx* ctx, const int32_t* d_parent, const int32_t* d_level, int32_t n,
                 const int32_t* d_qx, const int32_t* d_qy, int64_t q, int32_t* d_out, hipStream_t s);

/*
 * Bridges of an undirected graph (Section 4: edge e is a bridge iff
 * deleting it disconnects its endpoints), by Tarjan-Vishkin: spanning
 * forest by hooking connected components, Euler tour of the forest,
 * preorder and subtree sizes, per-node minimum / maximum preorder over
 * non-tree neighbours, low / high by range minimum / maximum over subtree
 * intervals, and the test on tree edges.
 *   d_row_ptr[n+1], d_col[nnz]  symmetric CSR: every edge {u, w} appears as
 *                  slot (u, w) in row u and slot (w, u) in row w; each row
 *                  sorted ascending; parallel edges repeat a column; a
 *                  self-loop {u, u} gives two (u, u) slots. n < 2^30,
 *                  nnz < 2^31.
 *   d_mask[ceil(nnz/32)]  output: bit k (word k/32, bit k%32) is set iff
 *                  slot k belongs to a bridge (both slots of a bridge set)
 *   h_count        optional host output: number of bridges. When non-NULL
 *                  the call waits for stream s before returning.
 * Graphs may be disconnected (one tour per component). A self-loop or an
 * edge with a parallel copy is never a bridge.
 */
int et_bridges(et_ctx* ctx, const int32_t* d_row_ptr, const int32_t* d_col, int32_t n,
               int32_t nnz, uint32_t* d_mask, int64_t* h_count, hipStream_t s);

/*
 * Bridges by the comparison methods of Section 4.1: Chaitanya-Kothapalli
 * marking. Every non-tree edge marks the tree edges on its path up to the
 * endpoints' lowest common ancestor; unmarked tree edges are bridges.
 *   spanning = 0   CK: a breadth-first-search forest (one root per
 *                  component, chosen by connectivity labels). The call
 *                  waits for stream s about once per 16 BFS levels.
 *   spanning = 1   hybrid: the connectivity forest of et_bridges, rooted and
 *                  levelled by its Euler tour.
 * Arguments, output and limits as for et_bridges (the result is the same).
 */
int et_bridges_ck(et_ctx* ctx, const int32_t* d_row_ptr, const int32_t* d_col, int32_t n, int32_t nnz,
                  int32_t spanning, uint32_t* d_mask, int64_t* h_count, hipStream_t s);

/*
 * Bridges of a batch of independent graphs in one pass (the bridge problem
 * of Section 4 for many instances at once, as the tree batch of Section 3.3
 * does for LCA). The batch runs as the disjoint union of its graphs, so
 * every graph gets the answer et_bridges gives it alone.
 *   d_row_ptr[n_total + n_graphs]  the graphs' own row-pointer arrays back to
 *                  back: graph t's n_t + 1 entries (0 .. nnz_t) start at
 *                  d_voff[t] + t
 *   d_col[nnz_total]  the graphs' column arrays back to back, ids local to
 *                  each graph; each graph a symmetric CSR as for et_bridges
 *   d_voff[n_graphs + 1], d_soff[n_graphs + 1]  device int64 vertex and slot
 *                  offsets: graph t owns vertices [voff[t], voff[t+1]) and
 *                  slots [soff[t], soff[t+1]); both start at 0 and end at
 *                  n_total and nnz_total; empty graphs are allowed
 *   d_mask[mask_words]  output, one word-aligned mask per graph: graph t's
 *                  ceil(nnz_t / 32) words follow those of graphs 0 .. t-1,
 *                  and its bit k is set iff its slot k belongs to a bridge.
 *                  mask_words >= the sum of ceil(nnz_t / 32); words past
 *                  that sum are zeroed
 *   d_counts[n_graphs]  optional device output: bridges per graph
 * n_total < 2^30, nnz_total < 2^31. Offsets that do not match the row
 * pointers, a column outside its own graph, or a mask_words below the
 * sum set ET_EINPUT in ctx's status (outputs are then undefined).
 * Scratch: n_total + 1 + nnz_total int32 and ceil(nnz_total / 32) words
 * beyond what et_bridges takes for the union.
 */
int et_bridges_batch(et_ctx* ctx, const int32_t* d_row_ptr, const int32_t* d_col, const int64_t* d_voff,
                     const int64_t* d_soff, int32_t n_graphs, int32_t n_total, int32_t nnz_total,
                     uint32_t* d_mask, int64_t mask_words, int64_t* d_counts, hipStream_t s);

/*
 * Bridges of many small graphs in one kernel launch (Section 4.1 for each
 * graph; batched as the tree batch of Section 3.3). Each graph is solved in
 * one workgroup's LDS -- spanning forest by union-find, the forest's Euler
 * tour (succ = next(twin), Section 2.1) ranked by pointer jumping,
 * preorder and subtree sizes, per-vertex non-forest extremes, low / high by
 * range minima and maxima, the bridge test -- so HBM sees only the CSR
 * arrays, the mask words and the counts. Workgroups take graphs from a
 * counter until none are left.
 *   d_row_ptr, d_col, d_voff, d_soff   as for et_bridges_batch (each graph's
 *                  own row pointers back to back, its columns back to back,
 *                  int64 vertex and slot offsets)
 *   d_moff[n_graphs + 1]  device int64 offsets of the graphs' mask words:
 *                  graph t's ceil(nnz_t / 32) words start at moff[t]
 *                  (moff[0] = 0; the layout et_bridges_batch uses when they
 *                  are the running sums of ceil(nnz_t / 32))
 *   max_graph_vertices, max_graph_slots  upper bounds on every graph's
 *                  vertex and slot counts, at most ET_FUSED_MAX_VERTICES and
 *                  ET_FUSED_MAX_SLOTS; they set the LDS each workgroup takes
 *   d_mask[mask_words]  output words (bit k of graph t's words = its slot k)
 *   d_counts[n_graphs]  optional device output: bridges per graph
 *   d_order[n_graphs]   optional (NULL = 0, 1, 2, ...): the order in which
 *                  workgroups take the graphs, a permutation of
 *                  0 .. n_graphs-1 (costly graphs first shortens the
 *                  launch's tail); an entry out of range sets ET_EINPUT and
 *                  is skipped, a repeated entry leaves the graph it
 *                  displaces unanswered
 * Same masks and counts as et_bridges_batch. ET_ESIZE if a bound exceeds
 * its maximum or the LDS it needs exceeds what one workgroup may take. A
 * graph larger than the bounds, offsets that do not match, rows that are
 * not sorted or a slot without its twin set ET_EINPUT in ctx's status (that
 * graph's words are then zero). Uses a counter pair of ctx: calls sharing
 * a context must be ordered on one stream.
 */
#define ET_FUSED_MAX_VERTICES 1024
#define ET_FUSED_MAX_SLOTS 8192
int et_bridges_batch_fused(et_ctx* ctx, const int32_t* d_row_ptr, const int32_t* d_col, const int64_t* d_voff,
                           const int64_t* d_soff, const int64_t* d_moff, int32_t n_graphs, int32_t n_total,
                           int32_t nnz_total, int32_t max_graph_vertices, int32_t max_graph_slots,
                           uint32_t* d_mask, int64_t mask_words, int64_t* d_counts, const int32_t* d_order,
                           hipStream_t s);

/* Device-side bridge count of the most recent et_bridges call (for a batch:
 * the total over its graphs) on ctx
 * (written to a caller-owned device int64). */
int et_bridges_count(et_ctx* ctx, int64_t* d_count, hipStream_t s);

#ifdef __cplusplus
}
#endif

#endif /* ET_H */

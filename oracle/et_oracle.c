/*
 * Plain sequential CPU oracle for the Euler-tour hot path.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do. It shares no code, header, table or helper with
 * the GPU path. Every routine computes the plain definition of its result
 * with the most obvious sequential algorithm, so that it can be checked
 * against the paper by eye:
 *
 *   - Euler tour of a rooted tree (Section 2, Fig. 1): an iterative
 *     depth-first search that visits the children of every node in
 *     ascending id order and emits the half-edge into a child on the way
 *     down and the half-edge out of it on the way back up. Half-edge ids:
 *     2c is (parent(c) -> c), 2c+1 is (c -> parent(c)); the root's two ids
 *     are unused. rank(e) is the position of e in the tour (head = 0).
 *   - depth (distance to the root), preorder (0-based discovery index) and
 *     subtree size (Section 2: a subtree is an interval of the tour).
 *   - List ranking (Section 2.2): walk each list from its head.
 *   - LCA (Section 3): parent climbing after levelling the depths (the
 *     query procedure of the naive method, Section 3.1), and Tarjan's
 *     offline union-find LCA for trees too deep to climb.
 *   - Inlabel tables (Section 3.1, Schieber-Vishkin): inlabel(v) is the
 *     member of [pre(v)+1, pre(v)+size(v)] with the most trailing zeros,
 *     found by trying the largest power of two first; ascendant(v) is the
 *     OR of 2^h(inlabel(u)) over all ancestors-or-self u; head[I] records
 *     the parent of the top node of the path labelled I and its depth.
 *   - Euler tour from an unordered edge list (Section 2.1, Fig. 2): the
 *     DCEL construction itself. Both directions of every edge become
 *     half-edges (2i and 2i+1 for edge i, twins of each other); B is the
 *     list of half-edges in lexicographic (source, target) order; next(e)
 *     is the half-edge after e in its source's run of B, wrapping to the
 *     run's first; succ(e) = next(twin(e)). The cycle is cut before the
 *     first half-edge of the root's run. Children are then visited in
 *     cyclic id order starting after the parent.
 *   - Bridges (Section 4.1): Tarjan's depth-first low-link algorithm. A
 *     tree edge {p, u} is a bridge iff low(u) > disc(p). Parallel edges
 *     are handled by skipping the parent only once; self-loops are ignored.
 *
 * Return codes: 0 ok, -1 bad argument, -4 malformed input (not a tree,
 * id out of range, list not a set of simple paths).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_EINPUT (-4)

/* children of every node in ascending id order, as a CSR built by a
 * sequential counting pass (ids visited in increasing order) */
static int build_children(const int32_t* parent, int32_t n, int32_t** cptr_out,
                          int32_t** cidx_out, int32_t* root_out) {
    int32_t root = -1;
    int32_t* cptr = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
    int32_t* cidx = (int32_t*)malloc(((size_t)n + 1) * sizeof(int32_t));
    int32_t* fill = (int32_t*)malloc(((size_t)n + 1) * sizeof(int32_t));
    if (!cptr || !cidx || !fill) { free(cptr); free(cidx); free(fill); return ORC_EINVAL; }
    for (int32_t v = 0; v < n; ++v) {
        int32_t p = parent[v];
        if (p == -1) {
            if (root != -1) { free(cptr); free(cidx); free(fill); return ORC_EINPUT; }
            root = v;
        } else if (p < 0 || p >= n || p == v) {
            free(cptr); free(cidx); free(fill); return ORC_EINPUT;
        } else {
            cptr[p + 1]++;
        }
    }
    if (root == -1) { free(cptr); free(cidx); free(fill); return ORC_EINPUT; }
    for (int32_t v = 0; v < n; ++v) cptr[v + 1] += cptr[v];
    memcpy(fill, cptr, (size_t)n * sizeof(int32_t));
    for (int32_t v = 0; v < n; ++v)
        if (parent[v] >= 0) cidx[fill[parent[v]]++] = v;
    free(fill);
    *cptr_out = cptr;
    *cidx_out = cidx;
    *root_out = root;
    return ORC_OK;
}

/* Euler tour by iterative DFS. Outputs (each may be NULL):
 *   tour[2(n-1)]  half-edge ids in tour order
 *   rank[2n]      position of each half-edge in the tour, -1 for the root's ids
 *   depth[n], pre[n], size[n], and *root_out. */
int oracle_euler_tour(const int32_t* parent, int32_t n, int32_t* tour, int32_t* rank,
                      int32_t* depth, int32_t* pre, int32_t* size, int32_t* root_out) {
    if (!parent || n < 1) return ORC_EINVAL;
    int32_t *cptr, *cidx, root;
    int rc = build_children(parent, n, &cptr, &cidx, &root);
    if (rc) return rc;
    int32_t* stack = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    int32_t* next_child = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    int32_t* d = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    int32_t* pr = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    int32_t* sz = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    if (!stack || !next_child || !d || !pr || !sz) {
        free(stack); free(next_child); free(d); free(pr); free(sz); free(cptr); free(cidx);
        return ORC_EINVAL;
    }
    if (rank) for (int64_t e = 0; e < 2 * (int64_t)n; ++e) rank[e] = -1;
    for (int32_t v = 0; v < n; ++v) next_child[v] = cptr[v];

    int64_t pos = 0;        /* next tour position */
    int32_t visited = 0;    /* next preorder number */
    int32_t top = 0;
    stack[top++] = root;
    d[root] = 0;
    pr[root] = visited++;
    while (top > 0) {
        int32_t u = stack[top - 1];
        if (next_child[u] < cptr[u + 1]) {
            int32_t c = cidx[next_child[u]++];
            /* descend along half-edge 2c = (u -> c) */
            if (tour) tour[pos] = 2 * c;
            if (rank) rank[2 * c] = (int32_t)pos;
            pos++;
            d[c] = d[u] + 1;
            pr[c] = visited++;
            stack[top++] = c;
        } else {
            /* every child of u is finished: size is one plus the sum */
            int32_t s = 1;
            for (int32_t k = cptr[u]; k < cptr[u + 1]; ++k) s += sz[cidx[k]];
            sz[u] = s;
            top--;
            if (u != root) {
                /* return along half-edge 2u+1 = (u -> parent(u)) */
                if (tour) tour[pos] = 2 * u + 1;
                if (rank) rank[2 * u + 1] = (int32_t)pos;
                pos++;
            }
        }
    }
    rc = ORC_OK;
    if (visited != n) rc = ORC_EINPUT; /* some node is not reachable from the root: a cycle */
    if (rc == ORC_OK) {
        if (depth) memcpy(depth, d, (size_t)n * sizeof(int32_t));
        if (pre) memcpy(pre, pr, (size_t)n * sizeof(int32_t));
        if (size) memcpy(size, sz, (size_t)n * sizeof(int32_t));
        if (root_out) *root_out = root;
    }
    free(stack); free(next_child); free(d); free(pr); free(sz); free(cptr); free(cidx);
    return rc;
}

/* List ranking by walking. succ[e] is the next element, -1 ends a list,
 * -2 marks an unused slot. rank[e] = number of steps from the head of e's
 * list; unused slots get -1. Every used slot must lie on exactly one list
 * that starts at one of heads[]; otherwise ORC_EINPUT. */
int oracle_list_rank(const int32_t* succ, int32_t len, const int32_t* heads, int32_t nheads,
                     int32_t* rank) {
    if (len < 0 || nheads < 0 || (len > 0 && (!succ || !rank)) || (nheads > 0 && !heads))
        return ORC_EINVAL;
    for (int32_t e = 0; e < len; ++e) rank[e] = -1;
    int64_t ranked = 0;
    for (int32_t h = 0; h < nheads; ++h) {
        int32_t e = heads[h];
        if (e < 0 || e >= len || succ[e] == -2) return ORC_EINPUT;
        int32_t r = 0;
        while (e != -1) {
            if (e < 0 || e >= len || succ[e] == -2 || rank[e] != -1) return ORC_EINPUT;
            rank[e] = r++;
            ranked++;
            e = succ[e];
        }
    }
    int64_t used = 0;
    for (int32_t e = 0; e < len; ++e) used += (succ[e] != -2);
    return used == ranked ? ORC_OK : ORC_EINPUT;
}

/* Weighted list ranking (Section 2.2): sum[e] = the weights from the head
 * of e's list through e, added in 32-bit two's complement; rank as in
 * oracle_list_rank. Unused slots (succ == -2) get rank -1 and sum 0. */
int oracle_list_scan(const int32_t* succ, const int32_t* weight, int32_t len, const int32_t* heads,
                     int32_t nheads, int32_t* rank, int32_t* sum) {
    if (len < 0 || (len > 0 && (!weight || !sum))) return ORC_EINVAL;
    int rc = oracle_list_rank(succ, len, heads, nheads, rank);
    if (rc) return rc;
    for (int32_t e = 0; e < len; ++e) sum[e] = 0;
    for (int32_t k = 0; k < nheads; ++k) {
        uint32_t acc = 0;
        for (int32_t e = heads[k]; e != -1; e = succ[e]) {
            acc += (uint32_t)weight[e];
            sum[e] = (int32_t)acc;
        }
    }
    return ORC_OK;
}

/* LCA by climbing: lift the deeper endpoint to the other's depth, then lift
 * both until they meet. depth[] must be the true depths. */
int oracle_lca_climb(const int32_t* parent, const int32_t* depth, int32_t n,
                     const int32_t* qx, const int32_t* qy, int64_t q, int32_t* out) {
    if (!parent || !depth || n < 1 || q < 0 || (q > 0 && (!qx || !qy || !out))) return ORC_EINVAL;
    for (int64_t i = 0; i < q; ++i) {
        int32_t x = qx[i], y = qy[i];
        if (x < 0 || x >= n || y < 0 || y >= n) return ORC_EINPUT;
        while (depth[x] > depth[y]) x = parent[x];
        while (depth[y] > depth[x]) y = parent[y];
        while (x != y) { x = parent[x]; y = parent[y]; }
        out[i] = x;
    }
    return ORC_OK;
}

static int32_t dsu_find(int32_t* up, int32_t x) {
    int32_t r = x;
    while (up[r] != r) r = up[r];
    while (up[x] != r) { int32_t nx = up[x]; up[x] = r; x = nx; }
    return r;
}

/* Tarjan's offline LCA. After the DFS finishes a child c of u, c's set is
 * merged into u's set and the set's representative remembers u as its
 * ancestor; a query (u, v) is answered when u finishes if v has already
 * finished: the answer is the remembered ancestor of v's set. */
int oracle_lca_offline(const int32_t* parent, int32_t n, const int32_t* qx, const int32_t* qy,
                       int64_t q, int32_t* out) {
    if (!parent || n < 1 || q < 0 || (q > 0 && (!qx || !qy || !out))) return ORC_EINVAL;
    int32_t *cptr, *cidx, root;
    int rc = build_children(parent, n, &cptr, &cidx, &root);
    if (rc) return rc;
    for (int64_t i = 0; i < q; ++i)
        if (qx[i] < 0 || qx[i] >= n || qy[i] < 0 || qy[i] >= n) {
            free(cptr); free(cidx); return ORC_EINPUT;
        }
    /* queries grouped by endpoint: each query is listed under both ends */
    int64_t* qptr = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t* qlist = (int64_t*)malloc((size_t)(2 * q + 1) * sizeof(int64_t));
    int64_t* qfill = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
    int32_t* up = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    int32_t* anc = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    char* done = (char*)calloc((size_t)n, 1);
    int32_t* stack = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    int32_t* next_child = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    if (!qptr || !qlist || !qfill || !up || !anc || !done || !stack || !next_child) {
        rc = ORC_EINVAL;
        goto out;
    }
    for (int64_t i = 0; i < q; ++i) { qptr[qx[i] + 1]++; qptr[qy[i] + 1]++; }
    for (int32_t v = 0; v < n; ++v) qptr[v + 1] += qptr[v];
    memcpy(qfill, qptr, (size_t)n * sizeof(int64_t));
    for (int64_t i = 0; i < q; ++i) { qlist[qfill[qx[i]]++] = i; qlist[qfill[qy[i]]++] = i; }
    for (int32_t v = 0; v < n; ++v) { up[v] = v; anc[v] = v; next_child[v] = cptr[v]; }

    int32_t top = 0, seen = 1;
    stack[top++] = root;
    while (top > 0) {
        int32_t u = stack[top - 1];
        if (next_child[u] < cptr[u + 1]) {
            stack[top++] = cidx[next_child[u]++];
            seen++;
            continue;
        }
        /* u is finished */
        top--;
        done[u] = 1;
        for (int64_t k = qptr[u]; k < qptr[u + 1]; ++k) {
            int64_t i = qlist[k];
            int32_t other = (qx[i] == u) ? qy[i] : qx[i];
            if (done[other]) out[i] = anc[dsu_find(up, other)];
        }
        if (u != root) {
            int32_t p = parent[u];
            int32_t a = dsu_find(up, u), b = dsu_find(up, p);
            up[a] = b;
            anc[b] = p;
        }
    }
    rc = (seen == n) ? ORC_OK : ORC_EINPUT;
out:
    free(qptr); free(qlist); free(qfill); free(up); free(anc); free(done); free(stack);
    free(next_child); free(cptr); free(cidx);
    return rc;
}

static uint32_t trailing_zeros(uint32_t x) { /* x != 0 */
    uint32_t t = 0;
    while (t < 31 && !(x & 1u)) { x >>= 1; t++; }
    return t;
}

/* Schieber-Vishkin tables from the definitions. Needs parent, depth, pre
 * and size of the tree. Outputs:
 *   inlabel[n]  the member of [pre+1, pre+size] with the most trailing zeros
 *   asc[n]      OR of 2^h(inlabel(u)) over the ancestors-or-self u of v
 *   head_parent[n+1], head_depth[n+1]  for every path label I: the parent
 *               of the path's top node and that parent's depth (-1, -1 for
 *               the root's path); entries of labels that no path uses = -3 */
int oracle_sv_tables(const int32_t* parent, const int32_t* depth, const int32_t* pre,
                     const int32_t* size, int32_t n, uint32_t* inlabel, uint32_t* asc,
                     int32_t* head_parent, int32_t* head_depth) {
    if (!parent || !depth || !pre || !size || n < 1 || !inlabel || !asc || !head_parent ||
        !head_depth)
        return ORC_EINVAL;
    for (int32_t v = 0; v < n; ++v) {
        uint32_t lo = (uint32_t)pre[v] + 1u, hi = (uint32_t)pre[v] + (uint32_t)size[v];
        uint32_t best = 0;
        for (int t = 31; t >= 0 && !best; --t) {
            uint32_t m = (hi >> t) << t; /* largest multiple of 2^t not above hi */
            if (m >= lo && m != 0) best = m;
        }
        if (!best) return ORC_EINPUT; /* [pre+1, pre+size] always holds a nonzero member */
        inlabel[v] = best;
    }
    /* nodes in preorder, so every parent comes before its children */
    int32_t* by_pre = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    if (!by_pre) return ORC_EINVAL;
    for (int32_t v = 0; v < n; ++v) by_pre[pre[v]] = v;
    for (int32_t k = 0; k < n; ++k) {
        int32_t v = by_pre[k];
        uint32_t own = 1u << trailing_zeros(inlabel[v]);
        asc[v] = (parent[v] < 0) ? own : (asc[parent[v]] | own);
    }
    free(by_pre);
    for (int32_t i = 0; i <= n; ++i) { head_parent[i] = -3; head_depth[i] = -3; }
    for (int32_t v = 0; v < n; ++v) {
        int32_t p = parent[v];
        if (p < 0 || inlabel[p] != inlabel[v]) {
            head_parent[inlabel[v]] = p;
            head_depth[inlabel[v]] = depth[v] - 1;
        }
    }
    return ORC_OK;
}

/* Euler tour from the unordered edge list of a tree (Section 2.1): the
 * DCEL of Fig. 2 built as described there. eu[i], ev[i] is edge i; half-edge
 * 2i is (eu[i] -> ev[i]) and 2i+1 its twin. Outputs: succ[2m] (-1 at the
 * tail), rank[2m], and per node parent (-1 at the root), depth, pre, size.
 * The edges must form one tree on n nodes (m = n - 1). */
int oracle_euler_tour_edges(int32_t n, int64_t m, const int32_t* eu, const int32_t* ev, int32_t root,
                            int32_t* succ, int32_t* rank, int32_t* parent, int32_t* depth, int32_t* pre,
                            int32_t* size) {
    if (n < 1 || m != (int64_t)n - 1 || root < 0 || root >= n) return ORC_EINPUT;
    const int64_t L = 2 * m;
    for (int64_t i = 0; i < m; ++i)
        if (eu[i] < 0 || eu[i] >= n || ev[i] < 0 || ev[i] >= n || eu[i] == ev[i]) return ORC_EINPUT;
    for (int32_t v = 0; v < n; ++v) { parent[v] = -1; depth[v] = 0; pre[v] = 0; size[v] = 1; }
    size[root] = n;
    if (L == 0) return ORC_OK;
    int32_t* src = malloc(L * sizeof(int32_t));
    int32_t* dst = malloc(L * sizeof(int32_t));
    int32_t* B = malloc(L * sizeof(int32_t));
    int32_t* tmp = malloc(L * sizeof(int32_t));
    int32_t* pos = malloc(L * sizeof(int32_t));
    int64_t* cnt = calloc((size_t)n + 1, sizeof(int64_t));
    int64_t* first = malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!src || !dst || !B || !tmp || !pos || !cnt || !first) {
        free(src); free(dst); free(B); free(tmp); free(pos); free(cnt); free(first);
        return ORC_EINVAL;
    }
    for (int64_t i = 0; i < m; ++i) {
        src[2 * i] = eu[i]; dst[2 * i] = ev[i];
        src[2 * i + 1] = ev[i]; dst[2 * i + 1] = eu[i];
    }
    /* B: lexicographic order of (source, target), as two stable counting
     * sorts (by target, then by source) */
    for (int64_t h = 0; h < L; ++h) cnt[dst[h] + 1]++;
    for (int32_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
    for (int64_t h = 0; h < L; ++h) tmp[cnt[dst[h]]++] = (int32_t)h;
    memset(cnt, 0, ((size_t)n + 1) * sizeof(int64_t));
    for (int64_t h = 0; h < L; ++h) cnt[src[h] + 1]++;
    for (int32_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
    for (int32_t v = 0; v <= n; ++v) first[v] = cnt[v];   /* first[x]: start of x's run in B */
    for (int64_t k = 0; k < L; ++k) {
        const int32_t h = tmp[k];
        B[cnt[src[h]]++] = h;
    }
    for (int64_t k = 0; k < L; ++k) pos[B[k]] = (int32_t)k;
    /* succ(e) = next(twin(e)); next wraps inside the source's run */
    for (int64_t e = 0; e < L; ++e) {
        const int32_t t = (int32_t)(e ^ 1);
        const int32_t x = src[t];
        const int64_t k = pos[t];
        succ[e] = (k + 1 < first[x + 1]) ? B[k + 1] : B[first[x]];
    }
    /* cut the cycle before the root's first half-edge */
    int rc = ORC_OK;
    if (first[root] == first[root + 1]) rc = ORC_EINPUT;          /* root has no edge */
    const int32_t head = (rc == ORC_OK) ? B[first[root]] : -1;
    for (int64_t e = 0; e < L && rc == ORC_OK; ++e)
        if (succ[e] == head) { succ[e] = -1; break; }
    /* walk: ranks, directions (a half-edge goes down iff it precedes its twin),
     * parent, depth, preorder, size */
    for (int64_t e = 0; e < L; ++e) rank[e] = -1;
    int64_t r = 0;
    for (int32_t e = head; rc == ORC_OK && e != -1; e = succ[e]) {
        if (r >= L || rank[e] != -1) { rc = ORC_EINPUT; break; }
        rank[e] = (int32_t)r++;
    }
    if (rc == ORC_OK && r != L) rc = ORC_EINPUT;                /* edges not one connected tree */
    if (rc == ORC_OK) {
        int32_t d = 0, visited = 1;
        for (int32_t e = head; e != -1; e = succ[e]) {
            const int32_t tw = e ^ 1;
            if (rank[e] < rank[tw]) {                          /* down into dst[e] */
                const int32_t c = dst[e];
                parent[c] = src[e];
                depth[c] = ++d;
                pre[c] = visited++;
                size[c] = (rank[tw] - rank[e] + 1) / 2;
            } else {
                --d;
            }
        }
    }
    free(src); free(dst); free(B); free(tmp); free(pos); free(cnt); free(first);
    return rc;
}

/* Bridges of an undirected multigraph in symmetric CSR form (rows need not
 * be sorted). mask has ceil(nnz/32) words; bit k (word k/32, bit k%32) is
 * set iff CSR slot k belongs to a bridge. *count = number of bridges. */
int oracle_bridges(const int64_t* row_ptr, const int32_t* col, int32_t n, int64_t nnz,
                   uint32_t* mask, int64_t* count) {
    if (!row_ptr || n < 0 || nnz < 0 || (nnz > 0 && (!col || !mask))) return ORC_EINVAL;
    if (row_ptr[0] != 0 || row_ptr[n] != nnz) return ORC_EINPUT;
    for (int64_t k = 0; k < (nnz + 31) / 32; ++k) mask[k] = 0;
    int64_t nb = 0;
    int32_t* disc = (int32_t*)malloc(((size_t)n + 1) * sizeof(int32_t));
    int32_t* low = (int32_t*)malloc(((size_t)n + 1) * sizeof(int32_t));
    int32_t* par = (int32_t*)malloc(((size_t)n + 1) * sizeof(int32_t));
    int64_t* par_slot = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));  /* slot (p -> u) */
    int64_t* back_slot = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t)); /* slot (u -> p) */
    int64_t* it = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
    int32_t* stack = (int32_t*)malloc(((size_t)n + 1) * sizeof(int32_t));
    if (!disc || !low || !par || !par_slot || !back_slot || !it || !stack) {
        free(disc); free(low); free(par); free(par_slot); free(back_slot); free(it); free(stack);
        return ORC_EINVAL;
    }
    for (int32_t v = 0; v < n; ++v) { disc[v] = -1; back_slot[v] = -1; }
    int32_t clock = 0;
    int rc = ORC_OK;
    for (int32_t s = 0; s < n && rc == ORC_OK; ++s) {
        if (disc[s] != -1) continue;
        int32_t top = 0;
        disc[s] = low[s] = clock++;
        par[s] = -1;
        it[s] = row_ptr[s];
        stack[top++] = s;
        while (top > 0) {
            int32_t u = stack[top - 1];
            if (it[u] < row_ptr[u + 1]) {
                int64_t k = it[u]++;
                int32_t w = col[k];
                if (w < 0 || w >= n) { rc = ORC_EINPUT; break; }
                if (w == u) continue;                                   /* self-loop */
                if (w == par[u] && back_slot[u] == -1) { back_slot[u] = k; continue; }
                if (disc[w] == -1) {
                    disc[w] = low[w] = clock++;
                    par[w] = u;
                    par_slot[w] = k;
                    it[w] = row_ptr[w];
                    stack[top++] = w;
                } else if (disc[w] < low[u]) {
                    low[u] = disc[w];
                }
            } else {
                top--;
                int32_t p = par[u];
                if (p >= 0) {
                    if (low[u] < low[p]) low[p] = low[u];
                    if (low[u] > disc[p]) {
                        /* the only way out of u's subtree is the tree edge {p, u} */
                        if (back_slot[u] < 0) { rc = ORC_EINPUT; break; } /* not symmetric */
                        int64_t a = par_slot[u], b = back_slot[u];
                        mask[a >> 5] |= 1u << (a & 31);
                        mask[b >> 5] |= 1u << (b & 31);
                        nb++;
                    }
                }
            }
        }
    }
    if (count) *count = nb;
    free(disc); free(low); free(par); free(par_slot); free(back_slot); free(it); free(stack);
    return rc;
}

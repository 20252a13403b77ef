/*
 * dc_struct.hip -- region-graph structuring (Section "Search for control
 * structures") of every kernel of a batch whose control flow graphs the
 * graph stages have built.
 *
 * The region graph starts as the reachable blocks.  Repeatedly, a depth-first
 * search from the entry region visits regions in preorder (fall-through
 * successor first) and the first region that heads a template has the
 * template's regions merged into a new one, until one region is left or no
 * region heads a template.  Templates at a header H, in this order:
 *   if-else  H's successors A, B have H as only predecessor and one common
 *            single successor J (J joins when A and B are its only
 *            predecessors);
 *   if       (Fig. 2) one successor T has H as only predecessor and the
 *            other, F, as only successor (F joins when H and T are its only
 *            predecessors -- the two cases of the Fig. 3 trace);
 *   while    a successor B has H as only predecessor and only successor;
 *   linear   H's only successor S is not H, has H as only predecessor and at
 *            most one successor, or H among them;
 *   loop     H has an edge to itself.
 * The entry counts the start as one more predecessor.
 *
 * One wavefront per kernel runs the search; every lane takes the same steps
 * (the search is a chain).  Two changes keep a round short without changing
 * which merge is made:
 *   - the search stops at the first region that heads a template, which is
 *     the first such region of the whole preorder (regions are tested as the
 *     search reaches them, in preorder);
 *   - edges are not rewritten when their target is merged: every region has
 *     a forwarding entry to the region it was merged into, followed (with
 *     path halving) when an edge is read.  Only the header of a template has
 *     predecessors outside it, so forwarding every member to the new region
 *     is the same graph as rewriting the edges into the header.
 * Marks of the search carry the round number, so nothing is cleared between
 * rounds.  A kernel's regions (4 per block + 2) sit in LDS up to SR_LDS
 * regions, else in global memory; the same code reads both through generic
 * pointers.
 */
#include "dc_device.h"

namespace dc {

constexpr uint32_t SR_LDS = 512;   /* regions of a kernel kept in LDS */
constexpr uint32_t SR_NONE = 0xFFFFFFFFu;

struct Rg {
    int32_t *succ;      /* 2 per region, -1 none */
    uint32_t *npred;    /* predecessors (the entry: + 1) */
    uint32_t *fwd;      /* the region it was merged into; itself while alive */
    uint32_t *mark;     /* round of the last visit */
    uint32_t *stack;    /* 2 per region */
    uint32_t entry, next;
};

__device__ __forceinline__ uint32_t rg_find(Rg &g, uint32_t x) {
    while (g.fwd[x] != x) {
        const uint32_t p = g.fwd[x], q = g.fwd[p];
        g.fwd[x] = q;   /* path halving */
        x = q;
    }
    return x;
}
__device__ __forceinline__ int32_t rg_succ(Rg &g, uint32_t x, int e) {
    const int32_t y = g.succ[2 * x + e];
    return y < 0 ? -1 : (int32_t)rg_find(g, (uint32_t)y);
}
__device__ __forceinline__ int32_t rg_only(Rg &g, uint32_t x) {
    const int32_t a = rg_succ(g, x, 0), b = rg_succ(g, x, 1);
    if ((a >= 0) + (b >= 0) != 1) return -1;
    return a >= 0 ? a : b;
}

/* the template headed by x: members into m, returns the kind (0 none) */
__device__ int rg_match(Rg &g, uint32_t x, uint32_t *m, int *n) {
    const int32_t a = rg_succ(g, x, 0), b = rg_succ(g, x, 1);
    if (a >= 0 && b >= 0 && a != (int32_t)x && b != (int32_t)x) {
        const int32_t ja = rg_only(g, (uint32_t)a), jb = rg_only(g, (uint32_t)b);
        if (g.npred[a] == 1 && g.npred[b] == 1 && ja >= 0 && ja == jb && ja != (int32_t)x && ja != a && ja != b) {
            m[0] = x;
            m[1] = (uint32_t)a;
            m[2] = (uint32_t)b;
            *n = 3;
            if (g.npred[ja] == 2) {
                m[3] = (uint32_t)ja;
                *n = 4;
            }
            return DC_RG_IFELSE;
        }
        for (int k = 0; k < 2; k++) {
            const int32_t t = k == 0 ? a : b, f = k == 0 ? b : a;
            if (g.npred[t] == 1 && rg_only(g, (uint32_t)t) == f) {
                m[0] = x;
                m[1] = (uint32_t)t;
                *n = 2;
                if (g.npred[f] == 2) {
                    m[2] = (uint32_t)f;
                    *n = 3;
                }
                return DC_RG_IF;
            }
        }
        for (int k = 0; k < 2; k++) {
            const int32_t t = k == 0 ? a : b;
            if (g.npred[t] == 1 && rg_only(g, (uint32_t)t) == (int32_t)x) {
                m[0] = x;
                m[1] = (uint32_t)t;
                *n = 2;
                return DC_RG_WHILE;
            }
        }
    }
    const int32_t s = rg_only(g, x);
    if (s >= 0 && s != (int32_t)x && g.npred[s] == 1) {
        const int32_t s0 = rg_succ(g, (uint32_t)s, 0), s1 = rg_succ(g, (uint32_t)s, 1);
        if ((s0 >= 0) + (s1 >= 0) <= 1 || s0 == (int32_t)x || s1 == (int32_t)x) {
            m[0] = x;
            m[1] = (uint32_t)s;
            *n = 2;
            return DC_RG_LINEAR;
        }
    }
    if (a == (int32_t)x || b == (int32_t)x) {
        m[0] = x;
        *n = 1;
        return DC_RG_LOOP;
    }
    return 0;
}

/* merge m[0..n) (m[0] the header) into a new region; returns it */
__device__ uint32_t rg_merge(Rg &g, const uint32_t *m, int n, int kind) {
    const uint32_t H = m[0], R = g.next++;
    int32_t out[2] = {-1, -1};
    int no = 0;
    bool self = false;
    uint32_t into_h = 0;
    for (int i = 0; i < n; i++)
        for (int e = 0; e < 2; e++) {
            const int32_t y = rg_succ(g, m[i], e);
            if (y < 0) continue;
            if ((uint32_t)y == H) {
                into_h++;
                if (kind != DC_RG_WHILE && kind != DC_RG_LOOP && !self) {
                    self = true;
                    if (no < 2) out[no++] = (int32_t)R;
                }
                continue;
            }
            bool inside = false;
            for (int j = 0; j < n; j++) inside |= (uint32_t)y == m[j];
            if (inside) continue;
            bool dup = false;
            for (int k = 0; k < no; k++) dup |= out[k] == y;
            if (!dup) {
                if (no < 2) out[no++] = y;
            } else {
                g.npred[y]--;   /* two edges from the members become one from R */
            }
        }
    g.succ[2 * R] = out[0];
    g.succ[2 * R + 1] = out[1];
    g.npred[R] = g.npred[H] - into_h + (self ? 1u : 0u);
    g.fwd[R] = R;
    g.mark[R] = 0;
    for (int i = 0; i < n; i++) g.fwd[m[i]] = R;
    if (g.entry == H) g.entry = R;
    return R;
}

__device__ __forceinline__ uint64_t st_item(uint32_t j, const dc_merge_t &M) {
    uint64_t v = ((uint64_t)M.kind << 56) ^ ((uint64_t)M.n << 48) ^ M.region;
    for (int k = 0; k < 4; k++) v = mix64(v + M.member[k] + 0x9E3779B97F4A7C15ull * (uint64_t)(k + 1));
    return mix64(mix64(0x5354ull * 0x9E3779B97F4A7C15ull + j) ^ v);
}

/* the search on one kernel's regions at g (in LDS or global memory: each
 * copy uses the memory instructions of its own address space) */
__device__ __forceinline__ void struct_body(const Plan &P, const StructPlan &S, uint32_t k, uint32_t nb, uint32_t fb,
                                            uint32_t cap, dc_merge_t *out, dc_struct_result_t res, Rg g) {
    const uint32_t l = lane_id();
    for (uint32_t r = l; r < cap; r += 64) {
        g.succ[2 * r] = g.succ[2 * r + 1] = -1;
        g.npred[r] = 0;
        g.fwd[r] = r;
        g.mark[r] = 0;
    }
    __syncthreads();
    /* the reachable blocks and their edges (every lane the same steps) */
    uint32_t n_alive = 0;
    for (uint32_t b = 0; b < nb; b++) {
        if (P.rpo_pos[fb + b] < 0) continue;
        n_alive++;
        for (int e = 0; e < 2; e++) {
            const int32_t y = P.succ[2 * (fb + b) + e];
            g.succ[2 * b + e] = y;
            if (y >= 0) g.npred[y]++;
        }
    }
    g.npred[0]++;   /* the start */
    g.entry = 0;
    g.next = nb;
    uint32_t nm = 0, round = 0;
    uint64_t h = 0;
    while (n_alive > 1) {
        round++;
        uint32_t sp = 0, m[4] = {0, 0, 0, 0};
        int n = 0, kind = 0;
        g.stack[sp++] = g.entry;
        while (sp) {
            const uint32_t x = g.stack[--sp];
            if (g.mark[x] == round) continue;
            g.mark[x] = round;
            kind = rg_match(g, x, m, &n);
            if (kind) break;
            for (int e = 1; e >= 0; e--) {
                const int32_t y = rg_succ(g, x, e);
                if (y >= 0 && g.mark[y] != round) g.stack[sp++] = (uint32_t)y;
            }
        }
        if (!kind) break;
        const uint32_t r = rg_merge(g, m, n, kind);
        dc_merge_t M;
        M.region = r;
        M.kind = (uint8_t)kind;
        M.n = (uint8_t)n;
        M.pad = 0;
        for (int j = 0; j < 4; j++) M.member[j] = j < n ? m[j] : SR_NONE;
        out[nm] = M;
        h += st_item(nm, M);
        nm++;
        n_alive -= (uint32_t)n - 1;
    }
    res.n_blocks = nb;
    res.n_merges = nm;
    res.n_left = n_alive;
    res.root = n_alive == 1 ? g.entry : SR_NONE;
    res.digest = h;
    S.res[k] = res;
}

__global__ __launch_bounds__(64) void k_struct(Plan P, StructPlan S) {
    __shared__ int32_t l_succ[2 * SR_LDS];
    __shared__ uint32_t l_npred[SR_LDS], l_fwd[SR_LDS], l_mark[SR_LDS], l_stack[2 * SR_LDS];
    const uint32_t k = blockIdx.x, l = lane_id();
    const int32_t st = P.status[k];
    dc_struct_result_t res = {st, 0, 0, 0, SR_NONE, 0, 0};
    if (st != DC_OK) {
        S.res[k] = res;
        return;
    }
    const uint32_t nb = P.n_blocks[k], fb = P.first_block[k];
    /* ids: blocks, then one per merge -- at most nb - 1 merges that join
     * regions and one loop merge per edge to itself (one per block at the
     * start, one per joining merge) */
    const uint32_t cap = 4 * nb + 2;
    const uint64_t base = 4ull * fb + 2ull * k;
    const bool lds = cap <= SR_LDS;
    dc_merge_t *out = S.merges + base;
    Rg g;
    if (lds) {   /* uniform */
        g.succ = l_succ;
        g.npred = l_npred;
        g.fwd = l_fwd;
        g.mark = l_mark;
        g.stack = l_stack;
        struct_body(P, S, k, nb, fb, cap, out, res, g);
    } else {
        g.succ = S.succ + 2 * base;
        g.npred = S.npred + base;
        g.fwd = S.fwd + base;
        g.mark = S.mark + base;
        g.stack = S.stack + 2 * base;
        struct_body(P, S, k, nb, fb, cap, out, res, g);
    }
}

hipError_t launch_struct(const Plan &P, const StructPlan &S, hipStream_t s) {
    if (!P.n_kernels) return hipSuccess;
    hipLaunchKernelGGL(k_struct, dim3(P.n_kernels), dim3(64), 0, s, P, S);
    return hipGetLastError();
}

}  // namespace dc

/* dc_internal.h -- device buffers and stage launchers shared by the HIP
 * kernels (dc_kernels.hip) and the host API (dc_api.cpp). */
#pragma once
#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "dc.h"

namespace dc {

constexpr int NSLOT = DC_NSLOT;
constexpr int N_OPS = 77;

/* Device-side view of one planned batch.  Positions are this batch's own
 * dense numbering of instructions: kernel k owns [pos_begin[k], pos_begin[k+1]).
 * Arrays are indexed by position (sized n_pos), by global block (sized by
 * blk_cap, the block count the plan was made for) or by record capacity. */
struct Plan {
    /* inputs (device) */
    const dc_instr_t *instrs;
    const dc_kernel_t *kernels;
    const dc_arg_t *args;
    const uint32_t *pos_begin;      /* K + 1 */
    const int32_t *desc_status;     /* K: descriptor check done on the host */
    const uint32_t *work_order;     /* K: the order in which the fixpoint takes kernels (longest first); null =
                                       index order */
    uint32_t n_kernels;
    uint32_t n_pos;                 /* total instructions */
    uint64_t n_records;
    uint64_t n_args;

    /* per position */
    uint8_t *leader;                /* n_pos: leader flag */
    uint8_t *pcap;                  /* n_pos: record capacity of the instruction: bit 0 one access record,
                                       bits 3:1 built-in records (explicit definition dwords of a rule that can
                                       yield a built-in) */
    uint32_t *block_id;             /* n_pos: global block id of each position */
    uint32_t *totals;               /* [0] blocks, [1] access capacity, [2] built-in capacity of the batch */
    uint32_t *kslots;               /* KSLOT_WORDS per kernel: bit s = some record names register slot s (null for
                                       graph-only plans) */
    uint32_t with_records;          /* an analysis plan (not graph-only): capacities, regions, fixpoint */
    /* per global block (blk_cap entries, +1 where noted) */
    uint32_t blk_cap;
    uint32_t *block_start;          /* +1: first position of each global block; [total] = n_pos */
    uint32_t *block_kernel;
    int32_t *succ;                  /* 2 per block: local ids */
    uint32_t *pred_cnt;             /* +1 (count, then exclusive offsets) */
    uint32_t *pred_fill;
    uint32_t *pred;                 /* 2 per block: local ids */
    uint32_t *rpo;                  /* local ids, per kernel at first_block */
    int32_t *rpo_pos;               /* position of each block in its kernel's RPO, -1 unreachable */
    uint32_t *dfs_stack;
    uint8_t *dfs_seen;
    uint32_t *blk_acc_base;         /* +1: first access-record slot of the block's region (exclusive scan of the
                                       access capacity of its instructions); [total] = access capacity */
    uint32_t *blk_sys_base;         /* +1: the same for built-in records */
    uint32_t *kbad;                 /* K: first bad record, (index << 2) | code */
    int32_t *status;                /* K */
    uint32_t *first_block;          /* K */
    uint32_t *n_blocks;             /* K */
    uint32_t *n_reach;              /* K */
    uint4 *binfo;                   /* 2 per block, per kernel at first_block, by RPO position: {local id, first
                                       position, end position, 0}, {RPO position of successor 0, of successor 1,
                                       chained successor (0, 1; 2 = none), 0} (-1 when absent); null for
                                       CFG-only batches */

    /* fixpoint + extraction */
    uint32_t *arena;                /* per main-pass wave: arena_rows state rows of 192 dwords */
    uint32_t arena_rows;
    uint32_t main_waves;
    uint32_t *ovf_arena;            /* per overflow wave: ovf_rows state rows */
    uint32_t ovf_rows;
    uint32_t *ovf_bitmaps;          /* per overflow wave: 2 * ceil(ovf_block_cap / 32) + 64 words */
    uint32_t ovf_block_cap;
    uint32_t ovf_waves;
    uint32_t *ovf_list;             /* K */
    uint4 *dummy;                   /* (main_waves + ovf_waves) * 64: per-lane scratch stores */
    uint32_t *counters;             /* [0] work counter, [1] overflow count, [2] overflow work counter; plain form:
                                       [4], [5] records written so far (8 words) */
    uint32_t sweep_cap;
    uint32_t flags;
    uint32_t acc_cap, sys_cap;      /* record slots allocated (acc_sparse/acc_dense, sys_sparse/sys_dense) */
    dc_access_t *acc_sparse;        /* acc_cap: a block's records in its region */
    dc_sysval_t *sys_sparse;        /* sys_cap */
    uint32_t *blk_acc;              /* per block: access records of the last visit */
    uint32_t *blk_sys;              /* per block: built-in records of the last visit */
    dc_kernel_result_t *results;    /* K */
    dc_reg_state_t *export_states;  /* total_blocks * NSLOT (DC_OPT_EXPORT_STATES) */
    uint8_t *export_reached;        /* total_blocks */

    /* compaction */
    uint32_t *blk_acc_off;          /* per block: exclusive scan of blk_acc over the blocks */
    uint32_t *blk_sys_off;          /* per block */
    uint32_t *acc_count;            /* K + 1 -> exclusive offsets */
    uint32_t *sys_count;            /* K + 1 */
    dc_access_t *acc_dense;         /* acc_cap */
    dc_sysval_t *sys_dense;         /* sys_cap */

    /* scan scratch */
    uint32_t *scan_tmp;             /* scan_tmp_words */
    uint64_t scan_tmp_words;
};

/* launch configuration of the fixpoint kernel */
struct FixCfg {
    int waves_per_group;
    int groups;
};

/* stage launchers (enqueue only; return hipSuccess or the launch error) */
hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s);
hipError_t launch_fill_u8(uint8_t *p, uint64_t n, uint8_t v, hipStream_t s);
hipError_t launch_decode(const Plan &P, hipStream_t s);                 /* decode, checks, leaders, capacities */
hipError_t launch_leader_scan(const Plan &P, hipStream_t s);            /* block count, record capacities (totals) */
hipError_t launch_number_blocks(const Plan &P, hipStream_t s);          /* block numbering, record regions */
hipError_t launch_edges(const Plan &P, hipStream_t s);                  /* edges, predecessors, RPO, statuses */
/* entry state, fixpoint, extraction; dP = device copy of P; optional events bracket the main launch */
hipError_t launch_fixpoint(const Plan &P, const Plan *dP, const FixCfg &c, hipStream_t s, hipEvent_t before,
                           hipEvent_t after);
hipError_t launch_compact(const Plan &P, hipStream_t s);                /* dense outputs */
/* the plain form: one launch per kernel (dc_plain.hip); events bracket the launches */
hipError_t launch_plain(const Plan &P, const Plan *dP, hipStream_t s, hipEvent_t before, hipEvent_t after);
uint32_t fixpoint_groups_per_cu(uint32_t waves_per_group);              /* resident fixpoint groups per CU */
size_t fixpoint_lds_per_wave();                                         /* LDS bytes per fixpoint wavefront */
constexpr uint32_t KSLOT_WORDS = 12;                                    /* 384 bits >= NSLOT */
constexpr uint32_t FIX_ROW_DWORDS = 192;                                /* arena dwords per state row */
constexpr uint32_t FIX_MAX_ROWS = 6;                                    /* state rows of the largest kernel */
constexpr uint32_t OVF_MAX_WAVES = 512;                                 /* waves of the overflow pass */
constexpr uint64_t ARENA_BUDGET = 8ull << 30;                           /* arena bytes of either pass */
uint64_t scan_tmp_words_needed(uint64_t n);
uint64_t cap_scan_words(uint64_t n);     /* extra scan words of the capacity scan of n positions */
void *noalloc_setup(int device);         /* device address of the no-allocation scratch array (current device) */

/* Device arrays of a register-version run (dc_ssa.hip) over a plan's graph.
 * Per-kernel counts and their offsets come in four arrays: 0 table words
 * (blocks x named slots), 1 merges, 2 merge arguments, 3 operand versions. */
struct SsaPlan {
    uint32_t *idom;                 /* per global block: immediate dominator (local id), block 0 -> 0,
                                       unreachable -> DC_SSA_NONE */
    uint32_t *scr;                  /* 3 per global block: preorder scratch of kernels whose graph is not in LDS */
    uint32_t *counts;               /* SSA_ARRAYS x K */
    uint64_t *offs;                 /* SSA_ARRAYS x (K + 1): exclusive scans of counts */
    int32_t *status;                /* K */
    uint32_t *tab_a;                /* per (block, slot): first version in the block | merge flag << 31 */
    uint32_t *tab_b;                /* per (block, slot): version live at the block's end */
    uint64_t tab_cap;
    dc_phi_t *phis;                 /* ascending (block, slot) per kernel */
    uint64_t phi_cap;
    uint32_t *phi_args;
    uint64_t arg_cap;
    uint32_t *vers;                 /* per instruction its use versions, then its definition versions */
    uint64_t ops_cap;
    uint8_t *opn;                   /* per position: uses | definitions << 4 */
    dc_ssa_result_t *res;           /* K */
    uint32_t digest;                /* compute the per-kernel digest */
    /* variables and types (null without them) */
    uint32_t *nver;                 /* per (kernel, register column): versions, version 0 included */
    uint64_t col_cap;
    uint32_t *aoff;                 /* per merge: its first argument, relative to the kernel's arguments */
    uint32_t *tscr;                 /* 3 per node of the kernels with more than TY_LDS_NODES nodes: variable and
                                       type-class parents, flags | type bits */
    uint64_t scr_cap;
    dc_var_t *vars;                 /* per node */
    uint64_t node_cap;
    dc_types_result_t *tres;        /* K */
};
/* count arrays of the version and type stages: table words, merges, merge
 * arguments, operands, register columns, nodes, nodes of kernels whose
 * nodes do not fit the type stage's LDS */
constexpr uint32_t SSA_ARRAYS = 7;
constexpr uint32_t TY_LDS_NODES = 2048;
/* Device arrays of a text front end run (dc_text.hip).  Sizes come from the
 * counts of the first run on a text (line ends, .kernel lines, then per
 * kernel instructions, label-table slots and user arguments). */
struct TextPlan {
    const uint8_t *text;            /* the listing (caller's device memory) */
    uint64_t n_bytes;
    uint32_t n_tiles;               /* 4 KiB tiles of text */
    uint32_t *tile_cnt;             /* n_tiles: line ends per tile */
    uint64_t *tile_off;             /* n_tiles + 1 */
    uint64_t n_lines;               /* line ends + 1 */
    uint64_t *line_start;           /* n_lines + 1 ([n_lines] = n_bytes + 1) */
    uint8_t *kind;                  /* n_lines */
    uint32_t n_ltiles;              /* tiles of 4096 lines */
    uint32_t *ltile_cnt;            /* .kernel lines per line tile */
    uint64_t *ltile_off;            /* n_ltiles + 1 */
    uint32_t n_kernels, k_cap;
    uint64_t *kline;                /* k_cap + 1: line of each .kernel; [K] = n_lines */
    uint32_t *kcounts;              /* 3 x K: instructions, label-table slots, user arguments */
    uint64_t *koffs;                /* 3 x (K + 1): exclusive scans of kcounts */
    unsigned long long *lab_key;    /* lab_cap: hash of the label name (0 = empty) */
    uint32_t *lab_idx;              /* lab_cap: instruction index the label names */
    uint32_t *lab_line;             /* lab_cap: its line, relative to the kernel's first line */
    uint64_t lab_cap;
    dc_kernel_t *kernels;           /* k_cap */
    uint64_t *name_off;             /* k_cap: byte offset of the kernel's name in the text */
    uint32_t *name_len;             /* k_cap */
    dc_instr_t *instrs;
    uint64_t instr_cap;
    dc_arg_t *args;
    uint64_t arg_cap;
    uint32_t *fail;                 /* set when the text does not fit the plan */
};
hipError_t launch_text_lines(const TextPlan &T, hipStream_t s);      /* line ends per tile, their scan */
hipError_t launch_text_classify(const TextPlan &T, hipStream_t s);   /* line starts, kinds, .kernel counts */
hipError_t launch_text_kernels1(const TextPlan &T, hipStream_t s);   /* kernel starts, per-kernel counts, scans */
hipError_t launch_text_kernels2(const TextPlan &T, hipStream_t s);   /* labels, configuration, records */

/* Device arrays of a structuring run (dc_struct.hip): kernel k's regions
 * are ids 0 .. 4 n_blocks + 1 at 4 first_block + 2 k of each array. */
struct StructPlan {
    int32_t *succ;                  /* 2 per region */
    uint32_t *npred, *fwd, *mark;
    uint32_t *stack;                /* 2 per region */
    dc_merge_t *merges;             /* per region slot: the kernel's merges in order */
    dc_struct_result_t *res;        /* K */
};
hipError_t launch_struct(const Plan &P, const StructPlan &S, hipStream_t s);

hipError_t launch_ssa_size(const Plan &P, const SsaPlan &S, hipStream_t s);    /* table sizes and offsets */
hipError_t launch_ssa_graph(const Plan &P, const SsaPlan &S, hipStream_t s);   /* dominators, merges, numbering */
hipError_t launch_ssa_emit(const Plan &P, const SsaPlan &S, hipStream_t s);    /* merges, arguments, versions */
hipError_t launch_types(const Plan &P, const SsaPlan &S, hipStream_t s);       /* variables and types */

}  // namespace dc

/*
 * dc.h -- C ABI of libdc, the MI355X engine for the register-state dataflow
 * analysis of GCN kernels (Mihajlenko, Lukin & Stankevich, "A method for
 * decompilation of AMD GCN kernels to OpenCL").
 *
 * The engine runs the part of the paper's method that its Section
 * "Statement of the problem" lists as steps 2 and 3 -- register and
 * kernel-parameter initialisation from the ABI, then instruction processing
 * that builds the control flow graph and determines what each register holds
 * -- together with the searches of Sections "Search for memory accesses"
 * (array accesses and work-item built-ins such as get_global_id) and "Data
 * type recovery" (types from .arg lines and from instruction suffixes).
 * Input is pre-tokenized: one 16-byte record per instruction (the text front
 * end of Section "The body extraction" is not part of this library).
 *
 * Conventions for every function:
 *   - the return value is a dc_status_t: DC_OK (0) or a negative code; no
 *     function aborts or throws;
 *   - pointers documented as "device" must be HIP device memory of the
 *     context's device (for example a torch tensor's data_ptr()); all others
 *     are host memory;
 *   - the caller owns every input buffer and must keep device inputs alive
 *     and unchanged until dc_batch_wait / dc_cfg_view returns;
 *   - the library owns dc_cfg_t / dc_batch_t and their results until the
 *     matching *_free call;
 *   - `stream` is a hipStream_t (NULL = the default stream); work is enqueued
 *     asynchronously on it.
 * Per-kernel problems (bad records, unsupported descriptors, no fixpoint
 * within the sweep cap) are reported per kernel and never fail the batch;
 * call-level errors (DC_E_INVAL, DC_E_HIP, DC_E_OOM) fail the call.
 */
#ifndef DC_H
#define DC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dc_status_t;
#define DC_OK 0
#define DC_E_INVAL (-1)        /* null pointer, size out of range, bad option */
#define DC_E_HIP (-2)          /* a HIP runtime call failed (no device, launch error) */
#define DC_E_OOM (-3)          /* device or host allocation failed */
#define DC_E_NOTREADY (-4)     /* result asked for before it exists (e.g. states not exported) */
#define DC_E_BADOP (-10)       /* per kernel: opcode id outside the instruction subset */
#define DC_E_BADREG (-11)      /* per kernel: operand id invalid for its role, width or alignment */
#define DC_E_BADTARGET (-12)   /* per kernel: branch target outside the kernel, or target on a non-branch */
#define DC_E_NOEND (-13)       /* per kernel: control can fall off the end (last record not s_endpgm/s_branch) */
#define DC_E_UNSUPPORTED (-14) /* per kernel: descriptor outside the described ABI (useargs=0, dims, cws, args) */
#define DC_E_NOFIX (-15)       /* per kernel: no fixpoint within the sweep cap */
#define DC_E_CAPACITY (-16)    /* per kernel: the records have more blocks or records than the batch was planned
                                  for (they changed in place after planning); analyse them in a new batch */

#define DC_NSLOT 368           /* s0..s103, vcc, exec, scc, m0, 2 reserved, v0..v255 */

/* One instruction (16 bytes, little endian).  Operand ids: 0..103 s0..s103,
 * 104/105 vcc_lo/hi, 106/107 exec_lo/hi, 108 scc, 109 m0, 112..367 v0..v255,
 * 0x8000+k inline integer k-16 (k <= 80), 0x8060..0x8067 inline floats
 * +-0.5, +-1, +-2, +-4, 0xFFFE a literal held in imm, 0xFFFF none.  A
 * multi-dword operand names its first register.  imm holds a byte offset for
 * memory instructions and the third source's operand id for three-source ops.
 * target is the branch target as an instruction index within the kernel, -1
 * for non-branches.  The opcode numbering is dc_opcode_name(). */
typedef struct { uint16_t op, r0, r1, r2; int32_t imm; int32_t target; } dc_instr_t;

/* One kernel (32 bytes): its records are instrs[instr_begin .. +n_instr),
 * its user arguments args[arg_begin .. +n_args).  dims, cws and useargs are
 * the .dims, .cws and .useargs entries of the kernel's .config section
 * (Listing 1 and Listing 3 of the paper). */
typedef struct {
    uint64_t instr_begin; uint32_t n_instr; uint8_t dims, useargs; uint16_t n_args;
    uint32_t cws[3]; uint32_t arg_begin;
} dc_kernel_t;

/* One user kernel argument (.arg line of Listing 3): byte offset in the
 * argument area addressed by s[4:5] (user arguments follow the six hidden
 * 8-byte slots, so they start at 0x30), size in bytes (4 or 8), type as a
 * type-tier bit set (DC_TY_*), flags = pointee type bits for pointers. */
typedef struct { uint32_t offset; uint16_t size; uint8_t type, flags; } dc_arg_t;

#define DC_TY_INT 1
#define DC_TY_UINT 2
#define DC_TY_FLOAT 4
#define DC_TY_DOUBLE 8
#define DC_TY_PTR 16

/* Abstract value of one register slot (16 bytes): provenance bits (where
 * the value came from: local, group and global-offset ids per dimension,
 * sizes, the argument pointer, constants, loads, kernel arguments), type
 * bits (DC_TY_*), and the payload: bits 63:60 tag, 59:58 dword of a 64-bit
 * value, 57:56 dimension, 55:52 id-term mask or built-in kind, 51:48 shift,
 * 47:40 argument slot, 31:0 constant; all ones = unknown (TOP). */
typedef struct { uint32_t prov; uint8_t type, flags, pad0, pad1; uint64_t val; } dc_reg_state_t;

/* A memory access (16 bytes): instruction index, kind (0 load, 1 store),
 * space (0 global, 1 flat, 2 LDS), width in bytes, data type bits, address
 * payload (TOP = 0xFFFFFFFFFFFFFFFF when unresolved). */
typedef struct { uint32_t instr; uint8_t kind, space, width, dtype; uint64_t addr; } dc_access_t;

/* A recognised work-item built-in (8 bytes): instruction index, register
 * slot that holds it after the instruction, kind (DC_SV_*), dimension. */
typedef struct { uint32_t instr; uint16_t slot; uint8_t kind, dim; } dc_sysval_t;

#define DC_SV_GLOBAL_ID 0
#define DC_SV_GLOBAL_ID_MINUS_OFFSET 1
#define DC_SV_GLOBAL_OFFSET 2
#define DC_SV_GLOBAL_SIZE 3
#define DC_SV_NUM_GROUPS 4
#define DC_SV_WORK_DIM 5
#define DC_SV_GROUP_BASE 6
#define DC_SV_LOCAL_ID 7
#define DC_SV_GROUP_ID 8

/* Per-kernel result summary (32 bytes).  For a failed kernel everything but
 * status is zero.  digest is filled only with DC_OPT_DIGEST. */
typedef struct {
    int32_t status; uint32_t n_blocks, sweeps, n_access, n_sysval, pad; uint64_t digest;
} dc_kernel_result_t;

/* Options.  flags: */
#define DC_OPT_EXPORT_STATES 1u  /* keep every block's fixpoint IN state for dc_get_block_state */
#define DC_OPT_DIGEST 2u         /* compute the per-kernel digest of the fixpoint states */
#define DC_OPT_TIMING 4u         /* record HIP events around the stages (dc_get_stats ms_*) */
#define DC_OPT_GRAPH 8u          /* dc_batch_run replays the stages as one captured HIP graph (from the second run
                                    on; not with DC_OPT_EXPORT_STATES or DC_OPT_TIMING, nor on the NULL stream,
                                    where runs stay eager) */
#define DC_OPT_LONGEST_FIRST 16u /* the fixpoint takes kernels longest first instead of in index order */
#define DC_OPT_PLAIN 32u         /* the plain form: one launch per kernel, one workgroup doing every stage of that
                                    kernel (the comparison point of the batched form; not with DC_OPT_EXPORT_STATES
                                    or DC_OPT_GRAPH) */
typedef struct {
    uint32_t flags;
    uint32_t sweep_cap;          /* 0 = 64 + 2 * n_blocks per kernel */
    uint32_t waves_per_group;    /* fixpoint kernel: waves per workgroup, at most 4 and within the device's LDS
                                    per workgroup (0 = the most that fit, up to 4) */
    uint32_t groups_per_cu;      /* fixpoint kernel: resident workgroups per CU in the persistent grid (0 = auto) */
    uint32_t block_cap;          /* blocks (of two state rows) a kernel may have in the main pass; larger go to the
                                    overflow pass.  0 = sized on the first run to the largest kernel of at most 2048
                                    blocks, within 8 GB and a quarter of the free device memory */
    uint32_t reserved[3];
} dc_options_t;

typedef struct {
    uint64_t n_kernels, n_instr, n_blocks, n_unreached, sweeps_sum, n_access, n_sysval, bytes_alg;
    uint32_t sweeps_max, n_failed, n_overflow, pad;
    float ms_total, ms_decode, ms_cfg, ms_fixpoint, ms_compact, ms_pad;
} dc_stats_t;

typedef struct {
    int32_t status;
    uint32_t n_blocks, n_reach, n_pred;
    const uint32_t *block_start;   /* n_blocks + 1 instruction indices */
    const int32_t *succ;           /* 2 per block: fall-through, taken (-1 = none) */
    const uint32_t *pred_off;      /* n_blocks + 1 */
    const uint32_t *pred;          /* predecessors per block, ascending */
    const uint32_t *rpo;           /* reachable blocks in reverse postorder (DFS from block 0, fall-through first) */
} dc_cfg_view_t;

typedef struct dc_ctx dc_ctx_t;
typedef struct dc_cfg dc_cfg_t;
typedef struct dc_batch dc_batch_t;

/* Context on one HIP device.  Fails with DC_E_HIP when the device is absent. */
dc_status_t dc_ctx_create(int hip_device, dc_ctx_t **out);
void dc_ctx_destroy(dc_ctx_t *ctx);

/* The graph part only (decode and validate, leaders, block numbering, edges,
 * predecessor CSR, reverse postorder) for n_kernels kernels whose records
 * are in `instrs` (device, n_records entries).  Section "Search for control
 * structures": the control flow graph is built first.  Synchronous w.r.t.
 * the returned object: dc_cfg_view waits for the stream. */
dc_status_t dc_build_cfg(dc_ctx_t *ctx, const dc_kernel_t *kernels, uint32_t n_kernels, const dc_instr_t *instrs,
                         uint64_t n_records, void *stream, dc_cfg_t **out);
/* Host view of kernel k's graph; the arrays stay valid until dc_cfg_free. */
dc_status_t dc_cfg_view(dc_cfg_t *cfg, uint32_t k, dc_cfg_view_t *view);
void dc_cfg_free(dc_cfg_t *cfg);

/* The whole analysis for a batch: steps 2 and 3 of Section "Statement of
 * the problem" (registers and kernel parameters initialised from the ABI,
 * then instruction processing that builds the control flow graph and
 * determines what every register holds) solved to the least fixpoint over
 * the graph, with the searches of Section "Search for memory accesses"
 * (array accesses, work-item built-ins) and the types of Section "Data type
 * recovery" (.arg lines of Listing 3, instruction suffixes).
 * kernels (n_kernels descriptors) and args (n_args_total entries) are host
 * arrays, copied before return; instrs is device memory holding n_records
 * records, which must stay alive and unchanged until the batch is freed.
 * opts may be NULL (defaults).  Plans the batch (allocates its device
 * memory), enqueues the first run on `stream` and returns; the first run
 * synchronises the stream once, after the graph stage, to size the
 * block-indexed arrays and the fixpoint arenas from the real block counts.
 * Results are ready after dc_batch_wait.  Errors: DC_E_INVAL (null pointer,
 * a descriptor's records or arguments outside the arrays, more than 2^32-16
 * instructions), DC_E_OOM, DC_E_HIP; per-kernel problems are per-kernel
 * statuses. */
dc_status_t dc_analyze_batch(dc_ctx_t *ctx, const dc_kernel_t *kernels, uint32_t n_kernels, const dc_instr_t *instrs,
                             uint64_t n_records, const dc_arg_t *args, uint64_t n_args_total,
                             const dc_options_t *opts, void *stream, dc_batch_t **out);
/* Autotuner for the fixpoint's launch.  Times whole runs of a sample of the
 * batch (every stride-th kernel, at most `sample` kernels; 0 = 8192) under
 * each launch shape -- waves per workgroup 1, 2 and the most that fit, each
 * with the most resident groups per CU and three quarters of that -- in both
 * kernel orders (index order, DC_OPT_LONGEST_FIRST), and writes the fastest
 * into *best (the other fields are copied from base, which may be NULL) and
 * its time per run of the sample into *best_ms.  The choice is cached per
 * device size (CUs), batch size bucket (log2 of the mean kernel length and of
 * the kernel count) and the DIGEST/EXPORT flags of base, in the process and,
 * when the environment names a file in DC_TUNE_CACHE, in that file; a cached
 * choice is returned without timing.  Synchronous; allocates and frees its
 * own trial batches. */
dc_status_t dc_autotune(dc_ctx_t *ctx, const dc_kernel_t *kernels, uint32_t n_kernels, const dc_instr_t *instrs,
                        uint64_t n_records, const dc_arg_t *args, uint64_t n_args_total, const dc_options_t *base,
                        uint32_t sample, void *stream, dc_options_t *best, float *best_ms);
/* Run the same batch again on `instrs` (device; the same descriptors and
 * layout; NULL = the previous pointer).  Results are overwritten.  On the
 * planned records it allocates nothing and does not synchronise.  A new
 * pointer holds other records, whose block counts and record capacities may
 * differ: the run then plans the batch again for them (it synchronises the
 * stream and may allocate), as its first run did.  Records changed in place
 * after planning are the caller's error: kernels whose records no longer fit
 * the plan report DC_E_CAPACITY. */
dc_status_t dc_batch_run(dc_batch_t *batch, const dc_instr_t *instrs, void *stream);
dc_status_t dc_batch_wait(dc_batch_t *batch);

dc_status_t dc_get_kernel_status(const dc_batch_t *batch, uint32_t k, dc_status_t *st);
dc_status_t dc_get_kernel_result(const dc_batch_t *batch, uint32_t k, dc_kernel_result_t *out);
/* All n_kernels summaries into out[cap]. */
dc_status_t dc_get_results(const dc_batch_t *batch, dc_kernel_result_t *out, uint32_t cap);
/* Memory accesses of kernel k (Section "Search for memory accesses": array
 * element accesses recognised from the address arithmetic), one record per
 * reachable global/flat/LDS instruction in instruction order, the address
 * resolved from the fixpoint state before it.  Two-call idiom: always sets
 * *n_total, copies min(cap, n_total) records into buf (host).  Waits for the
 * batch.  DC_E_INVAL for k out of range or a null n_total (or a null buf
 * with cap > 0).  A failed kernel has no records. */
dc_status_t dc_get_accesses(const dc_batch_t *batch, uint32_t k, dc_access_t *buf, uint32_t cap, uint32_t *n_total);
/* Work-item built-ins of kernel k (Section "Search for memory accesses":
 * get_global_id and its idx0 form, get_global_offset, get_global_size,
 * get_num_groups, get_work_dim, get_local_id, get_group_id and the
 * group-id-times-size term), one record per register definition whose value
 * is one of them, ordered by (instruction, register).  Same conventions as
 * dc_get_accesses. */
dc_status_t dc_get_sysvals(const dc_batch_t *batch, uint32_t k, dc_sysval_t *buf, uint32_t cap, uint32_t *n_total);
/* Every kernel's records packed in kernel order; offsets (n_kernels + 1
 * entries, may be NULL) give each kernel's range. */
dc_status_t dc_get_all_accesses(const dc_batch_t *batch, dc_access_t *buf, uint64_t cap, uint64_t *n_total,
                                uint64_t *offsets);
dc_status_t dc_get_all_sysvals(const dc_batch_t *batch, dc_sysval_t *buf, uint64_t cap, uint64_t *n_total,
                               uint64_t *offsets);
/* Fixpoint IN state of one block: for each of the 368 register slots the
 * paper's Register record (Section "Search for memory accesses": type and
 * integrity, here with the value's provenance and payload) and its type bits
 * (Section "Data type recovery").  out368 (host) receives DC_NSLOT entries;
 * *reached (may be NULL) = 1 when the block is reachable (an unreachable
 * block's state is all zero).  Needs DC_OPT_EXPORT_STATES (else
 * DC_E_NOTREADY); DC_E_INVAL for k or block out of range or a failed
 * kernel. */
dc_status_t dc_get_block_state(const dc_batch_t *batch, uint32_t k, uint32_t block, dc_reg_state_t *out368,
                               uint8_t *reached);
dc_status_t dc_get_stats(const dc_batch_t *batch, dc_stats_t *out);

/* Stage times summed over the runs enqueued since the last reset (at most
 * the last 64), from HIP events recorded on the batch's stream (needs
 * DC_OPT_TIMING).  ms_fixpoint brackets exactly the fixpoint's two launches
 * (the main pass and the overflow pass, which returns at once when no kernel
 * was deferred to it); with DC_OPT_PLAIN it brackets the per-kernel
 * launches.  Waits for the stream. */
typedef struct { uint32_t runs, pad; float ms_total, ms_decode, ms_cfg, ms_fixpoint, ms_compact, ms_pad; } dc_timing_t;
dc_status_t dc_get_timing(const dc_batch_t *batch, dc_timing_t *out);
dc_status_t dc_timing_reset(dc_batch_t *batch);
void dc_batch_free(dc_batch_t *batch);

/* ------------------------------------------------------------------ */
/* The analysis without device allocation.                              */
/* ------------------------------------------------------------------ */
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * analysis as dc_analyze_batch, with every intermediate array in a static
 * device array of the library of DC_NOALLOC_SCRATCH_BYTES per device
 * (reserved when the library's code loads on a device and held until the
 * process ends), and the results in the caller's device buffers.  The call
 * calls no hipMalloc, hipFree or other allocating routine and does not
 * synchronise: it enqueues on `stream` and returns.
 *
 * Inputs (all device memory): kernels (n_kernels descriptors, records
 * relative to instrs, arguments relative to args), instrs (n_records),
 * args (n_args_total).  n_instr_total must be the sum of the descriptors'
 * n_instr.  flags: 0 or DC_OPT_DIGEST.
 * Outputs (device memory, written when the stream reaches the work):
 * results[n_kernels]; accesses[acc_cap] and sysvals[sys_cap], every
 * kernel's records packed in kernel order; acc_off / sys_off (n_kernels + 1
 * entries): exclusive offsets of each kernel's records.
 * Limits: n_kernels <= DC_NOALLOC_MAX_KERNELS and n_instr_total <=
 * DC_NOALLOC_MAX_INSTR, else DC_E_INVAL (before anything is enqueued).
 * Per kernel: a kernel with more than 2048 blocks, or too many blocks for
 * the fixed state arenas (256 blocks of up to 128 named registers or 85 of
 * more in the main pass; 1024 blocks in the overflow pass), fails with
 * DC_E_CAPACITY, and so does every kernel when the records or built-ins
 * outgrow acc_cap or sys_cap (acc_cap = n_instr_total and
 * sys_cap = 4 * n_instr_total always suffice); a descriptor whose records or
 * arguments lie outside the arrays fails with DC_E_INVAL; when n_instr_total
 * differs from the descriptors' sum every kernel fails with DC_E_INVAL.
 * Every call on a device shares that device's scratch array: calls that
 * overlap on one device (other streams, other threads) race and must be
 * serialised by the caller; calls on one stream are ordered. */
#define DC_NOALLOC_MAX_KERNELS 4096u
#define DC_NOALLOC_MAX_INSTR 262144u
#define DC_NOALLOC_SCRATCH_BYTES (96ull << 20)
dc_status_t dc_analyze_noalloc(dc_ctx_t *ctx, const dc_kernel_t *kernels, uint32_t n_kernels, uint32_t n_instr_total,
                               const dc_instr_t *instrs, uint64_t n_records, const dc_arg_t *args,
                               uint64_t n_args_total, uint32_t flags, dc_kernel_result_t *results,
                               dc_access_t *accesses, uint32_t acc_cap, uint32_t *acc_off, dc_sysval_t *sysvals,
                               uint32_t sys_cap, uint32_t *sys_off, void *stream);

/* ------------------------------------------------------------------ */
/* Text front end.                                                      */
/* ------------------------------------------------------------------ */
/* Section "The body extraction": listings in the format of the paper's
 * Listings 1-3 become kernel descriptors, records and argument tables.  The
 * paper's extraction loop is followed: a ".kernel NAME" line opens a kernel,
 * ".config" and ".text" lines switch between collecting its configuration and
 * its body; lines before the first .kernel, and between .kernel and the first
 * switch, are skipped.  The grammar (the paper fixes none):
 *   - a comment runs from "//" or ";" to the end of the line; blanks are
 *     space, tab and carriage return; lines end at '\n';
 *   - configuration: ".dims" (or "dims") x | xy | xyz -> dims 1..3 (else 0);
 *     ".cws a[, b[, c]]" (integers; a missing later size is 1; without .cws
 *     all sizes are 0); ".useargs"; ".arg name, "ctype", type[, ...]" -- args
 *     named "_." are the six hidden 8-byte slots and take no entry, user
 *     arguments are laid out from 0x30, each at the next multiple of its size
 *     (char 1, short 2, int/uint/float 4, long/ulong/double/size_t/pointers
 *     8; other types 4 bytes, no type bits), type bits from the type (signed
 *     int -> DC_TY_INT, unsigned -> DC_TY_UINT, float, double; "T*" ->
 *     DC_TY_PTR with T's bits in flags); the last .dims / .cws wins; other
 *     lines are skipped;
 *   - body: a line "NAME:" is a label naming the index of the next
 *     instruction (the first definition of a name wins); every other line is
 *     one instruction: a mnemonic (case-insensitive, dc_opcode_name) and
 *     operands separated by commas (or, with no comma, by blanks); words
 *     "key:value" without '[' are modifiers, of which "offset:N" sets imm;
 *     operands: s<n>, v<n>, s[a:b], v[a:b] (the first register), vcc(_lo/_hi),
 *     exec(_lo/_hi), scc, m0, off (none), the integers -16..64 and the floats
 *     +-0.5, +-1.0, +-2.0, +-4.0 as inline constants, other integers (decimal
 *     or 0x hex) as a literal in imm; operand order per opcode as in
 *     s_load_dword sdst, sbase, offset / v_cmp vcc, a, b / v_add_co_u32 dst,
 *     vcc, a, b / global_load dst, vaddr, saddr|off / global_store vaddr,
 *     data, saddr|off / ds_write addr, data / three-source dst, a, b, c /
 *     two-operand dst, a / dst, a, b; a branch names a label (or an index);
 *   - a malformed line still yields its record: unknown mnemonic -> op
 *     0xFFFF, an operand that is none of the above -> operand id 0xFFFD, a
 *     malformed offset -> op 0xFFFF, an unknown label -> target 0x7FFFFFFF;
 *     the analysis' record checks then fail that kernel.
 * Labels are told apart by a 64-bit hash of their names (two names of one
 * kernel with the same hash would be taken for one).
 * `text` is device memory (n_bytes, no terminator needed); the outputs stay
 * in device memory owned by the object (dc_text_device_arrays: descriptors
 * with instr_begin / arg_begin into the record and argument arrays, ready for
 * dc_analyze_batch) and are copied to the host by the getters.  opts may be
 * NULL; its flags may hold DC_OPT_TIMING only.  The first run on a text sizes
 * the arrays from its counts (three waits for the stream); dc_text_run on the
 * same pointer and size allocates nothing and does not synchronise (a text
 * changed in place to other counts makes the getters return
 * DC_E_CAPACITY), on another it sizes them again. */
typedef struct dc_text dc_text_t;
typedef struct { uint32_t n_kernels, fail; uint64_t n_lines, n_instr, n_args; } dc_text_counts_t;
dc_status_t dc_parse_text(dc_ctx_t *ctx, const char *text, uint64_t n_bytes, const dc_options_t *opts, void *stream,
                          dc_text_t **out);
dc_status_t dc_text_run(dc_text_t *t, const char *text, uint64_t n_bytes);
dc_status_t dc_text_wait(dc_text_t *t);
dc_status_t dc_text_get_counts(dc_text_t *t, dc_text_counts_t *out);
dc_status_t dc_text_device_arrays(dc_text_t *t, const dc_kernel_t **kernels, const dc_instr_t **instrs,
                                  const dc_arg_t **args);
dc_status_t dc_text_get_kernels(dc_text_t *t, dc_kernel_t *buf, uint32_t cap, uint32_t *n_total);
dc_status_t dc_text_get_records(dc_text_t *t, dc_instr_t *buf, uint64_t cap, uint64_t *n_total);
dc_status_t dc_text_get_args(dc_text_t *t, dc_arg_t *buf, uint64_t cap, uint64_t *n_total);
/* each kernel's name as a byte offset into the text and a length */
dc_status_t dc_text_get_names(dc_text_t *t, uint64_t *name_off, uint32_t *name_len, uint32_t cap, uint32_t *n_total);
/* stage times (needs DC_OPT_TIMING): ms_decode = line starts and kinds,
 * ms_cfg = per-kernel counts, ms_fixpoint = labels, configuration and
 * records, ms_compact = 0 */
dc_status_t dc_text_get_timing(dc_text_t *t, dc_timing_t *out);
dc_status_t dc_text_timing_reset(dc_text_t *t);
void dc_text_free(dc_text_t *t);

/* ------------------------------------------------------------------ */
/* Structuring (region graph).                                          */
/* ------------------------------------------------------------------ */
/* Section "Search for control structures": the control flow graph becomes a
 * region graph (initially the reachable blocks; region id = block index);
 * a depth-first search from the entry region visits regions in preorder
 * (fall-through successor first) and the first region that heads one of the
 * templates below has the template's regions merged into a new region (ids
 * n_blocks, n_blocks + 1, ... in merge order); the search starts again until
 * one region is left or no region heads a template.  Templates at header H,
 * tried in this order:
 *   DC_RG_IFELSE  H's successors A, B have H as only predecessor and one
 *                 common single successor J (not H, A, B): members H, A, B,
 *                 and J when A and B are its only predecessors;
 *   DC_RG_IF      (Fig. 2) a successor T (the fall-through one first) has H
 *                 as only predecessor and H's other successor F as only
 *                 successor: members H, T, and F when H and T are its only
 *                 predecessors (the two cases of the Fig. 3 trace);
 *   DC_RG_WHILE   a successor B has H as only predecessor and only
 *                 successor: members H, B (the back edge disappears);
 *   DC_RG_LINEAR  H's only successor S (not H) has H as only predecessor
 *                 and at most one successor, or H among its successors
 *                 (closing a loop: the new region has an edge to itself);
 *   DC_RG_LOOP    H has an edge to itself: member H (the edge disappears).
 * The entry counts the start as one more predecessor.  The new region's
 * successors are the members' successors outside the template (and itself,
 * for an edge back to H), in member order, each once.  The paper's if
 * template and linear region are the two it names; its exec-mask forms of
 * if-else (figures missing) are read as the standard diamond, which the
 * compiler's exec-mask shape reduces to as two nested ifs; while and loop
 * are this reading's additions so that counted loops reduce.  A kernel
 * whose records fail their checks gets that status and no merges. */
#define DC_RG_LINEAR 1
#define DC_RG_IF 2
#define DC_RG_IFELSE 3
#define DC_RG_WHILE 4
#define DC_RG_LOOP 5
typedef struct {
    uint32_t region;             /* the new region's id */
    uint8_t kind, n;             /* DC_RG_*, members (1..4) */
    uint16_t pad;
    uint32_t member[4];          /* header first; DC_SSA_NONE past n */
} dc_merge_t;                    /* 24 B */
typedef struct {
    dc_status_t status;
    uint32_t n_blocks, n_merges;
    uint32_t n_left;             /* regions left: 1 when the kernel reduces to one region */
    uint32_t root;               /* the last region when one is left, else DC_SSA_NONE */
    uint32_t pad;
    uint64_t digest;             /* sum over merges j of splitmix64(splitmix64(0x5354 * 0x9E3779B97F4A7C15 + j)
                                    ^ v), v folding (kind << 56) ^ (n << 48) ^ region with the four members
                                    by v = splitmix64(v + member[k] + 0x9E3779B97F4A7C15 * (k + 1)) */
} dc_struct_result_t;            /* 32 B */
typedef struct dc_struct dc_struct_t;
/* Structuring of n_kernels kernels whose records are in `instrs` (device):
 * the graph stages of dc_build_cfg, then one search per kernel, on
 * `stream`.  opts may be NULL; its flags may hold DC_OPT_TIMING only.  The
 * first run sizes the region arrays from the block count (one wait);
 * dc_struct_run on the same records allocates nothing and does not
 * synchronise. */
dc_status_t dc_structure(dc_ctx_t *ctx, const dc_kernel_t *kernels, uint32_t n_kernels, const dc_instr_t *instrs,
                         uint64_t n_records, const dc_options_t *opts, void *stream, dc_struct_t **out);
dc_status_t dc_struct_run(dc_struct_t *st, const dc_instr_t *instrs);
dc_status_t dc_struct_wait(dc_struct_t *st);
dc_status_t dc_struct_get_results(dc_struct_t *st, dc_struct_result_t *out, uint32_t cap);
/* kernel k's merges in the order they were made (two-call idiom) */
dc_status_t dc_struct_get_merges(dc_struct_t *st, uint32_t k, dc_merge_t *buf, uint32_t cap, uint32_t *n_total);
/* stage times (needs DC_OPT_TIMING): ms_decode, ms_cfg as for a batch,
 * ms_fixpoint = the structuring */
dc_status_t dc_struct_get_timing(dc_struct_t *st, dc_timing_t *out);
dc_status_t dc_struct_timing_reset(dc_struct_t *st);
void dc_struct_free(dc_struct_t *st);

/* ------------------------------------------------------------------ */
/* Register versions (minimal SSA form).                                */
/* ------------------------------------------------------------------ */
/* Section "Search for control structures": at a block with several
 * predecessors a register can hold the values of different definitions, and
 * the method then introduces a variable; the Register record of Section
 * "Search for memory accesses" carries a version.  Read here as the minimal
 * SSA form (Cytron, Ferrante, Rosen, Wegman & Zadeck 1991) of each kernel's
 * control flow graph over the DC_NSLOT register slots:
 *   - a virtual start before block 0 defines version 0 of every slot (its
 *     ABI entry value);
 *   - each definition makes a new version: an instruction defines its
 *     destination dwords, then the implicit vcc (two slots), exec (two) and
 *     scc, in that order (a slot written twice by one instruction gets two
 *     versions);
 *   - a merge (phi) of a slot sits at every block of the iterated dominance
 *     frontier of the blocks that define it (the start counts as a
 *     predecessor of block 0); its arguments are, per incoming edge, the
 *     version live at the end of the edge's source (block 0's entry edge
 *     first, carrying version 0, then the reachable predecessors in
 *     ascending order);
 *   - versions of a slot are numbered 1, 2, ... in a preorder walk of the
 *     dominator tree (children by ascending block index), a block's merges
 *     first (by slot), then its instructions in order;
 *   - dominators are those of the reachable blocks; unreachable blocks have
 *     no dominator (DC_SSA_NONE), no merges and no versions.
 * Uses of an instruction, in order: the dwords of r1, r2, the third source
 * (imm) and a stored r0 that name register slots, then the implicit vcc,
 * exec and scc uses.  A kernel whose records fail their checks gets that
 * status and nothing else. */
#define DC_SSA_NU 13             /* uses of one instruction, at most */
#define DC_SSA_ND 9              /* definitions of one instruction, at most */
#define DC_SSA_NONE 0xFFFFFFFFu
typedef struct {
    uint32_t block;              /* the merge's block */
    uint16_t slot, pad;          /* register slot (0..DC_NSLOT-1) */
    uint32_t version;
} dc_phi_t;                      /* 12 B */
typedef struct {
    dc_status_t status;
    uint32_t n_blocks, n_phi, n_phi_args;
    uint32_t n_operands;         /* versions stored: the uses and definitions of every instruction */
    uint32_t pad;
    uint64_t digest;             /* sum over the items (kind, index, value) of splitmix64(splitmix64(kind *
                                    0x9E3779B97F4A7C15 + index) ^ value): kind 1 per block (index block, value
                                    its dominator), 2 per merge ((block << 16) | slot, version), 3 per merge
                                    argument ((block << 24) | (slot << 12) | edge, version), 4 per use entry and
                                    5 per definition entry of the fixed layouts of dc_ssa_get_versions (index
                                    instruction * DC_SSA_NU + q, resp. * DC_SSA_ND + q, value the version or
                                    DC_SSA_NONE); 0 for a failed kernel or without DC_OPT_DIGEST */
} dc_ssa_result_t;               /* 32 B */
typedef struct dc_ssa dc_ssa_t;

/* Versions for n_kernels kernels whose records are in `instrs` (device,
 * n_records entries): the graph stages of dc_build_cfg, then the versions,
 * on `stream`.  opts may be NULL; its flags may hold DC_OPT_TIMING and
 * DC_OPT_DIGEST (without it dc_ssa_result_t.digest is 0).
 * The first run sizes the version tables from the graph (it waits for the
 * stream twice); dc_ssa_run on the same records allocates nothing and does
 * not synchronise, on other records it sizes them again. */
dc_status_t dc_build_ssa(dc_ctx_t *ctx, const dc_kernel_t *kernels, uint32_t n_kernels, const dc_instr_t *instrs,
                         uint64_t n_records, const dc_options_t *opts, void *stream, dc_ssa_t **out);
dc_status_t dc_ssa_run(dc_ssa_t *ssa, const dc_instr_t *instrs);
dc_status_t dc_ssa_wait(dc_ssa_t *ssa);
/* Getters (wait for the stream; two-call idiom as dc_get_accesses).
 * results: the first min(cap, n_kernels) kernels.  idom: kernel k's
 * immediate dominators, one per block.  phis: ascending (block, slot).
 * phi_args: per merge in that order, one version per incoming edge.
 * versions: use_ver (DC_SSA_NU per instruction) and def_ver (DC_SSA_ND per
 * instruction, either may be NULL) in the orders above, DC_SSA_NONE past an
 * instruction's operands and for unreachable instructions; *n_instr = the
 * kernel's instruction count, and min(cap_instr, n_instr) instructions are
 * written. */
dc_status_t dc_ssa_get_results(dc_ssa_t *ssa, dc_ssa_result_t *out, uint32_t cap);
dc_status_t dc_ssa_get_idom(dc_ssa_t *ssa, uint32_t k, uint32_t *buf, uint32_t cap, uint32_t *n_total);
dc_status_t dc_ssa_get_phis(dc_ssa_t *ssa, uint32_t k, dc_phi_t *buf, uint32_t cap, uint32_t *n_total);
dc_status_t dc_ssa_get_phi_args(dc_ssa_t *ssa, uint32_t k, uint32_t *buf, uint32_t cap, uint32_t *n_total);
dc_status_t dc_ssa_get_versions(dc_ssa_t *ssa, uint32_t k, uint32_t *use_ver, uint32_t *def_ver, uint32_t cap_instr,
                                uint32_t *n_instr);
/* Stage times (needs DC_OPT_TIMING): ms_decode, ms_cfg as for a batch,
 * ms_fixpoint = the version stages, ms_compact = the variable and type
 * stage of an object made by dc_build_types (0 otherwise). */
dc_status_t dc_ssa_get_timing(dc_ssa_t *ssa, dc_timing_t *out);
dc_status_t dc_ssa_timing_reset(dc_ssa_t *ssa);
void dc_ssa_free(dc_ssa_t *ssa);

/* ------------------------------------------------------------------ */
/* Variables and types over the register versions.                      */
/* ------------------------------------------------------------------ */
/* Section "Data type recovery": types come from the .arg lines of the
 * configuration (Listing 3) and from instruction suffixes, a suffix typing
 * the values an instruction reads as well as the one it writes (an unsigned
 * add adds two unsigned integers).  Section "Search for control
 * structures": a register whose value at a join depends on the path becomes
 * a variable when it is used later; the ternary operator is one instruction
 * (v_cndmask_b32).  Read over the versions above, per kernel:
 *   - nodes: versions 0 .. n-1 of every register slot that some record of
 *     the kernel names as an operand, and of vcc, exec and scc; ordered by
 *     slot, then version (dc_var_t.slot, .version);
 *   - var: a merge and each of its arguments are one variable (the variable
 *     made at the join); the classes of that relation;
 *   - tclass: the same relation, plus a move's destination dword with the
 *     source dword it copies (s_mov_b32, s_mov_b64 dword by dword,
 *     v_mov_b32) and v_cndmask_b32's result with each of its two values;
 *   - a class is named by its first node (an index into the kernel's nodes);
 *   - type: the union over the node's tclass of the type each definition
 *     gives its destination dwords and each use gives the registers it
 *     reads (DC_TY_* bits):
 *       definition: the mnemonic's first type suffix (i INT, u UINT, f32
 *       FLOAT, f64 DOUBLE; b and none: nothing); a scalar load through the
 *       kernel-argument pointer (s4 and s5 both at version 0) at dword
 *       offset o: UINT for o < 0x18 and o = 0x20010, nothing for
 *       0x18 <= o < 0x30, else the .arg type of the argument covering o
 *       (nothing when none does);
 *       use: a mnemonic whose last suffix is typed gives it to every register
 *       read as an explicit source; a global or flat access's address pair is
 *       a pointer (the saddr pair when the record has one, the vaddr pair
 *       then UINT), an s_load base a pointer, an LDS address UINT;
 *   - flags: DC_VF_MERGE for a merge's version; DC_VF_LIVE for a node some
 *     reachable instruction reads or that is an argument of a live merge (a
 *     live merge is a variable the method creates);
 *   - records that no path reaches make no versions and take no part.
 * A kernel whose records fail their checks gets that status and nothing
 * else. */
#define DC_VF_MERGE 1u
#define DC_VF_LIVE 2u
typedef struct {
    uint16_t slot;
    uint8_t type;                /* DC_TY_* bits of the node's type class */
    uint8_t flags;               /* DC_VF_* */
    uint32_t version;
    uint32_t var;                /* first node of the node's variable */
    uint32_t tclass;             /* first node of the node's type class */
} dc_var_t;                      /* 16 B */
typedef struct {
    dc_status_t status;
    uint32_t n_nodes;
    uint32_t n_vars;             /* variables (classes of var) */
    uint32_t n_tclasses;         /* type classes */
    uint32_t n_live_merges;
    uint32_t n_ternary;          /* reachable v_cndmask_b32 records */
    uint64_t digest;             /* sum over the nodes x of splitmix64(splitmix64(6 * 0x9E3779B97F4A7C15 + x) ^
                                    (var << 32 | tclass)) and splitmix64(splitmix64(7 * 0x9E3779B97F4A7C15 + x) ^
                                    (slot << 48 | version << 16 | type << 8 | flags)); 0 for a failed kernel or
                                    without DC_OPT_DIGEST */
} dc_types_result_t;             /* 32 B */

/* As dc_build_ssa, plus the variables and types, for kernels whose
 * argument tables are `args` (host, n_args entries, as dc_analyze_batch
 * takes them; copied).  The object is a dc_ssa_t: dc_ssa_run, _wait, the
 * version getters, _get_timing and dc_ssa_free apply; the first run also
 * sizes the node arrays (one more wait for the stream). */
dc_status_t dc_build_types(dc_ctx_t *ctx, const dc_kernel_t *kernels, uint32_t n_kernels, const dc_instr_t *instrs,
                           uint64_t n_records, const dc_arg_t *args, uint64_t n_args, const dc_options_t *opts,
                           void *stream, dc_ssa_t **out);
/* results: the first min(cap, n_kernels) kernels; vars: kernel k's nodes in
 * order (two-call idiom).  DC_E_INVAL on an object dc_build_ssa made. */
dc_status_t dc_types_get_results(dc_ssa_t *ssa, dc_types_result_t *out, uint32_t cap);
dc_status_t dc_types_get_vars(dc_ssa_t *ssa, uint32_t k, dc_var_t *buf, uint32_t cap, uint32_t *n_total);

/* ------------------------------------------------------------------ */
/* Request server: continuous batching of single-kernel analyses.       */
/* ------------------------------------------------------------------ */
/* The server takes analysis requests one kernel at a time as they arrive
 * and returns each one's result on its own; the analysis is the same as
 * dc_analyze_batch's, so a request's result does not depend
 * on what it was batched with.
 *
 * A service thread admits waiting requests into lanes.  A lane is a
 * preallocated slice of device memory (the arrays of a batch of up to
 * `lane_instr` instructions and `max_batch_kernels` kernels, the fixpoint
 * arenas) with pinned host staging and its own HIP stream.  Whenever a lane
 * is free and requests wait, it takes as many of them as fit it, oldest
 * first, from one length class, and enqueues the whole analysis.  A batch
 * is done when its longest kernel is, so requests are batched with others of
 * similar length: four classes with upper bounds long_instr/16, long_instr/4
 * and long_instr, the two longer classes holding at most half and a quarter
 * of the lanes (at least one).  Lanes run concurrently on the device, so requests
 * that arrive while others are being analysed start as soon as a lane and
 * its memory free up, and their work overlaps with what is already on the
 * GPU.  Admission is therefore by device memory: the lanes are carved from
 * `pool_bytes` when the server is created and nothing is allocated per
 * request on the device. */
typedef struct dc_server dc_server_t;

typedef struct {
    uint64_t pool_bytes;         /* device memory for the lanes; 0 = what `lanes` lanes of the largest size need */
    uint32_t lanes;              /* concurrent batches in flight, at most 16; 0 = one less than the process's HIP
                                    hardware queues (GPU_MAX_HW_QUEUES, HIP's default 4), at most 8: lanes that
                                    share a hardware queue run in order, so a long batch holds up the other */
    uint32_t max_request_instr;  /* longest request accepted (0 = 100,000 instructions) */
    uint32_t max_batch_kernels;  /* requests per batch (0 = 2048) */
    uint32_t long_instr;         /* length class bounds long_instr/16, /4, /1 (0 = 16384) */
    uint32_t flags;              /* DC_OPT_DIGEST or 0 */
    uint32_t reserved[3];
} dc_server_opts_t;

/* One request: a kernel descriptor (instr_begin and arg_begin are ignored),
 * its n_instr records and n_args argument entries (host memory, copied by
 * dc_server_submit), and a caller value returned with the result. */
typedef struct {
    dc_kernel_t kernel;
    const dc_instr_t *instrs;
    const dc_arg_t *args;
    uint64_t tag;
} dc_request_t;

/* One completed request.  accesses/sysvals point at summary.n_access and
 * summary.n_sysval records owned by the server, valid until the next
 * dc_server_poll or dc_server_destroy.  Times are CLOCK_MONOTONIC
 * nanoseconds: submission, admission into a lane, its batch's work enqueued
 * (records packed), the batch's analysis seen complete on the device,
 * results on the host.
 * status is the request's per-kernel status, or DC_E_HIP when the device
 * failed while it was in flight. */
typedef struct {
    uint64_t ticket, tag;
    dc_kernel_result_t summary;
    const dc_access_t *accesses;
    const dc_sysval_t *sysvals;
    uint64_t t_submit_ns, t_admit_ns, t_enqueued_ns, t_device_ns, t_done_ns;
    uint64_t batch;              /* batch id (admission order) */
    uint32_t batch_kernels;      /* requests in that batch */
    uint32_t lane;
} dc_result_t;

typedef struct {
    uint64_t submitted, completed, waiting, batches, max_batch_kernels, device_bytes, lane_instr;
    uint32_t lanes, pad;
} dc_server_stats_t;

/* Create a server on the context's device and start its service thread.
 * DC_E_INVAL when an option is out of range or pool_bytes cannot hold the
 * lanes for max_request_instr; DC_E_OOM when the allocation fails. */
dc_status_t dc_server_create(dc_ctx_t *ctx, const dc_server_opts_t *opts, dc_server_t **out);
/* Queue a request (copies it; non-blocking).  *ticket identifies it in the
 * results.  DC_E_INVAL for a request longer than max_request_instr or null
 * buffers; DC_E_HIP once the device has failed. */
dc_status_t dc_server_submit(dc_server_t *srv, const dc_request_t *req, uint64_t *ticket);
/* Move up to `max` completed results into out[]; *n = how many.  Never
 * blocks.  Invalidates the record pointers of the previous call. */
dc_status_t dc_server_poll(dc_server_t *srv, dc_result_t *out, uint32_t max, uint32_t *n);
dc_status_t dc_server_get_stats(dc_server_t *srv, dc_server_stats_t *out);
/* Stop admitting, wait for the batches in flight, free everything.
 * Requests still waiting are dropped. */
void dc_server_destroy(dc_server_t *srv);

const char *dc_status_str(dc_status_t st);
int dc_opcode_count(void);
const char *dc_opcode_name(int id);

#ifdef __cplusplus
}
#endif
#endif

/* dc_opnames.h -- mnemonics of the opcode numbering of the record encoding
 * (dc_opcode_name), in id order, as one list for the host API and the text
 * front end's device tables. */
#pragma once

#define DC_OPNAME_LIST \
    "s_load_dword", "s_load_dwordx2", "s_load_dwordx4", "s_mov_b32", "s_mov_b64", "s_and_saveexec_b64", \
    "s_or_saveexec_b64", "s_add_u32", "s_add_i32", "s_addc_u32", "s_sub_u32", "s_mul_i32", "s_lshl_b32", \
    "s_lshr_b32", "s_and_b32", "s_or_b32", "s_and_b64", "s_or_b64", "s_xor_b64", "s_andn2_b64", \
    "s_cmp_eq_u32", "s_cmp_lt_u32", "s_cmp_gt_u32", "s_cmp_lt_i32", "s_branch", "s_cbranch_scc0", \
    "s_cbranch_scc1", "s_cbranch_vccz", "s_cbranch_vccnz", "s_cbranch_execz", "s_cbranch_execnz", \
    "s_waitcnt", "s_barrier", "s_nop", "s_endpgm", "v_mov_b32", "v_cvt_f32_u32", "v_cvt_u32_f32", \
    "v_cvt_f64_f32", "v_add_co_u32", "v_addc_co_u32", "v_sub_co_u32", "v_add_u32", "v_mul_lo_u32", \
    "v_mul_u32_u24", "v_mul_hi_u32", "v_mad_u32_u24", "v_lshlrev_b32", "v_lshrrev_b32", "v_ashrrev_i32", \
    "v_and_b32", "v_or_b32", "v_xor_b32", "v_lshlrev_b64", "v_cndmask_b32", "v_add_f32", "v_sub_f32", \
    "v_mul_f32", "v_max_f32", "v_mad_f32", "v_fma_f32", "v_add_f64", "v_mul_f64", "v_fma_f64", \
    "v_cmp_eq_u32", "v_cmp_gt_u32", "v_cmp_lt_u32", "v_cmp_lt_i32", "v_cmp_gt_f32", "global_load_dword", \
    "global_load_dwordx2", "flat_load_dword", "global_store_dword", "global_store_dwordx2", \
    "flat_store_dword", "ds_read_b32", "ds_write_b32",

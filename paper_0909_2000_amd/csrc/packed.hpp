// Packed 16-bit helpers for gfx950: two independent lanes of work per VGPR,
// on the VOP3P instructions (v_pk_add_u16, v_pk_sub_u16, v_pk_min_u16,
// v_pk_max_u16, v_pk_lshlrev_b16), and gfx950's three-input bitwise
// v_bitop3_b32, whose 8-bit immediate is the truth table of the operation
// (0x96: the XOR of all three operands).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wlcs {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ u16x2 as_v(uint32_t a) { return __builtin_bit_cast(u16x2, a); }
__device__ __forceinline__ uint32_t as_u(u16x2 a) { return __builtin_bit_cast(uint32_t, a); }

__device__ __forceinline__ uint32_t pk_add(uint32_t a, uint32_t b) { return as_u(as_v(a) + as_v(b)); }
__device__ __forceinline__ uint32_t pk_sub(uint32_t a, uint32_t b) { return as_u(as_v(a) - as_v(b)); }
__device__ __forceinline__ uint32_t pk_sub_sat(uint32_t a, uint32_t b) {
    return as_u(__builtin_elementwise_sub_sat(as_v(a), as_v(b)));
}
__device__ __forceinline__ uint32_t pk_min(uint32_t a, uint32_t b) {
    return as_u(__builtin_elementwise_min(as_v(a), as_v(b)));
}
__device__ __forceinline__ uint32_t pk_max(uint32_t a, uint32_t b) {
    return as_u(__builtin_elementwise_max(as_v(a), as_v(b)));
}
// per half: a << (b & 15)
__device__ __forceinline__ uint32_t pk_shl(uint32_t a, uint32_t b) {
    return as_u(as_v(a) << (as_v(b) & (unsigned short)15));
}
// a 16-bit value (taken mod 2^16) in both halves
__device__ __forceinline__ uint32_t pk_rep(int32_t v) { return ((uint32_t)v & 0xFFFFu) * 0x10001u; }

// (half `HI` of x, in both lanes) + y, per 16-bit lane.  The half is picked
// with the op_sel modifiers of v_pk_add_u16, so the broadcast costs nothing
// and no register holds the duplicated value.  Pure ALU, no memory access.
template <int HI>
__device__ __forceinline__ uint32_t pk_add_bcast(uint32_t x, uint32_t y) {
    uint32_t r;
    if (HI)
        asm("v_pk_add_u16 %0, %1, %2 op_sel:[1,0]" : "=v"(r) : "v"(x), "v"(y));
    else
        asm("v_pk_add_u16 %0, %1, %2 op_sel_hi:[0,1]" : "=v"(r) : "v"(x), "v"(y));
    return r;
}

// One seaweed cell for two tiles at once (see seaweed.hip):
//     z     = x_code (half HI of x, both lanes) + y_codes
//     down  = max(s, min(t, z))
//     s     = s ^ t ^ down          (the seaweed leaving to the right: one
//                                    v_bitop3_b32; down is s or t in each half)
// Written as one volatile block so that the four instructions stay together
// and the compiler cannot hoist the letter sums of a whole column into
// registers ahead of time.  The y codes of a column are the same in every
// lane, so they come from a scalar register.  Pure ALU, no memory access.
template <int HI>
__device__ __forceinline__ uint32_t seaweed_cell(uint32_t& s, uint32_t t, uint32_t x, uint32_t y) {
    uint32_t down;
    if (HI)
        asm volatile(
            "v_pk_add_u16 %1, %3, %4 op_sel:[1,0]\n\t"
            "v_pk_min_u16 %1, %2, %1\n\t"
            "v_pk_max_u16 %1, %0, %1\n\t"
            "v_bitop3_b32 %0, %0, %2, %1 bitop3:0x96"
            : "+v"(s), "=&v"(down)
            : "v"(t), "v"(x), "s"(y));
    else
        asm volatile(
            "v_pk_add_u16 %1, %3, %4 op_sel_hi:[0,1]\n\t"
            "v_pk_min_u16 %1, %2, %1\n\t"
            "v_pk_max_u16 %1, %0, %1\n\t"
            "v_bitop3_b32 %0, %0, %2, %1 bitop3:0x96"
            : "+v"(s), "=&v"(down)
            : "v"(t), "v"(x), "s"(y));
    return down;
}
// The cell of the top row: t is the label of the seaweed entering the column
// from the top, the same in every lane, so it too comes from a scalar register.
__device__ __forceinline__ uint32_t seaweed_cell_top(uint32_t& s, uint32_t t, uint32_t x, uint32_t y) {
    uint32_t down;
    asm volatile(
        "v_pk_add_u16 %1, %3, %4 op_sel_hi:[0,1]\n\t"
        "v_pk_min_u16 %1, %2, %1\n\t"
        "v_pk_max_u16 %1, %0, %1\n\t"
        "v_bitop3_b32 %0, %0, %2, %1 bitop3:0x96"
        : "+v"(s), "=&v"(down)
        : "s"(t), "v"(x), "s"(y));
    return down;
}

// One pair slot of the score-plot schedule for strings blown up with a
// separator before every letter: the separator column and the letter column
// after it, combed in one top-down pass.  Row 2r of the strip (label a) is a
// separator row, row 2r + 1 (label b) a letter row.
//   separator column:  mx = max(a, b) moves down to the next slot's
//                      separator row, b = min(a, b) stays
//   letter column:     its separator row is a mismatch:  d = max(c, t),
//                      a = min(c, t), where c is the label the separator
//                      column sent down from the slot above; its letter row is
//                      the general cell:  z = x + y,  down = max(b, min(d, z)),
//                      b = b ^ d ^ down (one v_bitop3_b32),  t = down
// Eight instructions per slot.  Returns mx (the next slot's c).  Pure ALU.
#define WLCS_FUSED_SLOT_BODY(XSEL)                 \
    "v_pk_add_u16 %5, %7, %8 " XSEL "\n\t"       \
    "v_pk_max_u16 %3, %0, %1\n\t"                \
    "v_pk_min_u16 %1, %0, %1\n\t"                \
    "v_pk_max_u16 %4, %6, %2\n\t"                \
    "v_pk_min_u16 %0, %6, %2\n\t"                \
    "v_pk_min_u16 %5, %4, %5\n\t"                \
    "v_pk_max_u16 %2, %1, %5\n\t"                \
    "v_bitop3_b32 %1, %1, %4, %2 bitop3:0x96"
template <int HI>
__device__ __forceinline__ uint32_t fused_slot(uint32_t& a, uint32_t& b, uint32_t& t, uint32_t c, uint32_t x,
                                               uint32_t y) {
    uint32_t mx, d, z;
    if (HI)
        asm volatile(WLCS_FUSED_SLOT_BODY("op_sel:[1,0]")
                     : "+v"(a), "+v"(b), "+v"(t), "=&v"(mx), "=&v"(d), "=&v"(z)
                     : "v"(c), "v"(x), "s"(y));
    else
        asm volatile(WLCS_FUSED_SLOT_BODY("op_sel_hi:[0,1]")
                     : "+v"(a), "+v"(b), "+v"(t), "=&v"(mx), "=&v"(d), "=&v"(z)
                     : "v"(c), "v"(x), "s"(y));
    return mx;
}
#undef WLCS_FUSED_SLOT_BODY

// Two such slots of two independent passes (P: operands 0-5 and 12-14, Q:
// operands 6-11 and 15-17), their instructions alternated so that no
// instruction directly follows the one it depends on.  HP picks the half of
// P's x register (Q takes the other).  Each pass's c becomes its mx.  Pure
// ALU.
#define WLCS_FUSED_SLOT2_BODY(PSEL, QSEL)             \
    "v_pk_add_u16 %5, %13, %14 " PSEL "\n\t"       \
    "v_pk_add_u16 %11, %16, %17 " QSEL "\n\t"      \
    "v_pk_max_u16 %3, %0, %1\n\t"                   \
    "v_pk_max_u16 %9, %6, %7\n\t"                   \
    "v_pk_min_u16 %1, %0, %1\n\t"                   \
    "v_pk_min_u16 %7, %6, %7\n\t"                   \
    "v_pk_max_u16 %4, %12, %2\n\t"                  \
    "v_pk_max_u16 %10, %15, %8\n\t"                 \
    "v_pk_min_u16 %0, %12, %2\n\t"                  \
    "v_pk_min_u16 %6, %15, %8\n\t"                  \
    "v_pk_min_u16 %5, %4, %5\n\t"                   \
    "v_pk_min_u16 %11, %10, %11\n\t"                \
    "v_pk_max_u16 %2, %1, %5\n\t"                   \
    "v_pk_max_u16 %8, %7, %11\n\t"                  \
    "v_bitop3_b32 %1, %1, %4, %2 bitop3:0x96\n\t"  \
    "v_bitop3_b32 %7, %7, %10, %8 bitop3:0x96"
#define WLCS_FUSED_SLOT2_OPS                                                                        \
    : "+v"(pa), "+v"(pb), "+v"(pt), "=&v"(pmx), "=&v"(pd), "=&v"(pz), "+v"(qa), "+v"(qb), "+v"(qt), \
      "=&v"(qmx), "=&v"(qd), "=&v"(qz)                                                               \
    : "v"(pc), "v"(px), "s"(py), "v"(qc), "v"(qx), "s"(qy)
// (the two passes are one slot apart, so their x halves always differ)
template <int HP>
__device__ __forceinline__ void fused_slot2(uint32_t& pa, uint32_t& pb, uint32_t& pt, uint32_t& pc, uint32_t px,
                                            uint32_t py, uint32_t& qa, uint32_t& qb, uint32_t& qt, uint32_t& qc,
                                            uint32_t qx, uint32_t qy) {
    uint32_t pmx, pd, pz, qmx, qd, qz;
    if (HP)
        asm volatile(WLCS_FUSED_SLOT2_BODY("op_sel:[1,0]", "op_sel_hi:[0,1]") WLCS_FUSED_SLOT2_OPS);
    else
        asm volatile(WLCS_FUSED_SLOT2_BODY("op_sel_hi:[0,1]", "op_sel:[1,0]") WLCS_FUSED_SLOT2_OPS);
    pc = pmx;
    qc = qmx;
}
#undef WLCS_FUSED_SLOT2_BODY
#undef WLCS_FUSED_SLOT2_OPS

// One cell of the plain LCS dynamic program for two windows at once:
//     z = x_code (half HI of x, both lanes) + y_codes    (0 iff the letters match)
//     L = max(up, left, sat(diag + 1 - z))               (diag + 1 on a match, else 0)
// one2 must hold 0x00010001.  Pure ALU, no memory access.
template <int HI>
__device__ __forceinline__ uint32_t dp_cell(uint32_t up, uint32_t left, uint32_t diag, uint32_t x, uint32_t y,
                                            uint32_t one2) {
    uint32_t v, z, d;
    if (HI)
        asm volatile(
            "v_pk_add_u16 %1, %6, %7 op_sel:[1,0]\n\t"
            "v_pk_add_u16 %2, %5, %8\n\t"
            "v_pk_sub_u16 %1, %2, %1 clamp\n\t"
            "v_pk_max_u16 %2, %3, %4\n\t"
            "v_pk_max_u16 %0, %2, %1"
            : "=&v"(v), "=&v"(z), "=&v"(d)
            : "v"(up), "v"(left), "v"(diag), "v"(x), "v"(y), "v"(one2));
    else
        asm volatile(
            "v_pk_add_u16 %1, %6, %7 op_sel_hi:[0,1]\n\t"
            "v_pk_add_u16 %2, %5, %8\n\t"
            "v_pk_sub_u16 %1, %2, %1 clamp\n\t"
            "v_pk_max_u16 %2, %3, %4\n\t"
            "v_pk_max_u16 %0, %2, %1"
            : "=&v"(v), "=&v"(z), "=&v"(d)
            : "v"(up), "v"(left), "v"(diag), "v"(x), "v"(y), "v"(one2));
    return v;
}

// Per half: 1 if p < w (unsigned), else 0 -- min(sat(w - p), 1).  Written as
// two packed instructions (the compiler would otherwise split the halves).
// w2 is wave-uniform and is read from a scalar register.
__device__ __forceinline__ uint32_t pk_below(uint32_t w2, uint32_t p2, uint32_t one2) {
    uint32_t v;
    asm("v_pk_sub_u16 %0, %1, %2 clamp\n\tv_pk_min_u16 %0, %0, %3"
        : "=&v"(v)
        : "s"(__builtin_amdgcn_readfirstlane(w2)), "v"(p2), "v"(one2));
    return v;
}

// Per half: 1 if a > b (unsigned), else 0 -- min(sat(a - b), 1).  b is
// wave-uniform and is read from a scalar register.
__device__ __forceinline__ uint32_t pk_above(uint32_t a2, uint32_t b2, uint32_t one2) {
    uint32_t v;
    asm("v_pk_sub_u16 %0, %1, %2 clamp\n\tv_pk_min_u16 %0, %0, %3"
        : "=&v"(v)
        : "v"(a2), "s"(__builtin_amdgcn_readfirstlane(b2)), "v"(one2));
    return v;
}

// Per half: a >> 1.
__device__ __forceinline__ uint32_t pk_shr1(uint32_t a) {
    return as_u(as_v(a) >> (u16x2){(unsigned short)1, (unsigned short)1});
}

// Per half: val << (amount & 15), one v_pk_lshlrev_b16.
__device__ __forceinline__ uint32_t pk_lshl(uint32_t amount, uint32_t val) {
    uint32_t r;
    asm("v_pk_lshlrev_b16 %0, %1, %2" : "=v"(r) : "v"(amount), "v"(val));
    return r;
}

// (x >> OFF) & ((1 << WIDTH) - 1) as one v_bfe_u32 (the compiler would
// otherwise split it into a shift and a mask).
template <int OFF, int WIDTH>
__device__ __forceinline__ uint32_t bfe(uint32_t x) {
    uint32_t r;
    asm("v_bfe_u32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "i"(OFF), "i"(WIDTH));
    return r;
}

// Read-only device memory seen through the constant address space: loads
// with a wave-uniform address become scalar loads (s_load), whose results
// stay in scalar registers.  Only for data that no kernel of the launch writes.
typedef const __attribute__((address_space(4))) uint32_t* const_u32p;
__device__ __forceinline__ const_u32p as_const(const uint32_t* p) { return (const_u32p)p; }

// A wave-uniform pointer, forced into scalar registers.
template <typename T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
    const uint64_t a = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    return (T*)(((uint64_t)hi << 32) | lo);
}

// 16-bit element i of a wave-uniform array, through a 32-bit (scalar) load
__device__ __forceinline__ uint32_t u16_at(const uint32_t* __restrict__ p, int64_t i) {
    return (p[i >> 1] >> ((uint32_t)(i & 1) * 16u)) & 0xFFFFu;
}

}  // namespace wlcs

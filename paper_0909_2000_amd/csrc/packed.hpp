// Packed 16-bit helpers for gfx950: two independent lanes of work per VGPR,
// on the VOP3P instructions (v_pk_add_u16, v_pk_sub_u16, v_pk_min_u16,
// v_pk_max_u16, v_pk_lshlrev_b16).
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
//     s     = s ^ t ^ down          (the seaweed leaving to the right)
// Written as one volatile block so that the five instructions stay together
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
            "v_xor_b32 %0, %0, %2\n\t"
            "v_xor_b32 %0, %0, %1"
            : "+v"(s), "=&v"(down)
            : "v"(t), "v"(x), "s"(y));
    else
        asm volatile(
            "v_pk_add_u16 %1, %3, %4 op_sel_hi:[0,1]\n\t"
            "v_pk_min_u16 %1, %2, %1\n\t"
            "v_pk_max_u16 %1, %0, %1\n\t"
            "v_xor_b32 %0, %0, %2\n\t"
            "v_xor_b32 %0, %0, %1"
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
        "v_xor_b32 %0, %2, %0\n\t"
        "v_xor_b32 %0, %0, %1"
        : "+v"(s), "=&v"(down)
        : "s"(t), "v"(x), "s"(y));
    return down;
}

// Sort two labels per half: lo <- min(lo, b), returns max(lo, b).  One
// volatile block per call keeps the calls in program order, so that a column
// of them does not keep many results live at once.  Pure ALU.
__device__ __forceinline__ uint32_t pk_sort2(uint32_t& lo, uint32_t b) {
    uint32_t hi;
    asm volatile(
        "v_pk_max_u16 %0, %1, %2\n\t"
        "v_pk_min_u16 %1, %1, %2"
        : "=&v"(hi), "+v"(lo)
        : "v"(b));
    return hi;
}

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
__device__ __forceinline__ uint32_t pk_below(uint32_t w2, uint32_t p2, uint32_t one2) {
    uint32_t v;
    asm("v_pk_sub_u16 %0, %1, %2 clamp\n\tv_pk_min_u16 %0, %0, %3" : "=&v"(v) : "v"(w2), "v"(p2), "v"(one2));
    return v;
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

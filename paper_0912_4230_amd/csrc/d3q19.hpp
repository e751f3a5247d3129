// d3q19.hpp -- D3Q19 velocity set and population storage codecs for gfx950.
//
// Direction order used on the GPU: 0 rest; 1..6 the axis vectors
// (+x,-x,+y,-y,+z,-z); 7..18 the twelve face diagonals, each followed by its
// opposite.  Weights: 1/3 (rest), 1/18 (axes), 1/36 (diagonals), Sec. 2.1 of
// the paper (sentence after Eq. equilc2).  Components are encoded in bit
// masks so that every lookup folds to a constant after unrolling.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// global (HBM) address space: loads and stores through such pointers compile
// to global_* instructions instead of flat_*
#define GL __attribute__((address_space(1)))

namespace plbm {

constexpr int NQ = 19;

constexpr uint32_t bit(int q) { return 1u << q; }
constexpr uint32_t XP = bit(1) | bit(7) | bit(9) | bit(11) | bit(13);
constexpr uint32_t XN = bit(2) | bit(8) | bit(10) | bit(12) | bit(14);
constexpr uint32_t YP = bit(3) | bit(7) | bit(10) | bit(15) | bit(17);
constexpr uint32_t YN = bit(4) | bit(8) | bit(9) | bit(16) | bit(18);
constexpr uint32_t ZP = bit(5) | bit(11) | bit(14) | bit(15) | bit(18);
constexpr uint32_t ZN = bit(6) | bit(12) | bit(13) | bit(16) | bit(17);

__host__ __device__ constexpr int cx(int q) { return int((XP >> q) & 1u) - int((XN >> q) & 1u); }
__host__ __device__ constexpr int cy(int q) { return int((YP >> q) & 1u) - int((YN >> q) & 1u); }
__host__ __device__ constexpr int cz(int q) { return int((ZP >> q) & 1u) - int((ZN >> q) & 1u); }
__host__ __device__ constexpr int opp(int q) { return q == 0 ? 0 : ((q & 1) ? q + 1 : q - 1); }
__host__ __device__ constexpr int speed2(int q) { return cx(q) * cx(q) + cy(q) * cy(q) + cz(q) * cz(q); }

template <class R>
__host__ __device__ constexpr R weight(int q)
{
    return q == 0 ? R(1) / R(3) : (q <= 6 ? R(1) / R(18) : R(1) / R(36));
}

// FP32 weights whose exact sum is 1.  The rounded 1/3, 1/18 and 1/36 sum to
// 1 + 1.49e-8, so every collision returned 1 + 1.49e-8 omega times the
// equilibrium mass of the cell: a bias that accumulates step after step (the
// FP32 solute mass of a closed box grew by 2.3e-8 per step at tau_d = 0.65).
// Here w_2 = 14913080 * 2^-29 (1/36 to 6e-8; its mantissa is even), w_1 = 2 w_2
// and w_0 = 1 - 24 w_2 = 11184812 * 2^-25, all exact in FP32, so that
// w_0 + 6 w_1 + 12 w_2 = 1 exactly.  The isotropy sums (Sum w v_a v_b = 1/3)
// then hold to 6e-8, below FP32 resolution.
template <>
__host__ __device__ constexpr float weight<float>(int q)
{
    return q == 0 ? 11184812.0f / 33554432.0f : (q <= 6 ? 29826160.0f / 536870912.0f : 14913080.0f / 536870912.0f);
}

// ---------------------------------------------------------------------------
// storage codecs: Codec<S>::R is the compute type, load/store convert.
// Populations are streamed: each value is read once, one step after it was
// written, long after it has left the caches, so both directions use the
// non-temporal cache policy by default.

#ifndef PLBM_NT_STORE
#define PLBM_NT_STORE 1
#endif
#ifndef PLBM_NT_LOAD
#define PLBM_NT_LOAD 1
#endif

template <class T>
__device__ inline void st(GL T *p, T v)
{
    if constexpr (PLBM_NT_STORE) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <class T>
__device__ inline T ld(const GL T *p)
{
    if constexpr (PLBM_NT_LOAD) return __builtin_nontemporal_load(p);
    else return *p;
}

struct bf16_t { uint16_t v; };
struct f16_t { uint16_t v; };

template <class S> struct Codec;

template <> struct Codec<double> {
    using R = double;
    static constexpr bool split = false;
    __device__ static R load(const GL double *p) { return ld(p); }
    __device__ static void store(GL double *p, R v) { st(p, v); }
};

template <> struct Codec<float> {
    using R = float;
    static constexpr bool split = false;
    __device__ static R load(const GL float *p) { return ld(p); }
    __device__ static void store(GL float *p, R v) { st(p, v); }
};

// bfloat16: the upper half of an IEEE float; the hardware conversion
// (v_cvt_pk_bf16_f32) rounds to nearest even.
template <> struct Codec<bf16_t> {
    using R = float;
    static constexpr bool split = false;
    __device__ static R load(const GL bf16_t *p)
    {
        return __uint_as_float(uint32_t(ld(reinterpret_cast<const GL uint16_t *>(p))) << 16);
    }
    __device__ static void store(GL bf16_t *p, R v)
    {
        st(reinterpret_cast<GL uint16_t *>(p), __builtin_bit_cast(uint16_t, (__bf16)v));
    }
};

// IEEE binary16: hardware conversion (round to nearest even).
template <> struct Codec<f16_t> {
    using R = float;
    static constexpr bool split = false;
    __device__ static R load(const GL f16_t *p)
    {
        return float(__builtin_bit_cast(_Float16, ld(reinterpret_cast<const GL uint16_t *>(p))));
    }
    __device__ static void store(GL f16_t *p, R v)
    {
        st(reinterpret_cast<GL uint16_t *>(p), __builtin_bit_cast(uint16_t, _Float16(v)));
    }
};

// Split 16-bit codecs: population q of a cell is w_q m + r_q, where m (about
// the cell's population sum, i.e. drho for the hydrodynamic lattice and eps C
// or rho_1 for the second one) is kept in an FP32 plane and only the
// remainder r_q -- the velocity and non-equilibrium part, orders of magnitude
// below w_q m in low-Mach porous flow -- is rounded to 16 bits.  The stored m
// absorbs the rounding of the remainders, so that the decoded populations sum
// to the cell's population sum (store_all in kernels.hpp).
struct bf16s_t { uint16_t v; };
struct f16s_t { uint16_t v; };

template <> struct Codec<bf16s_t> {
    using R = float;
    static constexpr bool split = true;
    __device__ static R load(const GL bf16s_t *p)
    {
        // Converting through the __bf16 type keeps this a plain 16-bit load
        // followed by a shift.  Written as an integer shift, the shift can be
        // folded into a load into the high half of a register (tied to that
        // register's old value), which serialised the split pulls.
        return float(__builtin_bit_cast(__bf16, ld(reinterpret_cast<const GL uint16_t *>(p))));
    }
    __device__ static void store(GL bf16s_t *p, R v) { Codec<bf16_t>::store(reinterpret_cast<GL bf16_t *>(p), v); }
    // the 16-bit word of v (rounded to nearest even) and its value
    __device__ static uint16_t enc(R v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
    __device__ static R dec(uint16_t b) { return float(__builtin_bit_cast(__bf16, b)); }
    __device__ static void store_bits(GL bf16s_t *p, uint16_t b) { st(reinterpret_cast<GL uint16_t *>(p), b); }
};

template <> struct Codec<f16s_t> {
    using R = float;
    static constexpr bool split = true;
    __device__ static R load(const GL f16s_t *p)
    {
        return Codec<f16_t>::load(reinterpret_cast<const GL f16_t *>(p));
    }
    __device__ static void store(GL f16s_t *p, R v) { Codec<f16_t>::store(reinterpret_cast<GL f16_t *>(p), v); }
    __device__ static uint16_t enc(R v) { return __builtin_bit_cast(uint16_t, _Float16(v)); }
    __device__ static R dec(uint16_t b) { return float(__builtin_bit_cast(_Float16, b)); }
    __device__ static void store_bits(GL f16s_t *p, uint16_t b) { st(reinterpret_cast<GL uint16_t *>(p), b); }
};

// Paired 16-bit storage: the value of a link in both lattices of the
// miscible model (f_q and h_q), which a step pulls from the same upstream
// cell, side by side in one 32-bit word (f_q in the low half).  One 32-bit
// access then serves the two 16-bit values: streams of 4-byte elements run at
// the rate of FP32 planes, while 2-byte elements cost a streaming probe 7% of
// its rate at 256^3 and 512^3.  Each half is rounded exactly as the unpaired
// codec rounds it.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));

template <class S> struct PairCodec;

template <> struct PairCodec<bf16_t> {
    using W = uint32_t;
    using R = float;
    __device__ static void decode(W w, R &a, R &b)
    {
        a = __uint_as_float(w << 16);
        b = __uint_as_float(w & 0xffff0000u);
    }
    __device__ static W encode(R a, R b)
    {
        const bf16x2_t v = {(__bf16)a, (__bf16)b};
        return __builtin_bit_cast(uint32_t, v);
    }
    __device__ static void load(const GL W *p, R &a, R &b) { decode(ld(p), a, b); }
    __device__ static void store(GL W *p, R a, R b) { st(p, encode(a, b)); }
};

template <> struct PairCodec<f16_t> {
    using W = uint32_t;
    using R = float;
    __device__ static void decode(W w, R &a, R &b)
    {
        const f16x2_t v = __builtin_bit_cast(f16x2_t, w);
        a = float(v.x);
        b = float(v.y);
    }
    __device__ static W encode(R a, R b)
    {
        const f16x2_t v = {_Float16(a), _Float16(b)};
        return __builtin_bit_cast(uint32_t, v);
    }
    __device__ static void load(const GL W *p, R &a, R &b) { decode(ld(p), a, b); }
    __device__ static void store(GL W *p, R a, R b) { st(p, encode(a, b)); }
};

// the split codecs pair their 16-bit remainders the same way (and their two
// FP32 masses as one 8-byte pair per cell)
template <> struct PairCodec<bf16s_t> : PairCodec<bf16_t> {};
template <> struct PairCodec<f16s_t> : PairCodec<f16_t> {};

}  // namespace plbm

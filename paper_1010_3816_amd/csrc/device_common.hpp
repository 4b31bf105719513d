// Device-side building blocks shared by the forward step kernel
// (lw_kernels.hip) and the adjoint step kernel (adjoint_kernels.hip):
// complex helpers, cross-lane moves, the coefficient reconstruction of
// Eq. (1) from the 1-D radial and angular tables, and the pieces of S and D.
#pragma once

#include "internal.hpp"

namespace teuk {
namespace {

struct cd {
    double re, im;
};

__device__ __forceinline__ cd cadd(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd csub(cd a, cd b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cd cscale(double s, cd a) { return {s * a.re, s * a.im}; }
__device__ __forceinline__ cd cavg(cd a, cd b) { return {0.5 * (a.re + b.re), 0.5 * (a.im + b.im)}; }

// Cross-lane moves: lane L receives the value held by lane L+1 / lane L-1,
// as two 32-bit DPP wavefront shifts (wave_shl:1 / wave_shr:1).  The edge
// lanes (63 and 0) receive 0; their results are never stored.
constexpr int kDppWaveShl1 = 0x130;
// Rows of input loaded ahead of the row being finished, and the minimum
// wavefronts per SIMD the register allocation must allow (build-time tuning).
#ifndef TEUK_ROWS_IN_FLIGHT
#define TEUK_ROWS_IN_FLIGHT 3
#endif
#ifndef TEUK_WAVES_PER_SIMD
#define TEUK_WAVES_PER_SIMD 2
#endif
constexpr int kRowsInFlight = TEUK_ROWS_IN_FLIGHT;
// The same for the two-step pass, whose row loop takes rows in pairs.
constexpr int kRowsInFlight2 = 2;
constexpr int kDppWaveShr1 = 0x138;

// bound_ctrl: a lane whose source lane does not exist reads 0, so the
// destination needs no initialisation.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_right(double v) { return dpp_move<kDppWaveShl1>(v); }
__device__ __forceinline__ double from_left(double v) { return dpp_move<kDppWaveShr1>(v); }
__device__ __forceinline__ cd from_right(cd v) { return {from_right(v.re), from_right(v.im)}; }
__device__ __forceinline__ cd from_left(cd v) { return {from_left(v.re), from_left(v.im)}; }

// The coefficients of the first-order system at one (position, row), with
// the difference-operator scalings folded in: a2s = A2/dth^2, a1s = A1/(2 dth).
struct Coef {
    double b, cre, cim, ctr, cti, a2s, a1s, v0r, v0i;
};

struct Rad {
    double rho, rho2, a2d, rb1, rb2, rb3, ctr, cti0, cti1, b1n, dl2, v0r, v0i;
};

struct Ang {
    double sn2, cs, cotp, pd;
};

// Typed pointers for the tile sweep: state in global memory (address space
// 1) and the coefficient tables, read-only for a launch, in the constant
// address space (4), so that wavefront-uniform table reads become scalar
// loads even where the pointers come from a descriptor in memory.
typedef double v2d __attribute__((ext_vector_type(2)));
typedef const __attribute__((address_space(1))) v2d* gin_t;
typedef __attribute__((address_space(1))) v2d* gout_t;
typedef const __attribute__((address_space(4))) double* ctab_t;
typedef const __attribute__((address_space(4))) ExtPoint* cext_t;

__device__ __forceinline__ Rad load_rad(ctab_t rad, int pitch, int kind, int pos) {
    auto f = [&](int field) { return rad[((size_t)field * 2 + kind) * pitch + pos]; };
    Rad R;
    R.rho = f(R_RHO);
    R.rho2 = f(R_RHO2);
    R.a2d = f(R_A2D);
    R.rb1 = f(R_RB1);
    R.rb2 = f(R_RB2);
    R.rb3 = f(R_RB3);
    R.ctr = f(R_CTR);
    R.cti0 = f(R_CTI0);
    R.cti1 = f(R_CTI1);
    R.b1n = f(R_B1N);
    R.dl2 = f(R_DL2);
    R.v0r = f(R_V0R);
    R.v0i = f(R_V0I);
    return R;
}

__device__ __forceinline__ Ang load_ang(ctab_t ang, int nth, int j) {
    (void)nth;
    const size_t o = (size_t)j * kNumAng;
    Ang G;
    G.sn2 = ang[o + A_SN2];
    G.cs = ang[o + A_CS];
    G.cotp = ang[o + A_COTP];
    G.pd = ang[o + A_PD];
    return G;
}

__device__ __forceinline__ Rad load_rad(const double* __restrict__ rad, int pitch, int kind, int pos) {
    auto f = [&](int field) { return rad[((size_t)field * 2 + kind) * pitch + pos]; };
    Rad R;
    R.rho = f(R_RHO);
    R.rho2 = f(R_RHO2);
    R.a2d = f(R_A2D);
    R.rb1 = f(R_RB1);
    R.rb2 = f(R_RB2);
    R.rb3 = f(R_RB3);
    R.ctr = f(R_CTR);
    R.cti0 = f(R_CTI0);
    R.cti1 = f(R_CTI1);
    R.b1n = f(R_B1N);
    R.dl2 = f(R_DL2);
    R.v0r = f(R_V0R);
    R.v0i = f(R_V0I);
    return R;
}

__device__ __forceinline__ Ang load_ang(const double* ang, int nth, int j) {
    (void)nth;
    const size_t o = (size_t)j * kNumAng;
    Ang G;
    G.sn2 = ang[o + A_SN2];
    G.cs = ang[o + A_CS];
    G.cotp = ang[o + A_COTP];
    G.pd = ang[o + A_PD];
    return G;
}

// 1/Sigma and 1/Sigma^2 at one (position, row).
struct Sig {
    double isig, inv;
};

// Sigma^2 = rho^2 - a^2 Delta sin^2(theta) > 0.  1/Sigma from the hardware
// reciprocal square root (about 23 correct bits) refined by two Newton steps
// for x^{-1/2}, y <- y + y (1 - x y^2) / 2, each of which doubles the number
// of correct bits; 1/Sigma^2 = y^2.  Both are within a few ulp of the
// correctly rounded values, in 10 instructions instead of the 28 of a
// division and a square root.
#ifndef TEUK_RSQ_NEWTON
#define TEUK_RSQ_NEWTON 1
#endif
__device__ __forceinline__ Sig kerr_sigma(const Rad& R, const Ang& G) {
    const double sig2 = fma(-R.a2d, G.sn2, R.rho2);
#if TEUK_RSQ_NEWTON
    double y = __builtin_amdgcn_rsq(sig2);
    double e = fma(-sig2 * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-sig2 * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    return {y, y * y};
#else
    const double inv = 1.0 / sig2;
    return {sqrt(inv), inv};
#endif
}

// Eq. (1) coefficients from the factored tables (see RadField / AngField).
__device__ __forceinline__ Coef kerr_coef(const Rad& R, const Ang& G, Sig s) {
    Coef c;
    c.b = R.rho * s.isig;
    const double bp = s.isig * fma(-fma(-R.rb3, G.sn2, R.rb2), s.inv, R.rb1);
    c.ctr = R.ctr * s.inv;
    c.cti = fma(R.cti1, G.cs, R.cti0) * s.inv;
    const double b1 = R.b1n * s.inv;
    c.cre = fma(c.b, bp - c.ctr, -b1);
    c.cim = -c.b * c.cti;
    c.a2s = R.dl2 * s.inv;
    c.a1s = c.a2s * G.cotp;
    c.v0r = fma(R.dl2, G.pd, R.v0r) * s.inv;
    c.v0i = R.v0i * s.inv;
    return c;
}

__device__ __forceinline__ Coef user_coef(ctab_t u, int nth, int pitch, int j, int pos, double inv_dth2,
                                          double inv_2dth) {
    auto f = [&](int k) { return u[((size_t)k * nth + j) * pitch + pos]; };
    Coef c;
    c.b = f(U_B);
    c.cre = f(U_CRE);
    c.cim = f(U_CIM);
    c.ctr = f(U_CTRE);
    c.cti = f(U_CTIM);
    c.a2s = f(U_A2) * inv_dth2;
    c.a1s = f(U_A1) * inv_2dth;
    c.v0r = f(U_V0RE);
    c.v0i = f(U_V0IM);
    return c;
}

// Pi row of S:  -Ct q + A2 (f_{j+1} - 2 f_j + f_{j-1})/dth^2
//               + A1 (f_{j+1} - f_{j-1})/(2 dth) - V0 f_j
__device__ __forceinline__ cd s_pi(const Coef& k, cd fm, cd f0, cd fp, cd q) {
    const double lr = (fp.re + fm.re) - 2.0 * f0.re;
    const double li = (fp.im + fm.im) - 2.0 * f0.im;
    const double gr = fp.re - fm.re;
    const double gi = fp.im - fm.im;
    double sr = fma(k.a2s, lr, k.a1s * gr);
    double si = fma(k.a2s, li, k.a1s * gi);
    sr -= fma(k.ctr, q.re, -k.cti * q.im);
    si -= fma(k.ctr, q.im, k.cti * q.re);
    sr -= fma(k.v0r, f0.re, -k.v0i * f0.im);
    si -= fma(k.v0r, f0.im, k.v0i * f0.re);
    return {sr, si};
}

// D applied to (dP, dQ), Pi row:  c dP - b dQ.
__device__ __forceinline__ cd d_pi(const Coef& k, cd dP, cd dQ) {
    return {fma(k.cre, dP.re, fma(-k.cim, dP.im, -k.b * dQ.re)),
            fma(k.cre, dP.im, fma(k.cim, dP.re, -k.b * dQ.im))};
}

// Workgroups are dispatched round-robin over the 8 XCDs; map them so that
// each XCD (own L2) receives a contiguous range of tiles, i.e. neighbouring
// strips whose halo columns overlap.  Used by the adjoint kernels (measured
// slightly faster with it); the forward passes keep dispatch order.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    constexpr int X = 8;
    const int x = b % X, idx = b / X, per = nb / X, rem = nb % X;
    return x * per + min(x, rem) + idx;
}

// Loads always read a valid (clamped) address, so the load itself is
// unconditional and stays in flight until it is needed; where a column's
// value must not be used it is zeroed by a bit mask at its point of use.
__device__ __forceinline__ cd ld(const double2* __restrict__ p, size_t o) {
    const double2 v = p[o];
    return {v.x, v.y};
}

__device__ __forceinline__ cd masked(cd v, unsigned long long mask) {
    return {__longlong_as_double(__double_as_longlong(v.re) & mask),
            __longlong_as_double(__double_as_longlong(v.im) & mask)};
}

__device__ __forceinline__ cd ld(gin_t p, size_t o) {
    const v2d v = p[o];
    return {v.x, v.y};
}

// Streaming store of one complex value (16 B, one dwordx4 per lane): the
// value is not read again by this launch and, for a window slot, not soon.
__device__ __forceinline__ void st(double2* p, size_t o, cd v) {
    v2d w;
    w.x = v.re;
    w.y = v.im;
    __builtin_nontemporal_store(w, reinterpret_cast<v2d*>(p + o));
}

__device__ __forceinline__ void st(gout_t p, size_t o, cd v) {
    v2d w;
    w.x = v.re;
    w.y = v.im;
    __builtin_nontemporal_store(w, p + o);
}

// Store of a state the next launch reads.  KEEP: an ordinary store, whose
// line stays in the device's last-level cache, so the next launch reads it
// from there when the states fit (the host picks the kernel instance);
// otherwise streaming, which leaves the cache to the input.  The choice is
// made at compile time: with a run-time branch between the two, the
// compiler merges them into one store to the same address and drops the
// non-temporal hint.
template <int KEEP>
__device__ __forceinline__ void st_state(double2* p, size_t o, cd v) {
    if constexpr (KEEP) {
        v2d w;
        w.x = v.re;
        w.y = v.im;
        *reinterpret_cast<v2d*>(p + o) = w;
    } else {
        st(p, o, v);
    }
}

template <int KEEP>
__device__ __forceinline__ void st_state(gout_t p, size_t o, cd v) {
    if constexpr (KEEP) {
        v2d w;
        w.x = v.re;
        w.y = v.im;
        p[o] = w;
    } else {
        st(p, o, v);
    }
}

// Row access through buffer resources.  A resource describes one row of one
// plane: its base address sits in scalar registers and each lane addresses
// its column by a fixed byte offset, so moving to another row costs scalar
// arithmetic only.  The hardware checks every lane's offset against the
// resource's size and drops a store that falls outside it: a lane that must
// not write gets the offset kOffNone, so stores need no branch on the lane
// mask, and the compiler's waits on the memory counter, which count every
// store on every path, stay as loose as the loads allow.
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
constexpr int kRsrcWord3 = 0x00020000;      // raw buffer, 32-bit data format
constexpr uint32_t kOffNone = 0x80000000u;  // past the end of any row (at most 2^24 columns, 256 MiB)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(gin_t row, int32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)row, (short)0, bytes, kRsrcWord3);
}
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const double2* row, int32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<double2*>(row), (short)0, bytes, kRsrcWord3);
}

__device__ __forceinline__ cd ld_row(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    const v2d v = __builtin_bit_cast(v2d, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
    return {v.x, v.y};
}

// Immediate of s_waitcnt (gfx9 encoding: vmcnt in bits 3:0 and 15:14,
// expcnt 6:4, lgkmcnt 11:8) that waits until at most n vector memory
// operations are outstanding and leaves the other counters alone.
constexpr int waitcnt_vm(int n) { return (n & 0xF) | (0x7 << 4) | (0xF << 8) | ((n >> 4) << 14); }

// KEEP as in st_state: 0 streaming (non-temporal), 1 an ordinary store.
template <int KEEP>
__device__ __forceinline__ void st_row(__amdgpu_buffer_rsrc_t r, uint32_t off, cd v) {
    v2d w;
    w.x = v.re;
    w.y = v.im;
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4u, w), r, off, 0, KEEP ? 0 : 2);
}

// All pointers are distinct allocations (restrict): the uniform reads of
// the angular tables and extraction descriptors become scalar loads.
}  // namespace
}  // namespace teuk

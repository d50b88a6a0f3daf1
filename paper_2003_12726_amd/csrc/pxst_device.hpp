// Device helpers: reference lookups, compensated sums, wave reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pxst {

__device__ inline float qnan() { return __int_as_float(0x7fc00000); }
__device__ inline bool valid(float v) { return v == v; }

// Nearest integer with halves rounded up, from floor and a fraction test (exact in
// float32, unlike floor(x + 0.5) just below one half).
__device__ inline int round_half_up(float x) {
    const float f = floorf(x);
    return (int)f + ((x - f) >= 0.5f ? 1 : 0);
}

// Candidate-window centre of a map value: round-half-up of the value clamped to
// +-1e8 (a map that far out has no valid lookups anyway).
__device__ inline int window_centre(float u) {
    return round_half_up(fminf(fmaxf(u, -1.0e8f), 1.0e8f));
}

// Integer part and non-negative fraction of a translation along one axis, arranged
// for a lookup at (integer target) - dx - origin: the lookup lands on corner
// target - e with fractional weight t in [0, 1).
struct AxisShift {
    int e;      // floor(dx) + origin + (frac(dx) > 0)
    float t;    // 1 - frac(dx) if frac(dx) > 0, else 0
};
__device__ inline AxisShift axis_shift(float d, int origin) {
    const float s = floorf(d);
    const float f = d - s;
    AxisShift r;
    r.e = (int)s + origin + (f > 0.f ? 1 : 0);
    r.t = f > 0.f ? 1.f - f : 0.f;
    return r;
}

// Masked bilinear interpolation (Sec. 4): corners (a0, b0) .. (a0+1, b0+1) of the
// reference with weights from the fractions (fa, fb).  Unknown corners (NaN) and
// corners outside the grid are dropped and the weights renormalised.  Returns NaN
// when no corner with non-zero weight is known.
__device__ inline float masked_bilinear(const float* __restrict__ refv, int Rs, int Rf, int a0,
                                        int b0, float fa, float fb) {
    const bool r0 = a0 >= 0 && a0 < Rs, r1 = a0 + 1 >= 0 && a0 + 1 < Rs;
    const bool c0 = b0 >= 0 && b0 < Rf, c1 = b0 + 1 >= 0 && b0 + 1 < Rf;
    const size_t base = (size_t)a0 * Rf + b0;
    const float v00 = (r0 && c0) ? refv[base] : qnan();
    const float v01 = (r0 && c1) ? refv[base + 1] : qnan();
    const float v10 = (r1 && c0) ? refv[base + Rf] : qnan();
    const float v11 = (r1 && c1) ? refv[base + Rf + 1] : qnan();
    if (valid(v00) && valid(v01) && valid(v10) && valid(v11)) {
        const float h0 = fmaf(fb, v01 - v00, v00);
        const float h1 = fmaf(fb, v11 - v10, v10);
        return fmaf(fa, h1 - h0, h0);
    }
    const float ga = 1.f - fa, gb = 1.f - fb;
    const float w00 = ga * gb, w01 = ga * fb, w10 = fa * gb, w11 = fa * fb;
    float num = 0.f, den = 0.f;
    if (valid(v00)) { num = fmaf(w00, v00, num); den += w00; }
    if (valid(v01)) { num = fmaf(w01, v01, num); den += w01; }
    if (valid(v10)) { num = fmaf(w10, v10, num); den += w10; }
    if (valid(v11)) { num = fmaf(w11, v11, num); den += w11; }
    return den > 0.f ? num / den : qnan();
}

// Same lookup with all four corners known to be valid and inside the grid.
__device__ inline float bilinear4(float v00, float v01, float v10, float v11, float fa, float fb) {
    const float h0 = fmaf(fb, v01 - v00, v00);
    const float h1 = fmaf(fb, v11 - v10, v10);
    return fmaf(fa, h1 - h0, h0);
}

// Error-free transformation of s + p: s <- fl(s + p), p <- the rounding error.  Used
// to fold a block partial sum into a running total, carrying the lost low part into
// the next block (compensated summation across blocks of frames).
__device__ inline void two_sum_fold(float& s, float& p) {
    const float t = s + p;
    const float bp = t - s;
    const float e = (s - (t - bp)) + (p - bp);
    s = t;
    p = e;
}

// Kahan step: add x to (s, c).
__device__ inline void kahan_add(float& s, float& c, float x) {
    const float y = x - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

// Normalised error of a candidate with the empty / zero-variance cases.
__device__ inline float normalised_error(float err, float var, int nv) {
    if (nv <= 0) return INFINITY;
    if (var > 0.f) return err / var;
    return err == 0.f ? 0.f : INFINITY;
}

// The same for a pixel whose white-field value is 0: every residual I - W g is then
// the count I itself, so over any set of valid frames the error equals the variance
// and E is exactly 1 (0 when every such count is 0).  Kernels that sum the error and
// the variance in different orders use this form, so that all candidates of such a
// pixel tie exactly and the first one wins, as the exact quotient has it.
__device__ inline float zero_white_error(float err, int nv) {
    if (nv <= 0) return INFINITY;
    return err > 0.f ? 1.f : 0.f;
}

// Paraboloid refinement on a 3x3 stencil E[x+1][y+1] (least-squares fit of
// q0 + q1 x + q2 y + q3 x^2 + q4 x y + q5 y^2 over x, y in {-1, 0, 1}); the vertex
// is accepted only for a minimum and clamped to +-0.5.
__device__ inline void refine_3x3(const float* E, float& ox, float& oy) {
    float s0 = 0.f, sxp = 0.f, sxm = 0.f, syp = 0.f, sym = 0.f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int b = 0; b < 3; ++b) s0 += E[a * 3 + b];
    }
#pragma unroll
    for (int b = 0; b < 3; ++b) { sxm += E[0 * 3 + b]; sxp += E[2 * 3 + b]; }
#pragma unroll
    for (int a = 0; a < 3; ++a) { sym += E[a * 3 + 0]; syp += E[a * 3 + 2]; }
    const float q1 = (sxp - sxm) / 6.f;
    const float q2 = (syp - sym) / 6.f;
    const float q4 = (E[8] - E[6] - E[2] + E[0]) / 4.f;
    const float q3 = (sxp + sxm) / 2.f - s0 / 3.f;
    const float q5 = (syp + sym) / 2.f - s0 / 3.f;
    const float D = 4.f * q3 * q5 - q4 * q4;
    ox = 0.f;
    oy = 0.f;
    if (q3 > 0.f && D > 0.f) {
        ox = fminf(fmaxf((q4 * q2 - 2.f * q5 * q1) / D, -0.5f), 0.5f);
        oy = fminf(fmaxf((q4 * q1 - 2.f * q3 * q2) / D, -0.5f), 0.5f);
    }
}

// Three-point parabola vertex, accepted only for a minimum, clamped to +-0.5.
__device__ inline float refine_3pt(float em, float e0, float ep) {
    const float c = em - 2.f * e0 + ep;
    if (!(c > 0.f)) return 0.f;
    return fminf(fmaxf((em - ep) / (2.f * c), -0.5f), 0.5f);
}

// Refinement offset at integer minimum (kx, ky) (0-based window indices) given the
// 3x3 stencil around it (entries outside the window unused).
__device__ inline void refine_at(const float* st, int kx, int ky, int nx, int ny, float& ox,
                                 float& oy) {
    ox = 0.f;
    oy = 0.f;
    const int rx = nx / 2, ry = ny / 2;
    const int kxs = kx - rx, kys = ky - ry;
    if (rx > 0 && ry > 0) {
        if (abs(kxs) < rx && abs(kys) < ry) {
            bool fin = true;
#pragma unroll
            for (int q = 0; q < 9; ++q) fin = fin && isfinite(st[q]);
            if (fin) refine_3x3(st, ox, oy);
        }
    } else if (rx > 0) {
        if (abs(kxs) < rx && isfinite(st[1]) && isfinite(st[4]) && isfinite(st[7]))
            ox = refine_3pt(st[1], st[4], st[7]);
    } else if (ry > 0) {
        if (abs(kys) < ry && isfinite(st[3]) && isfinite(st[4]) && isfinite(st[5]))
            oy = refine_3pt(st[3], st[4], st[5]);
    }
}

// (value, index) order: smaller value first, lower index on ties.
__device__ inline bool better(float e, int k, float be, int bk) {
    return e < be || (e == be && k < bk);
}

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over the 64 lanes of a wave with data-parallel-primitive moves instead of LDS
// permutes: xor 1 and xor 2 inside quads, then the mirrors of half-rows and rows (each
// lane then holds its 16-lane row's sum), then the four row sums read from lanes 0, 16,
// 32 and 48 and added in that order.  The result is uniform across the wave.  Every lane
// must be active.
template <int CTRL>
__device__ inline float dpp_f32(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, false));
}
__device__ inline float wave_total(float v) {
    v += dpp_f32<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp_f32<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp_f32<0x141>(v);   // row_half_mirror
    v += dpp_f32<0x140>(v);   // row_mirror
    const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return ((r0 + r1) + r2) + r3;
}
__device__ inline int wave_total(int v) {
    v += __builtin_amdgcn_mov_dpp(v, 0xB1, 0xf, 0xf, false);
    v += __builtin_amdgcn_mov_dpp(v, 0x4E, 0xf, 0xf, false);
    v += __builtin_amdgcn_mov_dpp(v, 0x141, 0xf, 0xf, false);
    v += __builtin_amdgcn_mov_dpp(v, 0x140, 0xf, 0xf, false);
    return ((__builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16)) +
            __builtin_amdgcn_readlane(v, 32)) + __builtin_amdgcn_readlane(v, 48);
}

__device__ inline int wave_min_i(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ inline int wave_max_i(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}


// Arguments of a kernel that serves one job (passed by value) or a table of jobs in
// device memory (the job index is blockIdx.z).  The form is a compile-time choice: a
// run-time select between the two would take the by-value arguments' address and move
// them from scalar to vector registers.
// The table is read through the constant address space, so that the loads are scalar
// and the arguments stay in scalar registers in both forms (the table is not written
// while a kernel runs).
// Entry j (wave-uniform) of a job table in device memory, read through the constant
// address space (scalar loads, arguments in scalar registers).
template <class X>
__device__ __forceinline__ X table_entry(const X* __restrict__ jobs, int j) {
    typedef const __attribute__((address_space(4))) X* ConstPtr;
    X out;
    __builtin_memcpy(&out, (ConstPtr)jobs + j, sizeof(X));
    return out;
}

template <bool BATCH, class X>
__device__ __forceinline__ X job_args(const X* __restrict__ jobs, const X& one) {
    if constexpr (BATCH) {
        typedef const __attribute__((address_space(4))) X* ConstPtr;
        X out;
        __builtin_memcpy(&out, (ConstPtr)jobs + blockIdx.z, sizeof(X));
        return out;
    } else {
        return one;
    }
}

// Work item of block b out of n items.  Work-groups go to the eight XCDs in turn
// (block b to XCD b mod 8) and each XCD has its own L2, so consecutive items of the
// work list -- neighbouring tiles, whose regions overlap -- would each be read into a
// different L2.  Instead each XCD takes one contiguous run of the list: XCD x holds
// the items [x q + min(x, r), ...) with q = n / 8, r = n mod 8 (a bijection of [0, n)).
__device__ inline int xcd_item(int b, int n) {
    if (b >= n) return b;
    const int x = b & 7, i = b >> 3, q = n >> 3, r = n & 7;
    return x * q + min(x, r) + i;
}

}  // namespace pxst

// Translation search (Sec. 2.2.3): for each frame, the error integrated over the
// detector for integer shifts of that frame's translation, first minimum and
// paraboloid refinement.
//
// Pass 0 (one work-group per 64 x 64 detector tile): the bounding box of the integer
// parts of the map over the tile's good pixels (it does not depend on the frame).
// Pass 1 (grid: tiles x frames): the work-group stages in LDS the reference region that
// the tile's lookups of this frame can reach, for every shift (the box moved by the
// frame's integer shift, widened by the window and one cell); each thread takes 16
// pixels of the tile (one column, every fourth row), reads each pixel's
// (2Tx+2) x (2Ty+2) neighbourhood from LDS and forms all shifted lookups from it (the
// bilinear fractions do not depend on the integer shift): the neighbourhood's rows are
// interpolated along the fast axis once and the results along the slow axis per shift;
// a neighbourhood with an invalid value (NaN: invalid reference pixel or outside the
// grid, which the sum of the row interpolations reveals) takes the masked form per
// shift instead.  A tile whose region exceeds the LDS reads the neighbourhoods from the
// reference directly.  Per-shift sums are reduced over the work-group and written as
// per-tile partials.  Pass 2 (one wave per frame) adds the partials with compensated
// float32 sums in a fixed order, normalises, takes the first minimum and refines.
#include "pxst_device.hpp"
#include "pxst_internal.hpp"

namespace pxst {

namespace {


// Pass 0: integer bounding box of the map over each tile's good pixels (min > max when
// the tile has none; |u| beyond 2^24 marks the box as unusable).
template <bool BATCH>
__global__ __launch_bounds__(256) void k_tr_bbox(const TrArgs* __restrict__ jobs, TrArgs one) {
    const TrArgs a = job_args<BATCH>(jobs, one);
    const int tile = blockIdx.x;
    if (tile >= a.nblk) return;
    const int ty = tile / a.tiles_x, tx = tile - ty * a.tiles_x;
    const size_t HW = (size_t)a.H * a.W;
    int mn0 = INT_MAX, mx0 = INT_MIN, mn1 = INT_MAX, mx1 = INT_MIN;
    for (int e = threadIdx.x; e < TR_TILE * TR_TILE; e += 256) {
        const int i = ty * TR_TILE + e / TR_TILE, j = tx * TR_TILE + e % TR_TILE;
        if (i >= a.H || j >= a.W) continue;
        const size_t pix = (size_t)i * a.W + j;
        if (a.mask[pix] == 0) continue;
        const float u0 = a.u[pix], u1 = a.u[HW + pix];
        const bool ok = fabsf(u0) < 16777216.f && fabsf(u1) < 16777216.f;
        const int f0 = ok ? (int)floorf(u0) : INT_MIN / 4, f1 = ok ? (int)floorf(u1) : INT_MIN / 4;
        mn0 = min(mn0, f0);
        mx0 = max(mx0, ok ? f0 : INT_MAX / 4);
        mn1 = min(mn1, f1);
        mx1 = max(mx1, ok ? f1 : INT_MAX / 4);
    }
    mn0 = wave_min_i(mn0);
    mx0 = wave_max_i(mx0);
    mn1 = wave_min_i(mn1);
    mx1 = wave_max_i(mx1);
    __shared__ int4 red[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = make_int4(mn0, mx0, mn1, mx1);
    __syncthreads();
    if (threadIdx.x == 0) {
        int4 b = red[0];
        for (int w = 1; w < 4; ++w) {
            b.x = min(b.x, red[w].x);
            b.y = max(b.y, red[w].y);
            b.z = min(b.z, red[w].z);
            b.w = max(b.w, red[w].w);
        }
        a.bbox[tile] = b;
    }
}

// One pixel's contribution to every shift's sums.  The neighbourhood holds rows
// a0 - TX .. a0 + TX + 1 and columns b0 - TY .. b0 + TY + 1; shift (sx, sy) looks up
// corner rows a0 - sx, a0 - sx + 1 and columns b0 - sy, b0 - sy + 1, i.e. neighbourhood
// rows and columns ix = TX - sx + {0, 1}, iy = TY - sy + {0, 1}.
//
// tr_fast: every lookup valid; h[r][c] is row r interpolated along the fast axis between
// columns c and c + 1 (the fractions do not depend on the shift).  With the white field
// folded into the slow-axis weights, the residual of a shift is I - W g =
// I + A h[ix][iy] + B h[ix + 1][iy] with A = -W (1 - fa), B = -W fa: two FMAs, and one
// more for its square.
template <int TX, int TY>
__device__ __forceinline__ void tr_fast(const float (&h)[2 * TX + 2][2 * TY + 1], float fa, float I, float Wp,
                                        bool good, float (&err)[(2 * TX + 1) * (2 * TY + 1)], float& vC,
                                        int& cC) {
    constexpr int NXs = 2 * TX + 1, NYs = 2 * TY + 1;
    const float v = I - Wp;
    const float A = -Wp * (1.f - fa), B = -Wp * fa;
#pragma unroll
    for (int ix = 0; ix < NXs; ++ix) {
#pragma unroll
        for (int iy = 0; iy < NYs; ++iy) {
            const int s = (TX - ix + TX) * NYs + (TY - iy + TY);
            const float rr = fmaf(B, h[ix + 1][iy], fmaf(A, h[ix][iy], I));
            err[s] = fmaf(rr, rr, err[s]);
        }
    }
    vC = fmaf(v, v, vC);
    cC += good ? 1 : 0;
}

// tr_masked: some neighbourhood value is invalid (NaN): the masked bilinear form of
// Sec. 4 per shift; a shift whose lookup has no valid corner drops the pixel.
template <int TX, int TY>
__device__ __forceinline__ void tr_masked(const float (&nb)[2 * TX + 2][2 * TY + 2], float fa, float fb,
                                          float I, float Wp, bool good,
                                          float (&err)[(2 * TX + 1) * (2 * TY + 1)],
                                          float (&var)[(2 * TX + 1) * (2 * TY + 1)], unsigned& anyv) {
    constexpr int NXs = 2 * TX + 1, NYs = 2 * TY + 1;
    const float v = I - Wp, v2 = v * v;
#pragma unroll
    for (int ix = 0; ix < NXs; ++ix) {
#pragma unroll
        for (int iy = 0; iy < NYs; ++iy) {
            const float v00 = nb[ix][iy], v01 = nb[ix][iy + 1], v10 = nb[ix + 1][iy],
                        v11 = nb[ix + 1][iy + 1];
            const float ga = 1.f - fa, gb = 1.f - fb;
            float num = 0.f, den = 0.f;
            if (valid(v00)) { num = fmaf(ga * gb, v00, num); den += ga * gb; }
            if (valid(v01)) { num = fmaf(ga * fb, v01, num); den += ga * fb; }
            if (valid(v10)) { num = fmaf(fa * gb, v10, num); den += fa * gb; }
            if (valid(v11)) { num = fmaf(fa * fb, v11, num); den += fa * fb; }
            const float g = den > 0.f ? num / den : qnan();
            const int s = (TX - ix + TX) * NYs + (TY - iy + TY);
            if (good && valid(g)) {
                const float rr = fmaf(-Wp, g, I);
                err[s] = fmaf(rr, rr, err[s]);
                var[s] += v2;
                anyv |= 1u << s;
            }
        }
    }
}

// a NaN anywhere in the neighbourhood reaches the sum of its row interpolations
template <int TX, int TY>
__device__ __forceinline__ bool rows_valid(const float (&h)[2 * TX + 2][2 * TY + 1]) {
    float chk = 0.f;
#pragma unroll
    for (int r = 0; r < 2 * TX + 2; ++r)
#pragma unroll
        for (int c = 0; c < 2 * TY + 1; ++c) chk += h[r][c];
    return valid(chk);
}

// Per-frame constants of the pixel loop.
struct TrFrame {
    const uint16_t* fr;
    float fd0, fd1;
    int is0, is1;
    const float* reg;   // staged region: rows from R0, columns from C0, pitch RW
    int R0, C0, RW;
};

// The 16 pixels of a thread (column j of its tile, rows wave, wave + 4, ...): each
// pixel's neighbourhood from the staged region (STAGED) or from the reference, then its
// contribution to every shift.  CHECK: the neighbourhoods may hold invalid values; a
// pixel whose neighbourhood does is noted and evaluated in the masked form after the
// others (so that the per-shift variance sums are live only then).  The next pixel's
// inputs are loaded while the current one is evaluated, and a pixel that is masked or
// outside the detector runs the same instructions with zero count and white-field, at
// the box corner (so that its reads stay inside the staged region), and adds nothing.
template <int TX, int TY, bool STAGED, bool CHECK>
__device__ __forceinline__ void tr_pixels(const TrArgs& a, const TrFrame& f, int i_first, int j, int4 bb,
                                          float (&err)[(2 * TX + 1) * (2 * TY + 1)],
                                          float (&var)[(2 * TX + 1) * (2 * TY + 1)], unsigned& anyv,
                                          float& vC, int& cC) {
    constexpr int CR = 2 * TY + 2, RR = 2 * TX + 2;
    constexpr int NM = TR_TILE / (TR_THREADS / 64);
    static_assert(NM <= 32, "one bit per pixel of a thread");
    const size_t HW = (size_t)a.H * a.W;
    auto fetch = [&](int m, bool& good, float& u0, float& u1, float& Wp, float& I) {
        const int i = i_first + (TR_THREADS / 64) * m;
        const bool in = m < NM && i < a.H && j < a.W;
        const size_t pix = in ? (size_t)i * a.W + j : 0;
        const unsigned mk = a.mask[pix];
        good = in & (mk != 0u);
        u0 = a.u[pix];
        u1 = a.u[HW + pix];
        Wp = a.white[pix];
        I = (float)f.fr[pix];
    };
    // lower corner of the neighbourhood's centre cell and the bilinear fractions
    auto place = [&](float u0, float u1, int& a0, int& b0, float& fa, float& fb) {
        const float f0 = floorf(u0), f1 = floorf(u1);
        const float t0 = (u0 - f0) - f.fd0, t1 = (u1 - f1) - f.fd1;
        a0 = (int)f0 - f.is0 - a.o0 - (t0 < 0.f ? 1 : 0);
        b0 = (int)f1 - f.is1 - a.o1 - (t1 < 0.f ? 1 : 0);
        fa = t0 < 0.f ? t0 + 1.f : t0;
        fb = t1 < 0.f ? t1 + 1.f : t1;
    };
    auto load_nb = [&](float (&nb)[RR][CR], int a0, int b0) {
        if (STAGED) {
            const float* q = f.reg + (a0 - TX - f.R0) * f.RW + (b0 - TY - f.C0);
#pragma unroll
            for (int r = 0; r < RR; ++r)
#pragma unroll
                for (int c = 0; c < CR; ++c) nb[r][c] = q[r * f.RW + c];
        } else {
#pragma unroll
            for (int r = 0; r < RR; ++r) {
                const int rr = a0 - TX + r;
#pragma unroll
                for (int c = 0; c < CR; ++c) {
                    const int cc = b0 - TY + c;
                    nb[r][c] = (rr >= 0 && rr < a.Rs && cc >= 0 && cc < a.Rf)
                                   ? a.refv[(size_t)rr * a.Rf + cc] : qnan();
                }
            }
        }
    };
    unsigned fail = 0u;   // pixels (bit m) left for the masked form
    bool g_n;
    float u0_n, u1_n, W_n, I_n;
    fetch(0, g_n, u0_n, u1_n, W_n, I_n);
#pragma unroll 2
    for (int m = 0; m < NM; ++m) {
        const bool good = g_n;
        const float u0 = good ? u0_n : (float)bb.x, u1 = good ? u1_n : (float)bb.z;
        const float Wp = good ? W_n : 0.f, I = good ? I_n : 0.f;
        fetch(m + 1, g_n, u0_n, u1_n, W_n, I_n);
        int a0, b0;
        float fa, fb;
        place(u0, u1, a0, b0, fa, fb);
        float h[RR][CR - 1];
        {
            float nb[RR][CR];
            load_nb(nb, a0, b0);
#pragma unroll
            for (int r = 0; r < RR; ++r)
#pragma unroll
                for (int c = 0; c < CR - 1; ++c) h[r][c] = fmaf(fb, nb[r][c + 1] - nb[r][c], nb[r][c]);
        }
        if (!CHECK || rows_valid<TX, TY>(h))
            tr_fast<TX, TY>(h, fa, I, Wp, good, err, vC, cC);
        else if (good)
            fail |= 1u << m;
    }
    if (CHECK) {
        while (fail) {
            const int m = __ffs(fail) - 1;
            fail &= fail - 1u;
            bool good;
            float u0, u1, Wp, I;
            fetch(m, good, u0, u1, Wp, I);
            int a0, b0;
            float fa, fb;
            place(u0, u1, a0, b0, fa, fb);
            float nb[RR][CR];
            load_nb(nb, a0, b0);
            tr_masked<TX, TY>(nb, fa, fb, I, Wp, good, err, var, anyv);
        }
    }
}

// Pass 1.  STAGED: the tiles whose region fits the LDS; the others (and tiles without a
// good pixel) in the launch without staging.  Every tile is written by exactly one.
template <int TX, int TY, bool STAGED, bool BATCH>
__global__ __launch_bounds__(TR_THREADS) void k_tr_partial(const TrArgs* __restrict__ jobs, TrArgs one) {
    constexpr int NXs = 2 * TX + 1, NYs = 2 * TY + 1, CT = NXs * NYs;
    __shared__ float reg[STAGED ? TR_LDS_FLOATS : 1];
    const TrArgs a = job_args<BATCH>(jobs, one);
    const int tile = blockIdx.x, n = blockIdx.y;
    if (tile >= a.nblk || n >= a.N) return;
    const int tyi = tile / a.tiles_x, txi = tile - tyi * a.tiles_x;
    const int4 bb = a.bbox[tile];
    const bool any_px = bb.x <= bb.y;
    const long long rh = (long long)bb.y - bb.x + 2 * TX + 3, rw = (long long)bb.w - bb.z + 2 * TY + 3;
    const bool fits = any_px && rh * rw <= TR_LDS_FLOATS;
    if (fits != STAGED) return;
    const size_t HW = (size_t)a.H * a.W;
    const float d0 = a.dx_in[2 * n], d1 = a.dx_in[2 * n + 1];
    const float s0 = floorf(d0), s1 = floorf(d1);
    TrFrame f;
    f.fr = a.frames + (size_t)n * HW;
    f.fd0 = d0 - s0;
    f.fd1 = d1 - s1;
    f.is0 = (int)s0;
    f.is1 = (int)s1;
    f.reg = reg;
    f.RW = STAGED ? (int)rw : 0;
    // the region of this frame's lookups: rows R0 .. R0 + rh - 1, columns C0 .. C0 + rw - 1
    f.R0 = bb.x - f.is0 - a.o0 - 1 - TX;
    f.C0 = bb.z - f.is1 - a.o1 - 1 - TY;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

    // staged region entirely valid (no invalid reference pixel, inside the grid): every
    // neighbourhood read from it is valid and skips the test
    bool region_ok = false;
    if (STAGED) {
        // wave w stages rows w, w + 4, ...: lanes take columns lane, lane + 64, ...; eight
        // rows' loads in flight at a time
        const int RH = (int)rh, RW = f.RW;
        bool bad = false;
        for (int r0 = wave; r0 < RH; r0 += 8 * (TR_THREADS / 64)) {
            for (int c = lane; c < RW; c += 64) {
                const int gc = f.C0 + c;
                const bool cin = gc >= 0 && gc < a.Rf;
                float vals[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int r = r0 + k * (TR_THREADS / 64), gr = f.R0 + r;
                    vals[k] = (r < RH && cin && gr >= 0 && gr < a.Rs) ? a.refv[(size_t)gr * a.Rf + gc] : qnan();
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int r = r0 + k * (TR_THREADS / 64);
                    if (r < RH) {
                        reg[r * RW + c] = vals[k];
                        bad = bad || !valid(vals[k]);
                    }
                }
            }
        }
        region_ok = !__syncthreads_or(bad ? 1 : 0);
    }

    // per shift: squared residuals; the variance of the pixels with a valid lookup is
    // common to all shifts for pixels whose whole neighbourhood is valid (vC, cC) and
    // kept per shift for the others (var, with a bit per shift set by any valid lookup)
    float err[CT], var[CT];
#pragma unroll
    for (int s = 0; s < CT; ++s) {
        err[s] = 0.f;
        var[s] = 0.f;
    }
    unsigned anyv = 0u;
    float vC = 0.f;
    int cC = 0;
    const int j = txi * TR_TILE + lane, i_first = tyi * TR_TILE + wave;
    if (any_px) {
        if (STAGED && region_ok)
            tr_pixels<TX, TY, STAGED, false>(a, f, i_first, j, bb, err, var, anyv, vC, cC);
        else
            tr_pixels<TX, TY, STAGED, true>(a, f, i_first, j, bb, err, var, anyv, vC, cC);
    }

    // work-group reduction of every per-shift sum; when no pixel of the work-group took
    // the masked form, the variance and count are the common ones for every shift
    // (a pixel's masked-form variance is non-zero only with its bit set)
    __shared__ float red[TR_THREADS / 64][CT * 3];
    const bool masked = __syncthreads_or(anyv != 0u ? 1 : 0);
    float* __restrict__ out = a.part + ((size_t)n * a.nblk + tile) * (CT * 3);
    if constexpr (STAGED) if (!masked) {
        // (the barrier above also ends every read of the staged region) each thread's
        // per-shift sums go to that region, shift by shift with a pitch of TR_THREADS + 8
        // floats; eight threads per shift then add 32 entries each (thread p: entries
        // p, p + 8, ...; the eight shifts a wave reads at a time fall on distinct banks)
        // and combine their sums in a fixed butterfly.  The variance and count are common
        // to all shifts.
        constexpr int RP = TR_THREADS + 8;
        static_assert(CT * RP <= TR_LDS_FLOATS, "per-shift sums fit the staged region");
        static_assert(CT * 8 <= TR_THREADS, "eight threads per shift");
#pragma unroll
        for (int s = 0; s < CT; ++s) reg[s * RP + threadIdx.x] = err[s];
        const float vv = wave_total(vC);
        const int c = wave_total(cC);
        if (lane == 0) {
            red[wave][0] = vv;
            red[wave][1] = (float)c;
        }
        __syncthreads();
        const int s = min((int)threadIdx.x >> 3, CT - 1), p = threadIdx.x & 7;
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < TR_THREADS / 8; ++k) acc += reg[s * RP + 8 * k + p];
        acc += __shfl_xor(acc, 1, 64);
        acc += __shfl_xor(acc, 2, 64);
        acc += __shfl_xor(acc, 4, 64);
        if (p == 0 && (int)threadIdx.x < CT * 8) {
            float v = 0.f, cn = 0.f;
#pragma unroll
            for (int w = 0; w < TR_THREADS / 64; ++w) {
                v += red[w][0];
                cn += red[w][1];
            }
            out[3 * s] = acc;
            out[3 * s + 1] = v;
            out[3 * s + 2] = cn;
        }
        return;
    }
    if (masked) {
#pragma unroll
        for (int s = 0; s < CT; ++s) {
            const float e = wave_total(err[s]);
            const float vv = wave_total(var[s] + vC);
            const int c = wave_total(cC + (int)((anyv >> s) & 1u));
            if (lane == 0) {
                red[wave][3 * s] = e;
                red[wave][3 * s + 1] = vv;
                red[wave][3 * s + 2] = (float)c;
            }
        }
    } else {
        const float vv = wave_total(vC);
        const int c = wave_total(cC);
#pragma unroll
        for (int s = 0; s < CT; ++s) {
            const float e = wave_total(err[s]);
            if (lane == 0) {
                red[wave][3 * s] = e;
                red[wave][3 * s + 1] = vv;
                red[wave][3 * s + 2] = (float)c;
            }
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < CT * 3; q += TR_THREADS) {
        float acc = 0.f;
#pragma unroll
        for (int w = 0; w < TR_THREADS / 64; ++w) acc += red[w][q];
        out[q] = acc;
    }
}

// One wave per frame: lanes add the block partials of each shift (compensated, blocks
// in lane-strided order), a fixed butterfly combines the lanes, lane 0 decides.
template <int TX, int TY, bool BATCH>
__global__ __launch_bounds__(64) void k_tr_final(const TrArgs* __restrict__ jobs, TrArgs one) {
    constexpr int NXs = 2 * TX + 1, NYs = 2 * TY + 1, CT = NXs * NYs;
    __shared__ float Es[CT];
    const TrArgs a = job_args<BATCH>(jobs, one);
    const int n = blockIdx.x;
    if (n >= a.N) return;
    const int lane = threadIdx.x;
    for (int s = 0; s < CT; ++s) {
        float eS = 0.f, eC = 0.f, vS = 0.f, vC = 0.f, c = 0.f;
        for (int b = lane; b < a.nblk; b += 64) {
            const float* p = a.part + ((size_t)n * a.nblk + b) * (CT * 3) + 3 * s;
            kahan_add(eS, eC, p[0]);
            kahan_add(vS, vC, p[1]);
            c += p[2];
        }
        const float e = wave_sum<float>(eS);
        const float v = wave_sum<float>(vS);
        const float cnt = wave_sum<float>(c);
        if (lane == 0) Es[s] = normalised_error(e, v, cnt > 0.f ? 1 : 0);
    }
    __syncthreads();
    if (lane != 0) return;
    float be = INFINITY;
    int bk = -1;
    for (int s = 0; s < CT; ++s) {
        if (Es[s] < be) {
            be = Es[s];
            bk = s;
        }
    }
    const float d0 = a.dx_in[2 * n], d1 = a.dx_in[2 * n + 1];
    if (bk < 0) {
        a.dx_out[2 * n] = d0;
        a.dx_out[2 * n + 1] = d1;
        if (a.err_out) a.err_out[n] = INFINITY;
        if (a.arg_out) a.arg_out[n] = -1;
        return;
    }
    const int bx = bk / NYs, by = bk - bx * NYs;
    float ox = 0.f, oy = 0.f;
    if (a.refine) {
        float st[9];
        for (int q = 0; q < 9; ++q) {
            const int kx = bx + q / 3 - 1, ky = by + q % 3 - 1;
            st[q] = (kx >= 0 && kx < NXs && ky >= 0 && ky < NYs) ? Es[kx * NYs + ky] : INFINITY;
        }
        refine_at(st, bx, by, NXs, NYs, ox, oy);
    }
    a.dx_out[2 * n] = d0 + (float)(bx - TX) + ox;
    a.dx_out[2 * n + 1] = d1 + (float)(by - TY) + oy;
    if (a.err_out) a.err_out[n] = be;
    if (a.arg_out) a.arg_out[n] = bk;
}

typedef void (*TrKernel)(const TrArgs*, TrArgs);

template <int TX, int TY, bool BATCH>
void pick(TrKernel& ps, TrKernel& pg, TrKernel& f) {
    ps = k_tr_partial<TX, TY, true, BATCH>;
    pg = k_tr_partial<TX, TY, false, BATCH>;
    f = k_tr_final<TX, TY, BATCH>;
}

template <bool BATCH>
bool pick_form(int tx, int ty, TrKernel& ps, TrKernel& pg, TrKernel& f) {
    switch (tx * 3 + ty) {
        case 0: pick<0, 0, BATCH>(ps, pg, f); return true;
        case 1: pick<0, 1, BATCH>(ps, pg, f); return true;
        case 2: pick<0, 2, BATCH>(ps, pg, f); return true;
        case 3: pick<1, 0, BATCH>(ps, pg, f); return true;
        case 4: pick<1, 1, BATCH>(ps, pg, f); return true;
        case 5: pick<1, 2, BATCH>(ps, pg, f); return true;
        case 6: pick<2, 0, BATCH>(ps, pg, f); return true;
        case 7: pick<2, 1, BATCH>(ps, pg, f); return true;
        case 8: pick<2, 2, BATCH>(ps, pg, f); return true;
    }
    return false;
}

bool pick_tr(int tx, int ty, bool batch, TrKernel& ps, TrKernel& pg, TrKernel& f) {
    return batch ? pick_form<true>(tx, ty, ps, pg, f) : pick_form<false>(tx, ty, ps, pg, f);
}

}  // namespace

TrArgs make_tr_args(const Geom& g, const pxst_scan& sc, const float* refv, const float* u, const float* dx_in,
                    const pxst_window& win, float* dx_out, float* err_min, int32_t* argmin, char* ws,
                    const Layout& L) {
    TrArgs a{};
    a.frames = sc.frames;
    a.white = sc.white;
    a.mask = sc.mask;
    a.refv = refv;
    a.u = u;
    a.dx_in = dx_in;
    a.dx_out = dx_out;
    a.err_out = err_min;
    a.arg_out = argmin;
    a.part = (float*)(ws + L.tr_part);
    a.N = g.N;
    a.H = g.H;
    a.W = g.W;
    a.Rs = g.Rs;
    a.Rf = g.Rf;
    a.o0 = g.o0;
    a.o1 = g.o1;
    a.tiles_x = (g.W + TR_TILE - 1) / TR_TILE;
    a.nblk = a.tiles_x * ((g.H + TR_TILE - 1) / TR_TILE);
    a.bbox = (int4*)(ws + L.tr_bbox);
    a.refine = win.refine != 0;
    a.tx = win.r_ss;
    a.ty = win.r_fs;
    return a;
}

int launch_translations_jobs(const TrArgs* host, int n, const TrArgs* dev, hipStream_t s) {
    TrKernel kp = nullptr, kg = nullptr, kf = nullptr;
    if (!pick_tr(host[0].tx, host[0].ty, dev != nullptr, kp, kg, kf)) {
        set_error("translation window radii must be in 0..%d", PXST_MAX_TR_RADIUS);
        return PXST_EUNSUPPORTED;
    }
    int nblk = 1, nf = 1;
    long long work = 0;
    for (int j = 0; j < n; ++j) {
        if (host[j].tx != host[0].tx || host[j].ty != host[0].ty) {
            set_error("batched translation search: jobs differ in window");
            return PXST_EINVAL;
        }
        nblk = std::max(nblk, host[j].nblk);
        nf = std::max(nf, host[j].N);
        work += (long long)host[j].H * host[j].W * host[j].N * (2 * host[j].tx + 1) * (2 * host[j].ty + 1);
    }
    const TrArgs one = dev ? TrArgs{} : host[0];
    PXST_LAUNCH_JOBS(k_tr_bbox, dim3(nblk, 1, n), dim3(256), 0, s, dev, one);
    profile_begin("tr_partial", s);
    hipLaunchKernelGGL(kp, dim3(nblk, nf, n), dim3(TR_THREADS), 0, s, dev, one);
    hipLaunchKernelGGL(kg, dim3(nblk, nf, n), dim3(TR_THREADS), 0, s, dev, one);
    profile_end("tr_partial", s, work, nullptr, 0);
    hipLaunchKernelGGL(kf, dim3(nf, 1, n), dim3(64), 0, s, dev, one);
    return check_hip(hipGetLastError(), "translation search");
}

int launch_translations(const Geom& g, const pxst_scan& sc, const float* refv, const float* u,
                        const float* dx_in, const pxst_window& win, float* dx_out, float* err_min,
                        int32_t* argmin, char* ws, const Layout& L, hipStream_t s) {
    const TrArgs a = make_tr_args(g, sc, refv, u, dx_in, win, dx_out, err_min, argmin, ws, L);
    return launch_translations_jobs(&a, 1, nullptr, s);
}

}  // namespace pxst

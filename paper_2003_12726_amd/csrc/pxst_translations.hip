// Translation search (Sec. 2.2.3): for each frame, the error integrated over the
// detector for integer shifts of that frame's translation, first minimum and
// paraboloid refinement.
//
// Pass 1 (grid: pixel blocks x frames): a thread walks 16 pixels of one frame; for
// each it loads the (2Tx+2) x (2Ty+2) reference neighbourhood of u - dx_n - origin
// once and forms all shifted lookups from it (the bilinear fractions do not depend on
// the integer shift): when the neighbourhood is fully valid, by interpolating its rows
// along the fast axis once and the results along the slow axis per shift.  Per-shift sums are reduced over the work-group and written as
// per-block partials.  Pass 2 (one wave per frame) adds the partials with compensated
// float32 sums in a fixed order, normalises, takes the first minimum and refines.
#include "pxst_device.hpp"
#include "pxst_internal.hpp"

namespace pxst {

namespace {

struct TrArgs {
    const uint16_t* frames;
    const float* white;
    const uint8_t* mask;
    const float* refv;
    const float* u;
    const float* dx_in;
    float* dx_out;
    float* err_out;
    int* arg_out;
    float* part;      // [N][nblk][Ct][3]
    int N, H, W, Rs, Rf, o0, o1;
    int nblk, refine;
};

template <int TX, int TY>
__global__ __launch_bounds__(TR_THREADS) void k_tr_partial(TrArgs a) {
    constexpr int NXs = 2 * TX + 1, NYs = 2 * TY + 1, CT = NXs * NYs;
    constexpr int CR = 2 * TY + 2;   // neighbourhood columns
    constexpr int RR = 2 * TX + 2;   // neighbourhood rows
    const int blk = blockIdx.x, n = blockIdx.y;
    const size_t HW = (size_t)a.H * a.W;
    const float d0 = a.dx_in[2 * n], d1 = a.dx_in[2 * n + 1];
    const float s0 = floorf(d0), s1 = floorf(d1);
    const float fd0 = d0 - s0, fd1 = d1 - s1;
    const uint16_t* fr = a.frames + (size_t)n * HW;

    // per shift: squared residuals; the variance and count of the pixels with a valid
    // lookup are common to all shifts for pixels whose whole neighbourhood is valid
    // (vC, cC) and kept per shift for the others (var, cnt)
    float err[CT], var[CT];
    int cnt[CT];
#pragma unroll
    for (int s = 0; s < CT; ++s) {
        err[s] = 0.f;
        var[s] = 0.f;
        cnt[s] = 0;
    }
    float vC = 0.f;
    int cC = 0;
    const size_t p_begin = (size_t)blk * TR_PIX_PER_BLOCK;
    for (int m = 0; m < TR_PIX_PER_BLOCK / TR_THREADS; ++m) {
        const size_t pix = p_begin + (size_t)m * TR_THREADS + threadIdx.x;
        if (pix >= HW || a.mask[pix] == 0) continue;
        const float u0 = a.u[pix], u1 = a.u[HW + pix];
        const float f0 = floorf(u0), f1 = floorf(u1);
        const float t0 = (u0 - f0) - fd0, t1 = (u1 - f1) - fd1;
        const int a0 = (int)f0 - (int)s0 - a.o0 - (t0 < 0.f ? 1 : 0);
        const int b0 = (int)f1 - (int)s1 - a.o1 - (t1 < 0.f ? 1 : 0);
        const float fa = t0 < 0.f ? t0 + 1.f : t0, fb = t1 < 0.f ? t1 + 1.f : t1;
        const float Wp = a.white[pix];
        const float I = (float)fr[pix];
        const float v = I - Wp, v2 = v * v;
        // neighbourhood rows a0 - TX .. a0 + TX + 1, columns b0 - TY .. b0 + TY + 1;
        // shift (sx, sy) looks up corner rows a0 - sx, a0 - sx + 1 and columns
        // b0 - sy, b0 - sy + 1
        float nb[RR][CR];
        bool all = a0 - TX >= 0 && a0 + TX + 1 < a.Rs && b0 - TY >= 0 && b0 + TY + 1 < a.Rf;
#pragma unroll
        for (int r = 0; r < RR; ++r) {
            const int rr = a0 - TX + r;
#pragma unroll
            for (int c = 0; c < CR; ++c) {
                const int cc = b0 - TY + c;
                nb[r][c] = (rr >= 0 && rr < a.Rs && cc >= 0 && cc < a.Rf) ? a.refv[(size_t)rr * a.Rf + cc]
                                                                         : qnan();
                all = all && valid(nb[r][c]);
            }
        }
        if (all) {
            // every lookup valid: interpolate along fs, then along ss (the fractions are
            // the same for every shift)
            float h[RR][CR - 1];
#pragma unroll
            for (int r = 0; r < RR; ++r)
#pragma unroll
                for (int c = 0; c < CR - 1; ++c) h[r][c] = fmaf(fb, nb[r][c + 1] - nb[r][c], nb[r][c]);
            const float nW = -Wp;
#pragma unroll
            for (int ix = 0; ix < NXs; ++ix) {
#pragma unroll
                for (int iy = 0; iy < NYs; ++iy) {
                    const float g = fmaf(fa, h[ix + 1][iy] - h[ix][iy], h[ix][iy]);
                    const int s = (TX - ix + TX) * NYs + (TY - iy + TY);
                    const float rr = fmaf(nW, g, I);
                    err[s] = fmaf(rr, rr, err[s]);
                }
            }
            vC += v2;
            cC += 1;
        } else {
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
                    // shift (sx, sy) = (TX - ix, TY - iy); candidate index (sx + TX) NYs + (sy + TY)
                    const int s = (TX - ix + TX) * NYs + (TY - iy + TY);
                    if (valid(g)) {
                        const float rr = fmaf(-Wp, g, I);
                        err[s] = fmaf(rr, rr, err[s]);
                        var[s] += v2;
                        cnt[s] += 1;
                    }
                }
            }
        }
    }
#pragma unroll
    for (int s = 0; s < CT; ++s) {
        var[s] += vC;
        cnt[s] += cC;
    }
    // work-group reduction of every per-shift sum
    __shared__ float red[TR_THREADS / 64][CT * 3];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int s = 0; s < CT; ++s) {
        const float e = wave_sum<float>(err[s]);
        const float vv = wave_sum<float>(var[s]);
        const int c = wave_sum<int>(cnt[s]);
        if (lane == 0) {
            red[wave][3 * s] = e;
            red[wave][3 * s + 1] = vv;
            red[wave][3 * s + 2] = (float)c;
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < CT * 3; q += TR_THREADS) {
        float acc = 0.f;
#pragma unroll
        for (int w = 0; w < TR_THREADS / 64; ++w) acc += red[w][q];
        a.part[((size_t)n * a.nblk + blk) * (CT * 3) + q] = acc;
    }
}

// One wave per frame: lanes add the block partials of each shift (compensated, blocks
// in lane-strided order), a fixed butterfly combines the lanes, lane 0 decides.
template <int TX, int TY>
__global__ __launch_bounds__(64) void k_tr_final(TrArgs a) {
    constexpr int NXs = 2 * TX + 1, NYs = 2 * TY + 1, CT = NXs * NYs;
    __shared__ float Es[CT];
    const int n = blockIdx.x;
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

typedef void (*TrKernel)(TrArgs);

template <int TX, int TY>
void pick(TrKernel& p, TrKernel& f) {
    p = k_tr_partial<TX, TY>;
    f = k_tr_final<TX, TY>;
}

bool pick_tr(int tx, int ty, TrKernel& p, TrKernel& f) {
    switch (tx * 3 + ty) {
        case 0: pick<0, 0>(p, f); return true;
        case 1: pick<0, 1>(p, f); return true;
        case 2: pick<0, 2>(p, f); return true;
        case 3: pick<1, 0>(p, f); return true;
        case 4: pick<1, 1>(p, f); return true;
        case 5: pick<1, 2>(p, f); return true;
        case 6: pick<2, 0>(p, f); return true;
        case 7: pick<2, 1>(p, f); return true;
        case 8: pick<2, 2>(p, f); return true;
    }
    return false;
}

}  // namespace

int launch_translations(const Geom& g, const pxst_scan& sc, const float* refv, const float* u,
                        const float* dx_in, const pxst_window& win, float* dx_out, float* err_min,
                        int32_t* argmin, char* ws, const Layout& L, hipStream_t s) {
    TrKernel kp = nullptr, kf = nullptr;
    if (!pick_tr(win.r_ss, win.r_fs, kp, kf)) {
        set_error("translation window radii must be in 0..%d", PXST_MAX_TR_RADIUS);
        return PXST_EUNSUPPORTED;
    }
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
    a.nblk = (int)((g.HW() + TR_PIX_PER_BLOCK - 1) / TR_PIX_PER_BLOCK);
    a.refine = win.refine != 0;
    profile_begin("tr_partial", s);
    hipLaunchKernelGGL(kp, dim3(a.nblk, g.N), dim3(TR_THREADS), 0, s, a);
    profile_end("tr_partial", s,
                (long long)g.HW() * g.N * (2 * win.r_ss + 1) * (2 * win.r_fs + 1), nullptr, 0);
    hipLaunchKernelGGL(kf, dim3(g.N), dim3(64), 0, s, a);
    return check_hip(hipGetLastError(), "translation search");
}

}  // namespace pxst

// Split-half analysis (Sec. 2.3, additional analysis): every (frame, pixel) term of
// the data set belongs to one of two halves; a pixel map is searched from each half
// against the same reference (the search of Sec. 2.2.2 with the other half's terms
// left out), and the differences of the two maps are histogrammed per axis.
//
// The halves are arbitrary per (frame, pixel), so the frame sums of a pixel differ from
// its neighbours' and the matrix-core contraction (one column sum per position) does
// not apply: one work-group per 8x8 tile, 64 pixels x 4 candidate strides, every
// candidate summing its pixel's terms of the half over the frames (compensated float32
// as in the scattered-tile search), first minimum, paraboloid on the 3x3 stencil.
#include "pxst_device.hpp"
#include "pxst_internal.hpp"

namespace pxst {

namespace {

struct SplitArgs {
    const uint16_t* frames;
    const float* white;
    const uint8_t* mask;
    const uint8_t* half;   // [N][H][W] 0 / 1
    const float* refv;
    const float* dx;
    const float* u_in;
    float* u_out;
    int* found;            // argmin, -1 when the pixel has no result
    int N, H, W, Rs, Rf, o0, o1, rx, ry, refine, hval, tiles_x;
};

__device__ float split_eval(const SplitArgs& a, size_t pix, size_t HW, int t0, int t1, float Wp) {
    float eS = 0.f, eP = 0.f, vS = 0.f, vP = 0.f;
    int nv = 0;
    for (int n = 0; n < a.N; ++n) {
        if (a.half[(size_t)n * HW + pix] != a.hval) continue;
        const AxisShift s0 = axis_shift(a.dx[2 * n], a.o0);
        const AxisShift s1 = axis_shift(a.dx[2 * n + 1], a.o1);
        const float g = masked_bilinear(a.refv, a.Rs, a.Rf, t0 - s0.e, t1 - s1.e, s0.t, s1.t);
        if (valid(g)) {
            const float I = (float)a.frames[(size_t)n * HW + pix];
            const float rr = fmaf(-Wp, g, I);
            eP = fmaf(rr, rr, eP);
            const float v = I - Wp;
            vP = fmaf(v, v, vP);
            ++nv;
            if ((nv % 32) == 0) {
                two_sum_fold(eS, eP);
                two_sum_fold(vS, vP);
            }
        }
    }
    return normalised_error(eS + eP, vS + vP, nv);
}

__global__ __launch_bounds__(256) void k_pm_split(SplitArgs a) {
    __shared__ float redE[4][64];
    __shared__ int redK[4][64];
    __shared__ float sten[64][9];
    const int tile = blockIdx.x;
    const int ty = tile / a.tiles_x, tx = tile - ty * a.tiles_x;
    const int p = threadIdx.x & 63, sub = threadIdx.x >> 6;
    const int i = ty * TILE + (p >> 3), j = tx * TILE + (p & 7);
    const size_t HW = (size_t)a.H * a.W;
    const bool inb = i < a.H && j < a.W;
    const size_t pix = inb ? (size_t)i * a.W + j : 0;
    const bool good = inb && a.mask[pix] != 0;
    const int NX = 2 * a.rx + 1, NY = 2 * a.ry + 1, C = NX * NY;
    int c0 = 0, c1 = 0;
    float Wp = 0.f;
    if (good) {
        c0 = window_centre(a.u_in[pix]);
        c1 = window_centre(a.u_in[HW + pix]);
        Wp = a.white[pix];
    }
    float be = INFINITY;
    int bk = INT_MAX;
    if (good) {
        for (int k = sub; k < C; k += 4) {
            const int kx = k / NY, ky = k - kx * NY;
            const float E = split_eval(a, pix, HW, c0 - a.rx + kx, c1 - a.ry + ky, Wp);
            if (E < be) {
                be = E;
                bk = k;
            }
        }
    }
    redE[sub][p] = be;
    redK[sub][p] = bk;
    __syncthreads();
    if (sub == 0) {
        for (int s = 1; s < 4; ++s)
            if (better(redE[s][p], redK[s][p], be, bk)) {
                be = redE[s][p];
                bk = redK[s][p];
            }
        redE[0][p] = be;
        redK[0][p] = isfinite(be) ? bk : -1;
    }
    __syncthreads();
    const int kb = redK[0][p];
    if (a.refine && good && kb >= 0) {
        const int bx = kb / NY, by = kb - bx * NY;
        for (int q = sub; q < 9; q += 4) {
            const int kx = bx + q / 3 - 1, ky = by + q % 3 - 1;
            float E = INFINITY;
            if (kx >= 0 && kx < NX && ky >= 0 && ky < NY)
                E = split_eval(a, pix, HW, c0 - a.rx + kx, c1 - a.ry + ky, Wp);
            sten[p][q] = E;
        }
    }
    __syncthreads();
    if (sub == 0 && inb) {
        if (!good || kb < 0) {
            a.u_out[pix] = a.u_in[pix];
            a.u_out[HW + pix] = a.u_in[HW + pix];
            a.found[pix] = -1;
        } else {
            const int bx = kb / NY, by = kb - bx * NY;
            float ox = 0.f, oy = 0.f;
            if (a.refine) refine_at(sten[p], bx, by, NX, NY, ox, oy);
            a.u_out[pix] = (float)(c0 + bx - a.rx) + ox;
            a.u_out[HW + pix] = (float)(c1 + by - a.ry) + oy;
            a.found[pix] = kb;
        }
    }
}

__global__ void k_fill_i32(int* __restrict__ p, int n, int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Equal bins over [-R, R] per axis with numpy's rule: edge k = -R + k (2R / nbins)
// (the last edge R exactly), index from the scaled offset then corrected against the
// edges; the last bin holds its upper edge; values outside are not counted.
__device__ inline int hist_bin(double d, double R, int nb) {
    if (!(d >= -R && d <= R)) return -1;
    const double step = (2.0 * R) / nb;
    auto edge = [&](int k) { return k >= nb ? R : -R + k * step; };
    int k = (int)((d + R) * (nb / (2.0 * R)));
    if (k >= nb) k = nb - 1;
    if (k < 0) k = 0;
    if (d < edge(k)) --k;
    else if (k != nb - 1 && d >= edge(k + 1)) ++k;
    return k;
}

// Counts per work-group in LDS (bins of both axes, up to HIST_LDS of them), then one
// global addition per non-empty bin; beyond that, global additions per value.
constexpr int HIST_LDS = 8192, HIST_THREADS = 256, HIST_PIX = 4096;
__global__ __launch_bounds__(HIST_THREADS) void k_split_hist(const float* __restrict__ ua, const float* __restrict__ ub,
                                                             const int* __restrict__ ka, const int* __restrict__ kb,
                                                             const uint8_t* __restrict__ mask, size_t HW, double R,
                                                             int nb, int* __restrict__ hist) {
    __shared__ int lh[HIST_LDS];
    const bool local = 2 * nb <= HIST_LDS;
    if (local)
        for (int i = threadIdx.x; i < 2 * nb; i += HIST_THREADS) lh[i] = 0;
    __syncthreads();
    const size_t p0 = (size_t)blockIdx.x * HIST_PIX;
    const size_t p1 = min(HW, p0 + HIST_PIX);
    for (size_t p = p0 + threadIdx.x; p < p1; p += HIST_THREADS) {
        if (!mask[p] || ka[p] < 0 || kb[p] < 0) continue;
        for (int ax = 0; ax < 2; ++ax) {
            const double d = (double)ua[ax * HW + p] - (double)ub[ax * HW + p];
            const int k = hist_bin(d, R, nb);
            if (k < 0) continue;
            if (local)
                atomicAdd(&lh[ax * nb + k], 1);
            else
                atomicAdd(&hist[ax * nb + k], 1);
        }
    }
    __syncthreads();
    if (local)
        for (int i = threadIdx.x; i < 2 * nb; i += HIST_THREADS)
            if (lh[i]) atomicAdd(&hist[i], lh[i]);
}

}  // namespace

int launch_split_half(const Geom& g, const pxst_scan& sc, const float* refv, const float* dx, const float* u_in,
                      const pxst_window& win, const uint8_t* half, float* u_a, float* u_b, double hist_range,
                      int nbins, int32_t* hist, char* ws, const Layout& L, hipStream_t s) {
    const size_t HW = g.HW();
    int* ka = (int*)(ws + L.frac_k);
    int* kb = (int*)(ws + L.frac_bk);
    SplitArgs a{};
    a.frames = sc.frames;
    a.white = sc.white;
    a.mask = sc.mask;
    a.half = half;
    a.refv = refv;
    a.dx = dx;
    a.u_in = u_in;
    a.N = g.N;
    a.H = g.H;
    a.W = g.W;
    a.Rs = g.Rs;
    a.Rf = g.Rf;
    a.o0 = g.o0;
    a.o1 = g.o1;
    a.rx = win.r_ss;
    a.ry = win.r_fs;
    a.refine = win.refine != 0;
    a.tiles_x = (g.W + TILE - 1) / TILE;
    const int ntiles = a.tiles_x * ((g.H + TILE - 1) / TILE);
    profile_begin("pm_split", s);
    for (int h = 0; h < 2; ++h) {
        a.hval = h;
        a.u_out = h ? u_b : u_a;
        a.found = h ? kb : ka;
        hipLaunchKernelGGL(k_pm_split, dim3(ntiles), dim3(256), 0, s, a);
    }
    profile_end("pm_split", s, 0, nullptr, 0);
    if (hist) {
        hipLaunchKernelGGL(k_fill_i32, dim3((2 * nbins + 255) / 256), dim3(256), 0, s, hist, 2 * nbins, 0);
        hipLaunchKernelGGL(k_split_hist, dim3((unsigned)((HW + HIST_PIX - 1) / HIST_PIX)), dim3(HIST_THREADS), 0, s,
                           u_a, u_b, ka, kb, sc.mask, HW, hist_range, nbins, hist);
    }
    return check_hip(hipGetLastError(), "split-half pixel maps");
}

}  // namespace pxst

// Split-half analysis (Sec. 2.3, additional analysis): every (frame, pixel) term of
// the data set belongs to one of two halves; a pixel map is searched from each half
// against the same reference (the search of Sec. 2.2.2 with the other half's terms
// left out), and the differences of the two maps are histogrammed per axis.
//
// Each half is the pixel-map search itself, run with the half mask: the halves are
// arbitrary per (frame, pixel), so the frame sums that the matrix-core contraction
// shares between the pixels of a tile do not exist, and the tiles go to the LDS-staged
// searches (the reference region of a tile staged once per frame for its 64 pixels;
// a term outside the half adds a zero residual and no variance), the tiles whose
// region does not fit to the generic search.
#include "pxst_device.hpp"
#include "pxst_internal.hpp"

namespace pxst {

namespace {

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

int launch_split_half(const Geom& g, const pxst_scan& sc, const float* refv, const int* sat, const float* dx,
                      const float* u_in, const pxst_window& win, const uint8_t* half, float* u_a, float* u_b,
                      double hist_range, int nbins, int32_t* hist, char* ws, const Layout& L, hipStream_t s) {
    const size_t HW = g.HW();
    int* ka = (int*)(ws + L.frac_k);
    int* kb = (int*)(ws + L.frac_bk);
    profile_begin("pm_split", s);
    for (int h = 0; h < 2; ++h) {
        const int rc = launch_pixel_map(g, sc, refv, sat, dx, u_in, win, h ? u_b : u_a, nullptr, h ? kb : ka, ws,
                                        L, s, half, h);
        if (rc) return rc;
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

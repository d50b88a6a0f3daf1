// Defocus by registration (Sec. 2.1): a reference image is built (Sec. 2.2.1) from the
// map of every candidate magnification and the candidate whose reference has the
// greatest contrast is chosen.  A candidate is a pair of per-axis scale factors of the
// linear map u = c + s (x - c) on the fixed reference grid; contrast is the variance
// over the squared mean of the reference pixels with a positive weight sum (float64
// sums in a fixed order).  Each candidate runs the reference update of the main loop.
#include "pxst_device.hpp"
#include "pxst_internal.hpp"

namespace pxst {

namespace {

constexpr int CT_THREADS = 256;

__global__ void k_linear_map(float* __restrict__ u, int H, int W, double s0, double s1, double c0, double c1) {
    const size_t HW = (size_t)H * W;
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= HW) return;
    const int i = (int)(p / W), j = (int)(p - (size_t)i * W);
    u[p] = (float)(c0 + s0 * ((double)i - c0));
    u[HW + p] = (float)(c1 + s1 * ((double)j - c1));
}

// Per block: count, sum and sum of squares of the weighted reference pixels.
__global__ __launch_bounds__(CT_THREADS) void k_contrast_partial(const float* __restrict__ ref,
                                                                  const double* __restrict__ wsum, size_t RR,
                                                                  double* __restrict__ part) {
    __shared__ double red[CT_THREADS / 64][3];
    double n = 0.0, s = 0.0, q = 0.0;
    for (size_t p = (size_t)blockIdx.x * CT_THREADS + threadIdx.x; p < RR; p += (size_t)gridDim.x * CT_THREADS) {
        if (wsum[p] > 0.0) {
            const double v = (double)ref[p];
            n += 1.0;
            s += v;
            q = fma(v, v, q);
        }
    }
    n = wave_sum<double>(n);
    s = wave_sum<double>(s);
    q = wave_sum<double>(q);
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6][0] = n;
        red[threadIdx.x >> 6][1] = s;
        red[threadIdx.x >> 6][2] = q;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0, c = 0.0;
        for (int w = 0; w < CT_THREADS / 64; ++w) {
            a += red[w][0];
            b += red[w][1];
            c += red[w][2];
        }
        part[3 * blockIdx.x] = a;
        part[3 * blockIdx.x + 1] = b;
        part[3 * blockIdx.x + 2] = c;
    }
}

__global__ void k_contrast_final(const double* __restrict__ part, int nblk, double* __restrict__ out) {
    if (threadIdx.x != 0) return;
    double n = 0.0, s = 0.0, q = 0.0;
    for (int b = 0; b < nblk; ++b) {
        n += part[3 * b];
        s += part[3 * b + 1];
        q += part[3 * b + 2];
    }
    double c = 0.0;
    if (n > 0.0) {
        const double m = s / n;
        if (m != 0.0) c = (q / n - m * m) / (m * m);
    }
    *out = c;
}

// First maximum of the contrasts.
__global__ void k_first_max(const double* __restrict__ c, int n, int* __restrict__ best) {
    if (threadIdx.x != 0) return;
    int k = 0;
    for (int i = 1; i < n; ++i)
        if (c[i] > c[k]) k = i;
    *best = k;
}

}  // namespace

int launch_defocus_sweep(const Geom& g, const pxst_scan& sc, const float* dx, const float* scales, int n_cand,
                         double c0, double c1, double* contrast, int32_t* best, char* ws, const Layout& L,
                         hipStream_t s) {
    const size_t HW = g.HW(), RR = g.RR();
    float* u = (float*)(ws + L.sweep_u);
    float* ref = (float*)(ws + L.sweep_ref);
    double* w = (double*)(ws + L.sweep_w);
    double* part = (double*)(ws + L.sweep_part);
    profile_begin("defocus_sweep", s);
    for (int k = 0; k < n_cand; ++k) {
        hipLaunchKernelGGL(k_linear_map, dim3((unsigned)((HW + 255) / 256)), dim3(256), 0, s, u, g.H, g.W,
                           (double)scales[2 * k], (double)scales[2 * k + 1], c0, c1);
        int rc = launch_update_reference(g, sc, u, dx, ref, w, nullptr, ws, L, s, PXST_REF_EXACT);
        if (rc) return rc;
        hipLaunchKernelGGL(k_contrast_partial, dim3(SWEEP_BLOCKS), dim3(CT_THREADS), 0, s, ref, w, RR, part);
        hipLaunchKernelGGL(k_contrast_final, dim3(1), dim3(64), 0, s, part, SWEEP_BLOCKS, contrast + k);
    }
    if (best) hipLaunchKernelGGL(k_first_max, dim3(1), dim3(64), 0, s, contrast, n_cand, best);
    profile_end("defocus_sweep", s, (long long)n_cand * (long long)HW * g.N, nullptr, 0);
    return check_hip(hipGetLastError(), "defocus sweep");
}

}  // namespace pxst

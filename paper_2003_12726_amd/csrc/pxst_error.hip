// Figures of merit (Sec. 2.2.4, integrand of Eq. 2) and the per-pixel variance.
//
// sigma2 = (1/N) sum_n M (I - W)^2 per pixel.  The error pass streams the frames
// once: every thread owns one pixel, forms eps = M (I - W g)^2 / sigma2 with the
// masked bilinear lookup at u - dx_n - origin, accumulates the pixel error with
// compensated float32 sums and adds the frame error in float64 per wave; the final
// passes add the per-block frame partials and then the frames, each in a fixed order,
// so the totals are reproducible.
#include "pxst_device.hpp"
#include "pxst_internal.hpp"

namespace pxst {

namespace {

constexpr int ERR_PIX_PER_THREAD = ERR_PIX_PER_THREAD_CFG;

__global__ void k_sigma2(const uint16_t* __restrict__ frames, const float* __restrict__ white,
                         const uint8_t* __restrict__ mask, int N, size_t HW, float* __restrict__ s2) {
    const size_t pix = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= HW) return;
    if (!mask[pix]) {
        s2[pix] = 0.f;
        return;
    }
    const float Wp = white[pix];
    float S = 0.f, P = 0.f;
    for (int n = 0; n < N; ++n) {
        const float v = (float)frames[(size_t)n * HW + pix] - Wp;
        P = fmaf(v, v, P);
        if (((n + 1) & 31) == 0) two_sum_fold(S, P);
    }
    s2[pix] = (S + P) / (float)N;
}

struct ErrArgs {
    const uint16_t* frames;
    const float* white;
    const uint8_t* mask;
    const float* refv;
    const float* s2;
    const float* u;
    const float* dx;
    float* pixel_err;
    double* part;       // [N][nblk]
    double* frame_err;  // [N] (workspace copy when the caller passes none)
    double* frame_out;  // caller's frame errors or null
    double* total;
    int N, H, W, Rs, Rf, o0, o1, nblk;
};

__global__ __launch_bounds__(ERR_THREADS) void k_err_pixels(ErrArgs a) {
    extern __shared__ double wsum_sh[];   // [N][waves]
    constexpr int WAVES = ERR_THREADS / 64;
    const size_t HW = (size_t)a.H * a.W;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    size_t pix[ERR_PIX_PER_THREAD];
    bool use[ERR_PIX_PER_THREAD];
    float Wp[ERR_PIX_PER_THREAD], s2[ERR_PIX_PER_THREAD], u0[ERR_PIX_PER_THREAD],
        u1[ERR_PIX_PER_THREAD];
    float pS[ERR_PIX_PER_THREAD], pC[ERR_PIX_PER_THREAD];
#pragma unroll
    for (int m = 0; m < ERR_PIX_PER_THREAD; ++m) {
        pix[m] = ((size_t)blockIdx.x * ERR_PIX_PER_THREAD + m) * ERR_THREADS + threadIdx.x;
        const bool inb = pix[m] < HW;
        use[m] = inb && a.mask[pix[m]] != 0 && a.s2[pix[m]] > 0.f;
        Wp[m] = inb ? a.white[pix[m]] : 0.f;
        s2[m] = inb ? a.s2[pix[m]] : 1.f;
        u0[m] = inb ? a.u[pix[m]] : 0.f;
        u1[m] = inb ? a.u[HW + pix[m]] : 0.f;
        pS[m] = 0.f;
        pC[m] = 0.f;
    }
    for (int n = 0; n < a.N; ++n) {
        const float d0 = a.dx[2 * n], d1 = a.dx[2 * n + 1];
        const float sd0 = floorf(d0), sd1 = floorf(d1);
        const float fd0 = d0 - sd0, fd1 = d1 - sd1;
        double fsum = 0.0;
#pragma unroll
        for (int m = 0; m < ERR_PIX_PER_THREAD; ++m) {
            if (!use[m]) continue;
            const float f0 = floorf(u0[m]), f1 = floorf(u1[m]);
            const float t0 = (u0[m] - f0) - fd0, t1 = (u1[m] - f1) - fd1;
            const int a0 = (int)f0 - (int)sd0 - a.o0 - (t0 < 0.f ? 1 : 0);
            const int b0 = (int)f1 - (int)sd1 - a.o1 - (t1 < 0.f ? 1 : 0);
            const float g = masked_bilinear(a.refv, a.Rs, a.Rf, a0, b0, t0 < 0.f ? t0 + 1.f : t0,
                                            t1 < 0.f ? t1 + 1.f : t1);
            if (valid(g)) {
                const float rr = fmaf(-Wp[m], g, (float)a.frames[(size_t)n * HW + pix[m]]);
                const float eps = rr * rr / s2[m];
                kahan_add(pS[m], pC[m], eps);
                fsum += (double)eps;
            }
        }
        fsum = wave_sum<double>(fsum);
        if (lane == 0) wsum_sh[(size_t)n * WAVES + wave] = fsum;
    }
    if (a.pixel_err) {
#pragma unroll
        for (int m = 0; m < ERR_PIX_PER_THREAD; ++m)
            if (pix[m] < HW) a.pixel_err[pix[m]] = use[m] ? pS[m] : 0.f;
    }
    __syncthreads();
    for (int n = threadIdx.x; n < a.N; n += ERR_THREADS) {
        double acc = 0.0;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) acc += wsum_sh[(size_t)n * WAVES + w];
        a.part[(size_t)n * a.nblk + blockIdx.x] = acc;
    }
}

// One wave per frame: lanes add the block partials in lane-strided order, a fixed
// butterfly combines the lanes.
__global__ __launch_bounds__(64) void k_err_frames(ErrArgs a) {
    const int n = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < a.nblk; b += 64) acc += a.part[(size_t)n * a.nblk + b];
    acc = wave_sum<double>(acc);
    if (threadIdx.x == 0) {
        a.frame_err[n] = acc;
        if (a.frame_out) a.frame_out[n] = acc;
    }
}

// Total: the frame errors added by one wave in the same fixed order.
__global__ __launch_bounds__(64) void k_err_total(ErrArgs a) {
    double acc = 0.0;
    for (int n = threadIdx.x; n < a.N; n += 64) acc += a.frame_err[n];
    acc = wave_sum<double>(acc);
    if (threadIdx.x == 0) *a.total = acc;
}

}  // namespace

int launch_sigma2(const Geom& g, const pxst_scan& sc, float* s2, hipStream_t s) {
    const size_t HW = g.HW();
    hipLaunchKernelGGL(k_sigma2, dim3((unsigned)((HW + 255) / 256)), dim3(256), 0, s, sc.frames,
                       sc.white, sc.mask, g.N, HW, s2);
    return check_hip(hipGetLastError(), "pixel variance");
}

int launch_error(const Geom& g, const pxst_scan& sc, const float* refv, const float* s2,
                 const float* u, const float* dx, float* pixel_err, double* frame_err,
                 double* total, char* ws, const Layout& L, hipStream_t s) {
    ErrArgs a{};
    a.frames = sc.frames;
    a.white = sc.white;
    a.mask = sc.mask;
    a.refv = refv;
    a.s2 = s2;
    a.u = u;
    a.dx = dx;
    a.pixel_err = pixel_err;
    a.N = g.N;
    a.H = g.H;
    a.W = g.W;
    a.Rs = g.Rs;
    a.Rf = g.Rf;
    a.o0 = g.o0;
    a.o1 = g.o1;
    const size_t per_block = (size_t)ERR_THREADS * ERR_PIX_PER_THREAD;
    a.nblk = (int)((g.HW() + per_block - 1) / per_block);
    a.part = (double*)(ws + L.err_part);
    a.frame_err = (double*)(ws + L.err_pix);
    a.frame_out = frame_err;
    a.total = total;
    const size_t sh = (size_t)g.N * (ERR_THREADS / 64) * sizeof(double);
    if (sh > 60 * 1024) {
        set_error("error evaluation supports at most %d frames", (int)(60 * 1024 / 32));
        return PXST_EUNSUPPORTED;
    }
    profile_begin("err_pixels", s);
    hipLaunchKernelGGL(k_err_pixels, dim3(a.nblk), dim3(ERR_THREADS), sh, s, a);
    profile_end("err_pixels", s, (long long)g.HW() * g.N, nullptr, 0);
    hipLaunchKernelGGL(k_err_frames, dim3(g.N), dim3(64), 0, s, a);
    hipLaunchKernelGGL(k_err_total, dim3(1), dim3(64), 0, s, a);
    return check_hip(hipGetLastError(), "error evaluation");
}

}  // namespace pxst

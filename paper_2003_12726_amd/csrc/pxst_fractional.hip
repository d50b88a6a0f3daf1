// Pixel-map search on a fine grid (Sec. 2.2.2: the error evaluated at non-integer
// positions through the interpolation of Sec. 4, in place of the paraboloid).
//
// The candidates of a pixel are c + m / s per axis (s odd, m over the integer window
// widened by (s-1)/2 fine points per side).  They fall into s^2 classes by the fine
// offset q / s, q in [-(s-1)/2, (s-1)/2]; the lookup of candidate c + k + q/s in frame
// n is at (c + k) - (dx_n - q/s) - origin, so a class is exactly the integer search
// with every translation moved by -q/s.  The classes run one after the other through
// the integer search (all its kernels, matrix cores included) and a combine kernel
// keeps, per pixel, the first minimum in fine-grid order: the smallest (error, fine
// index) pair.
#include "pxst_device.hpp"
#include "pxst_internal.hpp"

namespace pxst {

namespace {

__global__ void k_shift_dx(const float* __restrict__ dx, float* __restrict__ dxq, int N, float f0, float f1) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    dxq[2 * n] = dx[2 * n] - f0;
    dxq[2 * n + 1] = dx[2 * n + 1] - f1;
}

// Folds one class's search (error, local index) into the best (error, fine index).
__global__ void k_frac_combine(const float* __restrict__ e_run, const int* __restrict__ k_run, size_t HW,
                               int q0, int q1, int s, int rx, int ry, float* __restrict__ best_e,
                               int* __restrict__ best_k, int first) {
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= HW) return;
    float be = first ? INFINITY : best_e[p];
    int bk = first ? -1 : best_k[p];
    const int k = k_run[p];
    if (k >= 0) {
        const int h = (s - 1) / 2;
        const int Mx = rx * s + h, My = ry * s + h;
        const int kx = k / (2 * ry + 1) - rx, ky = k - (k / (2 * ry + 1)) * (2 * ry + 1) - ry;
        const int idx = (kx * s + q0 + Mx) * (2 * My + 1) + (ky * s + q1 + My);
        const float e = e_run[p];
        if (bk < 0 || e < be || (e == be && idx < bk)) {
            be = e;
            bk = idx;
        }
    }
    best_e[p] = be;
    best_k[p] = bk;
}

// u_out = c + m / s at the best fine index; pixels without one keep u_in.
__global__ void k_frac_finish(const float* u_in, const float* __restrict__ best_e, const int* __restrict__ best_k,
                              size_t HW, int s, int rx, int ry, float* u_out, float* __restrict__ err_out,
                              int* __restrict__ arg_out) {
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= HW) return;
    const int k = best_k[p];
    const float u0 = u_in[p], u1 = u_in[HW + p];
    float o0 = u0, o1 = u1;
    if (k >= 0) {
        const int h = (s - 1) / 2;
        const int Mx = rx * s + h, My = ry * s + h;
        const int m0 = k / (2 * My + 1) - Mx, m1 = k - (k / (2 * My + 1)) * (2 * My + 1) - My;
        o0 = (float)((double)window_centre(u0) + (double)m0 / s);
        o1 = (float)((double)window_centre(u1) + (double)m1 / s);
    }
    u_out[p] = o0;
    u_out[HW + p] = o1;
    if (err_out) err_out[p] = k >= 0 ? best_e[p] : INFINITY;
    if (arg_out) arg_out[p] = k;
}

}  // namespace

int launch_pixel_map_fractional(const Geom& g, const pxst_scan& sc, const float* refv, const int* sat,
                                const float* dx, const float* u_in, const pxst_window& win, int steps,
                                float* u_out, float* err_min, int32_t* argmin, char* ws, const Layout& L,
                                hipStream_t s) {
    const size_t HW = g.HW();
    const int h = (steps - 1) / 2;
    float* dxq = (float*)(ws + L.frac_dx);
    float* u_run = (float*)(ws + L.frac_u);
    float* e_run = (float*)(ws + L.frac_e);
    int* k_run = (int*)(ws + L.frac_k);
    float* be = (float*)(ws + L.frac_be);
    int* bk = (int*)(ws + L.frac_bk);
    const pxst_window wi{win.r_ss, win.r_fs, 0};
    const unsigned blocks = (unsigned)((HW + 255) / 256);
    bool first = true;
    profile_begin("pm_frac", s);
    for (int q0 = -h; q0 <= h; ++q0) {
        for (int q1 = -h; q1 <= h; ++q1) {
            hipLaunchKernelGGL(k_shift_dx, dim3((g.N + 255) / 256), dim3(256), 0, s, dx, dxq, g.N,
                               (float)q0 / (float)steps, (float)q1 / (float)steps);
            int rc = launch_pixel_map(g, sc, refv, sat, dxq, u_in, wi, u_run, e_run, k_run, ws, L, s);
            if (rc) return rc;
            hipLaunchKernelGGL(k_frac_combine, dim3(blocks), dim3(256), 0, s, e_run, k_run, HW, q0, q1, steps,
                               win.r_ss, win.r_fs, be, bk, first ? 1 : 0);
            first = false;
        }
    }
    hipLaunchKernelGGL(k_frac_finish, dim3(blocks), dim3(256), 0, s, u_in, be, bk, HW, steps, win.r_ss,
                       win.r_fs, u_out, err_min, argmin);
    profile_end("pm_frac", s, 0, nullptr, 0);
    return check_hip(hipGetLastError(), "fractional pixel-map search");
}

}  // namespace pxst

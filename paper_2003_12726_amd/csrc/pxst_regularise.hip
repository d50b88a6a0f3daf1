// Pixel-map regularisation (Sec. 2.2.2, closing paragraphs): a Gaussian filter of the
// map, then the irrotational constraint -- the map is replaced by the gradient of its
// least-squares potential.
//
// Filter: two passes (axis 0, then axis 1) of the sampled Gaussian exp(-k^2 / (2 s^2)),
// |k| <= int(4 s + 0.5), normalised to unit sum, nearest-pixel boundaries; float64
// sums, one thread per output value (the passes are bandwidth-bound).
//
// Potential: Phi minimises the squared misfit of its forward differences against the
// trapezoid means of u along each axis.  The paper solves the normal equations
// D^T D Phi = D^T t by conjugate gradients; here they are solved directly: D^T D is
// the Neumann Laplacian, diagonal in the orthonormal type-II DCT basis with
// eigenvalues (2 - 2 cos(pi k / H)) + (2 - 2 cos(pi l / W)).  The 2-D transforms are
// four float64 matrix products with the DCT matrices (plain library GEMMs); the
// right-hand side, the spectral division and the gradient are kernels of their own.
// The new map is the gradient of Phi: central differences inside, second-order
// one-sided differences at the edges, first order along an axis of two pixels; an
// axis of one pixel keeps its component.
#include <rocblas/rocblas.h>

#include <cmath>
#include <mutex>

#include "pxst_device.hpp"
#include "pxst_internal.hpp"

namespace pxst {

namespace {

// Filter weights w[k + R], k in [-R, R], normalised in index order (one thread).
__global__ void k_gauss_weights(double sigma, int R, double* __restrict__ w) {
    for (int k = threadIdx.x; k <= 2 * R; k += blockDim.x) {
        const double x = (double)(k - R);
        w[k] = exp(-(x * x) / (2.0 * sigma * sigma));
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k <= 2 * R; ++k) s += w[k];
        for (int k = 0; k <= 2 * R; ++k) w[k] /= s;
    }
}

// One filter pass along `axis` of both components: out[c][i][j] = sum_k w[k] in[...]
// with the index along the axis clamped to the detector.
template <typename Tin, typename Tout>
__global__ void k_gauss_axis(const Tin* __restrict__ in, Tout* __restrict__ out, int H, int W, int axis,
                             const double* __restrict__ w, int R) {
    const size_t HW = (size_t)H * W;
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 2 * HW) return;
    const size_t c = e / HW, p = e - c * HW;
    const int i = (int)(p / W), j = (int)(p - (size_t)i * W);
    const Tin* src = in + c * HW;
    double acc = 0.0;
    if (axis == 0) {
        for (int k = -R; k <= R; ++k) {
            const int ii = min(max(i + k, 0), H - 1);
            acc += w[k + R] * (double)src[(size_t)ii * W + j];
        }
    } else {
        for (int k = -R; k <= R; ++k) {
            const int jj = min(max(j + k, 0), W - 1);
            acc += w[k + R] * (double)src[(size_t)i * W + jj];
        }
    }
    out[e] = (Tout)acc;
}

// Orthonormal type-II DCT matrix, column-major n x n: C[k + i n] = s_k cos(pi k (2i+1) / 2n).
__global__ void k_dct_matrix(double* __restrict__ C, int n) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)n * n) return;
    const int k = (int)(e % n), i = (int)(e / n);
    const double s = k == 0 ? sqrt(1.0 / n) : sqrt(2.0 / n);
    C[e] = s * cos(M_PI * (double)k * (double)(2 * i + 1) / (2.0 * n));
}

// b = D^T t: at (i, j), t0[i-1] - t0[i] + t1[j-1] - t1[j] over the differences that
// exist, t the trapezoid means of u; row-major [H][W] float64.
__global__ void k_integ_rhs(const float* __restrict__ u, int H, int W, double* __restrict__ b) {
    const size_t HW = (size_t)H * W;
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= HW) return;
    const int i = (int)(p / W), j = (int)(p - (size_t)i * W);
    const float* u0 = u;
    const float* u1 = u + HW;
    auto t0 = [&](int ii) { return 0.5 * ((double)u0[(size_t)(ii + 1) * W + j] + (double)u0[(size_t)ii * W + j]); };
    auto t1 = [&](int jj) { return 0.5 * ((double)u1[(size_t)i * W + jj + 1] + (double)u1[(size_t)i * W + jj]); };
    double v = 0.0;
    if (i >= 1) v += t0(i - 1);
    if (i <= H - 2) v -= t0(i);
    if (j >= 1) v += t1(j - 1);
    if (j <= W - 2) v -= t1(j);
    b[p] = v;
}

// Spectral division of the transformed right-hand side (column-major W x H: element
// (l, k) at l + k W, l the frequency along axis 1, k along axis 0); the constant term
// (the null space) is set to zero.
__global__ void k_integ_scale(double* __restrict__ X, int H, int W) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)H * W) return;
    const int l = (int)(e % W), k = (int)(e / W);
    const double lam = (2.0 - 2.0 * cos(M_PI * (double)k / H)) + (2.0 - 2.0 * cos(M_PI * (double)l / W));
    X[e] = e == 0 ? 0.0 : X[e] / lam;
}

// Derivative of phi along one axis at index q of n samples with stride st.
__device__ inline double axis_gradient(const double* __restrict__ f, size_t base, int q, int n, size_t st) {
    if (n == 2) return q == 0 ? f[base + st] - f[base] : f[base] - f[base - st];
    if (q == 0) return -1.5 * f[base] + 2.0 * f[base + st] - 0.5 * f[base + 2 * st];
    if (q == n - 1) return 0.5 * f[base - 2 * st] - 2.0 * f[base - st] + 1.5 * f[base];
    return 0.5 * (f[base + st] - f[base - st]);
}

// u_out = gradient of phi (row-major [H][W]); an axis of one pixel keeps u_in's
// component (u_out may be u_in).
__global__ void k_integ_grad(const double* __restrict__ phi, const float* u_in, int H, int W, float* u_out) {
    const size_t HW = (size_t)H * W;
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= HW) return;
    const int i = (int)(p / W), j = (int)(p - (size_t)i * W);
    const float g0 = H == 1 ? u_in[p] : (float)axis_gradient(phi, p, i, H, (size_t)W);
    const float g1 = W == 1 ? u_in[HW + p] : (float)axis_gradient(phi, p, j, W, 1);
    u_out[p] = g0;
    u_out[HW + p] = g1;
}

inline unsigned blocks_of(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

// One library handle per device, shared by the calls of this process; the stream is set
// under the lock for every sequence of products.
std::mutex g_blas_mu;
rocblas_handle g_blas[64] = {};

int blas_status(rocblas_status st, const char* what) {
    if (st == rocblas_status_success) return PXST_OK;
    set_error("%s: rocBLAS status %d", what, (int)st);
    return PXST_EHIP;
}

}  // namespace

int launch_regularise(const Geom& g, const float* u_in, float* u_out, float sigma, int integrate, char* ws,
                      const Layout& L, hipStream_t s) {
    const int H = g.H, W = g.W;
    const size_t HW = g.HW();
    const float* src = u_in;
    if (sigma > 0.f) {
        const int R = (int)(4.0 * (double)sigma + 0.5);
        double* w = (double*)(ws + L.gw);
        double* tmp = (double*)(ws + L.gtmp);
        profile_begin("reg_filter", s);
        hipLaunchKernelGGL(k_gauss_weights, dim3(1), dim3(256), 0, s, (double)sigma, R, w);
        hipLaunchKernelGGL((k_gauss_axis<float, double>), dim3(blocks_of(2 * HW, 256)), dim3(256), 0, s, u_in,
                           tmp, H, W, 0, w, R);
        hipLaunchKernelGGL((k_gauss_axis<double, float>), dim3(blocks_of(2 * HW, 256)), dim3(256), 0, s, tmp,
                           u_out, H, W, 1, w, R);
        // work units: output values times taps, per pass
        profile_end("reg_filter", s, 2LL * 2 * (long long)HW * (2 * R + 1), nullptr, 0);
        src = u_out;
        int rc = check_hip(hipGetLastError(), "pixel-map filter");
        if (rc) return rc;
    } else if (!integrate && u_out != u_in) {
        hipMemcpyAsync(u_out, u_in, 2 * HW * sizeof(float), hipMemcpyDeviceToDevice, s);
    }
    if (!integrate) return check_hip(hipGetLastError(), "pixel-map regularisation");
    if (!L.integ) {
        set_error("workspace laid out without the integration buffers (pm_integrate = 0)");
        return PXST_EWORKSPACE;
    }
    double* CH = (double*)(ws + L.dct_h);
    double* CW = (double*)(ws + L.dct_w);
    double* X = (double*)(ws + L.ibuf0);
    double* T = (double*)(ws + L.ibuf1);
    profile_begin("reg_integrate", s);
    hipLaunchKernelGGL(k_dct_matrix, dim3(blocks_of((size_t)H * H, 256)), dim3(256), 0, s, CH, H);
    hipLaunchKernelGGL(k_dct_matrix, dim3(blocks_of((size_t)W * W, 256)), dim3(256), 0, s, CW, W);
    hipLaunchKernelGGL(k_integ_rhs, dim3(blocks_of(HW, 256)), dim3(256), 0, s, src, H, W, X);
    int rc = check_hip(hipGetLastError(), "pixel-map integration");
    if (rc) return rc;
    {
        // row-major [H][W] arrays are column-major W x H matrices: the 2-D transform of b
        // is C_W b^T C_H^T, its inverse C_W^T X C_H
        std::lock_guard<std::mutex> lock(g_blas_mu);
        int dev = 0;
        if ((rc = check_hip(hipGetDevice(&dev), "device"))) return rc;
        if (dev < 0 || dev >= 64) {
            set_error("device index %d out of range", dev);
            return PXST_EUNSUPPORTED;
        }
        if (!g_blas[dev] && (rc = blas_status(rocblas_create_handle(&g_blas[dev]), "rocblas_create_handle")))
            return rc;
        rocblas_handle h = g_blas[dev];
        if ((rc = blas_status(rocblas_set_stream(h, s), "rocblas_set_stream"))) return rc;
        const double one = 1.0, zero = 0.0;
        // T = C_W X ; X = T C_H^T ; scale ; T = C_W^T X ; X = T C_H
        if ((rc = blas_status(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, W, H, W, &one, CW,
                                            W, X, W, &zero, T, W),
                              "DCT (axis 1)")))
            return rc;
        if ((rc = blas_status(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, W, H, H, &one,
                                            T, W, CH, H, &zero, X, W),
                              "DCT (axis 0)")))
            return rc;
        hipLaunchKernelGGL(k_integ_scale, dim3(blocks_of(HW, 256)), dim3(256), 0, s, X, H, W);
        if ((rc = blas_status(rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, W, H, W, &one,
                                            CW, W, X, W, &zero, T, W),
                              "inverse DCT (axis 1)")))
            return rc;
        if ((rc = blas_status(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, W, H, H, &one, T,
                                            W, CH, H, &zero, X, W),
                              "inverse DCT (axis 0)")))
            return rc;
    }
    hipLaunchKernelGGL(k_integ_grad, dim3(blocks_of(HW, 256)), dim3(256), 0, s, X, src, H, W, u_out);
    // work units: float64 operations of the four transforms
    profile_end("reg_integrate", s, 4LL * (long long)HW * (H + W), nullptr, 0);
    return check_hip(hipGetLastError(), "pixel-map integration");
}

}  // namespace pxst

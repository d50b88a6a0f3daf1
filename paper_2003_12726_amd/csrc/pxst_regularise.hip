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

#include <cmath>

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

// ------------------------------------------------------------- transform products
// The four products of the integration, each a float64 matrix product in which one
// operand is the orthonormal type-II DCT matrix of length n,
//   C(k, i) = s_k cos(pi k (2 i + 1) / (2 n)),  s_0 = sqrt(1 / n), s_k = sqrt(2 / n),
// and the other a column-major data matrix D (ld = its row count):
//   mode 0: out = C D      (n x n times n x N)
//   mode 1: out = C^T D
//   mode 2: out = D C^T    (M x n times n x n)
//   mode 3: out = D C
// The DCT operand is not stored: it is generated from a table of cos(pi t / (2 n)),
// t = 0..n, in LDS (the argument k (2 i + 1) is reduced modulo 4 n exactly, in
// integers, then folded by the symmetries of the cosine).  The products run on the
// matrix cores (v_mfma_f64_16x16x4f64: a 16 x 4 block of the left operand times a 4 x
// 16 block of the right one per instruction; lane l holds L(l mod 16, l div 16) and
// R(l div 16, l mod 16) and receives out(4 j + l div 16, l mod 16) in its j-th
// accumulator element).  A work-group computes a 32 x 32 block of out: each of its
// eight waves (two per SIMD) takes an eighth of the contraction for all four 16 x 16
// sub-blocks (four independent accumulation chains), loading the next k-steps'
// operands before it issues the current ones' products, and the eighths are added in
// LDS in a fixed order.  Mode 2 can also apply the spectral division of the integration to its
// output (out(l, k) / lambda(k, l), the constant term set to zero).
typedef double dbl4 __attribute__((ext_vector_type(4)));
constexpr int DG_TILE = 32, DG_WAVES = 8, DG_THREADS = 64 * DG_WAVES, DG_UNROLL = 4;

// The table's bytes and the reduction's share one dynamic LDS buffer.
inline size_t dct_lds_bytes(int n) {
    const size_t tab = (size_t)(n + 1) * sizeof(double);
    const size_t red = (size_t)DG_WAVES * DG_TILE * DG_TILE * sizeof(double);
    return tab > red ? tab : red;
}

// cos(pi t / (2 n)) for t in [0, 4 n) from tab[s] = cos(pi s / (2 n)), s = 0..n.
__device__ inline double dct_cos(const double* tab, int t, int n) {
    int u = t <= 2 * n ? t : 4 * n - t;   // even about 2 n
    const bool neg = u > n;                // odd about n
    u = neg ? 2 * n - u : u;
    const double c = tab[u];
    return neg ? -c : c;
}

// t + d reduced into [0, 4 n), for t in [0, 4 n) and d in [0, 8 n).
__device__ inline int mod4n_add(int t, int d, int n4) {
    t += d;
    t = t >= n4 ? t - n4 : t;
    return t >= n4 ? t - n4 : t;
}

template <int MODE, bool SCALE>
__global__ __launch_bounds__(DG_THREADS) void k_dct_gemm(const double* __restrict__ D, int ldd,
                                                         double* __restrict__ out, int M, int N, int K,
                                                         int n, int H, int W) {
    extern __shared__ double lds[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = lane & 15, q = lane >> 4;
    const int m0 = blockIdx.x * DG_TILE, n0 = blockIdx.y * DG_TILE;
    const int n4 = 4 * n;
    for (int t = threadIdx.x; t <= n; t += DG_THREADS) lds[t] = cos(M_PI * (double)t / (2.0 * (double)n));
    const double s0 = sqrt(1.0 / (double)n), s1 = sqrt(2.0 / (double)n);
    __syncthreads();
    // this wave's share of the contraction: K / 8 rounded up to a multiple of 4
    const int kq = ((K + 4 * DG_WAVES - 1) / (4 * DG_WAVES)) * 4;
    const int kb = min(K, wave * kq), ke = min(K, kb + kq);
    // DCT operand of the lane's two fragments (rows m0 + r, m0 + 16 + r of the left
    // operand in modes 0 and 1, columns n0 + r, n0 + 16 + r of the right one in modes 2
    // and 3) at contraction index k = k0 + q: t = a k + b (mod 4 n), stepped by 4 a per
    // k-step of 4
    const int f0 = (MODE <= 1 ? m0 : n0) + r, f1 = f0 + 16;
    const bool in0 = f0 < (MODE <= 1 ? M : N), in1 = f1 < (MODE <= 1 ? M : N);
    // modes 0 and 2: C(f, k): t = f (2 k + 1);  modes 1 and 3: C(k, f): t = k (2 f + 1)
    const int a0 = (MODE == 0 || MODE == 2) ? 2 * f0 : 2 * f0 + 1;
    const int a1 = (MODE == 0 || MODE == 2) ? 2 * f1 : 2 * f1 + 1;
    const int c0 = (MODE == 0 || MODE == 2) ? f0 : 0, c1 = (MODE == 0 || MODE == 2) ? f1 : 0;
    auto start = [&](int a, int c, int k) { return (int)(((long long)a * k + c) % n4); };
    const int kq0 = kb + q;
    int t0 = start(a0 % n4, c0 % n4, kq0), t1 = start(a1 % n4, c1 % n4, kq0);
    const int d0 = (int)((4LL * a0) % n4), d1 = (int)((4LL * a1) % n4);
    // scale of a DCT entry: s of its row index (f in modes 0 and 2, k in modes 1 and 3)
    const double sf0 = f0 == 0 ? s0 : s1, sf1 = f1 == 0 ? s0 : s1;
    auto cop = [&](int t, int k, double sf, bool in) -> double {
        if (!in || k >= ke) return 0.0;
        const double c = dct_cos(lds, t, n);
        return (MODE == 0 || MODE == 2) ? sf * c : (k == 0 ? s0 : s1) * c;
    };
    // data operand: modes 0 and 1: D(k, col) for col = n0 + r (+16); modes 2 and 3:
    // D(row, k) for row = m0 + r (+16)
    auto dop = [&](int k, int idx) -> double {
        if (k >= ke) return 0.0;
        if (MODE <= 1) return idx < N ? D[(size_t)k + (size_t)idx * ldd] : 0.0;
        return idx < M ? D[(size_t)idx + (size_t)k * ldd] : 0.0;
    };
    const int g0 = (MODE <= 1 ? n0 : m0) + r, g1 = g0 + 16;
    dbl4 acc00 = {0.0, 0.0, 0.0, 0.0}, acc01 = acc00, acc10 = acc00, acc11 = acc00;
    double ca0[DG_UNROLL], ca1[DG_UNROLL], da0[DG_UNROLL], da1[DG_UNROLL];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int u = 0; u < DG_UNROLL; ++u) {
            const int k = k0 + 4 * u + q;
            ca0[u] = cop(t0, k, sf0, in0);
            ca1[u] = cop(t1, k, sf1, in1);
            t0 = mod4n_add(t0, d0, n4);
            t1 = mod4n_add(t1, d1, n4);
            da0[u] = dop(k, g0);
            da1[u] = dop(k, g1);
        }
    };
    if (kb < ke) fetch(kb);
    for (int k0 = kb; k0 < ke; k0 += 4 * DG_UNROLL) {
        double xa0[DG_UNROLL], xa1[DG_UNROLL], xb0[DG_UNROLL], xb1[DG_UNROLL];
#pragma unroll
        for (int u = 0; u < DG_UNROLL; ++u) {
            xa0[u] = ca0[u];
            xa1[u] = ca1[u];
            xb0[u] = da0[u];
            xb1[u] = da1[u];
        }
        if (k0 + 4 * DG_UNROLL < ke) fetch(k0 + 4 * DG_UNROLL);
#pragma unroll
        for (int u = 0; u < DG_UNROLL; ++u) {
            // left operand rows (16-blocks 0 and 1) times right operand columns
            const double l0 = MODE <= 1 ? xa0[u] : xb0[u], l1 = MODE <= 1 ? xa1[u] : xb1[u];
            const double r0 = MODE <= 1 ? xb0[u] : xa0[u], r1 = MODE <= 1 ? xb1[u] : xa1[u];
            acc00 = __builtin_amdgcn_mfma_f64_16x16x4f64(l0, r0, acc00, 0, 0, 0);
            acc01 = __builtin_amdgcn_mfma_f64_16x16x4f64(l0, r1, acc01, 0, 0, 0);
            acc10 = __builtin_amdgcn_mfma_f64_16x16x4f64(l1, r0, acc10, 0, 0, 0);
            acc11 = __builtin_amdgcn_mfma_f64_16x16x4f64(l1, r1, acc11, 0, 0, 0);
        }
    }
    // eighths of the contraction added in a fixed order through LDS (which the table no
    // longer needs); two output elements per thread
    __syncthreads();
    {
        double* red = lds + (size_t)wave * DG_TILE * DG_TILE;
        const dbl4* accs[4] = {&acc00, &acc01, &acc10, &acc11};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int bm = (t >> 1) * 16, bn = (t & 1) * 16;
#pragma unroll
            for (int j = 0; j < 4; ++j) red[(bm + 4 * j + q) * DG_TILE + bn + r] = (*accs[t])[j];
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < DG_TILE * DG_TILE; e += DG_THREADS) {
        const int i = e % DG_TILE, c = e / DG_TILE;
        const int gm = m0 + i, gn = n0 + c;
        if (gm >= M || gn >= N) continue;
        double v = 0.0;
#pragma unroll
        for (int w = 0; w < DG_WAVES; ++w) v += lds[(size_t)w * DG_TILE * DG_TILE + i * DG_TILE + c];
        if (SCALE) {
            // out(l, k): l the frequency along axis 1 (of W), k along axis 0 (of H)
            const double lam = (2.0 - 2.0 * cos(M_PI * (double)gn / H)) + (2.0 - 2.0 * cos(M_PI * (double)gm / W));
            v = (gm == 0 && gn == 0) ? 0.0 : v / lam;
        }
        out[(size_t)gm + (size_t)gn * M] = v;
    }
}

template <int MODE, bool SCALE>
void dct_gemm(const double* D, int ldd, double* out, int M, int N, int K, int n, int H, int W, hipStream_t s) {
    const size_t sh = dct_lds_bytes(n);
    (void)hipFuncSetAttribute((const void*)k_dct_gemm<MODE, SCALE>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)sh);
    const dim3 grid((M + DG_TILE - 1) / DG_TILE, (N + DG_TILE - 1) / DG_TILE);
    k_dct_gemm<MODE, SCALE><<<grid, dim3(DG_THREADS), sh, s>>>(D, ldd, out, M, N, K, n, H, W);
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
    double* X = (double*)(ws + L.ibuf0);
    double* T = (double*)(ws + L.ibuf1);
    profile_begin("reg_integrate", s);
    hipLaunchKernelGGL(k_integ_rhs, dim3(blocks_of(HW, 256)), dim3(256), 0, s, src, H, W, X);
    // row-major [H][W] arrays are column-major W x H matrices: the 2-D transform of b is
    // C_W b^T C_H^T, its inverse C_W^T X C_H (C_n the DCT matrix of length n).
    // T = C_W X ; X = T C_H^T / lambda ; T = C_W^T X ; X = T C_H
    dct_gemm<0, false>(X, W, T, W, H, W, W, H, W, s);
    dct_gemm<2, true>(T, W, X, W, H, H, H, H, W, s);
    dct_gemm<1, false>(X, W, T, W, H, W, W, H, W, s);
    dct_gemm<3, false>(T, W, X, W, H, H, H, H, W, s);
    hipLaunchKernelGGL(k_integ_grad, dim3(blocks_of(HW, 256)), dim3(256), 0, s, X, src, H, W, u_out);
    // work units: float64 operations of the four transforms
    profile_end("reg_integrate", s, 4LL * (long long)HW * (H + W), nullptr, 0);
    return check_hip(hipGetLastError(), "pixel-map integration");
}

}  // namespace pxst

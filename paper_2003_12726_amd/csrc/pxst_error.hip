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
    // (unrolled so that the loads of several frames are in flight; same order of sums)
#pragma unroll 8
    for (int n = 0; n < N; ++n) {
        const float v = (float)frames[(size_t)n * HW + pix] - Wp;
        P = fmaf(v, v, P);
        if (((n + 1) & 31) == 0) two_sum_fold(S, P);
    }
    s2[pix] = (S + P) / (float)N;
}


// Lookup of Sec. 4 from four corner values (NaN: invalid or outside the grid).
__device__ inline float masked_bilinear4(float v00, float v01, float v10, float v11, float fa, float fb) {
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

// The value of lane (this lane xor off) through the LDS permute unit; addr = 4 (lane
// xor off), formed once per exchange step rather than per 32-bit half of every value.
__device__ inline double lane_xor(double v, int addr) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)b);
    const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sums of ERR_FB per-lane values over the wave, fixed order: three exchange steps that
// each halve the values a lane keeps (lane bit 5, 4, 3 picks the half), then three
// plain steps over lane bits 2, 1, 0.  Lane l ends with the sum of value
// 4 b5 + 2 b4 + b3 (b = bits of l).
constexpr int ERR_FB = 8;
__device__ inline double wave_sum8(double (&v)[ERR_FB], int lane) {
#pragma unroll
    for (int st = 0; st < 3; ++st) {
        const int off = 32 >> st, half = ERR_FB >> (st + 1);
        const bool hi = (lane & off) != 0;
        const int addr = (lane ^ off) << 2;
#pragma unroll
        for (int k = 0; k < half; ++k) {
            // (the empty asm makes the two values opaque: otherwise the compiler turns the
            // selects into a read of the array at a run-time index, a compare-and-select
            // chain over all ERR_FB values)
            double a = v[k], b = v[k + half];
            asm("" : "+v"(a), "+v"(b));
            const double send = hi ? a : b;
            const double keep = hi ? b : a;
            v[k] = keep + lane_xor(send, addr);
        }
    }
    double r = v[0];
#pragma unroll
    for (int off = 4; off > 0; off >>= 1) r += lane_xor(r, (lane ^ off) << 2);
    return r;
}

// One thread per pixel; frames in groups of ERR_FB whose loads are all issued before
// the group is evaluated.  Per-frame sums of the wave go to LDS, then one partial per
// block and frame to the workspace.  PAIRS (a grid of at least 2x2): the four corners
// come from two 8-byte loads of the 2x2 block at the lookup clamped into the grid, each
// corner inside the grid at its own row and column of the block; otherwise four loads
// at the corners clamped one by one.
template <bool PAIRS, bool BATCH>
__global__ __launch_bounds__(ERR_THREADS) void k_err_pixels(const ErrArgs* __restrict__ jobs, ErrArgs one) {
    extern __shared__ double wsum_sh[];   // [N][waves], then the frame table [N]
    constexpr int WAVES = ERR_THREADS / 64;
    const ErrArgs a = job_args<BATCH>(jobs, one);
    if ((int)blockIdx.x >= a.nblk) return;
    // per frame: the fractions of its shift and the integer parts (bits of ints)
    float4* ftab = (float4*)(wsum_sh + (size_t)a.N * WAVES);
    for (int n = threadIdx.x; n < a.N; n += ERR_THREADS) {
        const float d0 = a.dx[2 * n], d1 = a.dx[2 * n + 1];
        const float sd0 = floorf(d0), sd1 = floorf(d1);
        ftab[n] = make_float4(d0 - sd0, d1 - sd1, __int_as_float((int)sd0), __int_as_float((int)sd1));
    }
    __syncthreads();
    const size_t HW = (size_t)a.H * a.W;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const size_t pix = (size_t)blockIdx.x * ERR_THREADS + threadIdx.x;
    const bool inb = pix < HW;
    const size_t pc = inb ? pix : 0;
    const bool use = inb && a.mask[pc] != 0 && a.s2[pc] > 0.f;
    const float Wp = a.white[pc];
    const float s2 = a.s2[pc];
    const float inv_s2 = use ? 1.f / s2 : 0.f;
    const float u0 = a.u[pc], u1 = a.u[HW + pc];
    const float f0 = floorf(u0), f1 = floorf(u1);
    const float fu0 = u0 - f0, fu1 = u1 - f1;
    const int i0 = (int)f0 - a.o0, i1 = (int)f1 - a.o1;
    // the pixel's error summed in float64 over its frames
    double pS = 0.0;
    for (int n0 = 0; n0 < a.N; n0 += ERR_FB) {
        // PAIRS: v holds the 2x2 block read at the lookup clamped into the grid; else the
        // four corners clamped one by one
        float v[ERR_FB][4], I[ERR_FB], fa[ERR_FB], fb[ERR_FB];
        int rr[ERR_FB], cq[ERR_FB];
#pragma unroll
        for (int t = 0; t < ERR_FB; ++t) {
            const int n = min(n0 + t, a.N - 1);
            const float4 ft = ftab[n];
            const float t0 = fu0 - ft.x, t1 = fu1 - ft.y;
            const int r = i0 - __float_as_int(ft.z) - (t0 < 0.f ? 1 : 0);
            const int c = i1 - __float_as_int(ft.w) - (t1 < 0.f ? 1 : 0);
            rr[t] = r;
            cq[t] = c;
            fa[t] = t0 < 0.f ? t0 + 1.f : t0;
            fb[t] = t1 < 0.f ? t1 + 1.f : t1;
            if constexpr (PAIRS) {
                const int rc = min(max(r, 0), a.Rs - 2), ccl = min(max(c, 0), a.Rf - 2);
                const float* bp = a.refv + ((unsigned)rc * (unsigned)a.Rf + (unsigned)ccl);
                const float2 top = *(const float2*)bp;
                const float2 bot = *(const float2*)(bp + a.Rf);
                v[t][0] = top.x;
                v[t][1] = top.y;
                v[t][2] = bot.x;
                v[t][3] = bot.y;
            } else {
                const int ra = min(max(r, 0), a.Rs - 1), rb = min(max(r + 1, 0), a.Rs - 1);
                const int ca = min(max(c, 0), a.Rf - 1), cb = min(max(c + 1, 0), a.Rf - 1);
                v[t][0] = a.refv[(size_t)ra * a.Rf + ca];
                v[t][1] = a.refv[(size_t)ra * a.Rf + cb];
                v[t][2] = a.refv[(size_t)rb * a.Rf + ca];
                v[t][3] = a.refv[(size_t)rb * a.Rf + cb];
            }
            I[t] = (float)a.frames[(size_t)n * HW + pc];
        }
        // the common case, taken when it holds for every lane of the wave: every frame's
        // four corners inside the grid and valid (a NaN reaches the corners' sum); lanes
        // whose pixel is not used contribute zeros either way
        bool fast = true;
#pragma unroll
        for (int t = 0; t < ERR_FB; ++t) {
            const bool in = (unsigned)rr[t] <= (unsigned)(a.Rs - 2) && (unsigned)cq[t] <= (unsigned)(a.Rf - 2);
            fast = fast && in && valid((v[t][0] + v[t][1]) + (v[t][2] + v[t][3]));
        }
        double e[ERR_FB];
        if (__all(fast || !use)) {
#pragma unroll
            for (int t = 0; t < ERR_FB; ++t) {
                const float h0 = fmaf(fb[t], v[t][1] - v[t][0], v[t][0]);
                const float h1 = fmaf(fb[t], v[t][3] - v[t][2], v[t][2]);
                const float g = fmaf(fa[t], h1 - h0, h0);
                const float res = fmaf(-Wp, g, I[t]);
                const float eps = (res * res) * inv_s2;
                e[t] = (double)(use && n0 + t < a.N ? eps : 0.f);
                pS += e[t];
            }
        } else {
#pragma unroll
        for (int t = 0; t < ERR_FB; ++t) {
            const int r = rr[t], c = cq[t];
            // all four corners inside the grid: the values read are the corners
            const bool in = (unsigned)r <= (unsigned)(a.Rs - 2) && (unsigned)c <= (unsigned)(a.Rf - 2);
            float g;
            if (in && valid(v[t][0]) && valid(v[t][1]) && valid(v[t][2]) && valid(v[t][3])) {
                const float h0 = fmaf(fb[t], v[t][1] - v[t][0], v[t][0]);
                const float h1 = fmaf(fb[t], v[t][3] - v[t][2], v[t][2]);
                g = fmaf(fa[t], h1 - h0, h0);
            } else {
                // corner flags: bit 0 row r, bit 1 row r + 1, bit 2 column c, bit 3 column c + 1
                const unsigned k = ((unsigned)r < (unsigned)a.Rs ? 1u : 0u) |
                                   ((unsigned)(r + 1) < (unsigned)a.Rs ? 2u : 0u) |
                                   ((unsigned)c < (unsigned)a.Rf ? 4u : 0u) |
                                   ((unsigned)(c + 1) < (unsigned)a.Rf ? 8u : 0u);
                float v00 = v[t][0], v01 = v[t][1], v10 = v[t][2], v11 = v[t][3];
                if constexpr (PAIRS) {
                    // the block row of the lookup's first row is 1 only where the clamp
                    // moved the block up (r = Rs - 1), that of its second row 0 only where
                    // it moved it down (r = -1); the same for the columns
                    const int rc = min(max(r, 0), a.Rs - 2), ccl = min(max(c, 0), a.Rf - 2);
                    const float2 top = make_float2(v[t][0], v[t][1]), bot = make_float2(v[t][2], v[t][3]);
                    const float2 h0 = r > rc ? bot : top, h1 = r < rc ? top : bot;
                    const bool x0 = c > ccl, x1 = c < ccl;
                    v00 = x0 ? h0.y : h0.x;
                    v01 = x1 ? h0.x : h0.y;
                    v10 = x0 ? h1.y : h1.x;
                    v11 = x1 ? h1.x : h1.y;
                }
                const float q = qnan();
                g = masked_bilinear4((k & 5u) == 5u ? v00 : q, (k & 9u) == 9u ? v01 : q, (k & 6u) == 6u ? v10 : q,
                                     (k & 10u) == 10u ? v11 : q, fa[t], fb[t]);
            }
            e[t] = 0.0;
            if (use && n0 + t < a.N && valid(g)) {
                const float res = fmaf(-Wp, g, I[t]);
                e[t] = (double)((res * res) * inv_s2);
            }
            pS += e[t];
        }
        }
        const double fsum = wave_sum8(e, lane);
        const int f = n0 + ((lane >> 3) & 7);
        if ((lane & 7) == 0 && f < a.N) wsum_sh[(size_t)f * WAVES + wave] = fsum;
    }
    if (a.pixel_err && inb) a.pixel_err[pix] = use ? (float)pS : 0.f;
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
template <bool BATCH>
__global__ __launch_bounds__(64) void k_err_frames(const ErrArgs* __restrict__ jobs, ErrArgs one) {
    const ErrArgs a = job_args<BATCH>(jobs, one);
    const int n = blockIdx.x;
    if (n >= a.N) return;
    double acc = 0.0;
    for (int b = threadIdx.x; b < a.nblk; b += 64) acc += a.part[(size_t)n * a.nblk + b];
    acc = wave_sum<double>(acc);
    if (threadIdx.x == 0) {
        a.frame_err[n] = acc;
        if (a.frame_out) a.frame_out[n] = acc;
    }
}

// Total: the frame errors added by one wave in the same fixed order.
template <bool BATCH>
__global__ __launch_bounds__(64) void k_err_total(const ErrArgs* __restrict__ jobs, ErrArgs one) {
    const ErrArgs a = job_args<BATCH>(jobs, one);
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

ErrArgs make_err_args(const Geom& g, const pxst_scan& sc, const float* refv, const float* s2, const float* u,
                      const float* dx, float* pixel_err, double* frame_err, double* total, char* ws,
                      const Layout& L) {
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
    a.nblk = (int)((g.HW() + ERR_THREADS - 1) / ERR_THREADS);
    a.part = (double*)(ws + L.err_part);
    a.frame_err = (double*)(ws + L.err_pix);
    a.frame_out = frame_err;
    a.total = total;
    return a;
}

// LDS of the pixel pass: per-wave frame sums and the frame table.
template <bool PAIRS, bool BATCH>
static void launch_err_pixels(int nblk, int n, size_t sh, hipStream_t s, const ErrArgs* dev, const ErrArgs& one) {
    // (up to 1920 frames: 92 KB, above the default limit of dynamic LDS)
    (void)hipFuncSetAttribute((const void*)k_err_pixels<PAIRS, BATCH>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    k_err_pixels<PAIRS, BATCH><<<dim3(nblk, 1, n), dim3(ERR_THREADS), sh, s>>>(dev, one);
}

static size_t err_lds(int N) { return (size_t)N * (ERR_THREADS / 64) * sizeof(double) + (size_t)N * sizeof(float4); }

// The three passes for the jobs of `host` (their arguments also in device memory at
// `dev`, or one job passed by value when dev is null).  Every job's grid is its own;
// the launch covers the largest and blocks past a job's grid return at once.
int launch_error_jobs(const ErrArgs* host, int n, const ErrArgs* dev, hipStream_t s) {
    int nblk = 1, nf = 1, maxN = 1;
    bool pairs = true;
    for (int j = 0; j < n; ++j) {
        nblk = std::max(nblk, host[j].nblk);
        nf = std::max(nf, host[j].N);
        maxN = std::max(maxN, host[j].N);
        pairs = pairs && host[j].Rs >= 2 && host[j].Rf >= 2;
    }
    for (int j = 0; j < n && dev; ++j)
        if ((host[j].Rs >= 2 && host[j].Rf >= 2) != pairs) {
            set_error("batched error pass: jobs differ in the reference lookup form");
            return PXST_EINVAL;
        }
    const size_t sh = err_lds(maxN);
    if (sh > 150 * 1024) {
        set_error("error evaluation supports at most %d frames", (int)(150 * 1024 / 48));
        return PXST_EUNSUPPORTED;
    }
    const ErrArgs one = dev ? ErrArgs{} : host[0];
    long long work = 0;
    for (int j = 0; j < n; ++j) work += (long long)host[j].H * host[j].W * host[j].N;
    profile_begin("err_pixels", s);
    if (pairs) {
        if (dev) launch_err_pixels<true, true>(nblk, n, sh, s, dev, one);
        else launch_err_pixels<true, false>(nblk, n, sh, s, dev, one);
    } else {
        if (dev) launch_err_pixels<false, true>(nblk, n, sh, s, dev, one);
        else launch_err_pixels<false, false>(nblk, n, sh, s, dev, one);
    }
    profile_end("err_pixels", s, work, nullptr, 0);
    PXST_LAUNCH_JOBS(k_err_frames, dim3(nf, 1, n), dim3(64), 0, s, dev, one);
    PXST_LAUNCH_JOBS(k_err_total, dim3(1, 1, n), dim3(64), 0, s, dev, one);
    return check_hip(hipGetLastError(), "error evaluation");
}

int launch_error(const Geom& g, const pxst_scan& sc, const float* refv, const float* s2,
                 const float* u, const float* dx, float* pixel_err, double* frame_err,
                 double* total, char* ws, const Layout& L, hipStream_t s) {
    const ErrArgs a = make_err_args(g, sc, refv, s2, u, dx, pixel_err, frame_err, total, ws, L);
    return launch_error_jobs(&a, 1, nullptr, s);
}

}  // namespace pxst

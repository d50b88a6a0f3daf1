// Pixel-map search (Sec. 2.2.2): brute-force integer candidates, normalised error,
// first minimum, paraboloid refinement.
//
// Candidates are integer points c + k, so for frame n every lookup has the same
// bilinear fractions (those of dx_n): the reference interpolated for frame n is a
// fixed image G_n, and the error of candidate k at a pixel is a sum over frames of
// (I - W G_n[c + k - shift_n])^2.  A work-group owns an 8 x 8 tile of pixels and all
// of their candidates; per frame it stages the part of G_n that the tile's windows
// touch into LDS (double buffered) and every lane then evaluates its block of
// candidates from LDS with two FMAs each.  Tiles are classified first:
//   FAST    every staged value of every frame is a valid lookup (no per-candidate
//           bookkeeping: the variance is the same for all candidates);
//   EDGE    some lookups are invalid: per-candidate variance and frame counts;
//   GENERIC the staged region does not fit the LDS budget (widely scattered map):
//           no staging, lookups straight from the reference.
#include <algorithm>

#include "pxst_device.hpp"
#include <memory>

#include "pxst_internal.hpp"

namespace pxst {

namespace {

constexpr int FOLD = 32;     // frames per block of plain accumulation
constexpr int PF = 2;        // staged elements per thread whose loads overlap compute

struct PmArgs {
    const uint16_t* frames;
    const float* white;
    const uint8_t* mask;
    const float* refv;
    const int* sat;
    const float* dx;
    const float* u_in;
    float* u_out;
    float* err_out;
    int* arg_out;
    TileDesc* tiles;
    int* lists;        // [4][ntiles]
    int* counters;
    int4* tinfo;       // per tile: class, good pixels, padded region positions
    int N, H, W, Rs, Rf, o0, o1;
    int rx, ry, NX, NY, refine;
    int tiles_x, ntiles;
    // LDS kernel launch shape
    int nchunks, nblocks, sub;
    int stage_cap;      // max RH * RW handled with staging (edge kernel)
    int fast_cap;       // max RH * RW of the fast kernel (staged elements per frame)
    // matrix-core search of interior tiles
    const uint4* ipk;   // packed frames [tile][kblock][4][2][64] x 16 bytes
    const double* pstat;  // per tile pixel: sum I^2, 32896 sum I, sum (I - W)^2, good
    const int* fscale;  // fixed-point exponent of the reference
    int kblocks;
    int mm_lds_a;       // the tile's packed frames are staged in LDS
    int mm_on;          // bits: interior tiles / edge tiles on the matrix cores, frames
                        // staged in LDS for interior / edge tiles
    int mm_slow_max;    // slow-frame capacity of a matrix-core edge tile
    // B operand precomputed per reference position (null: generated in the search
    // kernel): three byte planes [3][Rs Rf][NP] of the positions relative to the integer
    // shift of frame pl_ref (the middle frame), per position the column sums sum g~^2
    // and sum G~, and per (position, 16 frames) the lookups' validity bits
    const uint8_t* planes;
    const double* pcs;
    const double* pgu;
    const unsigned* pvb;
    int pl_ref;
    // split-half search: only the (frame, pixel) terms with half[n][pixel] == hval
    // count (null: all terms)
    const uint8_t* half;
    int hval;
};


__device__ inline void write_unchanged(const PmArgs& a, size_t pix, size_t HW) {
    a.u_out[pix] = a.u_in[pix];
    a.u_out[HW + pix] = a.u_in[HW + pix];
    if (a.err_out) a.err_out[pix] = INFINITY;
    if (a.arg_out) a.arg_out[pix] = -1;
}

// Rectangle [r0, r1] x [c0, c1] (inclusive) of the reference holds no invalid pixel.
__device__ inline bool rect_valid(const int* sat, int Rs, int Rf, int r0, int r1, int c0, int c1) {
    if (r0 < 0 || c0 < 0 || r1 >= Rs || c1 >= Rf) return false;
    const size_t ld = (size_t)Rf + 1;
    const int v = sat[(size_t)(r1 + 1) * ld + (c1 + 1)] - sat[(size_t)r0 * ld + (c1 + 1)] -
                  sat[(size_t)(r1 + 1) * ld + c0] + sat[(size_t)r0 * ld + c0];
    return v == 0;
}

// One wave per tile: candidate-centre range, LDS fit and validity of every frame.
__device__ void classify_item(const PmArgs& a, int tile) {
    const int lane = threadIdx.x;
    const int ty = tile / a.tiles_x, tx = tile - ty * a.tiles_x;
    const int i = ty * TILE + (lane >> 3), j = tx * TILE + (lane & 7);
    const size_t HW = (size_t)a.H * a.W;
    const bool inb = i < a.H && j < a.W;
    const size_t pix = inb ? (size_t)i * a.W + j : 0;
    const bool good = inb && a.mask[pix] != 0;
    int c0 = 0, c1 = 0;
    if (good) {
        c0 = window_centre(a.u_in[pix]);
        c1 = window_centre(a.u_in[HW + pix]);
    }
    const int ngood = wave_sum<int>(good ? 1 : 0);
    if (ngood == 0) {
        if (inb) write_unchanged(a, pix, HW);
        if (lane == 0) a.tinfo[tile] = make_int4(CNT_NONE, 0, 0, 0);
        return;
    }
    const int mn0 = wave_min_i(good ? c0 : INT_MAX), mx0 = wave_max_i(good ? c0 : INT_MIN);
    const int mn1 = wave_min_i(good ? c1 : INT_MAX), mx1 = wave_max_i(good ? c1 : INT_MIN);
    const long long rh = (long long)mx0 - mn0 + a.NX;
    const long long rw = (long long)mx1 - mn1 + a.NY;
    int cls;
    if (rh * rw > a.stage_cap || rh * (long long)lds_pitch((int)min(rw, (long long)1 << 20)) >
                                     PM_STAGE_FLOATS) {
        cls = CNT_GENERIC;
    } else {
        // FAST needs, for every frame, all corners of the staged region valid
        const int T0 = mn0 - a.rx, T1 = mn1 - a.ry;
        int nbad = 0;   // frames whose staged region holds an invalid lookup
        for (int n = lane; n < a.N; n += 64) {
            const AxisShift s0 = axis_shift(a.dx[2 * n], a.o0);
            const AxisShift s1 = axis_shift(a.dx[2 * n + 1], a.o1);
            const int r0 = T0 - s0.e, c0r = T1 - s1.e;
            nbad += rect_valid(a.sat, a.Rs, a.Rf, r0, r0 + (int)rh, c0r, c0r + (int)rw) ? 0 : 1;
        }
        const int bad = wave_sum<int>(nbad);
        if (a.mm_on & 1)
            cls = bad == 0 ? CNT_FAST
                           : ((a.mm_on & 2) && bad <= a.mm_slow_max && bad < a.N ? CNT_EDGE_MM : CNT_EDGE);
        else
            cls = (bad == 0 && rh * rw <= a.fast_cap) ? CNT_FAST : CNT_EDGE;
        if (lane == 0) a.tiles[tile] = TileDesc{mn0, mn1, (int)rh, (int)rw};
    }
    // positions the matrix cores go through, in units of 64 pixels: the region in
    // blocks of 16, or for tiles taken in halves the two halves' own regions at 32 pixels
    long long pos = cls == CNT_GENERIC ? 0 : (rh * rw + 15) / 16 * 16;
    if ((cls == CNT_FAST && (a.mm_on & 1) && (a.mm_on & 16)) || (cls == CNT_EDGE_MM && (a.mm_on & 32))) {
        pos = 0;
        for (int h = 0; h < 2; ++h) {
            const bool in = good && (lane >> 5) == h;
            const int hn0 = wave_min_i(in ? c0 : INT_MAX), hx0 = wave_max_i(in ? c0 : INT_MIN);
            const int hn1 = wave_min_i(in ? c1 : INT_MAX), hx1 = wave_max_i(in ? c1 : INT_MIN);
            if (hn0 <= hx0)
                pos += ((long long)(hx0 - hn0 + a.NX) * (hx1 - hn1 + a.NY) + 15) / 16 * 8;
        }
    }
    if (lane == 0) a.tinfo[tile] = make_int4(cls, ngood, (int)pos, 0);
}

// Work lists of the classes and the counters, by one work-group of 1024 threads per
// job (ordered compaction with wave ballots; no atomics).
constexpr int COMPACT_THREADS = 1024;

// Tile of position i in the order of the work lists: vertical strips of STRIP tiles,
// each taken row by row, so that a tile's neighbours below follow it within STRIP
// items; with the work items in contiguous per-XCD runs, the operand-plane regions
// that vertically neighbouring tiles share are then still in the XCD's L2.
constexpr int STRIP = 8;
__device__ inline int strip_tile(int i, int tiles_x, int ntiles) {
    const int tiles_y = ntiles / tiles_x, ns = tiles_x / STRIP, full = ns * STRIP * tiles_y;
    int tx, ty;
    if (i < full) {
        const int s = i / (STRIP * tiles_y), r = i - s * (STRIP * tiles_y);
        ty = r / STRIP;
        tx = s * STRIP + (r - ty * STRIP);
    } else {
        const int rw = tiles_x - ns * STRIP, r = i - full;
        ty = r / rw;
        tx = ns * STRIP + (r - ty * rw);
    }
    return ty * tiles_x + tx;
}

__device__ void compact_item(const PmArgs& a) {
    __shared__ int wcnt[COMPACT_THREADS / 64][4];
    __shared__ int base[4];
    __shared__ int red[COMPACT_THREADS / 64][8];
    const int cls_of[4] = {CNT_FAST, CNT_EDGE, CNT_GENERIC, CNT_EDGE_MM};
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const unsigned long long lt = (1ull << lane) - 1ull;
    if (tid < 4) base[tid] = 0;
    // per thread: good pixels of each list's tiles, positions of FAST / EDGE_MM, NONE
    int acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    __syncthreads();
    // two ordered passes over the tiles: the interior list in strip order (its tiles read
    // overlapping operand-plane regions, which vertical neighbours then find in L2), the
    // other lists in tile order (measured faster for the edge search, whose per-XCD runs
    // then spread the slow tiles more evenly)
    for (int pass = 0; pass < 2; ++pass) {
        const bool strip = pass == 0;
        for (int t0 = 0; t0 < a.ntiles; t0 += COMPACT_THREADS) {
            const int i = t0 + tid;
            const int tile = i < a.ntiles ? (strip ? strip_tile(i, a.tiles_x, a.ntiles) : i) : a.ntiles;
            int4 ti = make_int4(-1, 0, 0, 0);
            if (tile < a.ntiles) ti = a.tinfo[tile];
            const int cls = ti.x;
            // the classes of this pass
            if (strip ? cls != CNT_FAST : cls == CNT_FAST) ti.x = -1;
            int mine[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const unsigned long long m = __ballot(ti.x == cls_of[c]);
                mine[c] = __popcll(m & lt);
                if (lane == 0) wcnt[wave][c] = __popcll(m);
            }
            __syncthreads();
            if (tid < 4) {
                int run = base[tid];
                for (int w = 0; w < COMPACT_THREADS / 64; ++w) {
                    const int v = wcnt[w][tid];
                    wcnt[w][tid] = run;
                    run += v;
                }
                base[tid] = run;
            }
            __syncthreads();
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if (ti.x == cls_of[c]) {
                    a.lists[c * a.ntiles + wcnt[wave][c] + mine[c]] = tile;
                    acc[c] += ti.y;
                }
            }
            if (ti.x == CNT_FAST) acc[4] += ti.z;
            if (ti.x == CNT_EDGE_MM) acc[5] += ti.z;
            if (!strip && cls == CNT_NONE) acc[6] += 1;
            __syncthreads();
        }
    }
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        const int v = wave_sum<int>(acc[q]);
        if (lane == 0) red[wave][q] = v;
    }
    __syncthreads();
    if (tid == 0) {
        int tot[7] = {0, 0, 0, 0, 0, 0, 0};
        for (int w = 0; w < COMPACT_THREADS / 64; ++w)
            for (int q = 0; q < 7; ++q) tot[q] += red[w][q];
        a.counters[CNT_FAST] = base[0];
        a.counters[CNT_EDGE] = base[1];
        a.counters[CNT_GENERIC] = base[2];
        a.counters[CNT_EDGE_MM] = base[3];
        a.counters[CNT_GOOD_FAST] = tot[0];
        a.counters[CNT_GOOD_EDGE] = tot[1];
        a.counters[CNT_GOOD_GENERIC] = tot[2];
        a.counters[CNT_GOOD_EDGE_MM] = tot[3];
        a.counters[CNT_MM_POS] = tot[4];
        a.counters[CNT_MM_POS_EDGE] = tot[5];
        a.counters[CNT_NONE] = tot[6];
    }
}

__global__ __launch_bounds__(COMPACT_THREADS) void k_compact(const PmArgs a) { compact_item(a); }
__global__ __launch_bounds__(COMPACT_THREADS) void k_compact_batch(const PmArgs* __restrict__ jobs) {
    compact_item(table_entry(jobs, (int)blockIdx.x));
}

// Cross-thread first minimum, 3x3 stencil and refinement of one pass's pixels; E
// holds this thread's normalised errors (window rows kx0.., columns ky0..).
template <int KR, int CW>
__device__ inline void finish_pixel(const PmArgs& a, float* smem, const float (&E)[KR][CW],
                                    float bestE, int bestK, bool good, bool pgood, bool inb,
                                    size_t pix, size_t HW, int c0, int c1, int blk, bool blk_ok,
                                    int pip, int ppp, int kx0, int ky0) {
    const int NX = a.NX, NY = a.NY;
    float* redE = smem;
    int* redK = (int*)(smem + a.nblocks * ppp);
    int* best = redK + a.nblocks * ppp;
    float* bestv = (float*)(best + ppp);
    float* sten = bestv + ppp;
    if (blk_ok) {
        redE[blk * ppp + pip] = bestE;
        redK[blk * ppp + pip] = bestK;
    }
    __syncthreads();
    if (blk == 0) {
        float be = INFINITY;
        int bk = INT_MAX;
        for (int b = 0; b < a.nblocks; ++b) {
            const float e = redE[b * ppp + pip];
            const int k = redK[b * ppp + pip];
            if (better(e, k, be, bk)) {
                be = e;
                bk = k;
            }
        }
        best[pip] = isfinite(be) ? bk : -1;
        bestv[pip] = be;
#pragma unroll
        for (int q = 0; q < 9; ++q) sten[pip * 9 + q] = INFINITY;
    }
    __syncthreads();
    const int kb = best[pip];
    if (a.refine && good && kb >= 0) {
        const int bx = kb / NY, by = kb - bx * NY;
#pragma unroll
        for (int r = 0; r < KR; ++r)
#pragma unroll
            for (int m = 0; m < CW; ++m) {
                const int dxk = kx0 + r - bx, dyk = ky0 + m - by;
                if (dxk >= -1 && dxk <= 1 && dyk >= -1 && dyk <= 1 && kx0 + r < NX && ky0 + m < NY)
                    sten[pip * 9 + (dxk + 1) * 3 + (dyk + 1)] = E[r][m];
            }
    }
    __syncthreads();
    if (blk == 0 && inb) {
        if (!pgood || kb < 0) {
            write_unchanged(a, pix, HW);
        } else {
            const int bx = kb / NY, by = kb - bx * NY;
            float ox = 0.f, oy = 0.f;
            if (a.refine) refine_at(sten + pip * 9, bx, by, NX, NY, ox, oy);
            a.u_out[pix] = (float)(c0 + bx - a.rx) + ox;
            a.u_out[HW + pix] = (float)(c1 + by - a.ry) + oy;
            if (a.err_out) a.err_out[pix] = bestv[pip];
            if (a.arg_out) a.arg_out[pix] = kb;
        }
    }
    __syncthreads();
}

// Squared residuals of KR window rows of CW candidates for one frame, accumulated into
// acc.  Rows are software-pipelined through two register buffers chosen by the row's
// parity at compile time: the LDS reads of row r + 1 are issued before the FMAs of
// row r, and a scheduling barrier per row keeps at most two rows of loads live.
template <int KR, int CW>
__device__ inline void eval_rows(const float* G, const int (&rowoff)[KR], float nW, float I,
                                 float (&acc)[KR][CW]) {
    float b0[CW], b1[CW];
#pragma unroll
    for (int m = 0; m < CW; ++m) b0[m] = G[rowoff[0] + m];
#pragma unroll
    for (int r = 0; r < KR; ++r) {
        float(&cur)[CW] = (r & 1) ? b1 : b0;
        float(&nxt)[CW] = (r & 1) ? b0 : b1;
        if (r + 1 < KR) {
#pragma unroll
            for (int m = 0; m < CW; ++m) nxt[m] = G[rowoff[r + 1] + m];
        }
#pragma unroll
        for (int m = 0; m < CW; ++m) {
            const float rr = fmaf(nW, cur[m], I);
            acc[r][m] = fmaf(rr, rr, acc[r][m]);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// --------------------------------------------------------------- LDS-staged search
//
// FAST kernel: every staged value of every frame is a valid lookup.  Thread layout:
// lane -> (pixel of the current pass, sub-group); a candidate block is KR window rows
// of the full window width; block index = wave * sub + sub-group.  Rows past the
// window are clamped to its last row so that the frame loop is one branch-free block:
//   issue the global loads of the next frame's staged elements (PFS per thread),
//   evaluate this frame's candidates from LDS (rows software-pipelined),
//   interpolate and store the next frame's elements, barrier.
constexpr int PFS = 4;

// Per-frame shift table in LDS, after both staging buffers and the dump slots: for
// frame n, (e, t) of both axes (axis_shift of dx_n).  Built once per tile so that the
// frame loop reads it from LDS instead of waiting on a global load every frame.
constexpr int SHIFT_TAB_OFF = 2 * PM_STAGE_FLOATS + 512;   // floats

__device__ inline int4* shift_table(float* smem) { return (int4*)(smem + SHIFT_TAB_OFF); }

__device__ inline void build_shift_table(const PmArgs& a, float* smem) {
    int4* tab = shift_table(smem);
    for (int n = threadIdx.x; n < a.N; n += blockDim.x) {
        const AxisShift s0 = axis_shift(a.dx[2 * n], a.o0);
        const AxisShift s1 = axis_shift(a.dx[2 * n + 1], a.o1);
        tab[n] = make_int4(s0.e, s1.e, __float_as_int(s0.t), __float_as_int(s1.t));
    }
    __syncthreads();
}

struct FrameShift {
    int goff;       // e0 * Rf + e1 (work-group uniform)
    int e0, e1;
    float t0, t1;
};

__device__ inline FrameShift frame_shift(int4 v, int Rf) {
    FrameShift f;
    f.e0 = __builtin_amdgcn_readfirstlane(v.x);
    f.e1 = __builtin_amdgcn_readfirstlane(v.y);
    f.t0 = __int_as_float(__builtin_amdgcn_readfirstlane(v.z));
    f.t1 = __int_as_float(__builtin_amdgcn_readfirstlane(v.w));
    f.goff = f.e0 * Rf + f.e1;
    return f;
}

template <int CW, int KR>
__device__ void pm_fast_item(const PmArgs& a, int slot) {
    extern __shared__ float smem[];
    if (slot >= a.counters[CNT_FAST]) return;
    const int tile = a.lists[CNT_FAST * a.ntiles + slot];
    const TileDesc td = a.tiles[tile];
    const int ty = tile / a.tiles_x, tx = tile - ty * a.tiles_x;
    const int RH = td.rh, RW = td.rw, P = lds_pitch(RW);
    const int T0 = td.cmin0 - a.rx, T1 = td.cmin1 - a.ry;
    const int bufsz = RH * P;
    const int nel = RH * RW;
    const int NX = a.NX, N = a.N, Rf = a.Rf;

    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int ppp = 64 / a.sub;
    const int pip = lane & (ppp - 1);
    const int blk = wave * a.sub + lane / ppp;
    const bool blk_ok = blk < a.nblocks;
    const int kx0 = blk * KR;
    const size_t HW = (size_t)a.H * a.W;
    const float* __restrict__ refv = a.refv;

    int rowoff[KR];
#pragma unroll
    for (int r = 0; r < KR; ++r) rowoff[r] = min(kx0 + r, NX - 1) * P;

    // staged elements of this thread: LDS offset (a dump slot past both buffers when
    // the element does not exist) and reference offset relative to the frame shift
    const int nst = (nel + nthr - 1) / nthr;   // <= PFS (checked by the classification)
    int st_lds[PFS], st_glb[PFS];
#pragma unroll
    for (int s = 0; s < PFS; ++s) {
        const int e = tid + s * nthr;
        const int r = e < nel ? e / RW : 0, q = e < nel ? e - r * RW : 0;
        st_lds[s] = e < nel ? r * P + q : 2 * bufsz + tid;
        st_glb[s] = (T0 + r) * Rf + (T1 + q);
    }
    build_shift_table(a, smem);
    const int4* __restrict__ tab = shift_table(smem);

    for (int pass = 0; pass < a.sub; ++pass) {
        const int pidx = pass * ppp + pip;
        const int i = ty * TILE + (pidx >> 3), j = tx * TILE + (pidx & 7);
        const bool inb = i < a.H && j < a.W;
        const size_t pix = inb ? (size_t)i * a.W + j : 0;
        const bool pgood = inb && a.mask[pix] != 0;
        const bool good = pgood && blk_ok;
        int c0 = td.cmin0, c1 = td.cmin1;
        float Wp = 0.f;
        if (pgood) {
            c0 = window_centre(a.u_in[pix]);
            c1 = window_centre(a.u_in[HW + pix]);
            Wp = a.white[pix];
        }
        const float nW = -Wp;
        const int base = (c0 - td.cmin0) * P + (c1 - td.cmin1);

        float eS[KR][CW], eP[KR][CW];
#pragma unroll
        for (int r = 0; r < KR; ++r)
#pragma unroll
            for (int m = 0; m < CW; ++m) {
                eS[r][m] = 0.f;
                eP[r][m] = 0.f;
            }
        float vS = 0.f, vP = 0.f;

        // stage frame 0 into buffer 0
        {
            const FrameShift f = frame_shift(tab[0], Rf);
#pragma unroll
            for (int s = 0; s < PFS; ++s) {
                if (s < nst) {
                    const float* p = refv + (st_glb[s] - f.goff);
                    smem[st_lds[s]] = bilinear4(p[0], p[1], p[Rf], p[Rf + 1], f.t0, f.t1);
                }
            }
            __syncthreads();
        }
        int4 shn = tab[min(1, N - 1)];   // shift of the frame staged next

        const uint16_t* fp = a.frames + pix;
        float I = (float)fp[0];
        // split-half search: a term outside the half adds a zero residual and no variance
        const bool split = a.half != nullptr;
        const uint8_t* hp = split ? a.half + pix : nullptr;
        bool hin = !split || hp[0] == a.hval;
        int nv = 0;
        // blocks of FOLD frames: plain sums inside a block, compensated fold after it
        // (keeping the fold out of the frame loop keeps the accumulators in place)
        for (int n0 = 0; n0 < N; n0 += FOLD) {
        const int nend = min(n0 + FOLD, N);
        for (int n = n0; n < nend; ++n) {
            const int n1 = min(n + 1, N - 1);
            const float* G = smem + (n & 1) * bufsz + base;
            float* Gn = smem + ((n + 1) & 1) * bufsz;
            const float Inext = (float)fp[(size_t)n1 * HW];
            const bool hnext = !split || hp[(size_t)n1 * HW] == a.hval;
            const FrameShift fn = frame_shift(shn, Rf);
            shn = tab[min(n + 2, N - 1)];
            float pv[PFS][4];
#pragma unroll
            for (int s = 0; s < PFS; ++s) {
                if (s < nst) {
                    const float* p = refv + (st_glb[s] - fn.goff);
                    pv[s][0] = p[0];
                    pv[s][1] = p[1];
                    pv[s][2] = p[Rf];
                    pv[s][3] = p[Rf + 1];
                }
            }
            __builtin_amdgcn_sched_barrier(0);

            eval_rows<KR, CW>(G, rowoff, hin ? nW : 0.f, hin ? I : 0.f, eP);
            const float v = I - Wp;
            vP = fmaf(hin ? v : 0.f, v, vP);
            nv += hin ? 1 : 0;
            __builtin_amdgcn_sched_barrier(0);

#pragma unroll
            for (int s = 0; s < PFS; ++s)
                if (s < nst)
                    Gn[st_lds[s]] = bilinear4(pv[s][0], pv[s][1], pv[s][2], pv[s][3], fn.t0, fn.t1);
            I = Inext;
            hin = hnext;
            __syncthreads();
        }
#pragma unroll
        for (int r = 0; r < KR; ++r)
#pragma unroll
            for (int m = 0; m < CW; ++m) two_sum_fold(eS[r][m], eP[r][m]);
        two_sum_fold(vS, vP);
        }

        // per-thread first minimum over its candidates (index order); the normalised
        // errors replace the running sums in eS
        float bestE = INFINITY;
        int bestK = INT_MAX;
        const float var = vS + vP;
#pragma unroll
        for (int r = 0; r < KR; ++r)
#pragma unroll
            for (int m = 0; m < CW; ++m) {
                float E = INFINITY;
                if (good && kx0 + r < NX) {
                    E = normalised_error(eS[r][m] + eP[r][m], var, nv);
                    if (E < bestE) {
                        bestE = E;
                        bestK = (kx0 + r) * CW + m;
                    }
                }
                eS[r][m] = E;
            }
        finish_pixel<KR, CW>(a, smem, eS, bestE, bestK, good, pgood, inb, pix, HW, c0, c1, blk, blk_ok,
                             pip, ppp, kx0, 0);
    }
}

// EDGE kernel: some staged lookups are invalid (NaN) in some frames.  Same thread
// layout as the FAST kernel.  A frame whose staged region holds no invalid value is a
// "fast frame": every candidate is valid, so the variance and frame count are common
// to all candidates of a pixel.  In the other ("slow") frames each candidate adds its
// squared residual and (I - W)^2 only when its lookup is valid; the per-candidate
// variance of slow frames starts at -0.0, so its sign bit records whether any slow
// frame was valid (-0.0 + x is +0.0 or positive for every x >= +0.0).
template <int CW, int KR>
__device__ void pm_edge_item(const PmArgs& a, int slot) {
    extern __shared__ float smem[];
    if (slot >= a.counters[CNT_EDGE]) return;
    const int tile = a.lists[CNT_EDGE * a.ntiles + slot];
    const TileDesc td = a.tiles[tile];
    const int ty = tile / a.tiles_x, tx = tile - ty * a.tiles_x;
    const int RH = td.rh, RW = td.rw, P = lds_pitch(RW);
    const int T0 = td.cmin0 - a.rx, T1 = td.cmin1 - a.ry;
    const int bufsz = RH * P;
    const int nel = RH * RW;
    const int NX = a.NX, N = a.N, Rf = a.Rf;

    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int ppp = 64 / a.sub;
    const int pip = lane & (ppp - 1);
    const int blk = wave * a.sub + lane / ppp;
    const bool blk_ok = blk < a.nblocks;
    const int kx0 = blk * KR;
    const size_t HW = (size_t)a.H * a.W;
    const float* __restrict__ refv = a.refv;

    int rowoff[KR];
#pragma unroll
    for (int r = 0; r < KR; ++r) rowoff[r] = min(kx0 + r, NX - 1) * P;
    build_shift_table(a, smem);
    const int4* __restrict__ tab = shift_table(smem);

    for (int pass = 0; pass < a.sub; ++pass) {
        const int pidx = pass * ppp + pip;
        const int i = ty * TILE + (pidx >> 3), j = tx * TILE + (pidx & 7);
        const bool inb = i < a.H && j < a.W;
        const size_t pix = inb ? (size_t)i * a.W + j : 0;
        const bool pgood = inb && a.mask[pix] != 0;
        const bool good = pgood && blk_ok;
        int c0 = td.cmin0, c1 = td.cmin1;
        float Wp = 0.f;
        if (pgood) {
            c0 = window_centre(a.u_in[pix]);
            c1 = window_centre(a.u_in[HW + pix]);
            Wp = a.white[pix];
        }
        const float nW = -Wp;
        const int base = (c0 - td.cmin0) * P + (c1 - td.cmin1);

        float eS[KR][CW], eP[KR][CW], vK[KR][CW];
#pragma unroll
        for (int r = 0; r < KR; ++r)
#pragma unroll
            for (int m = 0; m < CW; ++m) {
                eS[r][m] = 0.f;
                eP[r][m] = 0.f;
                vK[r][m] = -0.f;
            }
        float vS = 0.f, vP = 0.f;
        int nfast = 0;

        // stage frame 0 into buffer 0
        int slow_cur;
        {
            const FrameShift f = frame_shift(tab[0], Rf);
            int mine = 0;
            for (int e = tid; e < nel; e += nthr) {
                const int r = e / RW, q = e - r * RW;
                const float g = masked_bilinear(refv, a.Rs, Rf, T0 + r - f.e0, T1 + q - f.e1, f.t0, f.t1);
                smem[r * P + q] = g;
                mine |= valid(g) ? 0 : 1;
            }
            slow_cur = __syncthreads_or(mine);
        }

        const uint16_t* fp = a.frames + pix;
        float I = (float)fp[0];
        // split-half search: a term outside the half adds a zero residual and no variance
        const bool split = a.half != nullptr;
        const uint8_t* hp = split ? a.half + pix : nullptr;
        bool hin = !split || hp[0] == a.hval;
        for (int n0 = 0; n0 < N; n0 += FOLD) {
        const int nend = min(n0 + FOLD, N);
        for (int n = n0; n < nend; ++n) {
            const int n1 = min(n + 1, N - 1);
            const float* G = smem + (n & 1) * bufsz + base;
            float* Gn = smem + ((n + 1) & 1) * bufsz;
            const float Inext = (float)fp[(size_t)n1 * HW];
            const bool hnext = !split || hp[(size_t)n1 * HW] == a.hval;
            const float v = I - Wp;
            if (!slow_cur) {
                eval_rows<KR, CW>(G, rowoff, hin ? nW : 0.f, hin ? I : 0.f, eP);
                vP = fmaf(hin ? v : 0.f, v, vP);
                nfast += hin ? 1 : 0;
            } else {
                const float v2 = v * v;
#pragma unroll
                for (int r = 0; r < KR; ++r) {
#pragma unroll
                    for (int m = 0; m < CW; ++m) {
                        const float gv = G[rowoff[r] + m];
                        const bool ok = valid(gv) && hin;
                        const float rr = ok ? fmaf(nW, gv, I) : 0.f;
                        eP[r][m] = fmaf(rr, rr, eP[r][m]);
                        vK[r][m] += ok ? v2 : -0.f;
                    }
                }
            }
            __builtin_amdgcn_sched_barrier(0);

            // stage frame n + 1 (the last frame is staged again harmlessly)
            const FrameShift fn = frame_shift(tab[n1], Rf);
            int mine = 0;
            for (int e = tid; e < nel; e += nthr) {
                const int r = e / RW, q = e - r * RW;
                const float g = masked_bilinear(refv, a.Rs, Rf, T0 + r - fn.e0, T1 + q - fn.e1, fn.t0,
                                                fn.t1);
                Gn[r * P + q] = g;
                mine |= valid(g) ? 0 : 1;
            }
            I = Inext;
            hin = hnext;
            slow_cur = __syncthreads_or(mine);
        }
#pragma unroll
        for (int r = 0; r < KR; ++r)
#pragma unroll
            for (int m = 0; m < CW; ++m) two_sum_fold(eS[r][m], eP[r][m]);
        two_sum_fold(vS, vP);
        }

        float bestE = INFINITY;
        int bestK = INT_MAX;
        const float vcommon = vS + vP;
#pragma unroll
        for (int r = 0; r < KR; ++r)
#pragma unroll
            for (int m = 0; m < CW; ++m) {
                float E = INFINITY;
                if (good && kx0 + r < NX) {
                    const bool any = nfast > 0 || !signbit(vK[r][m]);
                    E = Wp == 0.f ? zero_white_error(eS[r][m] + eP[r][m], any ? 1 : 0)
                                  : normalised_error(eS[r][m] + eP[r][m], vcommon + vK[r][m], any ? 1 : 0);
                    if (E < bestE) {
                        bestE = E;
                        bestK = (kx0 + r) * CW + m;
                    }
                }
                eS[r][m] = E;
            }
        finish_pixel<KR, CW>(a, smem, eS, bestE, bestK, good, pgood, inb, pix, HW, c0, c1, blk, blk_ok,
                             pip, ppp, kx0, 0);
    }
}

// ------------------------------------------------------------------ generic search
// One work-group of 256 threads per tile: 64 pixels x 4 candidate strides; lookups
// straight from the reference.  Used for tiles whose staged region would not fit.
__device__ inline float eval_candidate(const PmArgs& a, size_t pix, size_t HW, int t0, int t1,
                                       float Wp) {
    float eS = 0.f, eP = 0.f, vS = 0.f, vP = 0.f;
    int nv = 0;
    for (int n = 0; n < a.N; ++n) {
        const AxisShift s0 = axis_shift(a.dx[2 * n], a.o0);
        const AxisShift s1 = axis_shift(a.dx[2 * n + 1], a.o1);
        const float g = masked_bilinear(a.refv, a.Rs, a.Rf, t0 - s0.e, t1 - s1.e, s0.t, s1.t);
        // (split-half search: only the half's terms)
        if (valid(g) && (!a.half || a.half[(size_t)n * HW + pix] == a.hval)) {
            const float I = (float)a.frames[(size_t)n * HW + pix];
            const float rr = fmaf(-Wp, g, I);
            eP = fmaf(rr, rr, eP);
            const float v = I - Wp;
            vP = fmaf(v, v, vP);
            ++nv;
        }
        if (((n + 1) % FOLD) == 0) {
            two_sum_fold(eS, eP);
            two_sum_fold(vS, vP);
        }
    }
    return normalised_error(eS + eP, vS + vP, nv);
}

__device__ void pm_generic_item(const PmArgs& a, int slot) {
    __shared__ float redE[4][64];
    __shared__ int redK[4][64];
    __shared__ float sten[64][9];
    if (slot >= a.counters[CNT_GENERIC]) return;
    const int tile = a.lists[CNT_GENERIC * a.ntiles + slot];
    const int ty = tile / a.tiles_x, tx = tile - ty * a.tiles_x;
    const int p = threadIdx.x & 63, sub = threadIdx.x >> 6;
    const int i = ty * TILE + (p >> 3), j = tx * TILE + (p & 7);
    const size_t HW = (size_t)a.H * a.W;
    const bool inb = i < a.H && j < a.W;
    const size_t pix = inb ? (size_t)i * a.W + j : 0;
    const bool good = inb && a.mask[pix] != 0;
    int c0 = 0, c1 = 0;
    float Wp = 0.f;
    if (good) {
        c0 = window_centre(a.u_in[pix]);
        c1 = window_centre(a.u_in[HW + pix]);
        Wp = a.white[pix];
    }
    const int C = a.NX * a.NY;
    float be = INFINITY;
    int bk = INT_MAX;
    if (good) {
        for (int k = sub; k < C; k += 4) {
            const int kx = k / a.NY, ky = k - kx * a.NY;
            const float E = eval_candidate(a, pix, HW, c0 - a.rx + kx, c1 - a.ry + ky, Wp);
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
        const int bx = kb / a.NY, by = kb - bx * a.NY;
        for (int q = sub; q < 9; q += 4) {
            const int kx = bx + q / 3 - 1, ky = by + q % 3 - 1;
            float E = INFINITY;
            if (kx >= 0 && kx < a.NX && ky >= 0 && ky < a.NY)
                E = eval_candidate(a, pix, HW, c0 - a.rx + kx, c1 - a.ry + ky, Wp);
            sten[p][q] = E;
        }
    }
    __syncthreads();
    if (sub == 0 && inb) {
        if (!good || kb < 0) {
            write_unchanged(a, pix, HW);
        } else {
            const int bx = kb / a.NY, by = kb - bx * a.NY;
            float ox = 0.f, oy = 0.f;
            if (a.refine) refine_at(sten[p], bx, by, a.NX, a.NY, ox, oy);
            a.u_out[pix] = (float)(c0 + bx - a.rx) + ox;
            a.u_out[HW + pix] = (float)(c1 + by - a.ry) + oy;
            if (a.err_out) a.err_out[pix] = redE[0][p];
            if (a.arg_out) a.arg_out[pix] = kb;
        }
    }
    __syncthreads();
}

// ------------------------------------------------------ matrix-core search (interior)
//
// For an interior tile every lookup is valid, and with g_n(q) the reference interpolated
// for frame n at the tile-region position q of a candidate, the error of that candidate
// at pixel p expands as
//     sum_n (I_n - W g_n)^2 = sum_n I_n^2 - 2 W sum_n I_n g_n(q) + W^2 sum_n g_n(q)^2.
// The middle sum is a contraction over frames, S[p][q] = sum_n I[p][n] G[n][q], of the
// 64 x N count matrix of the tile with the N x Q matrix of interpolated reference values:
// it runs on the int8 matrix cores with exact int32 accumulation.  Counts are split into
// two bytes, g into a 24-bit fixed-point number G = rint(g 2^F) (F per reference, so
// that |G| < 2^22) offset by 2^23 and split into three bytes; every byte is stored
// biased by -128 so that it is a signed int8, and the bias is removed with row and
// column sums.  The three sums are exact (or FP64) and combined in FP64, so the
// cancellation between them costs no accuracy.  The errors of all candidates of the
// tile's 64 pixels go to LDS; the first minimum and the paraboloid refinement follow.
constexpr int MM_WAVES = 8;
constexpr int MM_THREADS = MM_WAVES * 64;

typedef int mm_v4i __attribute__((ext_vector_type(4)));

// Per-pixel coefficients of the error.  With S the combined int8 products of the pixel
// and a position, g_q and C_q the position's column terms, interior tiles use
//     E = al + be (S + g_q) + ga C_q            (the normalised error;
// when var = 0 the same coefficients give the error itself), edge tiles
//     err_fast = al + be (S + g_q) + ga C_q     (over the frames without invalid
// lookups, whose variance is vf) and add the remaining frames term by term.
struct MmPix {
    double al, be, ga, vf;
    float W;
    int dc0, dc1;  // window centre relative to the tile's smallest centre
    int zvar;      // var == 0
    int good;
    int eo;        // error-table index of position (r, c) is eo + r NY + c
};

// Frames of a tile as the A operand (rows = the tile's 64 pixels in four groups of 16,
// K = frames): lane l of group m holds pixel m*16 + l%16, frames 16*(l/16) .. +15 of the
// K-block, byte 0 (then byte 1) of each count, biased by -128.
__global__ __launch_bounds__(256) void k_pm_pack(const uint16_t* __restrict__ frames,
                                                 const uint8_t* __restrict__ mask, int N, int H, int W,
                                                 int tiles_x, int KB, uint4* __restrict__ ipk) {
    // (tile, K-block) items in contiguous runs per XCD: horizontally neighbouring tiles,
    // whose 16-byte row segments share lines, are read through one L2
    const int item = xcd_item((int)blockIdx.x, (int)gridDim.x);
    const int tile = item / KB, kb = item - tile * KB;
    const int m = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int p = m * 16 + (lane & 15);
    const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
    const int i = ty * TILE + (p >> 3), j = tx * TILE + (p & 7);
    const bool good = i < H && j < W && mask[(size_t)i * W + j] != 0;
    const size_t HW = (size_t)H * W;
    const size_t pix = good ? (size_t)i * W + j : 0;
    unsigned lo[4], hi[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        unsigned l = 0, h = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int n = kb * MM_KB + 16 * (lane >> 4) + 4 * w + b;
            const unsigned v = (good && n < N) ? (unsigned)frames[(size_t)n * HW + pix] : 0u;
            l |= (v & 255u) << (8 * b);
            h |= (v >> 8) << (8 * b);
        }
        lo[w] = l ^ 0x80808080u;
        hi[w] = h ^ 0x80808080u;
    }
    const size_t base = (((size_t)tile * KB + kb) * 4 + m) * 2 * 64 + lane;
    ipk[base] = make_uint4(lo[0], lo[1], lo[2], lo[3]);
    ipk[base + 64] = make_uint4(hi[0], hi[1], hi[2], hi[3]);
}

// Per-pixel frame sums (FP64, exact for the integer sums), stored per tile [tile][64
// pixels][4].  One thread per pixel of the detector padded to whole tiles, in row-major
// order, so that a wave's loads of a frame are contiguous; padding pixels get zeros.
__global__ __launch_bounds__(256) void k_pm_pixstats(const uint16_t* __restrict__ frames,
                                                     const float* __restrict__ white,
                                                     const uint8_t* __restrict__ mask, int N, int H,
                                                     int W, int tiles_x, double* __restrict__ pstat) {
    const int PW = tiles_x * TILE;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int tiles_y = (H + TILE - 1) / TILE;
    if (idx >= (size_t)tiles_y * TILE * PW) return;
    const int i = (int)(idx / PW), j = (int)(idx - (size_t)i * PW);
    const int tile = (i / TILE) * tiles_x + j / TILE, p = (i % TILE) * TILE + j % TILE;
    const bool good = i < H && j < W && mask[(size_t)i * W + j] != 0;
    const size_t HW = (size_t)H * W;
    double A = 0.0, S = 0.0, V = 0.0;
    if (good) {
        const size_t pix = (size_t)i * W + j;
        const double Wp = (double)white[pix];
        // (unrolled so that the loads of several frames are in flight; same order of sums)
#pragma unroll 8
        for (int n = 0; n < N; ++n) {
            const double I = (double)frames[(size_t)n * HW + pix];
            A = fma(I, I, A);
            S += I;
            const double v = I - Wp;
            V = fma(v, v, V);
        }
    }
    double* o = pstat + ((size_t)tile * 64 + p) * 4;
    o[0] = A;
    o[1] = 32896.0 * S;
    o[2] = V;
    o[3] = good ? 1.0 : 0.0;
}

__device__ inline mm_v4i mm_as_v4i(uint4 v) {
    mm_v4i r;
    r.x = (int)v.x;
    r.y = (int)v.y;
    r.z = (int)v.z;
    r.w = (int)v.w;
    return r;
}

// LDS of the matrix-core search: E [64][NC] floats | frame weights float4 [KB * 64] |
// frame offsets int [KB * 64] | pixel parameters MmPix [64].  Frames past N (padding of
// the last K-block) get zero weights and frame 0's offset.
__host__ __device__ inline int mm_frames_padded(int n_frames) {
    return (n_frames + MM_KB - 1) / MM_KB * MM_KB;
}
// Extra LDS of edge tiles: slow-frame flags [NP] | slow list [S] | slow shifts int4
// [S] | counts I [S][64] | nslow, first fast frame | per wave, per position of its
// current column block, a bit mask of the slow frames whose lookup is invalid.
__host__ __device__ inline int mm_mask_words(int smax) { return (smax + 31) / 32; }
__host__ __device__ inline size_t mm_edge_bytes(int np, int smax) {
    return (size_t)np * 4 + (size_t)smax * (4 + 16 + 64 * 4) + 16 +
           (size_t)MM_WAVES * 16 * mm_mask_words(smax) * 4;
}
// LDS of one work-group: error tables of 16 mh pixels | frame table | pixel coefficients
// | edge extras | staged packed frames.
__host__ __device__ inline size_t mm_lds_bytes(int nc, int n_frames, bool stage_a, bool edge,
                                               int smax, int mh) {
    const size_t np = (size_t)mm_frames_padded(n_frames);
    const size_t e = ((size_t)16 * mh * nc + 3) / 4 * 4 * sizeof(float);
    const size_t apk = stage_a ? np / MM_KB * MM_PACK_BYTES : 0;
    return e + np * 16 + np * 4 + 64 * sizeof(MmPix) + (edge ? mm_edge_bytes((int)np, smax) : 0) + apk;
}

// Matrix-core search of one job: whether interior (fast) and edge tiles go to it, whether
// the packed frames are staged in LDS, whether the tiles are searched in two halves of
// 32 pixels (windows whose error tables of 64 pixels do not fit the LDS), and the edge
// tiles' slow-frame capacity (the largest that fits the LDS, preferring staged frames).
// Depends on the job's own window and frame count, and on whether the interior tiles
// read precomputed operand planes: then a tile whose table of 64 pixels leaves room
// for only one work-group per CU is searched in halves of 32 pixels with the packed
// frames staged, so that two fit (each half's region is smaller than the tile's, so
// the halves issue fewer products in all; they read their operand from L2 twice).
constexpr size_t MM_LDS_MAX = 160 * 1024;
// jobs of at least this many 8x8 tiles are searched alone inside a batch
constexpr long long PM_SOLO_TILES = 1024;
struct MmPlan {
    bool fast, edge, fast_stage, edge_stage, fast_half, edge_half;
    int slow_max;
};
MmPlan mm_plan(int nx, int ny, int n_frames, bool planes) {
    MmPlan p{};
    const int nc = nx * ny;
    p.fast = mm_lds_bytes(nc, n_frames, false, false, 0, 4) <= MM_LDS_MAX;
    p.fast_stage = mm_lds_bytes(nc, n_frames, true, false, 0, 4) <= MM_LDS_MAX;
    if (!p.fast && mm_lds_bytes(nc, n_frames, false, false, 0, 2) <= MM_LDS_MAX) {
        p.fast = true;
        p.fast_half = true;
    } else if (planes && p.fast && mm_lds_bytes(nc, n_frames, true, false, 0, 4) > MM_LDS_MAX / 2 &&
               mm_lds_bytes(nc, n_frames, true, false, 0, 2) <= MM_LDS_MAX / 2) {
        p.fast_half = true;
        p.fast_stage = true;
    }
    // capacity: the largest multiple of 32 (keeps the LDS arrays 16-byte aligned) that fits
    auto cap = [&](bool stage, int mh) {
        for (int sm = MM_SLOW_CAP; sm >= 32; sm -= 32)
            if (mm_lds_bytes(nc, n_frames, stage, true, sm, mh) <= MM_LDS_MAX) return sm;
        return 0;
    };
    const int s_lds = cap(true, 4), s_glb = cap(false, 4);
    if (s_lds >= 64 || (s_lds >= MM_SLOW_MIN && s_glb < 64)) {
        p.edge = true;
        p.edge_stage = true;
        p.slow_max = s_lds;
    } else if (s_glb >= MM_SLOW_MIN) {
        p.edge = true;
        p.edge_stage = false;
        p.slow_max = s_glb;
    } else {
        const int s_half = cap(false, 2);
        if (s_half >= MM_SLOW_MIN) {
            p.edge = true;
            p.edge_half = true;
            p.slow_max = s_half;
        }
    }
    return p;
}

// Frame-table entry of the matrix-core search: the bilinear weights of the frame's
// fractional shift scaled by 2^F (zero weights for padding frames and frames left out),
// and the byte offset of its integer shift, 4 (e0 Rf + e1) modulo 2^32.
__device__ inline void mm_frame_entry(const PmArgs& a, int nn, bool zero, float fs, float4& w, unsigned& go4) {
    const AxisShift s0 = axis_shift(a.dx[2 * nn], a.o0);
    const AxisShift s1 = axis_shift(a.dx[2 * nn + 1], a.o1);
    go4 = 4u * (unsigned)(s0.e * a.Rf + s1.e);
    const float t0 = s0.t, t1 = s1.t;
    w = zero ? make_float4(0.f, 0.f, 0.f, 0.f)
             : make_float4((1.f - t0) * (1.f - t1) * fs, (1.f - t0) * t1 * fs, t0 * (1.f - t1) * fs, t0 * t1 * fs);
}

// The 16 values of one lane's (position, 16 frames) as the three biased byte operands,
// with the rounding of g 2^F to an integer offset by 2^23 (from the bits of
// v + 1.5 2^23, |v| < 2^22); gt = rounded value, gu = gt + 2^23.
__device__ inline void mm_pack_b(const float (&vals)[16], unsigned (&B0)[4], unsigned (&B1)[4], unsigned (&B2)[4],
                                 double& CS, unsigned& gsum) {
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        unsigned u[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int t = 4 * w + b;
            const unsigned gu = __float_as_uint(vals[t] + 12582912.f) - 0x4AC00000u;
            const int gt = (int)gu - (1 << 23);
            CS = fma((double)gt, (double)gt, CS);
            gsum += gu;
            u[b] = gu;
        }
        const unsigned t01l = __builtin_amdgcn_perm(u[1], u[0], 0x05010400u);
        const unsigned t01h = __builtin_amdgcn_perm(u[1], u[0], 0x07030602u);
        const unsigned t23l = __builtin_amdgcn_perm(u[3], u[2], 0x05010400u);
        const unsigned t23h = __builtin_amdgcn_perm(u[3], u[2], 0x07030602u);
        B0[w] = __builtin_amdgcn_perm(t23l, t01l, 0x05040100u) ^ 0x80808080u;
        B1[w] = __builtin_amdgcn_perm(t23l, t01l, 0x07060302u) ^ 0x80808080u;
        B2[w] = __builtin_amdgcn_perm(t23h, t01h, 0x05040100u) ^ 0x80808080u;
    }
}

// Corners of the lookup at reference (row, col) from the 2x2 block read at that position
// clamped into the grid (top-left corner (clamp(row, 0, Rs-2), clamp(col, 0, Rf-2))):
// a corner outside the grid is NaN; one inside sits in the block at its own row and
// column minus the block's (0 or 1 -- also where the clamp moved the block).
__device__ inline void block_corners(int row, int col, float2 top, float2 bot, int Rs, int Rf, float& v00,
                                     float& v01, float& v10, float& v11) {
    const int rc = min(max(row, 0), Rs - 2), ccl = min(max(col, 0), Rf - 2);
    // the block row holding the lookup's first row is 1 only where the clamp moved the
    // block up (row = Rs - 1); its second row is 0 only where it moved it down (row = -1)
    const float2 h0 = row > rc ? bot : top, h1 = row < rc ? top : bot;
    const bool r0 = (unsigned)row < (unsigned)Rs, r1 = (unsigned)(row + 1) < (unsigned)Rs;
    const bool c0 = (unsigned)col < (unsigned)Rf, c1 = (unsigned)(col + 1) < (unsigned)Rf;
    const bool x0 = col > ccl, x1 = col < ccl;   // same for the columns
    v00 = (r0 && c0) ? (x0 ? h0.y : h0.x) : qnan();
    v01 = (r0 && c1) ? (x1 ? h0.x : h0.y) : qnan();
    v10 = (r1 && c0) ? (x0 ? h1.y : h1.x) : qnan();
    v11 = (r1 && c1) ? (x1 ? h1.x : h1.y) : qnan();
}

// Masked lookup of an edge tile's slow frame (shift si: integer parts, fraction bits)
// at reference (row, col), from the block read at the clamped position: true when all
// four corners are valid (the caller keeps its plain interpolation); otherwise gm is
// Sec. 4's interpolation renormalised over the valid corners (the form masked_bilinear
// computes), NaN when none is valid.
__device__ inline bool slow_lookup(const int4 si, int row, int col, float2 top, float2 bot, int Rs, int Rf,
                                   float& gm) {
    float v00, v01, v10, v11;
    block_corners(row, col, top, bot, Rs, Rf, v00, v01, v10, v11);
    if (valid(v00) && valid(v01) && valid(v10) && valid(v11)) return true;
    const float fa = __int_as_float(si.z), fb = __int_as_float(si.w);
    const float ga = 1.f - fa, gb = 1.f - fb;
    const float w00 = ga * gb, w01 = ga * fb, w10 = fa * gb, w11 = fa * fb;
    float num = 0.f, den = 0.f;
    if (valid(v00)) { num = fmaf(w00, v00, num); den += w00; }
    if (valid(v01)) { num = fmaf(w01, v01, num); den += w01; }
    if (valid(v10)) { num = fmaf(w10, v10, num); den += w10; }
    if (valid(v11)) { num = fmaf(w11, v11, num); den += w11; }
    gm = den > 0.f ? num / den : qnan();
    return false;
}

// Integer shift of the planes' origin frame.
__device__ inline int2 planes_origin(const PmArgs& a) {
    return make_int2(axis_shift(a.dx[2 * a.pl_ref], a.o0).e, axis_shift(a.dx[2 * a.pl_ref + 1], a.o1).e);
}
// The tile's region, relative to the planes' origin, lies in the reference grid (so the
// planes have an entry for each of its positions).  Always true for interior tiles,
// whose lookups are all valid.
__device__ inline bool planes_cover(const PmArgs& a, const TileDesc& td, int2 eo) {
    const int r0 = td.cmin0 - a.rx - eo.x, c0 = td.cmin1 - a.ry - eo.y;
    return r0 >= 0 && c0 >= 0 && r0 + td.rh <= a.Rs && c0 + td.rw <= a.Rf;
}

// Column span [x, y] per plane row of the region positions (relative to the planes'
// origin) of the tiles that read the planes: interior tiles, and edge tiles searched
// whole whose region the planes cover; spans start empty (x > y).
__global__ void k_planes_span_clear(int2* __restrict__ prow, int Rs) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < Rs) prow[r] = make_int2(INT_MAX, INT_MIN);
}
// One work-group per row of tiles: the union of its interior tiles' regions (a band of
// plane rows with one column span, a superset of the exact spans), then one atomic pair
// per plane row of the band.
__global__ __launch_bounds__(256) void k_planes_span(const PmArgs a, int2* __restrict__ prow) {
    __shared__ int red[4][4];
    const int ty = blockIdx.x;
    const int2 eo = planes_origin(a);
    const bool edge_whole = (a.mm_on & 2) && !(a.mm_on & 32);
    int rlo = INT_MAX, rhi = INT_MIN, clo = INT_MAX, chi = INT_MIN;
    for (int tx = threadIdx.x; tx < a.tiles_x; tx += 256) {
        const int tile = ty * a.tiles_x + tx;
        const int cls = a.tinfo[tile].x;
        if (cls != CNT_FAST && !(cls == CNT_EDGE_MM && edge_whole)) continue;
        const TileDesc td = a.tiles[tile];
        if (cls == CNT_EDGE_MM && !planes_cover(a, td, eo)) continue;
        const int r0 = td.cmin0 - a.rx - eo.x, c0 = td.cmin1 - a.ry - eo.y;
        rlo = min(rlo, r0);
        rhi = max(rhi, r0 + td.rh - 1);
        clo = min(clo, c0);
        chi = max(chi, c0 + td.rw - 1);
    }
    rlo = wave_min_i(rlo);
    rhi = wave_max_i(rhi);
    clo = wave_min_i(clo);
    chi = wave_max_i(chi);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[w][0] = rlo;
        red[w][1] = rhi;
        red[w][2] = clo;
        red[w][3] = chi;
    }
    __syncthreads();
    rlo = min(min(red[0][0], red[1][0]), min(red[2][0], red[3][0]));
    rhi = max(max(red[0][1], red[1][1]), max(red[2][1], red[3][1]));
    clo = min(min(red[0][2], red[1][2]), min(red[2][2], red[3][2]));
    chi = max(max(red[0][3], red[1][3]), max(red[2][3], red[3][3]));
    if (rlo > rhi) return;
    clo = max(clo, 0);
    chi = min(chi, a.Rf - 1);
    for (int r = max(rlo, 0) + (int)threadIdx.x; r <= min(rhi, a.Rs - 1); r += 256) {
        atomicMin(&prow[r].x, clo);
        atomicMax(&prow[r].y, chi);
    }
}

// B operand of the tiles, precomputed once per search for every reference position P
// (coordinates relative to the integer shift e_c of the planes' origin frame c: the
// interior tiles' positions X all have X - e_c in the grid, since every lookup of theirs
// is valid; edge tiles use the planes where they cover them), over each plane row's
// span of positions of the tiles that read them (prow, from k_planes_span): the bytes
// the search kernel would generate for a lookup with all four corners valid, in planes
// [3][Rs Rf][NP] whose 16 bytes at (P, 64 kb + 16 g) are lane (c, g)'s operand, and 0
// for any other lookup; per position the sums sum_n g~_n^2 (exact 64-bit integer,
// converted once) and sum_n G~_n; and per (position, 16 frames) the validity bits
// (bits 0-15: all four corners valid, bits 16-31: at least one valid; padding frames
// count as valid).  A wave takes 16 positions x 4 frame groups, the layout of the
// search's B operand.
constexpr int PL_THREADS = 256;
constexpr int PL_COLS = 256;   // columns of a plane row per work-group
__global__ __launch_bounds__(PL_THREADS) void k_pm_planes(const PmArgs a, const int2* __restrict__ prow,
                                                          uint8_t* __restrict__ planes, double* __restrict__ pcs,
                                                          double* __restrict__ pgu, unsigned* __restrict__ pvb) {
    extern __shared__ float4 plsm[];
    const int NP = a.kblocks * MM_KB, KB = a.kblocks, Rf = a.Rf, Rs = a.Rs;
    // per frame: weights, the byte offset of this block's lookup row clamped into the
    // grid, the column offset of the lookup (e_c1 - e_n1) and the row of the lookup
    float4* fw = plsm;
    unsigned* rbase = (unsigned*)(fw + NP);
    int* dcol = (int*)(rbase + NP);
    int* lrow = dcol + NP;
    const int pr = blockIdx.y;
    const int2 span = prow[pr];
    const int cb = blockIdx.x * PL_COLS;
    if (span.x > span.y || cb + PL_COLS <= span.x || cb > span.y) return;
    const float fs = ldexpf(1.f, *a.fscale);
    const int2 eo = planes_origin(a);
    const int e00 = eo.x, e01 = eo.y;
    for (int n = threadIdx.x; n < NP; n += PL_THREADS) {
        const bool zero = n >= a.N;
        const int nn = zero ? 0 : n;
        unsigned go4;
        mm_frame_entry(a, nn, zero, fs, fw[n], go4);
        const int ex = axis_shift(a.dx[2 * nn], a.o0).e, ey = axis_shift(a.dx[2 * nn + 1], a.o1).e;
        const int rr = pr + e00 - ex;
        rbase[n] = 4u * (unsigned)(min(max(rr, 0), Rs - 2) * Rf);
        dcol[n] = e01 - ey;
        lrow[n] = rr;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, c = lane & 15, g = lane >> 4;
    const size_t RR = (size_t)Rs * Rf;
    const size_t stride = RR * NP;
    const char* __restrict__ refb = (const char*)a.refv;
    const unsigned rf4 = 4u * (unsigned)Rf;
    for (int col0 = cb + wave * 16; col0 < cb + PL_COLS; col0 += (PL_THREADS / 64) * 16) {
        const int pcol = col0 + c;
        const bool pv = pcol >= span.x && pcol <= span.y && pcol < Rf;
        const int pc = min(max(pcol, 0), Rf - 1);
        const size_t P = (size_t)pr * Rf + pc;
        long long cs = 0;
        unsigned long long gs = 0;
        for (int kb = 0; kb < KB; ++kb) {
            const int nb = kb * MM_KB + 16 * g;
            float vals[16];
            float2 top[16], bot[16];
            int col[16];
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                // the 2x2 block at the lookup, clamped into the grid
                col[t] = pc + dcol[nb + t];
                const unsigned e4 = rbase[nb + t] + 4u * (unsigned)min(max(col[t], 0), Rf - 2);
                top[t] = *(const float2*)(refb + e4);
                bot[t] = *(const float2*)(refb + (e4 + rf4));
            }
            double part = 0.0;
            // per frame: all four corners valid (bits 0-15; the value is the plain
            // interpolation) and at least one valid (bits 16-31); padding frames count as valid
            unsigned vbits = 0;
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const float4 wt = fw[nb + t];
                const float v = fmaf(wt.w, bot[t].y, fmaf(wt.z, bot[t].x, fmaf(wt.y, top[t].y, wt.x * top[t].x)));
                const int rr = lrow[nb + t];
                const bool in = (unsigned)rr <= (unsigned)(Rs - 2) && (unsigned)col[t] <= (unsigned)(Rf - 2);
                const bool all = in && v == v;
                vals[t] = all ? v : 0.f;
                bool any = all;
                if (!all) {
                    float v00, v01, v10, v11;
                    block_corners(rr, col[t], top[t], bot[t], Rs, Rf, v00, v01, v10, v11);
                    any = valid(v00) || valid(v01) || valid(v10) || valid(v11);
                }
                const bool pad = nb + t >= a.N;
                vbits |= ((all || pad) ? 1u : 0u) << t;
                vbits |= ((any || pad) ? 1u : 0u) << (16 + t);
            }
            unsigned B0[4], B1[4], B2[4];
            unsigned gsum = 0;
            // (16 squares below 2^44 each: the float64 partial is exact)
            mm_pack_b(vals, B0, B1, B2, part, gsum);
            cs += (long long)part;
            gs += gsum;
            if (pv) {
                const size_t off = P * NP + nb;
                *(uint4*)(planes + off) = make_uint4(B0[0], B0[1], B0[2], B0[3]);
                *(uint4*)(planes + stride + off) = make_uint4(B1[0], B1[1], B1[2], B1[3]);
                *(uint4*)(planes + 2 * stride + off) = make_uint4(B2[0], B2[1], B2[2], B2[3]);
                pvb[P * (NP / 16) + kb * 4 + g] = vbits;
            }
        }
        cs += __shfl_xor(cs, 16, 64);
        cs += __shfl_xor(cs, 32, 64);
        gs += __shfl_xor(gs, 16, 64);
        gs += __shfl_xor(gs, 32, 64);
        if (pv && g == 0) {
            pcs[P] = (double)cs;
            pgu[P] = (double)gs;
        }
    }
}

template <bool LDSA, bool EDGE, int MH, bool PLANES = false>
__device__ void pm_mma_item(const PmArgs& a, int slot) {
    extern __shared__ float smem[];
    const int cnt = EDGE ? CNT_EDGE_MM : CNT_FAST;
    if (slot >= a.counters[cnt]) return;
    const int tile = a.lists[(EDGE ? LIST_EDGE_MM : CNT_FAST) * a.ntiles + slot];
    const TileDesc td = a.tiles[tile];
    if constexpr (EDGE && MH == 4) {
        // with operand planes, the edge tiles searched whole whose region they cover go
        // to the planes kernel and the others to the kernel that generates its operand
        // (edge tiles searched in halves always generate it)
        if (PLANES ? !planes_cover(a, td, planes_origin(a))
                   : (a.planes != nullptr && planes_cover(a, td, planes_origin(a))))
            return;
    }
    const int ty = tile / a.tiles_x, tx = tile - ty * a.tiles_x;
    const int RW = td.rw, Q = td.rh * td.rw, NT = (Q + 15) >> 4;
    const int T0 = td.cmin0 - a.rx, T1 = td.cmin1 - a.ry;
    const int NX = a.NX, NY = a.NY, NC = NX * NY, N = a.N, Rf = a.Rf, KB = a.kblocks;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const size_t HW = (size_t)a.H * a.W;

    const int NP = KB * MM_KB;
    float* ebuf = smem;
    float4* fw = (float4*)(smem + ((size_t)16 * MH * NC + 3) / 4 * 4);
    unsigned* fgo4 = (unsigned*)(fw + NP);   // 4 * (e0 Rf + e1), modulo 2^32
    MmPix* pp = (MmPix*)(fgo4 + NP);
    char* ext = (char*)(pp + 64);
    int* sflag = (int*)ext;                                    // edge tiles only
    int* slist = sflag + NP;
    const int SMAX = a.mm_slow_max;
    int4* sinfo = (int4*)(slist + SMAX);
    float* sI = (float*)(sinfo + SMAX);                        // [SMAX][64]
    int* smisc = (int*)(sI + SMAX * 64);
    const int MW = mm_mask_words(SMAX);
    unsigned* imask = (unsigned*)(smisc + 4) + (size_t)wave * 16 * MW;   // this wave's [16][MW]
    uint4* apk = (uint4*)(EDGE ? ext + mm_edge_bytes(NP, SMAX) : ext);   // packed frames, if staged

    // edge tiles: the frames whose staged region holds an invalid lookup (the test of
    // the classification), in frame order, and the first frame without one
    int nslow = 0, nref = 0;
    if (EDGE) {
        for (int n = tid; n < NP; n += MM_THREADS) {
            int f = 0;
            if (n < N) {
                const AxisShift s0 = axis_shift(a.dx[2 * n], a.o0);
                const AxisShift s1 = axis_shift(a.dx[2 * n + 1], a.o1);
                const int r0 = T0 - s0.e, c0r = T1 - s1.e;
                f = rect_valid(a.sat, a.Rs, a.Rf, r0, r0 + td.rh, c0r, c0r + td.rw) ? 0 : 1;
            }
            sflag[n] = f;
        }
        __syncthreads();
        if (wave == 0) {
            int count = 0, first = -1;
            for (int b0 = 0; b0 < N; b0 += 64) {
                const int n = b0 + lane;
                const int f = n < N ? sflag[n] : 0;
                const unsigned long long m = __ballot(f);
                const unsigned long long fm = __ballot(n < N && !f);
                const int before = __popcll(m & ((1ull << lane) - 1ull));
                if (f && count + before < SMAX) {
                    slist[count + before] = n;
                    sflag[n] = count + before + 1;   // slot + 1
                }
                if (first < 0 && fm) first = b0 + __ffsll((long long)fm) - 1;
                count += __popcll(m);
            }
            if (lane == 0) {
                smisc[0] = min(count, SMAX);
                smisc[1] = first < 0 ? 0 : first;
            }
        }
        __syncthreads();
        nslow = smisc[0];
        nref = smisc[1];
    }

    // frame table: bilinear weights scaled by 2^F (exact: a power of two) and the
    // reference offset of the frame's shift; padding frames get zero weights and the
    // offset of a real frame (an edge tile's slow frames read their corners at their own
    // clamped positions, and keep the plain interpolation where all four are valid)
    const float fs = ldexpf(1.f, *a.fscale);
    for (int n = tid; n < NP; n += MM_THREADS) {
        const bool zero = n >= N;
        mm_frame_entry(a, zero ? nref : n, zero, fs, fw[n], fgo4[n]);
    }
    if (EDGE) {
        for (int e = tid; e < nslow * 64; e += MM_THREADS) {
            const int k = e >> 6, p = e & 63;
            const int n = slist[k];
            if (p == 0) {
                const AxisShift s0 = axis_shift(a.dx[2 * n], a.o0);
                const AxisShift s1 = axis_shift(a.dx[2 * n + 1], a.o1);
                sinfo[k] = make_int4(s0.e, s1.e, __float_as_int(s0.t), __float_as_int(s1.t));
            }
            const int i = ty * TILE + (p >> 3), j = tx * TILE + (p & 7);
            const bool good = i < a.H && j < a.W && a.mask[(size_t)i * a.W + j] != 0;
            const size_t pix = good ? (size_t)i * a.W + j : 0;
            sI[e] = good ? (float)a.frames[(size_t)n * HW + pix] : 0.f;
        }
    }
    const int F = *a.fscale;
    const double inv = ldexp(1.0, -F), inv2 = inv * inv;
    if (tid < 64) {
        const int p = tid;
        const int i = ty * TILE + (p >> 3), j = tx * TILE + (p & 7);
        const bool inb = i < a.H && j < a.W;
        const size_t pix = inb ? (size_t)i * a.W + j : 0;
        MmPix q;
        q.good = inb && a.mask[pix] != 0;
        q.dc0 = q.dc1 = -(1 << 28);
        q.al = q.be = q.ga = q.vf = 0.0;
        q.W = 0.f;
        q.zvar = 0;
        q.eo = 0;
        if (q.good) {
            q.dc0 = window_centre(a.u_in[pix]) - td.cmin0;
            q.dc1 = window_centre(a.u_in[HW + pix]) - td.cmin1;
            // this pixel's table (of the part of 16 MH pixels it belongs to) at candidate
            // (r - dc0, c - dc1)
            q.eo = (p & (16 * MH - 1)) * NC - (q.dc0 * NY + q.dc1);
            const double Wd = (double)a.white[pix];
            q.W = a.white[pix];
            const double* st = a.pstat + ((size_t)tile * 64 + p) * 4;
            // err = A - 2 W inv (S + g_q + Ib) + W^2 inv^2 C_q
            const double A = st[0], Ib = st[1], var = st[2];
            if (EDGE) q.vf = var;
            const double s = (EDGE || var <= 0.0) ? 1.0 : 1.0 / var;
            q.zvar = var > 0.0 ? 0 : 1;
            q.be = -2.0 * Wd * inv * s;
            q.ga = Wd * Wd * inv2 * s;
            q.al = fma(-2.0 * Wd * inv, Ib, A) * s;
        }
        pp[p] = q;
    }
    if (LDSA) {
        const uint4* src = a.ipk + (size_t)tile * KB * (4 * 2 * 64);
        for (int e = tid; e < KB * (4 * 2 * 64); e += MM_THREADS) apk[e] = src[e];
    }
    __syncthreads();

    const double kconst = 16384.0 * 257.0 * 65793.0 * (double)(KB * MM_KB);
    const int c = lane & 15, g = lane >> 4;
    const int2 peo = PLANES ? planes_origin(a) : make_int2(0, 0);
    const int pe00 = peo.x, pe01 = peo.y;
    const size_t pstride = (size_t)a.Rs * Rf * NP;
    const uint4* __restrict__ ipk =
        (LDSA ? (const uint4*)apk : a.ipk + (size_t)tile * KB * (4 * 2 * 64)) + lane;

    // the tile's pixels in 4 / MH parts of 16 MH pixels (row groups MH h .. MH h + MH - 1),
    // each with the region of its own windows and its own error table (every wave
    // finds the part's region from the pixel table)
#pragma unroll 1
    for (int h = 0; h < 4 / MH; ++h) {
        int h0 = 0, h1 = 0, RWh = RW, Qh = Q;
        if (MH < 4) {
            const bool in = (lane >> 4) / MH == h && pp[lane].good;
            const int mn0 = wave_min_i(in ? pp[lane].dc0 : INT_MAX);
            const int mx0 = wave_max_i(in ? pp[lane].dc0 : INT_MIN);
            const int mn1 = wave_min_i(in ? pp[lane].dc1 : INT_MAX);
            const int mx1 = wave_max_i(in ? pp[lane].dc1 : INT_MIN);
            const bool any_good = mn0 <= mx0;
            h0 = any_good ? mn0 : 0;
            h1 = any_good ? mn1 : 0;
            RWh = any_good ? mx1 - mn1 + NY : 1;
            Qh = any_good ? (mx0 - mn0 + NX) * RWh : 0;
        }
        const int NTh = (Qh + 15) >> 4;

        for (int nt = wave; nt < NTh; nt += MM_WAVES) {
            const int q = nt * 16 + c;
            const bool qv = q < Qh;
            // lanes past the region compute the region's last position and discard it;
            // (r, cc) are coordinates in the region of the whole tile
            const int qc = qv ? q : Qh - 1;
            const int rq = qc / RWh;
            const int r = rq + h0, cc = qc - rq * RWh + h1;
            // byte offset into the reference before the frame shift (every looked-up pixel
            // lies in the validated rectangle, so offsets are in [0, 4 Rs Rf))
            const unsigned roff4 = 4u * (unsigned)((T0 + r) * Rf + (T1 + cc));
            const unsigned rf4 = 4u * (unsigned)Rf;
            // precomputed planes: the position relative to frame 0's integer shift
            const int Pl = PLANES ? (T0 + r - pe00) * Rf + (T1 + cc - pe01) : 0;
            const char* __restrict__ refb = (const char*)a.refv;
            mm_v4i acc[MH][4];
#pragma unroll
            for (int m = 0; m < MH; ++m)
#pragma unroll
                for (int s = 0; s < 4; ++s) acc[m][s] = mm_v4i{0, 0, 0, 0};
            double GU = 0.0, CS = 0.0;
            if (EDGE) {
                for (int w = lane; w < 16 * MW; w += 64) imask[w] = 0u;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
            for (int kb = 0; kb < KB; ++kb) {
                mm_v4i b0, b1, b2;
                if constexpr (PLANES && !EDGE) {
                    // precomputed operand bytes of this lane's position and frames
                    const uint8_t* pb = a.planes + (size_t)Pl * NP + kb * MM_KB + 16 * g;
                    b0 = mm_as_v4i(*(const uint4*)pb);
                    b1 = mm_as_v4i(*(const uint4*)(pb + pstride));
                    b2 = mm_as_v4i(*(const uint4*)(pb + 2 * pstride));
                } else if constexpr (EDGE && PLANES) {
                    // edge tile covered by the planes: the planes hold the plain
                    // interpolation where all four corners are valid (every frame without
                    // invalid lookups in the region, and most positions of the others) and 0
                    // where none is; only a lookup with some corners valid, a slow frame near
                    // the edge of the valid reference, takes the renormalised form here, its
                    // bytes replaced and the column sums corrected by the difference (exact
                    // integers).  Invalid lookups are recorded for the epilogue.
                    const uint8_t* pb = a.planes + (size_t)Pl * NP + kb * MM_KB + 16 * g;
                    const uint4 q0 = *(const uint4*)pb;
                    const uint4 q1 = *(const uint4*)(pb + pstride);
                    const uint4 q2 = *(const uint4*)(pb + 2 * pstride);
                    const unsigned vb = a.pvb[(size_t)Pl * (NP / 16) + kb * 4 + g];
                    unsigned B0[4] = {q0.x, q0.y, q0.z, q0.w};
                    unsigned B1[4] = {q1.x, q1.y, q1.z, q1.w};
                    unsigned B2[4] = {q2.x, q2.y, q2.z, q2.w};
                    const int nb = kb * MM_KB + 16 * g;
                    unsigned none = ~(vb >> 16) & 0xffffu;
                    unsigned some = (vb >> 16) & ~vb & 0xffffu;
                    while (none) {
                        const int t = __ffs(none) - 1;
                        none &= none - 1u;
                        const int k = sflag[nb + t] - 1;
                        if (k >= 0) atomicOr(&imask[c * MW + (k >> 5)], 1u << (k & 31));
                    }
                    while (some) {
                        const int t = __ffs(some) - 1;
                        some &= some - 1u;
                        const int k = sflag[nb + t] - 1;
                        if (k < 0) continue;
                        const int4 si = sinfo[k];
                        const int row = T0 + r - si.x, col = T1 + cc - si.y;
                        const int rc = min(max(row, 0), a.Rs - 2), ccl = min(max(col, 0), Rf - 2);
                        const unsigned e4 = 4u * (unsigned)(rc * Rf + ccl);
                        const float2 top = *(const float2*)(refb + e4);
                        const float2 bot = *(const float2*)(refb + (e4 + rf4));
                        float gm = 0.f;
                        slow_lookup(si, row, col, top, bot, a.Rs, Rf, gm);
                        if (!valid(gm)) {
                            // (the planes hold 0 here, the value of an invalid lookup)
                            atomicOr(&imask[c * MW + (k >> 5)], 1u << (k & 31));
                            continue;
                        }
                        const unsigned gn = __float_as_uint(gm * fs + 12582912.f) - 0x4AC00000u;
                        const int w = t >> 2, sh = 8 * (t & 3);
                        const unsigned w0 = w == 0 ? B0[0] : w == 1 ? B0[1] : w == 2 ? B0[2] : B0[3];
                        const unsigned w1 = w == 0 ? B1[0] : w == 1 ? B1[1] : w == 2 ? B1[2] : B1[3];
                        const unsigned w2 = w == 0 ? B2[0] : w == 1 ? B2[1] : w == 2 ? B2[2] : B2[3];
                        const unsigned gold =
                            (((w0 >> sh) & 0xffu) | (((w1 >> sh) & 0xffu) << 8) | (((w2 >> sh) & 0xffu) << 16)) ^
                            0x808080u;
                        const double dn = (double)((int)gn - (1 << 23)), dold = (double)((int)gold - (1 << 23));
                        CS = fma(dn, dn, CS);
                        CS = fma(-dold, dold, CS);
                        GU += (double)gn - (double)gold;
                        const unsigned keep = ~(0xffu << sh);
                        const unsigned n0 = (w0 & keep) | (((gn ^ 0x80u) & 0xffu) << sh);
                        const unsigned n1 = (w1 & keep) | ((((gn >> 8) ^ 0x80u) & 0xffu) << sh);
                        const unsigned n2 = (w2 & keep) | ((((gn >> 16) ^ 0x80u) & 0xffu) << sh);
#pragma unroll
                        for (int x = 0; x < 4; ++x) {
                            B0[x] = x == w ? n0 : B0[x];
                            B1[x] = x == w ? n1 : B1[x];
                            B2[x] = x == w ? n2 : B2[x];
                        }
                    }
                    b0 = mm_v4i{(int)B0[0], (int)B0[1], (int)B0[2], (int)B0[3]};
                    b1 = mm_v4i{(int)B1[0], (int)B1[1], (int)B1[2], (int)B1[3]};
                    b2 = mm_v4i{(int)B2[0], (int)B2[1], (int)B2[2], (int)B2[3]};
                } else {
                    // B operand: 16 frames of this lane's position, three biased bytes each;
                    // branch-free so that the 32 loads of the 16 frames are in flight together
                    unsigned B0[4], B1[4], B2[4];
                    unsigned gsum = 0;
                    float2 top[16], bot[16];
                    const int nb = kb * MM_KB + 16 * g;
                    // edge tiles: a frame with invalid lookups in the region (slot sl > 0) reads
                    // the corners of its own lookup, clamped into the grid (out-of-grid corners
                    // are masked below), so that its loads join the batch
                    int slot[16], row[16], col[16];
#pragma unroll
                    for (int t = 0; t < 16; ++t) {
                        unsigned e4 = roff4 - fgo4[nb + t];
                        if (EDGE) {
                            slot[t] = sflag[nb + t];
                            const int4 si = sinfo[slot[t] > 0 ? slot[t] - 1 : 0];
                            row[t] = T0 + r - si.x;
                            col[t] = T1 + cc - si.y;
                            const int rc = min(max(row[t], 0), a.Rs - 2), ccl = min(max(col[t], 0), Rf - 2);
                            if (slot[t] > 0) e4 = 4u * (unsigned)(rc * Rf + ccl);
                        }
                        top[t] = *(const float2*)(refb + e4);
                        bot[t] = *(const float2*)(refb + (e4 + rf4));
                    }
                    float vals[16];
#pragma unroll
                    for (int t = 0; t < 16; ++t) {
                        const float4 wt = fw[nb + t];
                        vals[t] = fmaf(wt.w, bot[t].y, fmaf(wt.z, bot[t].x, fmaf(wt.y, top[t].y, wt.x * top[t].x)));
                        float gm;
                        if (EDGE && slot[t] > 0 &&
                            !slow_lookup(sinfo[slot[t] - 1], row[t], col[t], top[t], bot[t], a.Rs, Rf, gm)) {
                            if (valid(gm)) {
                                vals[t] = gm * fs;
                            } else {
                                vals[t] = 0.f;
                                const int k = slot[t] - 1;
                                atomicOr(&imask[c * MW + (k >> 5)], 1u << (k & 31));
                            }
                        }
                    }
#pragma unroll
                    for (int w = 0; w < 4; ++w) {
                        unsigned u[4];
#pragma unroll
                        for (int b = 0; b < 4; ++b) {
                            const int t = 4 * w + b;
                            const float v = vals[t];
                            // rint(v) + 2^23 from the bits of v + 1.5 * 2^23 (|v| < 2^22)
                            const unsigned gu = __float_as_uint(v + 12582912.f) - 0x4AC00000u;
                            const int gt = (int)gu - (1 << 23);
                            CS = fma((double)gt, (double)gt, CS);
                            gsum += gu;
                            u[b] = gu;
                        }
                        const unsigned t01l = __builtin_amdgcn_perm(u[1], u[0], 0x05010400u);
                        const unsigned t01h = __builtin_amdgcn_perm(u[1], u[0], 0x07030602u);
                        const unsigned t23l = __builtin_amdgcn_perm(u[3], u[2], 0x05010400u);
                        const unsigned t23h = __builtin_amdgcn_perm(u[3], u[2], 0x07030602u);
                        B0[w] = __builtin_amdgcn_perm(t23l, t01l, 0x05040100u) ^ 0x80808080u;
                        B1[w] = __builtin_amdgcn_perm(t23l, t01l, 0x07060302u) ^ 0x80808080u;
                        B2[w] = __builtin_amdgcn_perm(t23h, t01h, 0x05040100u) ^ 0x80808080u;
                    }
                    GU += (double)gsum;
                    b0 = mm_v4i{(int)B0[0], (int)B0[1], (int)B0[2], (int)B0[3]};
                    b1 = mm_v4i{(int)B1[0], (int)B1[1], (int)B1[2], (int)B1[3]};
                    b2 = mm_v4i{(int)B2[0], (int)B2[1], (int)B2[2], (int)B2[3]};
                }
                const uint4* ak = ipk + (size_t)kb * (4 * 2 * 64);
#pragma unroll
                for (int m = 0; m < MH; ++m) {
                    const int mg = h * MH + m;   // row group of the tile
                    const mm_v4i a0 = mm_as_v4i(ak[(mg * 2) * 64]);
                    const mm_v4i a1 = mm_as_v4i(ak[(mg * 2 + 1) * 64]);
                    acc[m][0] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a0, b0, acc[m][0], 0, 0, 0);
                    acc[m][1] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a0, b1, acc[m][1], 0, 0, 0);
                    acc[m][1] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a1, b0, acc[m][1], 0, 0, 0);
                    acc[m][2] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a0, b2, acc[m][2], 0, 0, 0);
                    acc[m][2] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a1, b1, acc[m][2], 0, 0, 0);
                    acc[m][3] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a1, b2, acc[m][3], 0, 0, 0);
                }
            }
            if constexpr (PLANES && !EDGE) {
                // the position's column sums over all frames, precomputed
                GU = a.pgu[Pl];
                CS = a.pcs[Pl];
            } else {
                // column sums of the position over the four lane groups (same sum in all four)
                GU += __shfl_xor(GU, 16, 64);
                GU += __shfl_xor(GU, 32, 64);
                CS += __shfl_xor(CS, 16, 64);
                CS += __shfl_xor(CS, 32, 64);
                if constexpr (EDGE && PLANES) {
                    // (the lanes' sums are the slow frames' corrections)
                    GU += a.pgu[Pl];
                    CS += a.pcs[Pl];
                }
            }
            const double gq = 128.0 * 257.0 * GU - kconst;
            const int rN = r * NY + cc;
            // S = sum_s 256^s acc_s; with at most 3 K-blocks |acc_s| <= 2^21 KB, so the two
            // low and the two high classes can be combined exactly in 32 bits first
            auto contraction = [&](int m, int i) -> double {
                if (KB <= 3) {
                    const int lo = acc[m][0][i] + (acc[m][1][i] << 8);
                    const int hi = acc[m][2][i] + (acc[m][3][i] << 8);
                    return fma(65536.0, (double)hi, (double)lo);
                }
                return (double)acc[m][0][i] + 256.0 * (double)acc[m][1][i] + 65536.0 * (double)acc[m][2][i] +
                       16777216.0 * (double)acc[m][3][i];
            };
            if (!EDGE) {
#pragma unroll
                for (int m = 0; m < MH; ++m) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int p = h * MH * 16 + m * 16 + 4 * g + i;
                        // (the error formed on every lane and the table index from the
                        // candidate: measured faster for interior tiles than the edge
                        // tiles' form below)
                        const MmPix& P = pp[p];
                        const int kx = r - P.dc0, ky = cc - P.dc1;
                        const double S = (double)acc[m][0][i] + 256.0 * (double)acc[m][1][i] +
                                         65536.0 * (double)acc[m][2][i] + 16777216.0 * (double)acc[m][3][i];
                        double v = fma(P.be, S + gq, fma(P.ga, CS, P.al));
                        v = v > 0.0 ? v : 0.0;
                        const float E = P.zvar ? (v == 0.0 ? 0.f : INFINITY) : (float)v;
                        if (qv && (unsigned)kx < (unsigned)NX && (unsigned)ky < (unsigned)NY)
                            ebuf[(size_t)(m * 16 + 4 * g + i) * NC + kx * NY + ky] = E;
                    }
                }
            } else {
                // every valid lookup is in the products (an invalid one entered as g = 0, so
                // its frame added I^2 to the error and (I - W)^2 to the variance); those
                // terms are taken out again for the invalid (position, frame) pairs, which
                // only frames with invalid lookups in the region can have.  FP64 where the
                // subtraction can cancel.
                double ef[4 * MH], ai[4 * MH];
                float vi[4 * MH], Wl[4 * MH];
#pragma unroll
                for (int m = 0; m < MH; ++m) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int e = m * 4 + i, p = h * MH * 16 + m * 16 + 4 * g + i;
                        const MmPix& P = pp[p];
                        ef[e] = fma(P.be, contraction(m, i) + gq, fma(P.ga, CS, P.al));
                        ai[e] = 0.0;
                        vi[e] = 0.f;
                        Wl[e] = P.W;
                    }
                }
                // the invalid (position, slow frame) pairs recorded by the B operand lanes
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                int ninv = 0;
                for (int w = 0; w < MW; ++w) {
                    unsigned bits = imask[c * MW + w];
                    ninv += __popc(bits);
                    while (bits) {
                        const int k = w * 32 + __ffs(bits) - 1;
                        bits &= bits - 1u;
#pragma unroll
                        for (int m = 0; m < MH; ++m) {
#pragma unroll
                            for (int i = 0; i < 4; ++i) {
                                const int e = m * 4 + i, p = h * MH * 16 + m * 16 + 4 * g + i;
                                const float I = sI[k * 64 + p];
                                ai[e] = fma((double)I, (double)I, ai[e]);
                                const float v = I - Wl[e];
                                vi[e] = fmaf(v, v, vi[e]);
                            }
                        }
                    }
                }
                const int nv = N - ninv;
#pragma unroll
                for (int m = 0; m < MH; ++m) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int e = m * 4 + i, p = h * MH * 16 + m * 16 + 4 * g + i;
                        const int kx = r - pp[p].dc0, ky = cc - pp[p].dc1;
                        if (qv && (unsigned)kx < (unsigned)NX && (unsigned)ky < (unsigned)NY) {
                            double err = ef[e] - ai[e];
                            err = err > 0.0 ? err : 0.0;
                            const float var = (float)(pp[p].vf - (double)vi[e]);
                            ebuf[pp[p].eo + rN] = Wl[e] == 0.f ? zero_white_error((float)err, nv)
                                                               : normalised_error((float)err, var, nv);
                        }
                    }
                }
            }
        }
        __syncthreads();

        // first minimum per pixel (TPP lanes per pixel), then refinement and output
        {
            constexpr int TPP = MM_THREADS / (16 * MH);
            const int pl = tid / TPP, sub = tid % TPP, p = h * MH * 16 + pl;
            const MmPix P = pp[p];
            float be = INFINITY;
            int bk = INT_MAX;
            if (P.good) {
                const float* e = ebuf + (size_t)pl * NC;
                for (int k = sub; k < NC; k += TPP) {
                    const float v = e[k];
                    if (better(v, k, be, bk)) {
                        be = v;
                        bk = k;
                    }
                }
            }
#pragma unroll
            for (int o = 1; o < TPP; o <<= 1) {
                const float e2 = __shfl_xor(be, o, 64);
                const int k2 = __shfl_xor(bk, o, 64);
                if (better(e2, k2, be, bk)) {
                    be = e2;
                    bk = k2;
                }
            }
            const int i = ty * TILE + (p >> 3), j = tx * TILE + (p & 7);
            if (sub == 0 && i < a.H && j < a.W) {
                const size_t pix = (size_t)i * a.W + j;
                if (!P.good || !isfinite(be)) {
                    write_unchanged(a, pix, HW);
                } else {
                    const int bx = bk / NY, by = bk - bx * NY;
                    float ox = 0.f, oy = 0.f;
                    if (a.refine) {
                        float st[9];
                        const float* e = ebuf + (size_t)pl * NC;
#pragma unroll
                        for (int t = 0; t < 9; ++t) {
                            const int kx = bx + t / 3 - 1, ky = by + t % 3 - 1;
                            st[t] = (kx >= 0 && kx < NX && ky >= 0 && ky < NY) ? e[kx * NY + ky] : INFINITY;
                        }
                        refine_at(st, bx, by, NX, NY, ox, oy);
                    }
                    const int c0 = P.dc0 + td.cmin0, c1 = P.dc1 + td.cmin1;
                    a.u_out[pix] = (float)(c0 + bx - a.rx) + ox;
                    a.u_out[HW + pix] = (float)(c1 + by - a.ry) + oy;
                    if (a.err_out) a.err_out[pix] = be;
                    if (a.arg_out) a.arg_out[pix] = bk;
                }
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------ wrappers
// Single-job launches (one work-group per item) and shared launches over the items of
// several jobs, also one work-group per item (item i of the batch belongs to job j with
// off[j] <= i < off[j + 1]; each job's arguments come from a device table; a loop of
// persistent work-groups over the items had kept the item state live around the body,
// which pushed the edge search past its registers).  A job's items and their results do
// not depend on the other jobs of the batch.
__device__ inline int batch_job(const int* __restrict__ off, int njobs, int item) {
    int lo = 0, hi = njobs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= item) lo = mid; else hi = mid;
    }
    return lo;
}

#define PXST_WRAP(NAME, BOUND, BODY)                                                          \
    __global__ __launch_bounds__(BOUND) void NAME(const PmArgs a) { BODY(a, (int)blockIdx.x); } \
    __global__ __launch_bounds__(BOUND) void NAME##_batch(const PmArgs* __restrict__ jobs,       \
                                                          const int* __restrict__ off, int njobs) { \
        const int item = blockIdx.x;                                                          \
        if (item >= off[njobs]) return;                                                       \
        const int j = batch_job(off, njobs, item);                                            \
        BODY(table_entry(jobs, j), item - off[j]);                                            \
    }

// single-job launch of a matrix-core search over the list counted by CNT, items in
// contiguous runs per XCD
#define PXST_WRAP_XCD(NAME, BODY, CNT)                                                        \
    __global__ __launch_bounds__(MM_THREADS) void NAME(const PmArgs a) {                      \
        BODY(a, xcd_item((int)blockIdx.x, a.counters[CNT]));                                 \
    }

PXST_WRAP(k_classify, 64, classify_item)
PXST_WRAP(k_pm_generic, 256, pm_generic_item)
__device__ void pm_mma_fast_lds(const PmArgs& a, int slot) { pm_mma_item<true, false, 4>(a, slot); }
__device__ void pm_mma_fast_glb(const PmArgs& a, int slot) { pm_mma_item<false, false, 4>(a, slot); }
__device__ void pm_mma_edge_lds(const PmArgs& a, int slot) { pm_mma_item<true, true, 4>(a, slot); }
__device__ void pm_mma_edge_glb(const PmArgs& a, int slot) { pm_mma_item<false, true, 4>(a, slot); }
__device__ void pm_mma_fast_half(const PmArgs& a, int slot) { pm_mma_item<false, false, 2>(a, slot); }
__device__ void pm_mma_edge_half(const PmArgs& a, int slot) { pm_mma_item<false, true, 2>(a, slot); }
PXST_WRAP(k_pm_mma_lds, MM_THREADS, pm_mma_fast_lds)
PXST_WRAP(k_pm_mma_glb, MM_THREADS, pm_mma_fast_glb)
PXST_WRAP(k_pm_mma_edge_lds, MM_THREADS, pm_mma_edge_lds)
PXST_WRAP(k_pm_mma_edge_glb, MM_THREADS, pm_mma_edge_glb)
PXST_WRAP(k_pm_mma_half, MM_THREADS, pm_mma_fast_half)
__device__ void pm_mma_planes_lds(const PmArgs& a, int slot) { pm_mma_item<true, false, 4, true>(a, slot); }
__device__ void pm_mma_planes_glb(const PmArgs& a, int slot) { pm_mma_item<false, false, 4, true>(a, slot); }
__device__ void pm_mma_half_planes_lds(const PmArgs& a, int slot) { pm_mma_item<true, false, 2, true>(a, slot); }
__device__ void pm_mma_half_planes_glb(const PmArgs& a, int slot) { pm_mma_item<false, false, 2, true>(a, slot); }
PXST_WRAP_XCD(k_pm_mma_planes_lds, pm_mma_planes_lds, CNT_FAST)
PXST_WRAP_XCD(k_pm_mma_planes_glb, pm_mma_planes_glb, CNT_FAST)
PXST_WRAP_XCD(k_pm_mma_half_planes_lds, pm_mma_half_planes_lds, CNT_FAST)
PXST_WRAP_XCD(k_pm_mma_half_planes_glb, pm_mma_half_planes_glb, CNT_FAST)
__device__ void pm_mma_edge_planes_lds(const PmArgs& a, int slot) { pm_mma_item<true, true, 4, true>(a, slot); }
__device__ void pm_mma_edge_planes_glb(const PmArgs& a, int slot) { pm_mma_item<false, true, 4, true>(a, slot); }
PXST_WRAP_XCD(k_pm_mma_edge_planes_lds, pm_mma_edge_planes_lds, CNT_EDGE_MM)
PXST_WRAP_XCD(k_pm_mma_edge_planes_glb, pm_mma_edge_planes_glb, CNT_EDGE_MM)
PXST_WRAP(k_pm_mma_edge_half, MM_THREADS, pm_mma_edge_half)

template <int CW, int KR>
__global__ __launch_bounds__(512) void k_pm_fast(const PmArgs a) {
    pm_fast_item<CW, KR>(a, (int)blockIdx.x);
}
template <int CW, int KR>
__global__ __launch_bounds__(512) void k_pm_fast_batch(const PmArgs* __restrict__ jobs,
                                                       const int* __restrict__ off, int njobs) {
    const int item = blockIdx.x;
    if (item >= off[njobs]) return;
    const int j = batch_job(off, njobs, item);
    pm_fast_item<CW, KR>(table_entry(jobs, j), item - off[j]);
}
template <int CW, int KR>
__global__ __launch_bounds__(512) void k_pm_edge(const PmArgs a) {
    pm_edge_item<CW, KR>(a, (int)blockIdx.x);
}
template <int CW, int KR>
__global__ __launch_bounds__(512) void k_pm_edge_batch(const PmArgs* __restrict__ jobs,
                                                       const int* __restrict__ off, int njobs) {
    const int item = blockIdx.x;
    if (item >= off[njobs]) return;
    const int j = batch_job(off, njobs, item);
    pm_edge_item<CW, KR>(table_entry(jobs, j), item - off[j]);
}

// ------------------------------------------------------------------------ dispatch
typedef void (*PmKernel)(PmArgs);
typedef void (*PmBatchKernel)(const PmArgs*, const int*, int);

struct LdsShape {
    PmKernel fn;
    PmBatchKernel batch;
    int cw, kr;
};

template <int CW, int KR>
constexpr LdsShape fast_shape() { return LdsShape{k_pm_fast<CW, KR>, k_pm_fast_batch<CW, KR>, CW, KR}; }
template <int CW, int KR>
constexpr LdsShape edge_shape() { return LdsShape{k_pm_edge<CW, KR>, k_pm_edge_batch<CW, KR>, CW, KR}; }

// FAST: full window rows per thread (CW = 2 r_fs + 1), rows per thread chosen so that
// two accumulators per candidate stay within about 100 registers.
LdsShape pick_fast(int ny) {
    switch (ny) {
        case 1: return fast_shape<1, 8>();
        case 3: return fast_shape<3, 8>();
        case 5: return fast_shape<5, 8>();
        case 7: return fast_shape<7, 8>();
        case 9: return fast_shape<9, 5>();
        case 11: return fast_shape<11, 4>();
        case 13: return fast_shape<13, 4>();
        case 15: return fast_shape<15, 4>();
        case 17: return fast_shape<17, 3>();
        case 19: return fast_shape<19, 3>();
        case 21: return fast_shape<21, 3>();
        case 23: return fast_shape<23, 2>();
        case 25: return fast_shape<25, 2>();
        case 27: return fast_shape<27, 2>();
        case 29: return fast_shape<29, 2>();
        default: return fast_shape<31, 2>();
    }
}

// EDGE: three registers per candidate (two for the compensated error, one for the
// variance of frames with invalid lookups), full window rows.
LdsShape pick_edge(int ny) {
    switch (ny) {
        case 1: return edge_shape<1, 8>();
        case 3: return edge_shape<3, 8>();
        case 5: return edge_shape<5, 8>();
        case 7: return edge_shape<7, 5>();
        case 9: return edge_shape<9, 4>();
        case 11: return edge_shape<11, 3>();
        case 13: return edge_shape<13, 3>();
        case 15: return edge_shape<15, 2>();
        case 17: return edge_shape<17, 2>();
        case 19: return edge_shape<19, 2>();
        case 21: return edge_shape<21, 2>();
        case 23: return edge_shape<23, 1>();
        case 25: return edge_shape<25, 1>();
        case 27: return edge_shape<27, 1>();
        case 29: return edge_shape<29, 1>();
        default: return edge_shape<31, 1>();
    }
}

struct Launch {
    int nchunks, nblocks, sub, waves;
};

Launch plan_launch(int nx, int ny, int cw, int kr) {
    Launch l;
    l.nchunks = (ny + cw - 1) / cw;
    l.nblocks = ((nx + kr - 1) / kr) * l.nchunks;
    l.sub = 1;
    while ((l.nblocks + l.sub - 1) / l.sub > 8 && l.sub < 8) l.sub *= 2;
    l.waves = (l.nblocks + l.sub - 1) / l.sub;
    return l;
}

size_t lds_bytes(const Launch& l, int n_frames) {
    const size_t stage = (size_t)SHIFT_TAB_OFF * sizeof(float) + (size_t)n_frames * sizeof(int4);
    const int ppp = 64 / l.sub;
    const size_t red = (size_t)l.nblocks * ppp * 8 + (size_t)ppp * 8 + (size_t)ppp * 9 * 4;
    return stage > red ? stage : red;
}


PmArgs make_pm_args(const Geom& g, const pxst_scan& sc, const float* refv, const int* sat,
                    const float* dx, const float* u_in, const pxst_window& win, float* u_out,
                    float* err_min, int32_t* argmin, char* ws, const Layout& L, bool planes) {
    PmArgs a{};
    a.frames = sc.frames;
    a.white = sc.white;
    a.mask = sc.mask;
    a.refv = refv;
    a.sat = sat;
    a.dx = dx;
    a.u_in = u_in;
    a.u_out = u_out;
    a.err_out = err_min;
    a.arg_out = argmin;
    a.tiles = (TileDesc*)(ws + L.tiles);
    a.lists = (int*)(ws + L.lists);
    a.counters = (int*)(ws + L.counters);
    a.tinfo = (int4*)(ws + L.tinfo);
    a.N = g.N;
    a.H = g.H;
    a.W = g.W;
    a.Rs = g.Rs;
    a.Rf = g.Rf;
    a.o0 = g.o0;
    a.o1 = g.o1;
    a.rx = win.r_ss;
    a.ry = win.r_fs;
    a.NX = 2 * win.r_ss + 1;
    a.NY = 2 * win.r_fs + 1;
    a.refine = win.refine != 0;
    a.tiles_x = (g.W + TILE - 1) / TILE;
    const int tiles_y = (g.H + TILE - 1) / TILE;
    a.ntiles = a.tiles_x * tiles_y;
    const LdsShape fs = pick_fast(a.NY), es = pick_edge(a.NY);
    const Launch lf = plan_launch(a.NX, a.NY, fs.cw, fs.kr);
    const Launch le = plan_launch(a.NX, a.NY, es.cw, es.kr);
    a.stage_cap = 8 * le.waves * 64;
    a.fast_cap = PFS * lf.waves * 64;
    a.ipk = (const uint4*)(ws + L.ipk);
    a.pstat = (const double*)(ws + L.pstat);
    a.fscale = (const int*)(ws + L.fscale);
    a.kblocks = L.kblocks;
    a.pl_ref = g.N / 2;
    const MmPlan mp = mm_plan(a.NX, a.NY, g.N, planes);
    a.mm_on = (mp.fast ? 1 : 0) | (mp.edge ? 2 : 0) | (mp.fast_stage ? 4 : 0) | (mp.edge_stage ? 8 : 0) |
              (mp.fast_half ? 16 : 0) | (mp.edge_half ? 32 : 0);
    a.mm_slow_max = mp.slow_max;
    return a;
}

// One launch of the matrix-core search (interior or edge tiles) for one job
// (dev_jobs == nullptr: host_args[0] is passed by value) or a batch of jobs with the
// same window and the same kernel choice (their host-side arguments in host_args; all
// of them search whole tiles or all of them halves).
// The frames are staged in LDS when every job of the launch stages them; the LDS size
// is the largest any job needs.
int launch_mma(const PmArgs* host_args, int nargs, const PmArgs* dev_jobs, const int* off, int grid,
               bool edge, hipStream_t s) {
    const bool half = (host_args[0].mm_on & (edge ? 32 : 16)) != 0;
    // (the plan stages the frames of interior-tile halves only where they fit)
    bool stage = !(half && edge);
    for (int j = 0; j < nargs; ++j) {
        stage = stage && (host_args[j].mm_on & (edge ? 8 : 4)) != 0;
        if (((host_args[j].mm_on & (edge ? 32 : 16)) != 0) != half) {
            set_error("matrix-core search: jobs of one launch differ in tile halves");
            return PXST_EINVAL;
        }
    }
    size_t sh = 0;
    for (int j = 0; j < nargs; ++j) {
        const PmArgs& x = host_args[j];
        sh = std::max(sh, mm_lds_bytes(x.NX * x.NY, x.N, stage, edge, x.mm_slow_max, half ? 2 : 4));
    }
    if (sh > MM_LDS_MAX) {
        set_error("matrix-core search: %zu bytes of LDS exceed the limit", sh);
        return PXST_EINVAL;
    }
    if (dev_jobs == nullptr) {
        const bool planes = host_args[0].planes != nullptr;
        const PmKernel kern = half ? (edge ? k_pm_mma_edge_half
                                      : planes ? (stage ? k_pm_mma_half_planes_lds : k_pm_mma_half_planes_glb)
                                               : k_pm_mma_half)
                              : edge ? (planes ? (stage ? k_pm_mma_edge_planes_lds : k_pm_mma_edge_planes_glb)
                                               : (stage ? k_pm_mma_edge_lds : k_pm_mma_edge_glb))
                              : planes ? (stage ? k_pm_mma_planes_lds : k_pm_mma_planes_glb)
                                       : (stage ? k_pm_mma_lds : k_pm_mma_glb);
        hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
        hipLaunchKernelGGL(kern, dim3(grid), dim3(MM_THREADS), sh, s, host_args[0]);
        if (edge && !half && planes) {
            // the edge tiles the planes do not cover
            const PmKernel rest = stage ? k_pm_mma_edge_lds : k_pm_mma_edge_glb;
            hipFuncSetAttribute((const void*)rest, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
            hipLaunchKernelGGL(rest, dim3(grid), dim3(MM_THREADS), sh, s, host_args[0]);
        }
    } else {
        const PmBatchKernel kern = half ? (edge ? k_pm_mma_edge_half_batch : k_pm_mma_half_batch)
                                   : edge ? (stage ? k_pm_mma_edge_lds_batch : k_pm_mma_edge_glb_batch)
                                          : (stage ? k_pm_mma_lds_batch : k_pm_mma_glb_batch);
        hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
        hipLaunchKernelGGL(kern, dim3(grid), dim3(MM_THREADS), sh, s, dev_jobs, off, nargs);
    }
    return check_hip(hipGetLastError(), edge ? "pixel-map search (edge tiles, matrix cores)"
                                             : "pixel-map search (interior tiles, matrix cores)");
}

// Launch shapes of the fast and edge kernels for a window (same for every job with
// that window).
struct PmPlan {
    LdsShape fs, es;
    Launch lf, le;
    PmArgs fast_args(const PmArgs& a) const {
        PmArgs b = a;
        b.nchunks = lf.nchunks;
        b.nblocks = lf.nblocks;
        b.sub = lf.sub;
        return b;
    }
    PmArgs edge_args(const PmArgs& a) const {
        PmArgs b = a;
        b.nchunks = le.nchunks;
        b.nblocks = le.nblocks;
        b.sub = le.sub;
        return b;
    }
};

PmPlan pm_plan(int NX, int NY) {
    PmPlan p;
    p.fs = pick_fast(NY);
    p.es = pick_edge(NY);
    p.lf = plan_launch(NX, NY, p.fs.cw, p.fs.kr);
    p.le = plan_launch(NX, NY, p.es.cw, p.es.kr);
    return p;
}

}  // namespace

int launch_pixel_map(const Geom& g, const pxst_scan& sc, const float* refv, const int* sat,
                     const float* dx, const float* u_in, const pxst_window& win, float* u_out,
                     float* err_min, int32_t* argmin, char* ws, const Layout& L, hipStream_t s,
                     const uint8_t* half, int hval) {
    // interior tiles read precomputed operand planes when the workspace holds them
    const bool use_planes = !half && L.planes_on && g.Rs >= 2 && g.Rf >= 2;
    PmArgs a = make_pm_args(g, sc, refv, sat, dx, u_in, win, u_out, err_min, argmin, ws, L, use_planes);
    if (half) {
        // split-half search: the halves differ per (frame, pixel), so the frame sums of
        // the matrix-core contraction do not apply; the tiles go to the LDS-staged
        // kernels (which skip the terms outside the half) and the generic one
        a.half = half;
        a.hval = hval;
        a.mm_on = 0;
    }
    const PmPlan pl = pm_plan(a.NX, a.NY);
    hipLaunchKernelGGL(k_classify, dim3(a.ntiles), dim3(64), 0, s, a);
    hipLaunchKernelGGL(k_compact, dim3(1), dim3(COMPACT_THREADS), 0, s, a);
    int rc = check_hip(hipGetLastError(), "pixel-map classification");
    if (rc) return rc;
    // (profiling: the launches' work counts, final once the lists are built, in one copy)
    const int snap = profile_snapshot(a.counters, CNT_N, s);

    const long long evals_per_good_px = (long long)a.NX * a.NY * g.N;
    // with the operand planes (interior tiles, and edge tiles searched whole)
    PmArgs ap = a;
    if (a.mm_on & 1) {
        // the operand planes, when they fit the workspace
        if (use_planes) {
            uint8_t* planes = (uint8_t*)(ws + L.planes);
            double* pcs = (double*)(ws + L.pcs);
            double* pgu = (double*)(ws + L.pgu);
            unsigned* pvb = (unsigned*)(ws + L.pvb);
            ap.planes = planes;
            ap.pcs = pcs;
            ap.pgu = pgu;
            ap.pvb = pvb;
            const size_t sh = (size_t)L.kblocks * MM_KB * (16 + 4 + 4 + 4);
            int2* prow = (int2*)(ws + L.prow);
            hipFuncSetAttribute((const void*)k_pm_planes, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
            profile_begin("pm_planes", s);
            hipLaunchKernelGGL(k_planes_span_clear, dim3((g.Rs + 255) / 256), dim3(256), 0, s, prow, g.Rs);
            hipLaunchKernelGGL(k_planes_span, dim3(a.ntiles / a.tiles_x), dim3(256), 0, s, a, prow);
            hipLaunchKernelGGL(k_pm_planes, dim3((g.Rf + PL_COLS - 1) / PL_COLS, g.Rs), dim3(PL_THREADS), sh, s, a,
                               (const int2*)prow, planes, pcs, pgu, pvb);
            profile_end("pm_planes", s, 0, nullptr, 0);
            rc = check_hip(hipGetLastError(), "operand planes");
            if (rc) return rc;
        }
        profile_begin("pm_fast", s);
        profile_begin("pm_fast_int8_ops", s);
        rc = launch_mma(&ap, 1, nullptr, nullptr, a.ntiles, false, s);
        // int8 operations issued on the matrix cores: 2 per multiply-add, 64 pixels x
        // positions x padded frames x 6 byte pairs
        profile_end_snap("pm_fast_int8_ops", s, snap, CNT_MM_POS, a.counters + CNT_MM_POS,
                    2LL * 64 * 6 * (long long)mm_frames_padded(g.N));
        profile_end_snap("pm_fast", s, snap, CNT_GOOD_FAST, a.counters + CNT_GOOD_FAST, evals_per_good_px);
        if (rc) return rc;
    } else {
        const size_t sh = lds_bytes(pl.lf, g.N);
        hipFuncSetAttribute((const void*)pl.fs.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
        profile_begin("pm_fast", s);
        hipLaunchKernelGGL(pl.fs.fn, dim3(a.ntiles), dim3(pl.lf.waves * 64), sh, s, pl.fast_args(a));
        profile_end_snap("pm_fast", s, snap, CNT_GOOD_FAST, a.counters + CNT_GOOD_FAST, evals_per_good_px);
        rc = check_hip(hipGetLastError(), "pixel-map search (interior tiles)");
        if (rc) return rc;
    }
    if (a.mm_on & 2) {
        profile_begin("pm_edge_mma", s);
        rc = launch_mma(&ap, 1, nullptr, nullptr, a.ntiles, true, s);
        profile_end_snap("pm_edge_mma", s, snap, CNT_GOOD_EDGE_MM, a.counters + CNT_GOOD_EDGE_MM, evals_per_good_px);
        if (rc) return rc;
    }
    {
        const size_t sh = lds_bytes(pl.le, g.N);
        hipFuncSetAttribute((const void*)pl.es.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
        profile_begin("pm_edge", s);
        hipLaunchKernelGGL(pl.es.fn, dim3(a.ntiles), dim3(pl.le.waves * 64), sh, s, pl.edge_args(a));
        profile_end_snap("pm_edge", s, snap, CNT_GOOD_EDGE, a.counters + CNT_GOOD_EDGE, evals_per_good_px);
        rc = check_hip(hipGetLastError(), "pixel-map search (edge tiles)");
        if (rc) return rc;
    }
    profile_begin("pm_generic", s);
    hipLaunchKernelGGL(k_pm_generic, dim3(a.ntiles), dim3(256), 0, s, a);
    profile_end_snap("pm_generic", s, snap, CNT_GOOD_GENERIC, a.counters + CNT_GOOD_GENERIC, evals_per_good_px);
    return check_hip(hipGetLastError(), "pixel-map search (scattered tiles)");
}

int launch_pm_setup(const Geom& g, const pxst_scan& sc, char* ws, const Layout& L, hipStream_t s) {
    const int tiles_x = (g.W + TILE - 1) / TILE;
    const int ntiles = tiles_x * ((g.H + TILE - 1) / TILE);
    hipLaunchKernelGGL(k_pm_pack, dim3((unsigned)(ntiles * L.kblocks)), dim3(256), 0, s, sc.frames,
                       sc.mask, g.N, g.H, g.W, tiles_x, L.kblocks, (uint4*)(ws + L.ipk));
    hipLaunchKernelGGL(k_pm_pixstats, dim3((unsigned)(((size_t)ntiles * 64 + 255) / 256)), dim3(256), 0, s,
                       sc.frames, sc.white, sc.mask, g.N, g.H, g.W, tiles_x, (double*)(ws + L.pstat));
    return check_hip(hipGetLastError(), "pixel-map setup");
}

// Batched pixel-map search of several jobs, in two phases so that a caller can stage the
// argument tables of all its batched stages before one copy: staging (host only) and
// launching.  Per group of jobs sharing a window: counters reset and one shared
// classification over every tile of every job, then one shared launch of each kernel
// class.
struct PmGroup {
    PmPlan pl;
    int m = 0, grid = 0, max_n = 1, mm_on = 0;
    std::vector<PmArgs> ga;
    BatchUpload g, f, e;     // tables: plain, fast-kernel and edge-kernel arguments
};
struct PmBatchImpl {
    std::vector<PmJobDesc> solo;
    int n = 0, cls_grid = 0;
    BatchUpload cls;
    std::vector<PmGroup> groups;
};

size_t pixel_map_batch_table_bytes(int n) {
    // classification table and offsets, then at most three tables with offsets per group
    // (each rounded up to 256 bytes; at most n groups)
    const size_t P = sizeof(PmArgs);
    return (size_t)n * P + 256 + (size_t)(n + 1) * 4 + 256 +
           3 * ((size_t)n * P + (size_t)n * 256 + (size_t)2 * n * 4 + (size_t)n * 256);
}

int stage_pixel_map_batch(const PmJobDesc* jobs_in, int n_in, BatchArena& ar,
                          std::shared_ptr<PmBatchImpl>& out) {
    auto b = std::make_shared<PmBatchImpl>();
    // A job of at least PM_SOLO_TILES tiles whose workspace holds the operand planes fills
    // the device by itself: it is searched as it would be alone (planes, tile halves,
    // per-XCD work runs), each such job in its own launches; the smaller jobs share the
    // batched launches, where launch overhead is what they save.
    std::vector<PmJobDesc> small;
    small.reserve(n_in);
    for (int j = 0; j < n_in; ++j) {
        const PmJobDesc& d = jobs_in[j];
        const long long tiles = (long long)((d.g.H + TILE - 1) / TILE) * ((d.g.W + TILE - 1) / TILE);
        if (d.L->planes_on && d.g.Rs >= 2 && d.g.Rf >= 2 && tiles >= PM_SOLO_TILES)
            b->solo.push_back(d);
        else
            small.push_back(d);
    }
    const int n = (int)small.size();
    b->n = n;
    if (n > 0) {
        std::vector<PmArgs> base(n);
        for (int j = 0; j < n; ++j) {
            const PmJobDesc& d = small[j];
            base[j] = make_pm_args(d.g, d.sc, d.refv, d.sat, d.dx, d.u_in, d.win, d.u_out, nullptr,
                                   nullptr, d.ws, *d.L, false);
        }
        std::vector<int> off(n + 1, 0);
        for (int j = 0; j < n; ++j) off[j + 1] = off[j] + base[j].ntiles;
        b->cls = stage_table(ar, base.data(), n * sizeof(PmArgs), off);
        b->cls_grid = off[n];
        // groups of jobs with the same window and the same kernel choice (each job's
        // choice depends on its own sizes only, so a job is classified and searched the
        // same way alone and in a batch)
        std::vector<int> done(n, 0);
        for (int j0 = 0; j0 < n; ++j0) {
            if (done[j0]) continue;
            std::vector<int> grp;
            for (int j = j0; j < n; ++j)
                if (!done[j] && base[j].NX == base[j0].NX && base[j].NY == base[j0].NY &&
                    base[j].mm_on == base[j0].mm_on) {
                    grp.push_back(j);
                    done[j] = 1;
                }
            PmGroup G;
            G.pl = pm_plan(base[j0].NX, base[j0].NY);
            G.m = (int)grp.size();
            G.mm_on = base[j0].mm_on;
            std::vector<PmArgs> fa(G.m), ea(G.m);
            G.ga.resize(G.m);
            std::vector<int> go(G.m + 1, 0);
            for (int q = 0; q < G.m; ++q) {
                fa[q] = G.pl.fast_args(base[grp[q]]);
                ea[q] = G.pl.edge_args(base[grp[q]]);
                G.ga[q] = base[grp[q]];
                go[q + 1] = go[q] + base[grp[q]].ntiles;
                G.max_n = std::max(G.max_n, base[grp[q]].N);
            }
            G.grid = go[G.m];
            G.g = stage_table(ar, G.ga.data(), G.m * sizeof(PmArgs), go);
            if (!(G.mm_on & 1)) G.f = stage_table(ar, fa.data(), G.m * sizeof(PmArgs), go);
            G.e = stage_table(ar, ea.data(), G.m * sizeof(PmArgs), go);
            b->groups.push_back(std::move(G));
        }
    }
    if (ar.overflow) {
        set_error("batch workspace too small for the argument tables");
        return PXST_EWORKSPACE;
    }
    out = b;
    return PXST_OK;
}

int run_pixel_map_batch(const PmBatchImpl& b, hipStream_t s) {
    for (const PmJobDesc& d : b.solo) {
        const int rc = launch_pixel_map(d.g, d.sc, d.refv, d.sat, d.dx, d.u_in, d.win, d.u_out, nullptr,
                                        nullptr, d.ws, *d.L, s);
        if (rc) return rc;
    }
    if (b.n <= 0) return PXST_OK;
    hipLaunchKernelGGL(k_classify_batch, dim3(b.cls_grid), dim3(64), 0, s, (const PmArgs*)b.cls.args_dev,
                       b.cls.off_dev, b.n);
    hipLaunchKernelGGL(k_compact_batch, dim3(b.n), dim3(COMPACT_THREADS), 0, s,
                       (const PmArgs*)b.cls.args_dev);
    int rc = check_hip(hipGetLastError(), "batched pixel-map classification");
    if (rc) return rc;
    for (const PmGroup& G : b.groups) {
        const PmArgs* gd = (const PmArgs*)G.g.args_dev;
        if (G.mm_on & 1) {
            profile_begin("pm_fast", s);
            rc = launch_mma(G.ga.data(), G.m, gd, G.g.off_dev, G.grid, false, s);
            profile_end("pm_fast", s, 0, nullptr, 0);
            if (rc) return rc;
        } else {
            const size_t sh = lds_bytes(G.pl.lf, G.max_n);
            hipFuncSetAttribute((const void*)G.pl.fs.batch, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)sh);
            profile_begin("pm_fast", s);
            hipLaunchKernelGGL(G.pl.fs.batch, dim3(G.grid), dim3(G.pl.lf.waves * 64), sh, s,
                               (const PmArgs*)G.f.args_dev, G.f.off_dev, G.m);
            profile_end("pm_fast", s, 0, nullptr, 0);
        }
        if (G.mm_on & 2) {
            profile_begin("pm_edge_mma", s);
            rc = launch_mma(G.ga.data(), G.m, gd, G.g.off_dev, G.grid, true, s);
            profile_end("pm_edge_mma", s, 0, nullptr, 0);
            if (rc) return rc;
        }
        const size_t sh = lds_bytes(G.pl.le, G.max_n);
        hipFuncSetAttribute((const void*)G.pl.es.batch, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
        hipLaunchKernelGGL(G.pl.es.batch, dim3(G.grid), dim3(G.pl.le.waves * 64), sh, s,
                           (const PmArgs*)G.e.args_dev, G.e.off_dev, G.m);
        hipLaunchKernelGGL(k_pm_generic_batch, dim3(G.grid), dim3(256), 0, s, gd, G.g.off_dev, G.m);
        rc = check_hip(hipGetLastError(), "batched pixel-map search");
        if (rc) return rc;
    }
    return PXST_OK;
}

}  // namespace pxst

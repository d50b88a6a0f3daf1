// Reference update (Sec. 2.2.1 with the bilinear splat of Sec. 4) and the
// reference-plane error (Sec. 2.2.4).
//
// Both start from an inverted map: the good pixels are binned by floor(u) - origin
// into a cell grid by a counting sort that leaves every cell's pixels in pixel order,
// so a row of cells is a contiguous run of entries; an entry carries its pixel index,
// through which the frames are read in their own order.
//
// Reference update: a work-group owns a tile of reference pixels and, frame by frame,
// walks the rows of cells whose points can put a bilinear corner on the tile, adding
// the corners' value and weight into LDS bins with terms rounded to a power-of-two
// quantum, so that the FP64 sums are exact and independent of the order of the atomic
// additions (see k_ref_splat).
//
// Reference-plane error: every reference pixel p gathers, frame by frame, from the 3x3
// cells around p + floor(dx_n) (only those can put a corner on p), with compensated
// float32 sums over frames and float64 weight sums; frame chunks (grid z) are combined
// in chunk order, so every sum has a fixed order.
#include "pxst_device.hpp"
#include "pxst_internal.hpp"

namespace pxst {

namespace {

constexpr unsigned KEY_INVALID_OFF = 1;  // key = ncells + 1: bad pixel
constexpr unsigned KEY_OVERFLOW_OFF = 0;  // key = ncells: good pixel outside the grid

// Bounding box, sum and count of the cells of the good pixels: one partial per block
// (no atomics), then one block reduces the partials in block order.
__device__ inline int cell_coord(float u, int o) {
    float f = floorf(u);
    f = fminf(fmaxf(f, -1.0e9f), 1.0e9f);
    return (int)f - o;
}

template <bool BATCH>
__global__ __launch_bounds__(GRID_THREADS) void k_grid_bbox(const MapArgs* __restrict__ jobs, MapArgs one) {
    const MapArgs a = job_args<BATCH>(jobs, one);
    if ((int)blockIdx.x >= a.nparts) return;
    const float* __restrict__ u = a.u;
    const uint8_t* __restrict__ mask = a.mask;
    const float* __restrict__ white = a.white;
    const int HW = a.HW, o0 = a.o0, o1 = a.o1;
    GridPart* __restrict__ part = a.gpart;
    __shared__ GridPart wp[GRID_THREADS / 64];
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const bool good = k < HW && mask[k] != 0;
    int b0 = 0, b1 = 0;
    if (good) {
        b0 = cell_coord(u[k], o0);
        b1 = cell_coord(u[HW + k], o1);
    }
    GridPart g;
    g.bmin0 = wave_min_i(good ? b0 : INT_MAX);
    g.bmax0 = wave_max_i(good ? b0 : INT_MIN);
    g.bmin1 = wave_min_i(good ? b1 : INT_MAX);
    g.bmax1 = wave_max_i(good ? b1 : INT_MIN);
    g.sum0 = wave_sum<long long>(good ? (long long)b0 : 0);
    g.sum1 = wave_sum<long long>(good ? (long long)b1 : 0);
    g.n_good = wave_sum<int>(good ? 1 : 0);
    float wm = good ? fabsf(white[k]) : 0.f;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) wm = fmaxf(wm, __shfl_xor(wm, o, 64));
    g.wmax = wm;
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) wp[w] = g;
    __syncthreads();
    if (threadIdx.x == 0) {
        GridPart t = wp[0];
        for (int q = 1; q < GRID_THREADS / 64; ++q) {
            t.bmin0 = min(t.bmin0, wp[q].bmin0);
            t.bmax0 = max(t.bmax0, wp[q].bmax0);
            t.bmin1 = min(t.bmin1, wp[q].bmin1);
            t.bmax1 = max(t.bmax1, wp[q].bmax1);
            t.sum0 += wp[q].sum0;
            t.sum1 += wp[q].sum1;
            t.n_good += wp[q].n_good;
            t.wmax = fmaxf(t.wmax, wp[q].wmax);
        }
        part[blockIdx.x] = t;
    }
}

// Reduces the partials and sets the grid origin: the bounding box (plus a one-cell
// margin) when it fits the capacity, else a window of the capacity centred on the
// mean cell.
template <bool BATCH>
__global__ __launch_bounds__(GRID_THREADS) void k_grid_origin(const MapArgs* __restrict__ jobs, MapArgs one) {
    const MapArgs a = job_args<BATCH>(jobs, one);
    const GridPart* __restrict__ part = a.gpart;
    const int nparts = a.nparts, GH = a.GH, GW = a.GW;
    GridInfo* gi = a.gi;
    __shared__ GridPart wp[GRID_THREADS / 64];
    GridPart t;
    t.bmin0 = t.bmin1 = INT_MAX;
    t.bmax0 = t.bmax1 = INT_MIN;
    t.sum0 = t.sum1 = 0;
    t.n_good = 0;
    t.wmax = 0.f;
    for (int q = threadIdx.x; q < nparts; q += GRID_THREADS) {
        const GridPart p = part[q];
        t.wmax = fmaxf(t.wmax, p.wmax);
        t.bmin0 = min(t.bmin0, p.bmin0);
        t.bmax0 = max(t.bmax0, p.bmax0);
        t.bmin1 = min(t.bmin1, p.bmin1);
        t.bmax1 = max(t.bmax1, p.bmax1);
        t.sum0 += p.sum0;
        t.sum1 += p.sum1;
        t.n_good += p.n_good;
    }
    // exact operations (min, max, integer sums): the order does not change the result
    t.bmin0 = wave_min_i(t.bmin0);
    t.bmax0 = wave_max_i(t.bmax0);
    t.bmin1 = wave_min_i(t.bmin1);
    t.bmax1 = wave_max_i(t.bmax1);
    t.sum0 = wave_sum<long long>(t.sum0);
    t.sum1 = wave_sum<long long>(t.sum1);
    t.n_good = wave_sum<int>(t.n_good);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) t.wmax = fmaxf(t.wmax, __shfl_xor(t.wmax, o, 64));
    if ((threadIdx.x & 63) == 0) wp[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int q = 1; q < GRID_THREADS / 64; ++q) {
        t.bmin0 = min(t.bmin0, wp[q].bmin0);
        t.bmax0 = max(t.bmax0, wp[q].bmax0);
        t.bmin1 = min(t.bmin1, wp[q].bmin1);
        t.bmax1 = max(t.bmax1, wp[q].bmax1);
        t.sum0 += wp[q].sum0;
        t.sum1 += wp[q].sum1;
        t.n_good += wp[q].n_good;
        t.wmax = fmaxf(t.wmax, wp[q].wmax);
    }
    gi->wmax = t.wmax;
    gi->bmin0 = t.bmin0;
    gi->bmin1 = t.bmin1;
    gi->bmax0 = t.bmax0;
    gi->bmax1 = t.bmax1;
    gi->sum0 = t.sum0;
    gi->sum1 = t.sum1;
    gi->n_good = t.n_good;
    if (t.n_good == 0) {
        gi->g0 = 0;
        gi->g1 = 0;
        return;
    }
    const long long e0 = (long long)t.bmax0 - t.bmin0 + 3;
    const long long e1 = (long long)t.bmax1 - t.bmin1 + 3;
    gi->g0 = e0 <= GH ? t.bmin0 - 1 : (int)(t.sum0 / t.n_good) - GH / 2;
    gi->g1 = e1 <= GW ? t.bmin1 - 1 : (int)(t.sum1 / t.n_good) - GW / 2;
}

// The inverted map is a counting sort of the pixels by cell key (cell index in the
// grid; ncells: good pixel outside the grid; ncells + 1: bad pixel) that leaves the
// pixels of every key in pixel order, as a stable sort would.  Only the cells of the
// good pixels' bounding box (clipped to the grid) are touched:
//   counts cleared -> counts per key (integer atomics) -> per row of cells an exclusive
//   scan of its counts (cstart, one more entry for the row's end) and the row's total ->
//   one work-group scans the row totals (rstart) and sets the starts of the two other
//   keys (kstart) -> pixels of grid cells placed with atomic slot counters (which returns
//   every count to 0) -> per cell its few entries sorted by pixel index and the entries'
//   data written; good pixels outside the grid placed in pixel order by one work-group.
// The first entry of cell (r, c) is rstart[r] + cstart[r (GW + 1) + c].  Bad pixels are
// counted but not placed (no pass reads them).
__device__ inline void grid_region(const GridInfo& gi, int GH, int GW, int& r0, int& r1, int& c0, int& c1) {
    r0 = max(gi.bmin0 - gi.g0, 0);
    r1 = min(gi.bmax0 - gi.g0, GH - 1);
    c0 = max(gi.bmin1 - gi.g1, 0);
    c1 = min(gi.bmax1 - gi.g1, GW - 1);
}

// One work-group per row of cells: clears the counts of the region's cells (and the two
// other keys' counts).
template <bool BATCH>
__global__ __launch_bounds__(256) void k_count_clear(const MapArgs* __restrict__ jobs, MapArgs one) {
    const MapArgs a = job_args<BATCH>(jobs, one);
    const int GH = a.GH, GW = a.GW;
    unsigned* __restrict__ cnt = a.cnt;
    if ((int)blockIdx.x >= GH) return;
    const GridInfo gi = *a.gi;
    int r0, r1, c0, c1;
    grid_region(gi, GH, GW, r0, r1, c0, c1);
    const int r = blockIdx.x;
    if (r == 0 && threadIdx.x < 2) cnt[(size_t)GH * GW + threadIdx.x] = 0u;
    if (r < r0 || r > r1) return;
    for (int c = c0 + (int)threadIdx.x; c <= c1; c += 256) cnt[(size_t)r * GW + c] = 0u;
}

template <bool BATCH>
__global__ __launch_bounds__(256) void k_keys(const MapArgs* __restrict__ jobs, MapArgs one) {
    const MapArgs a = job_args<BATCH>(jobs, one);
    const float* __restrict__ u = a.u;
    const uint8_t* __restrict__ mask = a.mask;
    const int HW = a.HW, o0 = a.o0, o1 = a.o1, GH = a.GH, GW = a.GW;
    const GridInfo* __restrict__ gi = a.gi;
    unsigned* __restrict__ keys = a.keys;
    unsigned* __restrict__ cnt = a.cnt;
    if ((int)(blockIdx.x * blockDim.x) >= HW) return;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned ncells = (unsigned)GH * (unsigned)GW;
    unsigned key = ncells + KEY_INVALID_OFF;
    if (k < HW && mask[k]) {
        const int c0 = cell_coord(u[k], o0) - gi->g0;
        const int c1 = cell_coord(u[HW + k], o1) - gi->g1;
        key = (c0 >= 0 && c0 < GH && c1 >= 0 && c1 < GW) ? (unsigned)c0 * GW + c1
                                                          : ncells + KEY_OVERFLOW_OFF;
    }
    if (k < HW) {
        keys[k] = key;
        if (key < ncells) atomicAdd(&cnt[key], 1u);
    }
    // the two special keys: one addition per wave
    const unsigned long long mo = __ballot(k < HW && key == ncells + KEY_OVERFLOW_OFF);
    const unsigned long long mi = __ballot(k < HW && key == ncells + KEY_INVALID_OFF);
    if ((threadIdx.x & 63) == 0) {
        if (mo) atomicAdd(&cnt[ncells + KEY_OVERFLOW_OFF], (unsigned)__popcll(mo));
        if (mi) atomicAdd(&cnt[ncells + KEY_INVALID_OFF], (unsigned)__popcll(mi));
    }
}

// Inclusive scan over the 64 lanes of a wave (row_shr steps inside rows of 16, then the
// row ends broadcast to the rows above them).
__device__ inline unsigned wave_incl_scan(unsigned v) {
    const unsigned lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const unsigned t = __shfl_up(v, d, 64);
        if (lane >= (unsigned)d) v += t;
    }
    return v;
}

// Exclusive scan of a work-group's 256 values (one per thread); total returned.
__device__ inline unsigned block_excl_scan(unsigned v, unsigned* tmp4, unsigned& total) {
    const unsigned lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned inc = wave_incl_scan(v);
    if (lane == 63) tmp4[wave] = inc;
    __syncthreads();
    unsigned before = 0;
    total = 0;
#pragma unroll
    for (unsigned w = 0; w < 4; ++w) {
        before += w < wave ? tmp4[w] : 0u;
        total += tmp4[w];
    }
    __syncthreads();
    return before + inc - v;
}

// One work-group per row of cells: in-row exclusive scan of the region's counts, with
// the row's end after its last cell, and the row's total (0 outside the region).
template <bool BATCH>
__global__ __launch_bounds__(256) void k_scan_rows(const MapArgs* __restrict__ jobs, MapArgs one) {
    __shared__ unsigned tmp4[4];
    const MapArgs a = job_args<BATCH>(jobs, one);
    const int GH = a.GH, GW = a.GW;
    const unsigned* __restrict__ cnt = a.cnt;
    unsigned* __restrict__ cstart = a.cstart;
    unsigned* __restrict__ rtot = a.rtot;
    if ((int)blockIdx.x >= GH) return;
    const GridInfo gi = *a.gi;
    int r0, r1, c0, c1;
    grid_region(gi, GH, GW, r0, r1, c0, c1);
    const int r = blockIdx.x;
    if (r < r0 || r > r1) {
        if (threadIdx.x == 0) rtot[r] = 0u;
        return;
    }
    const unsigned* cr = cnt + (size_t)r * GW;
    unsigned* sr = cstart + (size_t)r * (GW + 1);
    unsigned run = 0;
    for (int cb = c0; cb <= c1; cb += 256) {
        const int c = cb + (int)threadIdx.x;
        const unsigned v = c <= c1 ? cr[c] : 0u;
        unsigned tot;
        const unsigned ex = block_excl_scan(v, tmp4, tot);
        if (c <= c1) sr[c] = run + ex;
        run += tot;
    }
    if (threadIdx.x == 0) {
        sr[c1 + 1] = run;
        rtot[r] = run;
    }
}

// One work-group: exclusive scan of the row totals into rstart[0 .. GH] and the starts
// of the other keys: kstart[0] = first entry outside the grid, kstart[1] = number of
// good pixels, kstart[2] = end.
template <bool BATCH>
__global__ __launch_bounds__(256) void k_scan_top(const MapArgs* __restrict__ jobs, MapArgs one) {
    __shared__ unsigned tmp4[4];
    const MapArgs a = job_args<BATCH>(jobs, one);
    const int GH = a.GH;
    const unsigned* __restrict__ rtot = a.rtot;
    const unsigned* __restrict__ cnt = a.cnt;
    const unsigned ncells = (unsigned)a.GH * (unsigned)a.GW;
    unsigned* __restrict__ rstart = a.rstart;
    unsigned* __restrict__ kstart = a.kstart;
    unsigned run = 0;
    for (int rb = 0; rb < GH; rb += 256) {
        const int r = rb + (int)threadIdx.x;
        const unsigned v = r < GH ? rtot[r] : 0u;
        unsigned tot;
        const unsigned ex = block_excl_scan(v, tmp4, tot);
        if (r < GH) rstart[r] = run + ex;
        run += tot;
    }
    if (threadIdx.x == 0) {
        rstart[GH] = run;
        const unsigned nov = cnt[ncells + KEY_OVERFLOW_OFF], nbad = cnt[ncells + KEY_INVALID_OFF];
        kstart[0] = run;
        kstart[1] = run + nov;
        kstart[2] = run + nov + nbad;
    }
}

__device__ inline unsigned cell_first(const unsigned* __restrict__ cstart, const unsigned* __restrict__ rstart,
                                      int GW, int r, int c) {
    return rstart[r] + cstart[(size_t)r * (GW + 1) + c];
}

// Places the pixels of grid cells: slot = remaining count - 1 (the order inside a cell
// is fixed afterwards); the counts end at 0.
template <bool BATCH>
__global__ void k_cell_scatter(const MapArgs* __restrict__ jobs, MapArgs one) {
    const MapArgs a = job_args<BATCH>(jobs, one);
    const unsigned* __restrict__ keys = a.keys;
    const int HW = a.HW, GW = a.GW;
    const unsigned ncells = (unsigned)a.GH * (unsigned)a.GW;
    const unsigned* __restrict__ cstart = a.cstart;
    const unsigned* __restrict__ rstart = a.rstart;
    unsigned* __restrict__ cnt = a.cnt;
    unsigned* __restrict__ vals = a.vals;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= HW) return;
    const unsigned key = keys[k];
    if (key < ncells) {
        const unsigned r = key / (unsigned)GW, c = key - r * (unsigned)GW;
        const unsigned slot = atomicSub(&cnt[key], 1u) - 1u;
        vals[cell_first(cstart, rstart, GW, (int)r, (int)c) + slot] = (unsigned)k;
    }
}

// Entry data: fractions of u, white-field and the cell in grid coordinates packed as
// (row << 16) | column (all 1s outside the grid; both fit 16 bits since detector and
// reference sides are at most 16384), plus the cell coordinates themselves.
__device__ inline void entry_data(const float* __restrict__ u, const float* __restrict__ white, unsigned k,
                                  int HW, int o0, int o1, const GridInfo& gi, int GH, int GW, float4& pd, int2& bs) {
    const float u0 = u[k], u1 = u[HW + k];
    const float f0 = floorf(u0), f1 = floorf(u1);
    const int b0 = cell_coord(u0, o0), b1 = cell_coord(u1, o1);
    const int r = b0 - gi.g0, c = b1 - gi.g1;
    const unsigned pack = (r >= 0 && r < GH && c >= 0 && c < GW) ? ((unsigned)r << 16) | (unsigned)c : ~0u;
    pd = make_float4(u0 - f0, u1 - f1, white[k], __uint_as_float(pack));
    bs = make_int2(b0, b1);
}

// One thread per cell of the grid (work-groups 0 .. ceil(GH GW / 256) - 1) and one more
// work-group for the good pixels outside the grid.  A region cell's thread sorts the
// cell's entries by pixel index (a cell holds one or two pixels when u maps about one
// pixel per reference pixel) and writes their data.  The last work-group places the
// pixels outside the grid in pixel order and writes theirs (nothing to do for a
// sensible map).
template <bool BATCH>
__global__ __launch_bounds__(256) void k_cell_finish(const MapArgs* __restrict__ jobs, MapArgs one) {
    __shared__ unsigned wc[4];
    const MapArgs a = job_args<BATCH>(jobs, one);
    const float* __restrict__ u = a.u;
    const float* __restrict__ white = a.white;
    const unsigned* __restrict__ keys = a.keys;
    const int HW = a.HW, o0 = a.o0, o1 = a.o1, GH = a.GH, GW = a.GW;
    const unsigned* __restrict__ cstart = a.cstart;
    const unsigned* __restrict__ rstart = a.rstart;
    const unsigned* __restrict__ kstart = a.kstart;
    unsigned* __restrict__ vals = a.vals;
    float4* __restrict__ pdata = a.pdata;
    int2* __restrict__ bsort = a.bsort;
    const int ncell = GH * GW, cblocks = (ncell + 255) / 256;
    if ((int)blockIdx.x > cblocks) return;
    const GridInfo gi = *a.gi;
    if ((int)blockIdx.x < cblocks) {
        const int q = (int)blockIdx.x * 256 + (int)threadIdx.x;
        if (q >= ncell) return;
        const int r = q / GW, c = q - r * GW;
        int r0, r1, c0, c1;
        grid_region(gi, GH, GW, r0, r1, c0, c1);
        if (r < r0 || r > r1 || c < c0 || c > c1) return;
        const unsigned b = cell_first(cstart, rstart, GW, r, c);
        const unsigned n = cell_first(cstart, rstart, GW, r, c + 1) - b;
        unsigned* v = vals + b;
        for (unsigned i = 1; i < n; ++i) {   // insertion sort of a few entries
            const unsigned x = v[i];
            unsigned j = i;
            while (j > 0 && v[j - 1] > x) {
                v[j] = v[j - 1];
                --j;
            }
            v[j] = x;
        }
        for (unsigned i = 0; i < n; ++i) entry_data(u, white, v[i], HW, o0, o1, gi, GH, GW, pdata[b + i], bsort[b + i]);
        return;
    }
    const unsigned ob = kstart[0], oe = kstart[1];
    if (oe == ob) return;
    const unsigned ncells = (unsigned)GH * (unsigned)GW;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned base = ob;
    for (int k0 = 0; k0 < HW; k0 += 256) {
        const int k = k0 + threadIdx.x;
        const bool f = k < HW && keys[k] == ncells + KEY_OVERFLOW_OFF;
        const unsigned long long m = __ballot(f);
        if (lane == 0) wc[wave] = (unsigned)__popcll(m);
        __syncthreads();
        unsigned before = 0, total = 0;
        for (int w = 0; w < 4; ++w) {
            before += w < wave ? wc[w] : 0u;
            total += wc[w];
        }
        if (f) {
            const unsigned e = base + before + (unsigned)__popcll(m & ((1ull << lane) - 1ull));
            vals[e] = (unsigned)k;
            entry_data(u, white, (unsigned)k, HW, o0, o1, gi, GH, GW, pdata[e], bsort[e]);
        }
        base += total;
        __syncthreads();
    }
}

// Bilinear weight that reference coordinate p receives from a point whose position
// along this axis is (cell - floor(dx)) + t, t = frac(u) - frac(dx) in (-1, 1).
__device__ inline float splat_weight(int p, int base, float t) {
    // floor of the point = base - (t < 0); fraction = t or t + 1
    if (t >= 0.f) {
        if (p == base) return 1.f - t;
        if (p == base + 1) return t;
        return 0.f;
    }
    if (p == base) return 1.f + t;
    if (p == base - 1) return -t;
    return 0.f;
}

struct GatherArgs {
    const uint16_t* frames;
    const float* dx;
    const float* u;           // error mode: map for the lookups of eps
    const float* refv_in;     // error mode: reference for the lookups
    const float* s2;          // error mode: sigma^2
    const unsigned* cstart;   // in-row first entries of the cells ([GH][GW + 1])
    const unsigned* rstart;   // first entry of every row of cells
    const unsigned* kstart;   // first entries of the pixels outside the grid, of the bad ones
    const float4* pdata;
    const int2* bsort;
    const unsigned* pidx;     // pixel index of each sorted entry
    const GridInfo* gi;
    int N, H, W, Rs, Rf, o0, o1, GH, GW;
    int nchunks;              // frame chunks (grid z); partials go to part when > 1
    RefPart* part;            // [nchunks][Rs * Rf]
    float* out;               // ref (or ref_err)
    double* wsum;             // weight sums (reference mode)
    float* refv_out;          // reference mode: ref with NaN for invalid (may be null)
};

// Contribution of sorted entry e in frame n to reference pixel (p0, p1): value and weight.
template <int MODE>
__device__ inline void gather_entry(const GatherArgs& a, unsigned e, int n, size_t HW, int p0, int p1,
                                    int s0, int s1, float fd0, float fd1, float& part, double& dpart) {
    const float4 pd = a.pdata[e];
    const int2 b = a.bsort[e];
    const float w0 = splat_weight(p0, b.x - s0, pd.x - fd0);
    const float w1 = splat_weight(p1, b.y - s1, pd.y - fd1);
    const float w = w0 * w1;
    if (w == 0.f) return;
    const unsigned k = a.pidx[e];
    const float I = (float)a.frames[(size_t)n * HW + k];
    if (MODE == 0) {
        const float wi = w * pd.z;
        part = fmaf(wi, I, part);
        dpart += (double)wi * (double)pd.z;
    } else {
        const float u0 = a.u[k], u1 = a.u[HW + k];
        const float f0 = floorf(u0), f1 = floorf(u1);
        const float t0 = (u0 - f0) - fd0, t1 = (u1 - f1) - fd1;
        const int a0 = (int)f0 - s0 - a.o0 - (t0 < 0.f ? 1 : 0);
        const int b0 = (int)f1 - s1 - a.o1 - (t1 < 0.f ? 1 : 0);
        const float g = masked_bilinear(a.refv_in, a.Rs, a.Rf, a0, b0, t0 < 0.f ? t0 + 1.f : t0,
                                        t1 < 0.f ? t1 + 1.f : t1);
        const float s2 = a.s2[k];
        float eps = 0.f;
        if (valid(g) && s2 > 0.f) {
            const float rr = fmaf(-pd.z, g, I);
            eps = rr * rr / s2;
        }
        part = fmaf(w, eps, part);
        dpart += (double)w;
    }
}

__device__ inline void write_reference(const GatherArgs& a, size_t p, float S, float C, double den,
                                       int mode) {
    const float num = S - C;
    const float val = den > 0.0 ? (float)((double)num / den) : 0.f;
    a.out[p] = val;
    if (mode == 0) {
        a.wsum[p] = den;
        if (a.refv_out) a.refv_out[p] = den > 0.0 ? val : qnan();
    }
}

// MODE 0: reference update (value M W I, weight M W^2).
// MODE 1: reference-plane error (value M eps, weight M).
// Grid: 16 x 16 reference pixels per work-group, frame chunk in z.
template <int MODE>
__global__ __launch_bounds__(256) void k_ref_gather(GatherArgs a) {
    const int p1 = blockIdx.x * 16 + (threadIdx.x & 15);
    const int p0 = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (p0 >= a.Rs || p1 >= a.Rf) return;
    const GridInfo gi = *a.gi;
    int gr0, gr1, gc0, gc1;
    grid_region(gi, a.GH, a.GW, gr0, gr1, gc0, gc1);
    const unsigned ov_begin = a.kstart[0], ov_end = a.kstart[1];
    const size_t HW = (size_t)a.H * a.W;
    const int F = (a.N + a.nchunks - 1) / a.nchunks;
    const int n_begin = blockIdx.z * F, n_end = min(a.N, n_begin + F);
    float S = 0.f, C = 0.f;      // compensated numerator over frames
    double den = 0.0;
    for (int n = n_begin; n < n_end; ++n) {
        const float d0 = a.dx[2 * n], d1 = a.dx[2 * n + 1];
        const float fs0 = floorf(d0), fs1 = floorf(d1);
        const float fd0 = d0 - fs0, fd1 = d1 - fs1;
        const int s0 = (int)fs0, s1 = (int)fs1;
        const int q0 = p0 + s0, q1 = p1 + s1;   // cell of a point landing on p
        if (q0 < gi.bmin0 - 1 || q0 > gi.bmax0 + 1 || q1 < gi.bmin1 - 1 || q1 > gi.bmax1 + 1)
            continue;
        float part = 0.f;
        double dpart = 0.0;
        // the three cell rows around q0; in each, the cells q1-1 .. q1+1 are contiguous
        unsigned eb[3], ee[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int r = q0 + d - 1 - gi.g0;
            const int c_lo = max(q1 - 1 - gi.g1, gc0), c_hi = min(q1 + 1 - gi.g1, gc1);
            eb[d] = ee[d] = 0;
            if (r >= gr0 && r <= gr1 && c_lo <= c_hi) {
                eb[d] = cell_first(a.cstart, a.rstart, a.GW, r, c_lo);
                ee[d] = cell_first(a.cstart, a.rstart, a.GW, r, c_hi + 1);
            }
        }
#pragma unroll
        for (int d = 0; d < 3; ++d)
            for (unsigned e = eb[d]; e < ee[d]; ++e)
                gather_entry<MODE>(a, e, n, HW, p0, p1, s0, s1, fd0, fd1, part, dpart);
        // good pixels outside the cell grid (none for a sensible map)
        for (unsigned e = ov_begin; e < ov_end; ++e)
            gather_entry<MODE>(a, e, n, HW, p0, p1, s0, s1, fd0, fd1, part, dpart);
        kahan_add(S, C, part);
        den += dpart;
    }
    const size_t p = (size_t)p0 * a.Rf + p1;
    if (a.nchunks == 1) {
        write_reference(a, p, S, C, den, MODE);
    } else {
        a.part[(size_t)blockIdx.z * ((size_t)a.Rs * a.Rf) + p] = RefPart{S, C, den};
    }
}

// Adds the frame-chunk partials of every reference pixel in chunk order.
__global__ void k_ref_combine(GatherArgs a, int mode) {
    const size_t RR = (size_t)a.Rs * a.Rf;
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= RR) return;
    float S = 0.f, C = 0.f;
    double den = 0.0;
    for (int c = 0; c < a.nchunks; ++c) {
        const RefPart q = a.part[(size_t)c * RR + p];
        kahan_add(S, C, q.s);
        kahan_add(S, C, -q.c);
        den += q.den;
    }
    write_reference(a, p, S, C, den, mode);
}

__global__ void k_prep_refv(const float* __restrict__ ref, const double* __restrict__ wsum, int n,
                            float* __restrict__ refv) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) refv[p] = wsum[p] > 0.0 ? ref[p] : qnan();
}

// Inclusive prefix sums of the invalid flags along each reference row, written
// transposed: tmp[c][r]; rowmax[r] = max |refv| over the valid pixels of row r.
template <bool BATCH>
__global__ __launch_bounds__(256) void k_sat_rows(const SatArgs* __restrict__ jobs, SatArgs one) {
    __shared__ int part[256];
    __shared__ float pmax[256 / 64];
    const SatArgs a = job_args<BATCH>(jobs, one);
    const float* __restrict__ refv = a.refv;
    const int Rs = a.Rs, Rf = a.Rf;
    int* __restrict__ tmp = a.tmp;
    float* __restrict__ rowmax = a.fscale ? a.rowmax : nullptr;
    const int r = blockIdx.x;
    if (r >= Rs) return;
    const int per = (Rf + 255) / 256;
    const int c0 = threadIdx.x * per;
    int s = 0;
    float mx = 0.f;
    for (int c = c0; c < min(c0 + per, Rf); ++c) {
        const float v = refv[(size_t)r * Rf + c];
        s += valid(v) ? 0 : 1;
        if (valid(v)) mx = fmaxf(mx, fabsf(v));
    }
    if (rowmax) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
        if ((threadIdx.x & 63) == 0) pmax[threadIdx.x >> 6] = mx;
    }
    part[threadIdx.x] = s;
    __syncthreads();
    if (rowmax && threadIdx.x == 0) {
        float m = pmax[0];
        for (int w = 1; w < 256 / 64; ++w) m = fmaxf(m, pmax[w]);
        rowmax[r] = m;
    }
    for (int off = 1; off < 256; off <<= 1) {
        const int v = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int run = threadIdx.x > 0 ? part[threadIdx.x - 1] : 0;
    for (int c = c0; c < min(c0 + per, Rf); ++c) {
        run += valid(refv[(size_t)r * Rf + c]) ? 0 : 1;
        tmp[(size_t)c * Rs + r] = run;
    }
}

// Column prefix sums of tmp[c][:] into sat[(r+1)][(c+1)] (row 0 and column 0 are 0).
template <bool BATCH>
__global__ __launch_bounds__(256) void k_sat_cols(const SatArgs* __restrict__ jobs, SatArgs one) {
    const SatArgs a = job_args<BATCH>(jobs, one);
    const int* __restrict__ tmp = a.tmp;
    const int Rs = a.Rs, Rf = a.Rf;
    int* __restrict__ sat = a.sat;
    const float* __restrict__ rowmax = a.rowmax;
    int* __restrict__ fscale = a.fscale;
    if ((int)blockIdx.x >= Rf) return;
    __shared__ int part[256];
    const int c = blockIdx.x;
    if (c == 0 && fscale) {
        // fixed-point exponent F: |refv| * 2^F < 2^21 for every valid pixel, so that a
        // bilinear value (a convex combination of pixels, weights rounded) stays well
        // inside |G| < 2^22
        __shared__ float pm[256];
        float m = 0.f;
        for (int r = threadIdx.x; r < Rs; r += 256) m = fmaxf(m, rowmax[r]);
        pm[threadIdx.x] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            float mm = 0.f;
            for (int t = 0; t < 256; ++t) mm = fmaxf(mm, pm[t]);
            int e = 0;
            if (mm > 0.f && isfinite(mm)) frexpf(mm, &e);   // mm < 2^e
            *fscale = mm > 0.f && isfinite(mm) ? min(100, max(-100, 21 - e)) : 0;
        }
        __syncthreads();
    }
    const int per = (Rs + 255) / 256;
    const int r0 = threadIdx.x * per;
    int s = 0;
    for (int r = r0; r < min(r0 + per, Rs); ++r) s += tmp[(size_t)c * Rs + r];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int v = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int run = threadIdx.x > 0 ? part[threadIdx.x - 1] : 0;
    const size_t ld = (size_t)Rf + 1;
    for (int r = r0; r < min(r0 + per, Rs); ++r) {
        run += tmp[(size_t)c * Rs + r];
        sat[(size_t)(r + 1) * ld + (c + 1)] = run;
    }
    if (c == 0) {
        for (int r = threadIdx.x; r <= Rs; r += 256) sat[(size_t)r * ld] = 0;
    }
    if (threadIdx.x == 0) sat[c + 1] = 0;
}

// ------------------------------------------------------------ reference update (splat)
//
// The reference update proper: every work-group owns a tile of RS_TR x RS_TC reference
// pixels and, frame by frame, walks the cells of the inverted map whose points can put
// a bilinear corner on the tile (rows of cells are contiguous runs of sorted entries,
// streamed 64 at a time per wave), adding each corner's value M W I w and weight
// M W^2 w into LDS bins.  The terms are rounded to integer multiples of a power-of-two quantum and
// summed as 64-bit integers.  The quantum comes from max |W| and from the number of
// terms a reference pixel can receive at most (frames x good pixels), so that no sum
// can leave the 63-bit range: terms get 43 bits when that bound allows (36 bits for a
// 512 x 512 detector with 400 frames; the rounding is 2^-bits of the largest possible
// term).  The sums are exact, so the LDS atomic additions give the same result in any
// order (bitwise reproducible).  Frame chunks (grid z) write exact partial sums that a
// second pass adds; the quotient is formed in FP64.
constexpr int RS_THREADS = 256;


// Quantum exponents: |W I| 2^fn < 2^T and W^2 2^fd < 2^T for every term (counts are at
// most 65535), T = min(43, 62 - bits(N n_good)): a sum of at most N n_good terms stays
// below 2^62.
__device__ inline void splat_scales(float wmax, int n_frames, int n_good, int& fn, int& fd) {
    int e1 = 0, e2 = 0, et = 0;
    if (wmax > 0.f && isfinite(wmax)) {
        frexp((double)wmax * 65535.0, &e1);
        frexp((double)wmax * (double)wmax, &e2);
    }
    frexp((double)n_frames * (double)(n_good > 0 ? n_good : 1), &et);
    const int T = min(43, 62 - et);
    fn = T - e1;
    fd = T - e2;
}

// The product a b rounded once to the nearest integer (ties to even), as a 64-bit two's
// complement integer, for |a b| < 2^51: the fused a b + 1.5 2^52 leaves that integer in
// the low mantissa bits of a double whose exponent stays fixed, so the difference of
// the bit patterns is the integer.
__device__ inline unsigned long long quantise(double a, double b) {
    constexpr double MAGIC = 6755399441055744.0;   // 1.5 * 2^52, bits 0x4338000000000000
    const unsigned long long x = (unsigned long long)__double_as_longlong(__fma_rn(a, b, MAGIC));
    // the low word of MAGIC's bits is zero: the subtraction only touches the high word
    const unsigned hi = (unsigned)(x >> 32) - 0x43380000u;
    return ((unsigned long long)hi << 32) | (unsigned)x;
}

// Bins of a tile with a border of 2 pixels on every side: a point of the cell block of a
// tile (cells whose points can reach the tile) has all four corners inside, so adding
// them needs no test; the border's sums are discarded.
constexpr int RS_PR = RS_TR + 4, RS_PC = RS_TC + 4;
// Cell rows of a tile's block per wave: RS_TR + 2 rows over 4 waves.
constexpr int RS_KR = (RS_TR + 2 + 3) / 4;
static_assert(RS_THREADS == 256, "four waves per tile");

// Lower corner (tile coordinates) and weights of a point along one axis: cell c minus
// the frame shift, t the fraction of u minus that of the shift, in (-1, 1).
__device__ inline void splat_axis(int c, float t, int& lo, float& wl, float& wh) {
    if (t >= 0.f) {
        lo = c;
        wl = 1.f - t;
        wh = t;
    } else {
        lo = c - 1;
        wl = -t;
        wh = 1.f + t;
    }
}

// Adds the four corners of a point of the cell block (i0 in [-1, RS_TR], j0 in
// [-1, RS_TC]); vn / vd: the quantised value and weight before the bilinear factor.
__device__ inline void splat_block(int i0, int j0, float t0, float t1, double vn, double vd,
                                   unsigned long long* bn, unsigned long long* bd) {
    int i, j;
    float wl0, wh0, wl1, wh1;
    splat_axis(i0, t0, i, wl0, wh0);
    splat_axis(j0, t1, j, wl1, wh1);
    const int b = (i + 2) * RS_PC + (j + 2);
#pragma unroll
    for (int di = 0; di < 2; ++di) {
#pragma unroll
        for (int dj = 0; dj < 2; ++dj) {
            const double w = (double)((di ? wh0 : wl0) * (dj ? wh1 : wl1));
            const int q = b + di * RS_PC + dj;
            atomicAdd(&bn[q], quantise(w, vn));
            atomicAdd(&bd[q], quantise(w, vd));
        }
    }
}

// Same for a point anywhere (good pixels outside the cell grid): corners outside the
// tile are skipped.
__device__ inline void splat_any(int i0, int j0, float t0, float t1, double vn, double vd,
                                 unsigned long long* bn, unsigned long long* bd) {
    int i, j;
    float wl0, wh0, wl1, wh1;
    splat_axis(i0, t0, i, wl0, wh0);
    splat_axis(j0, t1, j, wl1, wh1);
#pragma unroll
    for (int di = 0; di < 2; ++di) {
#pragma unroll
        for (int dj = 0; dj < 2; ++dj) {
            const int ii = i + di, jj = j + dj;
            if ((unsigned)ii < (unsigned)RS_TR && (unsigned)jj < (unsigned)RS_TC) {
                const double w = (double)((di ? wh0 : wl0) * (dj ? wh1 : wl1));
                const int q = (ii + 2) * RS_PC + (jj + 2);
                atomicAdd(&bn[q], quantise(w, vn));
                atomicAdd(&bd[q], quantise(w, vd));
            }
        }
    }
}

// Reference tile of RS_TR x RS_TC pixels, frames of one chunk (grid z).  For each frame
// whose shifted cell block meets the cells' region, wave w takes the block's cell rows
// w, w + 4, ... and each row's entries 64 at a time (a row of the block holds about
// RS_TC + 2 entries when u maps one detector pixel per reference pixel): the rows'
// entry ranges, then the first 64 entries of every row (fractions, white-field, cell,
// pixel index), then their frame values, read through the pixel index, are loaded
// together.  Everything a frame needs is read with vector loads and made uniform with
// lane reads (the frame's shift from a lane holding it, a row's range from the lane
// that loaded it), never with scalar or LDS reads: those share a wait counter with the
// LDS additions, so each frame would first wait for the previous frame's additions.
__device__ inline float lane_f(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

template <bool BATCH>
__global__ __launch_bounds__(RS_THREADS) void k_ref_splat(const SplatArgs* __restrict__ jobs, SplatArgs one) {
    constexpr int WAVES = RS_THREADS / 64;
    // value and weight sums (separate arrays: a wave's 64-bit additions to neighbouring
    // pixels then fall on neighbouring 8-byte words)
    __shared__ unsigned long long bn[RS_PR * RS_PC], bd[RS_PR * RS_PC];
    const SplatArgs a = job_args<BATCH>(jobs, one);
    // grid: x = tile column, y = tile row + tile rows x frame chunk
    if ((int)blockIdx.x >= a.tiles_x || (int)blockIdx.y >= a.tiles_y * a.nchunks) return;
    const int chunk = (int)blockIdx.y / a.tiles_y, trow = (int)blockIdx.y - chunk * a.tiles_y;
    const int P1 = blockIdx.x * RS_TC, P0 = trow * RS_TR;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    for (int i = tid; i < RS_PR * RS_PC; i += RS_THREADS) {
        bn[i] = 0ull;
        bd[i] = 0ull;
    }
    const GridInfo gi = *a.gi;
    int fn, fd;
    splat_scales(gi.wmax, a.N, gi.n_good, fn, fd);
    const double sn = ldexp(1.0, fn), sd = ldexp(1.0, fd);
    int gr0, gr1, gc0, gc1;
    grid_region(gi, a.GH, a.GW, gr0, gr1, gc0, gc1);
    const unsigned ov_begin = a.kstart[0], ov_end = a.kstart[1];
    const int F = (a.N + a.nchunks - 1) / a.nchunks;
    const int n_begin = chunk * F, n_end = min(a.N, n_begin + F);
    __syncthreads();
    float dl0 = 0.f, dl1 = 0.f;   // shift of frame (group start + lane)
    for (int n = n_begin; n < n_end; ++n) {
        const int fl = (n - n_begin) & 63;
        if (fl == 0) {
            const int m = min(n + lane, n_end - 1);
            dl0 = a.dx[2 * m];
            dl1 = a.dx[2 * m + 1];
        }
        const float d0 = lane_f(dl0, fl), d1 = lane_f(dl1, fl);
        const float fs0 = floorf(d0), fs1 = floorf(d1);
        const float fd0 = d0 - fs0, fd1 = d1 - fs1;
        const int s0 = (int)fs0, s1 = (int)fs1;
        // cells whose points can reach the tile: rows P0 - 1 + s0 .. P0 + RS_TR + s0 and
        // columns P1 - 1 + s1 .. P1 + RS_TC + s1, within the cells' region
        const int r_lo = max(P0 - 1 + s0 - gi.g0, gr0);
        const int r_hi = min(P0 + RS_TR + s0 - gi.g0, gr1);
        const int c_lo = max(P1 - 1 + s1 - gi.g1, gc0);
        const int c_hi = min(P1 + RS_TC + s1 - gi.g1, gc1);
        if (c_lo <= c_hi && r_lo + wave <= r_hi) {
            const int K0 = gi.g0 - s0 - P0, K1 = gi.g1 - s1 - P1;
            const uint16_t* __restrict__ fr = a.frames + (size_t)n * a.HW;
            // lane k < RS_KR loads the entry range of the wave's row k
            unsigned lb = 0u, le = 0u;
            {
                const int r = r_lo + wave + lane * WAVES;
                if (lane < RS_KR && r <= r_hi) {
                    const unsigned rs = a.rstart[r];
                    const unsigned* cr = a.cstart + (size_t)r * (a.GW + 1);
                    lb = rs + cr[c_lo];
                    le = rs + cr[c_hi + 1];
                }
            }
            unsigned eb[RS_KR], ee[RS_KR];
#pragma unroll
            for (int k = 0; k < RS_KR; ++k) {
                eb[k] = (unsigned)__builtin_amdgcn_readlane((int)lb, k);
                ee[k] = (unsigned)__builtin_amdgcn_readlane((int)le, k);
            }
            float4 pd[RS_KR];
            unsigned px[RS_KR];
#pragma unroll
            for (int k = 0; k < RS_KR; ++k) {
                const unsigned e = eb[k] + (unsigned)lane;
                pd[k] = make_float4(0.f, 0.f, 0.f, 0.f);
                px[k] = 0u;
                if (e < ee[k]) {
                    pd[k] = a.pdata[e];
                    px[k] = a.pidx[e];
                }
            }
            unsigned I[RS_KR];
#pragma unroll
            for (int k = 0; k < RS_KR; ++k) I[k] = eb[k] + (unsigned)lane < ee[k] ? (unsigned)fr[px[k]] : 0u;
#pragma unroll
            for (int k = 0; k < RS_KR; ++k) {
                if (eb[k] + (unsigned)lane < ee[k]) {
                    const unsigned pk = __float_as_uint(pd[k].w);
                    const double Wd = (double)pd[k].z;
                    splat_block((int)(pk >> 16) + K0, (int)(pk & 0xFFFFu) + K1, pd[k].x - fd0, pd[k].y - fd1,
                                Wd * (double)I[k] * sn, Wd * Wd * sd, bn, bd);
                }
            }
            for (int k = 0; k < RS_KR; ++k) {
                for (unsigned e0 = eb[k] + 64u; e0 < ee[k]; e0 += 64u) {
                    const unsigned e = e0 + (unsigned)lane;
                    if (e < ee[k]) {
                        const float4 q = a.pdata[e];
                        const unsigned pk = __float_as_uint(q.w);
                        const double Wd = (double)q.z;
                        splat_block((int)(pk >> 16) + K0, (int)(pk & 0xFFFFu) + K1, q.x - fd0, q.y - fd1,
                                    Wd * (double)fr[a.pidx[e]] * sn, Wd * Wd * sd, bn, bd);
                    }
                }
            }
        }
        // good pixels outside the cell grid (none for a sensible map)
        for (unsigned eo = ov_begin + tid; eo < ov_end; eo += RS_THREADS) {
            const float4 po = a.pdata[eo];
            const int2 b = a.bsort[eo];
            const double Wd = (double)po.z;
            splat_any(b.x - s0 - P0, b.y - s1 - P1, po.x - fd0, po.y - fd1,
                      Wd * (double)a.frames[(size_t)n * a.HW + a.pidx[eo]] * sn, Wd * Wd * sd, bn, bd);
        }
    }
    __syncthreads();
    const size_t RR = (size_t)a.Rs * a.Rf;
    for (int i = tid; i < RS_TR * RS_TC; i += RS_THREADS) {
        const int ti = i / RS_TC, tj = i % RS_TC;
        const int p0 = P0 + ti, p1 = P1 + tj;
        if (p0 >= a.Rs || p1 >= a.Rf) continue;
        const size_t p = (size_t)p0 * a.Rf + p1;
        const int q = (ti + 2) * RS_PC + (tj + 2);
        if (a.nchunks > 1) {
            a.part[(size_t)chunk * RR + p] = make_longlong2((long long)bn[q], (long long)bd[q]);
        } else {
            const double num = (double)(long long)bn[q] * ldexp(1.0, -fn);
            const double den = (double)(long long)bd[q] * ldexp(1.0, -fd);
            const float val = den > 0.0 ? (float)(num / den) : 0.f;
            a.ref[p] = val;
            a.wsum[p] = den;
            if (a.refv) a.refv[p] = den > 0.0 ? val : qnan();
        }
    }
}

// Reference values rounded to the nearest bfloat16 (ties to even), NaN kept.
__device__ inline float round_bf16(float x) {
    if (!(x == x) || isinf(x)) return x;
    unsigned b = __float_as_uint(x);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return __uint_as_float(b & 0xFFFF0000u);
}

__global__ void k_round_bf16(float* __restrict__ ref, float* __restrict__ refv, size_t n) {
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    ref[p] = round_bf16(ref[p]);
    if (refv) refv[p] = round_bf16(refv[p]);
}

// Adds the exact chunk partials and writes the reference.
template <bool BATCH>
__global__ void k_ref_splat_combine(const SplatArgs* __restrict__ jobs, SplatArgs one) {
    const SplatArgs a = job_args<BATCH>(jobs, one);
    const size_t RR = (size_t)a.Rs * a.Rf;
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= RR) return;
    unsigned long long sn = 0ull, sdd = 0ull;
    for (int c = 0; c < a.nchunks; ++c) {
        const longlong2 q = a.part[(size_t)c * RR + p];
        sn += (unsigned long long)q.x;
        sdd += (unsigned long long)q.y;
    }
    int fn, fd;
    splat_scales(a.gi->wmax, a.N, a.gi->n_good, fn, fd);
    const double num = (double)(long long)sn * ldexp(1.0, -fn);
    const double den = (double)(long long)sdd * ldexp(1.0, -fd);
    const float val = den > 0.0 ? (float)(num / den) : 0.f;
    a.ref[p] = val;
    a.wsum[p] = den;
    if (a.refv) a.refv[p] = den > 0.0 ? val : qnan();
}

inline unsigned grid_blocks(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

SatArgs make_sat_args(const Geom& g, float* refv, char* ws, const Layout& L) {
    SatArgs a{};
    a.refv = refv;
    a.Rs = g.Rs;
    a.Rf = g.Rf;
    a.tmp = (int*)(ws + L.sat_tmp);
    a.sat = (int*)(ws + L.sat);
    a.rowmax = (float*)(ws + L.rowmax);
    a.fscale = (int*)(ws + L.fscale);
    return a;
}

int launch_sat_jobs(const SatArgs* h, int n, const SatArgs* d, hipStream_t s) {
    int rs = 1, rf = 1;
    for (int j = 0; j < n; ++j) {
        rs = std::max(rs, h[j].Rs);
        rf = std::max(rf, h[j].Rf);
    }
    const SatArgs one = d ? SatArgs{} : h[0];
    PXST_LAUNCH_JOBS(k_sat_rows, dim3(rs, 1, n), dim3(256), 0, s, d, one);
    PXST_LAUNCH_JOBS(k_sat_cols, dim3(rf, 1, n), dim3(256), 0, s, d, one);
    return check_hip(hipGetLastError(), "prepare reference");
}

int launch_prep_reference(const Geom& g, const float* ref, const double* wsum, float* refv, int* sat,
                          int* sat_tmp, float* rowmax, int* fscale, hipStream_t s) {
    const size_t RR = g.RR();
    if (ref != nullptr)
        hipLaunchKernelGGL(k_prep_refv, dim3(grid_blocks(RR, 256)), dim3(256), 0, s, ref, wsum,
                           (int)RR, refv);
    if (sat != nullptr) {
        SatArgs a{};
        a.refv = refv;
        a.Rs = g.Rs;
        a.Rf = g.Rf;
        a.tmp = sat_tmp;
        a.sat = sat;
        a.rowmax = rowmax;
        a.fscale = fscale;
        return launch_sat_jobs(&a, 1, nullptr, s);
    }
    return check_hip(hipGetLastError(), "prepare reference");
}

// Builds the inverted map (sorted cells) of u; shared by the reference update and
// the reference-plane error.
MapArgs make_map_args(const Geom& g, const pxst_scan& sc, const float* u, char* ws, const Layout& L) {
    MapArgs a{};
    a.u = u;
    a.mask = sc.mask;
    a.white = sc.white;
    a.HW = (int)g.HW();
    a.o0 = g.o0;
    a.o1 = g.o1;
    a.GH = grid_h(g);
    a.GW = grid_w(g);
    a.nparts = (int)grid_blocks(g.HW(), GRID_THREADS);
    a.gi = (GridInfo*)(ws + L.ginfo);
    a.gpart = (GridPart*)(ws + L.gpart);
    a.keys = (unsigned*)(ws + L.keys);
    a.cnt = (unsigned*)(ws + L.ccount);
    a.vals = (unsigned*)(ws + L.vals2);
    a.cstart = (unsigned*)(ws + L.cstart);
    a.rtot = (unsigned*)(ws + L.rtot);
    a.rstart = (unsigned*)(ws + L.rstart);
    a.kstart = (unsigned*)(ws + L.kstart);
    a.pdata = (float4*)(ws + L.pdata);
    a.bsort = (int2*)(ws + L.bsort);
    return a;
}

// The inverted maps of n jobs (one launch per kernel; blocks past a job's grid return).
static int launch_maps(const MapArgs* h, int n, const MapArgs* d, hipStream_t s) {
    int parts = 1, gh = 1, hwb = 1, cb = 1;
    for (int j = 0; j < n; ++j) {
        parts = std::max(parts, h[j].nparts);
        gh = std::max(gh, h[j].GH);
        hwb = std::max(hwb, (int)grid_blocks((size_t)h[j].HW, 256));
        cb = std::max(cb, (int)grid_blocks((size_t)h[j].GH * h[j].GW, 256));
    }
    const MapArgs one = d ? MapArgs{} : h[0];
    PXST_LAUNCH_JOBS(k_grid_bbox, dim3(parts, 1, n), dim3(GRID_THREADS), 0, s, d, one);
    PXST_LAUNCH_JOBS(k_grid_origin, dim3(1, 1, n), dim3(GRID_THREADS), 0, s, d, one);
    PXST_LAUNCH_JOBS(k_count_clear, dim3(gh, 1, n), dim3(256), 0, s, d, one);
    PXST_LAUNCH_JOBS(k_keys, dim3(hwb, 1, n), dim3(256), 0, s, d, one);
    PXST_LAUNCH_JOBS(k_scan_rows, dim3(gh, 1, n), dim3(256), 0, s, d, one);
    PXST_LAUNCH_JOBS(k_scan_top, dim3(1, 1, n), dim3(256), 0, s, d, one);
    PXST_LAUNCH_JOBS(k_cell_scatter, dim3(hwb, 1, n), dim3(256), 0, s, d, one);
    PXST_LAUNCH_JOBS(k_cell_finish, dim3(cb + 1, 1, n), dim3(256), 0, s, d, one);
    return check_hip(hipGetLastError(), "inverse map");
}

// The reference-plane error and the float32 update use the same map.
static int build_inverse_map(const Geom& g, const pxst_scan& sc, const float* u, char* ws,
                             const Layout& L, hipStream_t s) {
    const MapArgs a = make_map_args(g, sc, u, ws, L);
    return launch_maps(&a, 1, nullptr, s);
}

static GatherArgs gather_args(const Geom& g, const pxst_scan& sc, const float* u, const float* dx,
                              char* ws, const Layout& L) {
    GatherArgs a{};
    a.frames = sc.frames;
    a.dx = dx;
    a.u = u;
    a.cstart = (const unsigned*)(ws + L.cstart);
    a.rstart = (const unsigned*)(ws + L.rstart);
    a.kstart = (const unsigned*)(ws + L.kstart);
    a.pdata = (const float4*)(ws + L.pdata);
    a.bsort = (const int2*)(ws + L.bsort);
    a.pidx = (const unsigned*)(ws + L.vals2);
    a.gi = (const GridInfo*)(ws + L.ginfo);
    a.N = g.N;
    a.H = g.H;
    a.W = g.W;
    a.Rs = g.Rs;
    a.Rf = g.Rf;
    a.o0 = g.o0;
    a.o1 = g.o1;
    a.GH = grid_h(g);
    a.GW = grid_w(g);
    a.nchunks = L.ref_chunks;
    a.part = (RefPart*)(ws + L.rpart);
    return a;
}

static void launch_gather(const GatherArgs& a, int mode, const Geom& g, hipStream_t s) {
    dim3 grid((g.Rf + 15) / 16, (g.Rs + 15) / 16, a.nchunks);
    if (mode == 0)
        hipLaunchKernelGGL(k_ref_gather<0>, grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_ref_gather<1>, grid, dim3(256), 0, s, a);
    if (a.nchunks > 1)
        hipLaunchKernelGGL(k_ref_combine, dim3(grid_blocks(g.RR(), 256)), dim3(256), 0, s, a, mode);
}

SplatArgs make_splat_args(const Geom& g, const pxst_scan& sc, const float* dx, float* ref, double* wsum,
                          float* refv, char* ws, const Layout& L) {
    SplatArgs a{};
    a.frames = sc.frames;
    a.dx = dx;
    a.cstart = (const unsigned*)(ws + L.cstart);
    a.rstart = (const unsigned*)(ws + L.rstart);
    a.kstart = (const unsigned*)(ws + L.kstart);
    a.pidx = (const unsigned*)(ws + L.vals2);
    a.pdata = (const float4*)(ws + L.pdata);
    a.bsort = (const int2*)(ws + L.bsort);
    a.gi = (const GridInfo*)(ws + L.ginfo);
    a.N = g.N;
    a.HW = (int)g.HW();
    a.Rs = g.Rs;
    a.Rf = g.Rf;
    a.GH = grid_h(g);
    a.GW = grid_w(g);
    a.nchunks = L.splat_chunks;
    a.tiles_x = (g.Rf + RS_TC - 1) / RS_TC;
    a.tiles_y = (g.Rs + RS_TR - 1) / RS_TR;
    a.part = (longlong2*)(ws + L.rpart);
    a.ref = ref;
    a.wsum = wsum;
    a.refv = refv;
    return a;
}

// The splat and combine of n jobs whose inverted maps are built.
static int launch_splats(const SplatArgs* hs, int n, const SplatArgs* ds, hipStream_t s) {
    for (int j = 1; j < n; ++j)
        if ((hs[j].nchunks > 1) != (hs[0].nchunks > 1)) {
            set_error("batched reference update: the jobs differ in frame chunking");
            return PXST_EINVAL;
        }
    int tx = 1, tyc = 1, rrb = 1;
    long long work = 0;
    for (int j = 0; j < n; ++j) {
        tx = std::max(tx, hs[j].tiles_x);
        tyc = std::max(tyc, hs[j].tiles_y * hs[j].nchunks);
        rrb = std::max(rrb, (int)grid_blocks((size_t)hs[j].Rs * hs[j].Rf, 256));
        work += (long long)hs[j].HW * hs[j].N;
    }
    const SplatArgs one = ds ? SplatArgs{} : hs[0];
    profile_begin("ref_gather", s);
    PXST_LAUNCH_JOBS(k_ref_splat, dim3(tx, tyc, n), dim3(RS_THREADS), 0, s, ds, one);
    if (hs[0].nchunks > 1)
        PXST_LAUNCH_JOBS(k_ref_splat_combine, dim3(rrb, 1, n), dim3(256), 0, s, ds, one);
    profile_end("ref_gather", s, work, nullptr, 0);
    return check_hip(hipGetLastError(), "reference update");
}

int launch_reference_jobs(const MapArgs* hm, const SplatArgs* hs, int n, const MapArgs* dm,
                          const SplatArgs* ds, hipStream_t s) {
    for (int j = 1; j < n; ++j)
        if ((hs[j].nchunks > 1) != (hs[0].nchunks > 1)) {
            set_error("batched reference update: the jobs differ in frame chunking");
            return PXST_EINVAL;
        }
    const int rc = launch_maps(hm, n, dm, s);
    return rc ? rc : launch_splats(hs, n, ds, s);
}

int launch_inverse_map(const Geom& g, const pxst_scan& sc, const float* u, char* ws, const Layout& L,
                       hipStream_t s) {
    return build_inverse_map(g, sc, u, ws, L, s);
}

int launch_update_reference(const Geom& g, const pxst_scan& sc, const float* u, const float* dx,
                            float* ref, double* wsum, float* refv, char* ws, const Layout& L,
                            hipStream_t s, int ref_mode, bool build_map) {
    if (ref_mode == PXST_REF_FP32) {
        int rc = build_map ? build_inverse_map(g, sc, u, ws, L, s) : PXST_OK;
        if (rc) return rc;
        GatherArgs b = gather_args(g, sc, u, dx, ws, L);
        b.out = ref;
        b.wsum = wsum;
        b.refv_out = refv;
        profile_begin("ref_gather", s);
        launch_gather(b, 0, g, s);
        profile_end("ref_gather", s, (long long)g.HW() * g.N, nullptr, 0);
        return check_hip(hipGetLastError(), "reference update (float32 gather)");
    }
    const MapArgs m = make_map_args(g, sc, u, ws, L);
    const SplatArgs a = make_splat_args(g, sc, dx, ref, wsum, refv, ws, L);
    int rc = build_map ? launch_reference_jobs(&m, &a, 1, nullptr, nullptr, s) : launch_splats(&a, 1, nullptr, s);
    if (rc || ref_mode != PXST_REF_BF16) return rc;
    return launch_round_bf16(g, ref, refv, s);
}

int launch_round_bf16(const Geom& g, float* ref, float* refv, hipStream_t s) {
    hipLaunchKernelGGL(k_round_bf16, dim3(grid_blocks(g.RR(), 256)), dim3(256), 0, s, ref, refv, g.RR());
    return check_hip(hipGetLastError(), "reference update (bfloat16)");
}

int launch_reference_error(const Geom& g, const pxst_scan& sc, const float* u, const float* dx,
                           const float* refv, float* ref_err, char* ws, const Layout& L,
                           hipStream_t s) {
    int rc = build_inverse_map(g, sc, u, ws, L, s);
    if (rc) return rc;
    GatherArgs a = gather_args(g, sc, u, dx, ws, L);
    a.refv_in = refv;
    a.s2 = (const float*)(ws + L.s2);
    a.out = ref_err;
    launch_gather(a, 1, g, s);
    return check_hip(hipGetLastError(), "reference-plane error");
}

}  // namespace pxst

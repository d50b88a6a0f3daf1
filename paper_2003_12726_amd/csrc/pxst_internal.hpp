// Internal declarations shared by the libpxst host code and kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <memory>
#include <vector>

#include "../../include/pxst.h"

namespace pxst {

// ----------------------------------------------------------------------------- geometry
struct Geom {
    int N, H, W, Rs, Rf, o0, o1;
    size_t HW() const { return (size_t)H * (size_t)W; }
    size_t RR() const { return (size_t)Rs * (size_t)Rf; }
};

inline Geom geom_of(const pxst_geom& g) {
    return Geom{g.n_frames, g.det_ss, g.det_fs, g.ref_ss, g.ref_fs, g.org_ss, g.org_fs};
}

// Pixel-map tiles are 8 x 8 detector pixels.
constexpr int TILE = 8;
// Staging budget of one LDS buffer of the pixel-map search (floats); two are used.
constexpr int PM_STAGE_FLOATS = 7936;
// Pixel-map search on the matrix cores: frames per K-block of the int8 products.
constexpr int MM_KB = 64;
// Packed frames of one tile and K-block: 4 row groups x 2 bytes x 64 lanes x 16 bytes.
constexpr size_t MM_PACK_BYTES = 4 * 2 * 64 * 16;
// Translation partial sums: detector pixels per work-group.
constexpr int TR_TILE = 64;          // translation search: 64 x 64 detector pixels per work-group
constexpr int TR_LDS_FLOATS = 8192;  // its staged reference region (32 KB)
constexpr int TR_THREADS = 256;
constexpr int TR_CT_MAX = (2 * PXST_MAX_TR_RADIUS + 1) * (2 * PXST_MAX_TR_RADIUS + 1);
// Error evaluation: pixels per work-group.
constexpr int ERR_THREADS = 256;

// Inverse-map (reference gather) cell grid: capacity per axis.
inline int grid_h(const Geom& g) { return 2 * (g.H > g.Rs ? g.H : g.Rs) + 8; }
inline int grid_w(const Geom& g) { return 2 * (g.W > g.Rf ? g.W : g.Rf) + 8; }

// Grid information computed on the device before the gather.
struct GridInfo {
    int bmin0, bmin1, bmax0, bmax1;   // bounding box of floor(u) - origin over good pixels
    int g0, g1;                       // cell-grid origin
    int n_good;
    float wmax;                       // max |W| over good pixels (fixed-point scale of the splat)
    long long sum0, sum1;             // sums of the cell coordinates (for a centred origin)
};

// Per-block partial of the bounding-box reduction.
struct GridPart {
    int bmin0, bmin1, bmax0, bmax1, n_good;
    float wmax;
    long long sum0, sum1;
};
constexpr int GRID_THREADS = 256;
// Reference gather: partial results of at most this many (pixel, frame-chunk) pairs.
constexpr size_t REF_PART_MAX = (size_t)8 << 20;

// Reference tiles of the splat (rows x columns of reference pixels per work-group), and
// the work-groups its frame chunks aim at: 3.5 times the 2048 resident at once (8 per
// CU) -- about half of a reference's tiles receive points, and finer chunks cost more
// partial sums to add.
constexpr int RS_TR = 16, RS_TC = 56;
constexpr size_t SPLAT_GROUPS = 7168;

struct RefPart {
    float s, c;     // compensated float32 numerator of the chunk
    double den;     // float64 weight sum of the chunk
};

// Workspace layout: every section at a 256-byte aligned offset.
struct Layout {
    // common
    size_t refv, refv2, sat, sat_tmp, s2;   // refv2: the solve loop's second reference copy
    // reference update
    size_t ginfo, gpart, keys, ccount, vals2, cstart, rtot, rstart, kstart, pdata, bsort, rpart;
    int ref_chunks;   // frame chunks of the reference gather
    int splat_chunks; // frame chunks of the reference tile splat
    // pixel map
    size_t tiles, lists, counters, tinfo;
    size_t ipk, pstat;        // frames packed as int8 matrix operands; per-pixel frame sums
    size_t rowmax, fscale;    // per-row max |reference| and the fixed-point exponent
    int kblocks;              // frame K-blocks of the packed frames
    // the search's B operand planes per reference position, their column sums, the
    // row spans they cover and the lookups' validity bits (when planes_on: 3 Rs Rf NP
    // bytes within PLANES_MAX)
    bool planes_on;
    size_t planes, pcs, pgu, prow, pvb;
    // translations
    size_t tr_part, tr_bbox;
    // error
    size_t err_part, err_pix;
    // pixel-map regularisation: filter weights and pass buffer; DCT matrices and two
    // [H][W] float64 buffers of the integration (only when integ)
    size_t gw, gtmp;
    // fractional-step search: shifted translations, one class's result, the best so far
    size_t frac_dx, frac_u, frac_e, frac_k, frac_be, frac_bk;
    // defocus sweep: a candidate's map, reference, weights and contrast partials
    size_t sweep_u, sweep_ref, sweep_w, sweep_part;
    bool integ;
    size_t ibuf0, ibuf1;
    size_t total;
};

// Largest precomputed operand planes (3 Rs Rf x padded frames bytes).
constexpr size_t PLANES_MAX = (size_t)2 << 30;
// Work-groups of the contrast reduction of the defocus sweep.
constexpr int SWEEP_BLOCKS = 256;
// Largest filter radius (|k| <= int(4 sigma + 0.5)) of the pixel-map regularisation.
constexpr int GF_MAXR = 256;

Layout make_layout(const Geom& g, int tr_ct, bool integ = false);

// Tile descriptor of the pixel-map search.
struct TileDesc {
    int cmin0, cmin1, rh, rw;
};

// Counters written by the tile classification.
// CNT_MM_POS: region positions (padded to 16) of the interior tiles, the column count of
// the matrix-core search's products.
// CNT_EDGE_MM: tiles with a few frames of invalid lookups, searched on the matrix cores
// (list 3).
enum { CNT_FAST = 0, CNT_EDGE = 1, CNT_GENERIC = 2, CNT_NONE = 3, CNT_GOOD_FAST = 4,
       CNT_GOOD_EDGE = 5, CNT_GOOD_GENERIC = 6, CNT_MM_POS = 7, CNT_EDGE_MM = 8,
       CNT_GOOD_EDGE_MM = 9, CNT_MM_POS_EDGE = 10, CNT_N = 12 };
constexpr int LIST_EDGE_MM = 3;
// Frames with invalid lookups that a matrix-core edge tile may have: chosen per job
// to fill the LDS, a multiple of 32 between these bounds.
constexpr int MM_SLOW_MIN = 32, MM_SLOW_CAP = 256;

// Round up to a multiple of a such that the row pitch is 8 (mod 32) floats: an 8-wide
// row of lanes then spans distinct LDS banks in each half-wave.
__host__ __device__ inline int lds_pitch(int rw) { return rw + ((8 - (rw & 31)) + 32) % 32; }

// ------------------------------------------------------------------------- host helpers
void set_error(const char* fmt, ...);
int check_hip(hipError_t e, const char* what);
void profile_begin(const char* family, hipStream_t s);
// work: literal work units, or (when dev_count is given) *dev_count * scale read after
// the launch (profiling synchronises anyway).
void profile_end(const char* family, hipStream_t s, long long work, const int* dev_count,
                 long long scale);
bool profiling();
// One asynchronous copy of n device counters for the spans of one call (id, or -1 when
// profiling is off or the copy could not be made); profile_end_snap then takes its work
// count from entry index of that copy (or, for id -1, copies dev_count itself).
int profile_snapshot(const int* dev_counters, int n, hipStream_t s);
void profile_end_snap(const char* family, hipStream_t s, int snap, int index, const int* dev_count,
                      long long scale);

// ------------------------------------------------------------------- batched launches
// Argument tables of a batched launch live in the caller's batch workspace; they are
// written into a pinned host buffer owned by the library and copied with
// hipMemcpyAsync on the launch stream just before the launch that reads them.
// Launches the batched form (job table `dev` in device memory, job index blockIdx.z) or
// the single-job form (arguments `one` by value) of a kernel templated on <bool BATCH>.
#define PXST_LAUNCH_JOBS(K, grid, block, sh, s, dev, one)                \
    do {                                                                  \
        if (dev)                                                          \
            K<true><<<(grid), (block), (sh), (s)>>>((dev), (one));        \
        else                                                              \
            K<false><<<(grid), (block), (sh), (s)>>>((dev), (one));       \
    } while (0)

struct BatchArena {
    char* host = nullptr;       // pinned staging memory
    char* dev = nullptr;        // batch workspace
    size_t cap = 0, used = 0;
    size_t flushed = 0;         // bytes already copied to the device
    hipStream_t stream = nullptr;
    bool overflow = false;
};
struct BatchUpload {
    const void* args_dev = nullptr;
    const int* off_dev = nullptr;
};
// Places `bytes` of arguments and the item offsets (njobs + 1 ints) in the staging
// memory and returns where they will be on the device; flush_tables copies everything
// staged since the last flush in one transfer, before the launches that read it.
BatchUpload stage_table(BatchArena& ar, const void* args, size_t bytes, const std::vector<int>& off);
// As stage_table, without offsets; returns the device address (null on overflow).
const void* stage_raw(BatchArena& ar, const void* args, size_t bytes);
int flush_tables(BatchArena& ar);
// One job of a batched pixel-map search.
struct PmJobDesc {
    Geom g;
    pxst_scan sc;
    const float* refv;
    const int* sat;
    const float* dx;
    const float* u_in;
    float* u_out;
    pxst_window win;
    char* ws;
    const Layout* L;
};

// ------------------------------------------------------------------------ kernel entry
// Each returns PXST_OK or a negative code (and sets the message).

// Arguments of the kernels that build a job's inverted map (cell sort of the pixels).
struct MapArgs {
    const float* u;
    const uint8_t* mask;
    const float* white;
    int HW, o0, o1, GH, GW, nparts;
    GridInfo* gi;
    GridPart* gpart;
    unsigned* keys;
    unsigned* cnt;
    unsigned* vals;
    unsigned* cstart;
    unsigned* rtot;
    unsigned* rstart;
    unsigned* kstart;
    float4* pdata;
    int2* bsort;
};
// Arguments of the reference splat of one job.
struct SplatArgs {
    const uint16_t* frames;
    const float* dx;
    const unsigned* cstart;
    const unsigned* rstart;
    const unsigned* kstart;
    const unsigned* pidx;     // pixel index of each entry
    const float4* pdata;
    const int2* bsort;
    const GridInfo* gi;
    int N, HW, Rs, Rf, GH, GW, nchunks;
    int tiles_x, tiles_y;     // reference tiles of the splat
    longlong2* part;   // [nchunks][Rs * Rf] quantised (numerator, weight) sums
    float* ref;
    double* wsum;
    float* refv;
};
// Arguments of the summed-area table of invalid reference pixels (and the fixed-point
// exponent of the matrix-core search) of one job.
struct SatArgs {
    const float* refv;
    int Rs, Rf;
    int* tmp;
    int* sat;
    float* rowmax;
    int* fscale;
};
MapArgs make_map_args(const Geom& g, const pxst_scan& sc, const float* u, char* ws, const Layout& L);
SplatArgs make_splat_args(const Geom& g, const pxst_scan& sc, const float* dx, float* ref, double* wsum,
                          float* refv, char* ws, const Layout& L);
SatArgs make_sat_args(const Geom& g, float* refv, char* ws, const Layout& L);
// The reference update (exact arithmetic) of n jobs: inverted maps, splat, combine; one
// launch per kernel covers all of them when the tables are in device memory (dev*
// non-null), else one job by value.
int launch_reference_jobs(const MapArgs* hm, const SplatArgs* hs, int n, const MapArgs* dm,
                          const SplatArgs* ds, hipStream_t s);
// bfloat16 storage of an exact reference update: ref and refv rounded in place.
int launch_round_bf16(const Geom& g, float* ref, float* refv, hipStream_t s);
// The summed-area tables and fixed-point exponents of n jobs.
int launch_sat_jobs(const SatArgs* h, int n, const SatArgs* d, hipStream_t s);
// refv = reference with NaN where the weight sum is 0; when sat is given also the
// summed-area table of invalid pixels and, from the per-row maxima of |refv|, the
// exponent F of the fixed-point reference used by the matrix-core search.
int launch_prep_reference(const Geom& g, const float* ref, const double* wsum, float* refv,
                          int* sat, int* sat_tmp, float* rowmax, int* fscale, hipStream_t s);

// Job setup of the matrix-core pixel-map search (depends on the frames only): frames
// packed as biased int8 operands per tile and K-block, and per-pixel frame sums.
int launch_pm_setup(const Geom& g, const pxst_scan& sc, char* ws, const Layout& L, hipStream_t s);

// Reference update (splat as a deterministic gather over the inverted map).
// build_map = false: the inverted map of u is already in the workspace (launch_inverse_map).
int launch_update_reference(const Geom& g, const pxst_scan& sc, const float* u, const float* dx,
                            float* ref, double* wsum, float* refv, char* ws, const Layout& L,
                            hipStream_t s, int ref_mode = PXST_REF_EXACT, bool build_map = true);
// The inverted map of u (the reference update's first part, independent of the shifts).
int launch_inverse_map(const Geom& g, const pxst_scan& sc, const float* u, char* ws, const Layout& L,
                       hipStream_t s);

// Reference-plane error: ref_err = sum w M eps / sum w M (needs sigma2 in ws s2).
int launch_reference_error(const Geom& g, const pxst_scan& sc, const float* u, const float* dx,
                           const float* refv, float* ref_err, char* ws, const Layout& L,
                           hipStream_t s);

// Pixel-map search.
// With `half` non-null, the split-half search: only the (frame, pixel) terms whose
// half[n][pixel] equals hval count.
int launch_pixel_map(const Geom& g, const pxst_scan& sc, const float* refv, const int* sat,
                     const float* dx, const float* u_in, const pxst_window& win, float* u_out,
                     float* err_min, int32_t* argmin, char* ws, const Layout& L, hipStream_t s,
                     const uint8_t* half = nullptr, int hval = 0);

// Batched pixel-map search in two phases: argument tables staged (host only; copied by
// flush_tables), then the launches.  Jobs large enough to fill the device are searched
// in launches of their own.
struct PmBatchImpl;
int stage_pixel_map_batch(const PmJobDesc* jobs, int n, BatchArena& ar, std::shared_ptr<PmBatchImpl>& out);
int run_pixel_map_batch(const PmBatchImpl& b, hipStream_t s);
// Upper bound of the table bytes stage_pixel_map_batch takes for n jobs.
size_t pixel_map_batch_table_bytes(int n);

// Translation search.
// Arguments of the translation search of one job.
struct TrArgs {
    const uint16_t* frames;
    const float* white;
    const uint8_t* mask;
    const float* refv;
    const float* u;
    const float* dx_in;
    float* dx_out;
    float* err_out;
    int* arg_out;
    float* part;      // [N][nblk][Ct][3]: error, variance, a positive value when any lookup was valid
    int4* bbox;       // [nblk]: min / max of floor(u0), min / max of floor(u1) over good pixels
    int N, H, W, Rs, Rf, o0, o1;
    int nblk, tiles_x, refine;
    int tx, ty;       // window radii (the kernels are compiled per window)
};

TrArgs make_tr_args(const Geom& g, const pxst_scan& sc, const float* refv, const float* u, const float* dx_in,
                    const pxst_window& win, float* dx_out, float* err_min, int32_t* argmin, char* ws,
                    const Layout& L);
// The translation search of n jobs with the same window (device table as for the error).
int launch_translations_jobs(const TrArgs* host, int n, const TrArgs* dev, hipStream_t s);
int launch_translations(const Geom& g, const pxst_scan& sc, const float* refv, const float* u,
                        const float* dx_in, const pxst_window& win, float* dx_out,
                        float* err_min, int32_t* argmin, char* ws, const Layout& L,
                        hipStream_t s);

// sigma2[i, j] = (1/N) sum M (I - W)^2 into ws s2.
// Pixel-map regularisation: filter (sigma > 0), then the irrotational constraint
// (integrate != 0; the layout must hold the integration buffers).  u_out may be u_in.
int launch_regularise(const Geom& g, const float* u_in, float* u_out, float sigma, int integrate, char* ws,
                      const Layout& L, hipStream_t s);
// Fractional-step pixel-map search: steps^2 integer searches with shifted translations,
// combined per pixel (no paraboloid).  u_out may be u_in.
int launch_pixel_map_fractional(const Geom& g, const pxst_scan& sc, const float* refv, const int* sat,
                                const float* dx, const float* u_in, const pxst_window& win, int steps,
                                float* u_out, float* err_min, int32_t* argmin, char* ws, const Layout& L,
                                hipStream_t s);
// Split-half analysis: two pixel-map searches, one per half of the (frame, pixel) terms,
// and the histogram of their differences (hist may be null).
int launch_split_half(const Geom& g, const pxst_scan& sc, const float* refv, const int* sat, const float* dx,
                      const float* u_in, const pxst_window& win, const uint8_t* half, float* u_a, float* u_b,
                      double hist_range, int nbins, int32_t* hist, char* ws, const Layout& L, hipStream_t s);
// Defocus sweep: reference update and contrast for every candidate scale pair (scales
// in host memory), first maximum into best (may be null).
int launch_defocus_sweep(const Geom& g, const pxst_scan& sc, const float* dx, const float* scales, int n_cand,
                         double c0, double c1, double* contrast, int32_t* best, char* ws, const Layout& L,
                         hipStream_t s);
int launch_sigma2(const Geom& g, const pxst_scan& sc, float* s2, hipStream_t s);

// Figures of merit.
// Arguments of the error passes of one job.
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

ErrArgs make_err_args(const Geom& g, const pxst_scan& sc, const float* refv, const float* s2, const float* u,
                      const float* dx, float* pixel_err, double* frame_err, double* total, char* ws,
                      const Layout& L);
// The error passes of n jobs (arguments in host memory and, when dev is non-null, the
// same table in device memory: then one launch per pass covers all of them).
int launch_error_jobs(const ErrArgs* host, int n, const ErrArgs* dev, hipStream_t s);
int launch_error(const Geom& g, const pxst_scan& sc, const float* refv, const float* s2,
                 const float* u, const float* dx, float* pixel_err, double* frame_err,
                 double* total, char* ws, const Layout& L, hipStream_t s);

}  // namespace pxst

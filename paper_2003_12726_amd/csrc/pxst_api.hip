// C entry points of libpxst: argument validation, workspace layout, the main loop
// and kernel timing.  Kernels live in the other translation units.
#include <cstdarg>
#include <cstdio>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "pxst_internal.hpp"

namespace pxst {


// ---------------------------------------------------------------------------- errors
static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int check_hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return PXST_OK;
    set_error("%s: %s", what, hipGetErrorString(e));
    return PXST_EHIP;
}

// -------------------------------------------------------------------------- profiling
namespace {
struct Span {
    hipEvent_t a, b;
    long long work;
    int* pinned;        // device counter copied here asynchronously (or null)
    long long scale;
    int snap;           // counter snapshot pinned points into (or -1: its own copy)
};
// Pinned copies of a block of device counters, shared by the spans that read them and
// reused once every such span has been read.
constexpr int SNAP_INTS = 64;
struct Snap {
    int* host = nullptr;
    int refs = 0;
    bool busy = false;
};
std::vector<Snap> g_snaps;
struct Family {
    std::vector<Span> spans;
    std::vector<hipEvent_t> pool;
    std::vector<int*> pinned_pool;
    hipEvent_t open = nullptr;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::map<std::string, Family> g_prof;
// families that record (all when g_prof_all); a restricted selection takes no device
// work counters
bool g_prof_all = true;
std::vector<std::string> g_prof_sel;

bool selected(const char* family) {
    if (g_prof_all) return true;
    for (const std::string& s : g_prof_sel)
        if (s == family) return true;
    return false;
}

hipEvent_t take_event(Family& f) {
    if (!f.pool.empty()) {
        hipEvent_t e = f.pool.back();
        f.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

int* take_pinned(Family& f) {
    if (!f.pinned_pool.empty()) {
        int* p = f.pinned_pool.back();
        f.pinned_pool.pop_back();
        return p;
    }
    void* p = nullptr;
    if (hipHostMalloc(&p, sizeof(int), hipHostMallocDefault) != hipSuccess) return nullptr;
    return (int*)p;
}
}  // namespace

bool profiling() { return g_prof_on; }

int profile_snapshot(const int* dev_counters, int n, hipStream_t s) {
    if (!g_prof_on || n <= 0 || n > SNAP_INTS) return -1;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_all) return -1;
    int id = -1;
    for (size_t i = 0; i < g_snaps.size(); ++i)
        if (!g_snaps[i].busy) {
            id = (int)i;
            break;
        }
    if (id < 0) {
        void* p = nullptr;
        if (hipHostMalloc(&p, SNAP_INTS * sizeof(int), hipHostMallocDefault) != hipSuccess) return -1;
        g_snaps.push_back(Snap{(int*)p, 0, false});
        id = (int)g_snaps.size() - 1;
    }
    Snap& sn = g_snaps[id];
    if (hipMemcpyAsync(sn.host, dev_counters, (size_t)n * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess)
        return -1;
    sn.busy = true;
    sn.refs = 0;
    return id;
}

void profile_end_snap(const char* family, hipStream_t s, int snap, int index, const int* dev_count,
                      long long scale) {
    if (!g_prof_on) return;
    if (snap < 0) {
        profile_end(family, s, 0, dev_count, scale);
        return;
    }
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!selected(family)) return;
    Family& f = g_prof[family];
    if (!f.open) return;
    hipEvent_t b = take_event(f);
    if (!b) return;
    hipEventRecord(b, s);
    g_snaps[snap].refs += 1;
    f.spans.push_back(Span{f.open, b, 0, g_snaps[snap].host + index, scale, snap});
    f.open = nullptr;
}

void profile_begin(const char* family, hipStream_t s) {
    if (!g_prof_on) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!selected(family)) return;
    Family& f = g_prof[family];
    f.open = take_event(f);
    if (f.open) hipEventRecord(f.open, s);
}

// Records the end event; a device work counter is copied asynchronously into pinned
// host memory (read when the family is read), so timing adds no synchronisation.
void profile_end(const char* family, hipStream_t s, long long work, const int* dev_count,
                 long long scale) {
    if (!g_prof_on) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!selected(family)) return;
    Family& f = g_prof[family];
    if (!f.open) return;
    hipEvent_t b = take_event(f);
    if (!b) return;
    hipEventRecord(b, s);
    int* pin = nullptr;
    if (dev_count && g_prof_all) {
        pin = take_pinned(f);
        if (pin) hipMemcpyAsync(pin, dev_count, sizeof(int), hipMemcpyDeviceToHost, s);
    }
    f.spans.push_back(Span{f.open, b, work, pin, scale, -1});
    f.open = nullptr;
}

// -------------------------------------------------------------------- batch staging
namespace {
std::mutex g_batch_mu;
char* g_batch_host = nullptr;      // pinned staging buffer of argument tables
size_t g_batch_cap = 0;
hipEvent_t g_batch_done = nullptr; // recorded after the last batch's table copies
}  // namespace

static size_t align256(size_t x);

BatchUpload stage_table(BatchArena& ar, const void* args, size_t bytes, const std::vector<int>& off) {
    const size_t a_bytes = align256(bytes), o_bytes = align256(off.size() * sizeof(int));
    if (ar.overflow || ar.used + a_bytes + o_bytes > ar.cap) {
        ar.overflow = true;
        return BatchUpload{};
    }
    char* h = ar.host + ar.used;
    char* d = ar.dev + ar.used;
    std::memcpy(h, args, bytes);
    std::memcpy(h + a_bytes, off.data(), off.size() * sizeof(int));
    ar.used += a_bytes + o_bytes;
    return BatchUpload{d, (const int*)(d + a_bytes)};
}

const void* stage_raw(BatchArena& ar, const void* args, size_t bytes) {
    const size_t a_bytes = align256(bytes);
    if (ar.overflow || ar.used + a_bytes > ar.cap) {
        ar.overflow = true;
        return nullptr;
    }
    std::memcpy(ar.host + ar.used, args, bytes);
    const void* d = ar.dev + ar.used;
    ar.used += a_bytes;
    return d;
}

int flush_tables(BatchArena& ar) {
    hipError_t e = hipSuccess;
    if (ar.used > ar.flushed)
        e = hipMemcpyAsync(ar.dev + ar.flushed, ar.host + ar.flushed, ar.used - ar.flushed,
                           hipMemcpyHostToDevice, ar.stream);
    ar.flushed = ar.used;
    return check_hip(e, "argument table copy");
}

// --------------------------------------------------------------------------- layout
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

Layout make_layout(const Geom& g, int tr_ct, bool integ) {
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + (bytes ? bytes : 1));
        return o;
    };
    const size_t HW = g.HW(), RR = g.RR();
    L.refv = take(RR * sizeof(float));
    L.refv2 = take(RR * sizeof(float));
    L.sat = take((size_t)(g.Rs + 1) * (g.Rf + 1) * sizeof(int));
    L.sat_tmp = take(RR * sizeof(int));
    L.s2 = take(HW * sizeof(float));
    L.ginfo = take(sizeof(GridInfo));
    L.gpart = take(((HW + GRID_THREADS - 1) / GRID_THREADS) * sizeof(GridPart));
    L.keys = take(HW * 4);
    L.vals2 = take(HW * 4);
    const size_t ncells = (size_t)grid_h(g) * (size_t)grid_w(g);
    L.ccount = take((ncells + 2) * 4);
    L.cstart = take((size_t)grid_h(g) * (grid_w(g) + 1) * 4);
    L.rtot = take((size_t)grid_h(g) * 4);
    L.rstart = take(((size_t)grid_h(g) + 1) * 4);
    L.kstart = take(4 * 4);
    L.pdata = take(HW * 16);
    L.bsort = take(HW * 8);
    {
        // frame chunks of the reference gather: enough (pixel, chunk) work items to fill
        // the device, bounded by the partial-result buffer
        const size_t RRs = RR > 0 ? RR : 1;
        size_t chunks = (size_t)(4u << 20) / RRs;
        if (chunks > REF_PART_MAX / RRs) chunks = REF_PART_MAX / RRs;
        if (chunks > (size_t)g.N) chunks = (size_t)g.N;
        if (chunks < 1) chunks = 1;
        L.ref_chunks = (int)chunks;
        // frame chunks of the tile splat (its partial sums share the buffer)
        const size_t stiles = (size_t)((g.Rs + RS_TR - 1) / RS_TR) * (size_t)((g.Rf + RS_TC - 1) / RS_TC);
        size_t sch = (SPLAT_GROUPS + stiles - 1) / (stiles > 0 ? stiles : 1);
        if (sch > REF_PART_MAX / RRs) sch = REF_PART_MAX / RRs;
        if (sch > (size_t)g.N) sch = (size_t)g.N;
        if (sch < 1) sch = 1;
        L.splat_chunks = (int)sch;
        const size_t pch = chunks > sch ? chunks : sch;
        static_assert(sizeof(RefPart) == sizeof(longlong2), "one partial buffer for both updates");
        L.rpart = take(pch > 1 ? pch * RRs * sizeof(RefPart) : 1);
    }
    const size_t ntiles = (size_t)((g.H + TILE - 1) / TILE) * ((g.W + TILE - 1) / TILE);
    L.tiles = take(ntiles * sizeof(TileDesc));
    L.lists = take(4 * ntiles * sizeof(int));
    L.tinfo = take(ntiles * 4 * sizeof(int));
    L.counters = take(CNT_N * sizeof(int));
    L.kblocks = (g.N + MM_KB - 1) / MM_KB;
    L.ipk = take(ntiles * (size_t)L.kblocks * MM_PACK_BYTES);
    L.pstat = take(ntiles * 64 * 4 * sizeof(double));
    {
        const size_t pb = 3 * RR * (size_t)L.kblocks * MM_KB;
        L.planes_on = pb <= PLANES_MAX;
        if (L.planes_on) {
            L.planes = take(pb);
            L.pcs = take(RR * sizeof(double));
            L.pgu = take(RR * sizeof(double));
            L.prow = take((size_t)g.Rs * 2 * sizeof(int));
            L.pvb = take(RR * (size_t)L.kblocks * 4 * sizeof(unsigned));
        }
    }
    L.rowmax = take((size_t)g.Rs * sizeof(float));
    L.fscale = take(sizeof(int));
    const size_t nblk_tr = (size_t)((g.H + TR_TILE - 1) / TR_TILE) * ((g.W + TR_TILE - 1) / TR_TILE);
    L.tr_part = take((size_t)g.N * nblk_tr * (tr_ct > 0 ? tr_ct : 1) * 3 * sizeof(float));
    L.tr_bbox = take(nblk_tr * 4 * sizeof(int));
    const size_t per_err = (size_t)ERR_THREADS;
    const size_t nblk_err = (HW + per_err - 1) / per_err;
    L.err_part = take((size_t)g.N * nblk_err * sizeof(double));
    L.err_pix = take((size_t)g.N * sizeof(double) + sizeof(double));
    L.frac_dx = take((size_t)g.N * 2 * sizeof(float));
    L.frac_u = take(2 * HW * sizeof(float));
    L.frac_e = take(HW * sizeof(float));
    L.frac_k = take(HW * sizeof(int));
    L.frac_be = take(HW * sizeof(float));
    L.frac_bk = take(HW * sizeof(int));
    L.sweep_u = take(2 * HW * sizeof(float));
    L.sweep_ref = take(RR * sizeof(float));
    L.sweep_w = take(RR * sizeof(double));
    L.sweep_part = take(3 * SWEEP_BLOCKS * sizeof(double));
    L.gw = take((2 * GF_MAXR + 1) * sizeof(double));
    L.gtmp = take(2 * HW * sizeof(double));
    // the integration buffers come last: a workspace laid out with them also serves
    // every call that does not integrate
    L.integ = integ;
    if (integ) {
        L.ibuf0 = take(HW * sizeof(double));
        L.ibuf1 = take(HW * sizeof(double));
    }
    L.total = off;
    return L;
}

// ------------------------------------------------------------------------ validation
static bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

static int check_geom(const pxst_geom* g) {
    if (!g) {
        set_error("geometry is null");
        return PXST_EINVAL;
    }
    if (g->n_frames < 1 || g->det_ss < 1 || g->det_fs < 1 || g->ref_ss < 1 || g->ref_fs < 1) {
        set_error("sizes must be positive (N=%d H=%d W=%d Rs=%d Rf=%d)", g->n_frames, g->det_ss,
                  g->det_fs, g->ref_ss, g->ref_fs);
        return PXST_EINVAL;
    }
    if ((long long)g->det_ss * g->det_fs >= (1LL << 24) || g->det_ss > 16384 || g->det_fs > 16384 ||
        g->ref_ss > 16384 || g->ref_fs > 16384) {
        set_error("sizes exceed the implemented limits (detector < 2^24 pixels, sides <= 16384)");
        return PXST_EUNSUPPORTED;
    }
    if (g->n_frames > 1920) {
        set_error("at most 1920 frames are supported");
        return PXST_EUNSUPPORTED;
    }
    const long long lim = 1LL << 28;
    if (g->org_ss < -lim || g->org_ss > lim || g->org_fs < -lim || g->org_fs > lim) {
        set_error("origin out of range");
        return PXST_EINVAL;
    }
    return PXST_OK;
}

static int check_scan(const pxst_scan* sc) {
    if (!sc) {
        set_error("scan is null");
        return PXST_EINVAL;
    }
    int rc = check_geom(&sc->geom);
    if (rc) return rc;
    if (!sc->frames || !sc->white || !sc->mask) {
        set_error("frames, white-field and mask must be non-null");
        return PXST_EINVAL;
    }
    if (!aligned(sc->frames, 2) || !aligned(sc->white, 4)) {
        set_error("frames or white-field misaligned");
        return PXST_EINVAL;
    }
    return PXST_OK;
}

static int check_window(const pxst_window& w, int maxr, const char* what) {
    if (w.r_ss < 0 || w.r_fs < 0) {
        set_error("%s window radii must be >= 0", what);
        return PXST_EINVAL;
    }
    if (w.r_ss > maxr || w.r_fs > maxr) {
        set_error("%s window radii must be <= %d", what, maxr);
        return PXST_EUNSUPPORTED;
    }
    return PXST_OK;
}

static int check_ptr(const void* p, size_t a, const char* what, bool required = true) {
    if (!p) {
        if (!required) return PXST_OK;
        set_error("%s is null", what);
        return PXST_EINVAL;
    }
    if (!aligned(p, a)) {
        set_error("%s is misaligned", what);
        return PXST_EINVAL;
    }
    return PXST_OK;
}

// Every entry point uses one layout per geometry: the translation partial sums are
// sized for the largest translation window.
static int tr_ct_of(const pxst_solve_opts*) { return TR_CT_MAX; }

static int check_ws(const void* ws, size_t bytes, size_t need) {
    if (!ws || bytes < need) {
        set_error("workspace of %zu bytes given, %zu needed", ws ? bytes : (size_t)0, need);
        return PXST_EWORKSPACE;
    }
    if (!aligned(ws, 256)) {
        set_error("workspace must be 256-byte aligned");
        return PXST_EINVAL;
    }
    return PXST_OK;
}

// ------------------------------------------------------- allocation-free error pass
// Scratch of pxst_error_noalloc: a fixed device array, one copy per GPU that the library
// runs on, held until the process ends.  In host code `scratch` names only a stand-in:
// its device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[PXST_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static std::map<int, char*> g_scratch_dev;   // device ordinal -> address of its copy

// Address of the current device's copy of `scratch` (looked up on its first use there,
// with that device current).
static int scratch_address(char** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_error("hipGetDevice: %s", hipGetErrorString(e));
        return PXST_EHIP;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_dev.find(dev);
    if (it == g_scratch_dev.end()) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("hipGetSymbolAddress of the scratch array: %s", hipGetErrorString(e));
            return PXST_EHIP;
        }
        it = g_scratch_dev.emplace(dev, (char*)p).first;
    }
    *out = it->second;
    return PXST_OK;
}

// The error pass's sections of the scratch array, each 256-byte aligned: the reference
// with invalid pixels as NaN, sigma^2, the per-(frame, block) partial sums and the
// per-frame sums.  Every section is written in full before it is read, so nothing is
// cleared between calls.
struct NoallocLayout {
    size_t refv, s2, err_part, err_pix, total;
};

static NoallocLayout noalloc_layout(const Geom& g) {
    NoallocLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += (bytes + 255) & ~(size_t)255;
        return at;
    };
    L.refv = take((size_t)g.Rs * g.Rf * sizeof(float));
    L.s2 = take(g.HW() * sizeof(float));
    const size_t nblk = (g.HW() + ERR_THREADS - 1) / ERR_THREADS;
    L.err_part = take((size_t)g.N * nblk * sizeof(double));
    L.err_pix = take((size_t)g.N * sizeof(double) + sizeof(double));
    L.total = off;
    return L;
}

}  // namespace pxst

using namespace pxst;

extern "C" {

int32_t pxst_abi_version(void) { return PXST_ABI_VERSION; }

const char* pxst_last_error(void) { return g_err; }

static int check_regularise_opts(float sigma, int integrate) {
    if (!(sigma >= 0.f) || !std::isfinite(sigma)) {
        set_error("sigma must be finite and >= 0 (got %g)", (double)sigma);
        return PXST_EINVAL;
    }
    if ((int)(4.0 * (double)sigma + 0.5) > GF_MAXR) {
        set_error("sigma %g exceeds the filter limit (radius int(4 sigma + 0.5) <= %d)", (double)sigma, GF_MAXR);
        return PXST_EUNSUPPORTED;
    }
    if (integrate != 0 && integrate != 1) {
        set_error("integrate must be 0 or 1 (got %d)", integrate);
        return PXST_EINVAL;
    }
    return PXST_OK;
}

size_t pxst_workspace_bytes(const pxst_geom* geom, const pxst_solve_opts* opts) {
    if (check_geom(geom)) return 0;
    if (opts) {
        if (check_window(opts->pm, PXST_MAX_PM_RADIUS, "pixel-map")) return 0;
        if (opts->update_dx && check_window(opts->tr, PXST_MAX_TR_RADIUS, "translation")) return 0;
    }
    if (opts && check_regularise_opts(opts->pm_sigma, opts->pm_integrate)) return 0;
    return make_layout(geom_of(*geom), tr_ct_of(opts), opts && opts->pm_integrate).total;
}

static int check_ref_mode(int mode) {
    if (mode != PXST_REF_EXACT && mode != PXST_REF_FP32 && mode != PXST_REF_BF16) {
        set_error("unknown reference-update mode %d", mode);
        return PXST_EINVAL;
    }
    return PXST_OK;
}

int pxst_update_reference_ex(const pxst_scan* scan, const float* u, const float* dx, int32_t ref_mode,
                             float* ref, double* wsum, void* ws, size_t ws_bytes, hipStream_t stream) {
    int rc;
    if ((rc = check_scan(scan))) return rc;
    if ((rc = check_ptr(u, 4, "u")) || (rc = check_ptr(dx, 4, "dx")) ||
        (rc = check_ptr(ref, 4, "ref")) || (rc = check_ptr(wsum, 8, "wsum")))
        return rc;
    if ((rc = check_ref_mode(ref_mode))) return rc;
    const Geom g = geom_of(scan->geom);
    const Layout L = make_layout(g, TR_CT_MAX);
    if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
    return launch_update_reference(g, *scan, u, dx, ref, wsum, nullptr, (char*)ws, L, stream,
                                   ref_mode);
}

int pxst_update_reference(const pxst_scan* scan, const float* u, const float* dx, float* ref,
                          double* wsum, void* ws, size_t ws_bytes, hipStream_t stream) {
    return pxst_update_reference_ex(scan, u, dx, PXST_REF_EXACT, ref, wsum, ws, ws_bytes, stream);
}

int pxst_update_pixel_map(const pxst_scan* scan, const float* ref, const double* wsum,
                          const float* dx, const float* u_in, pxst_window window, float* u_out,
                          float* err_min, int32_t* argmin, void* ws, size_t ws_bytes,
                          hipStream_t stream) {
    int rc;
    if ((rc = check_scan(scan))) return rc;
    if ((rc = check_ptr(ref, 4, "ref")) || (rc = check_ptr(wsum, 8, "wsum")) ||
        (rc = check_ptr(dx, 4, "dx")) || (rc = check_ptr(u_in, 4, "u_in")) ||
        (rc = check_ptr(u_out, 4, "u_out")) || (rc = check_ptr(err_min, 4, "err_min", false)) ||
        (rc = check_ptr(argmin, 4, "argmin", false)))
        return rc;
    if ((rc = check_window(window, PXST_MAX_PM_RADIUS, "pixel-map"))) return rc;
    const Geom g = geom_of(scan->geom);
    const Layout L = make_layout(g, TR_CT_MAX);
    if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
    char* w = (char*)ws;
    float* refv = (float*)(w + L.refv);
    int* sat = (int*)(w + L.sat);
    if ((rc = launch_prep_reference(g, ref, wsum, refv, sat, (int*)(w + L.sat_tmp),
                                        (float*)(w + L.rowmax), (int*)(w + L.fscale), stream)))
        return rc;
    if ((rc = launch_pm_setup(g, *scan, w, L, stream))) return rc;
    return launch_pixel_map(g, *scan, refv, sat, dx, u_in, window, u_out, err_min, argmin, w, L,
                            stream);
}

int pxst_update_pixel_map_fractional(const pxst_scan* scan, const float* ref, const double* wsum,
                                     const float* dx, const float* u_in, pxst_window window, int32_t steps,
                                     float* u_out, float* err_min, int32_t* argmin, void* ws, size_t ws_bytes,
                                     hipStream_t stream) {
    int rc;
    if ((rc = check_scan(scan))) return rc;
    if ((rc = check_ptr(ref, 4, "ref")) || (rc = check_ptr(wsum, 8, "wsum")) ||
        (rc = check_ptr(dx, 4, "dx")) || (rc = check_ptr(u_in, 4, "u_in")) ||
        (rc = check_ptr(u_out, 4, "u_out")) || (rc = check_ptr(err_min, 4, "err_min", false)) ||
        (rc = check_ptr(argmin, 4, "argmin", false)))
        return rc;
    if ((rc = check_window(window, PXST_MAX_PM_RADIUS, "pixel-map"))) return rc;
    if (steps < 1 || steps % 2 == 0) {
        set_error("steps must be odd and >= 1 (got %d)", steps);
        return PXST_EINVAL;
    }
    if (steps > PXST_MAX_FRAC_STEPS) {
        set_error("at most %d steps per pixel are supported", PXST_MAX_FRAC_STEPS);
        return PXST_EUNSUPPORTED;
    }
    const Geom g = geom_of(scan->geom);
    const Layout L = make_layout(g, TR_CT_MAX);
    if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
    char* w = (char*)ws;
    float* refv = (float*)(w + L.refv);
    int* sat = (int*)(w + L.sat);
    if ((rc = launch_prep_reference(g, ref, wsum, refv, sat, (int*)(w + L.sat_tmp),
                                        (float*)(w + L.rowmax), (int*)(w + L.fscale), stream)))
        return rc;
    if ((rc = launch_pm_setup(g, *scan, w, L, stream))) return rc;
    return launch_pixel_map_fractional(g, *scan, refv, sat, dx, u_in, window, steps, u_out, err_min, argmin, w,
                                       L, stream);
}

int pxst_split_half_pixel_map(const pxst_scan* scan, const float* ref, const double* wsum, const float* dx,
                              const float* u_in, pxst_window window, const uint8_t* half, float* u_a, float* u_b,
                              float hist_range, int32_t nbins, int32_t* hist, void* ws, size_t ws_bytes,
                              hipStream_t stream) {
    int rc;
    if ((rc = check_scan(scan))) return rc;
    if ((rc = check_ptr(ref, 4, "ref")) || (rc = check_ptr(wsum, 8, "wsum")) ||
        (rc = check_ptr(dx, 4, "dx")) || (rc = check_ptr(u_in, 4, "u_in")) || (rc = check_ptr(half, 1, "half")) ||
        (rc = check_ptr(u_a, 4, "u_a")) || (rc = check_ptr(u_b, 4, "u_b")) ||
        (rc = check_ptr(hist, 4, "hist", false)))
        return rc;
    if (u_a == u_in || u_b == u_in || u_a == u_b) {
        set_error("u_a, u_b and u_in must be distinct arrays");
        return PXST_EINVAL;
    }
    if ((rc = check_window(window, PXST_MAX_PM_RADIUS, "pixel-map"))) return rc;
    if (hist && (!(hist_range > 0.f) || !std::isfinite(hist_range) || nbins < 1 || nbins > 65536)) {
        set_error("histogram: range must be finite and > 0, 1 <= nbins <= 65536");
        return PXST_EINVAL;
    }
    const Geom g = geom_of(scan->geom);
    const Layout L = make_layout(g, TR_CT_MAX);
    if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
    char* w = (char*)ws;
    float* refv = (float*)(w + L.refv);
    int* sat = (int*)(w + L.sat);
    if ((rc = launch_prep_reference(g, ref, wsum, refv, sat, (int*)(w + L.sat_tmp), (float*)(w + L.rowmax),
                                    (int*)(w + L.fscale), stream)))
        return rc;
    return launch_split_half(g, *scan, refv, sat, dx, u_in, window, half, u_a, u_b, (double)hist_range, nbins, hist,
                             w, L, stream);
}

int pxst_defocus_sweep(const pxst_scan* scan, const float* dx, const float* scales, int32_t n_cand,
                       float centre_ss, float centre_fs, double* contrast, int32_t* best, void* ws,
                       size_t ws_bytes, hipStream_t stream) {
    int rc;
    if ((rc = check_scan(scan))) return rc;
    if ((rc = check_ptr(dx, 4, "dx")) || (rc = check_ptr(contrast, 8, "contrast")) ||
        (rc = check_ptr(best, 4, "best", false)))
        return rc;
    if (n_cand < 1 || !scales) {
        set_error("the sweep needs at least one candidate (n_cand = %d) and its scales", n_cand);
        return PXST_EINVAL;
    }
    for (int k = 0; k < 2 * n_cand; ++k)
        if (!std::isfinite(scales[k])) {
            set_error("scale %d is not finite", k);
            return PXST_EINVAL;
        }
    const Geom g = geom_of(scan->geom);
    const Layout L = make_layout(g, TR_CT_MAX);
    if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
    const double c0 = std::isnan(centre_ss) ? 0.5 * (g.H - 1) : (double)centre_ss;
    const double c1 = std::isnan(centre_fs) ? 0.5 * (g.W - 1) : (double)centre_fs;
    if (!std::isfinite(c0) || !std::isfinite(c1)) {
        set_error("centre must be finite or NaN");
        return PXST_EINVAL;
    }
    return launch_defocus_sweep(g, *scan, dx, scales, n_cand, c0, c1, contrast, best, (char*)ws, L, stream);
}

int pxst_update_translations(const pxst_scan* scan, const float* ref, const double* wsum,
                             const float* u, const float* dx_in, pxst_window window, float* dx_out,
                             float* err_min, int32_t* argmin, void* ws, size_t ws_bytes,
                             hipStream_t stream) {
    int rc;
    if ((rc = check_scan(scan))) return rc;
    if ((rc = check_ptr(ref, 4, "ref")) || (rc = check_ptr(wsum, 8, "wsum")) ||
        (rc = check_ptr(u, 4, "u")) || (rc = check_ptr(dx_in, 4, "dx_in")) ||
        (rc = check_ptr(dx_out, 4, "dx_out")) || (rc = check_ptr(err_min, 4, "err_min", false)) ||
        (rc = check_ptr(argmin, 4, "argmin", false)))
        return rc;
    if ((rc = check_window(window, PXST_MAX_TR_RADIUS, "translation"))) return rc;
    const Geom g = geom_of(scan->geom);
    const Layout L = make_layout(g, TR_CT_MAX);
    if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
    char* w = (char*)ws;
    float* refv = (float*)(w + L.refv);
    if ((rc = launch_prep_reference(g, ref, wsum, refv, nullptr, nullptr, nullptr, nullptr, stream))) return rc;
    return launch_translations(g, *scan, refv, u, dx_in, window, dx_out, err_min, argmin, w, L,
                               stream);
}

int pxst_error(const pxst_scan* scan, const float* ref, const double* wsum, const float* u,
               const float* dx, float* pixel_err, double* frame_err, double* total, float* ref_err,
               void* ws, size_t ws_bytes, hipStream_t stream) {
    int rc;
    if ((rc = check_scan(scan))) return rc;
    if ((rc = check_ptr(ref, 4, "ref")) || (rc = check_ptr(wsum, 8, "wsum")) ||
        (rc = check_ptr(u, 4, "u")) || (rc = check_ptr(dx, 4, "dx")) ||
        (rc = check_ptr(total, 8, "total")) || (rc = check_ptr(pixel_err, 4, "pixel_err", false)) ||
        (rc = check_ptr(frame_err, 8, "frame_err", false)) ||
        (rc = check_ptr(ref_err, 4, "ref_err", false)))
        return rc;
    const Geom g = geom_of(scan->geom);
    const Layout L = make_layout(g, TR_CT_MAX);
    if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
    char* w = (char*)ws;
    float* refv = (float*)(w + L.refv);
    float* s2 = (float*)(w + L.s2);
    if ((rc = launch_prep_reference(g, ref, wsum, refv, nullptr, nullptr, nullptr, nullptr, stream))) return rc;
    if ((rc = launch_sigma2(g, *scan, s2, stream))) return rc;
    if ((rc = launch_error(g, *scan, refv, s2, u, dx, pixel_err, frame_err, total, w, L, stream)))
        return rc;
    if (ref_err) return launch_reference_error(g, *scan, u, dx, refv, ref_err, w, L, stream);
    return PXST_OK;
}

int pxst_error_noalloc(const pxst_scan* scan, const float* ref, const double* wsum, const float* u,
                       const float* dx, float* pixel_err, double* frame_err, double* total,
                       hipStream_t stream) {
    int rc;
    if ((rc = check_scan(scan))) return rc;
    if ((rc = check_ptr(ref, 4, "ref")) || (rc = check_ptr(wsum, 8, "wsum")) ||
        (rc = check_ptr(u, 4, "u")) || (rc = check_ptr(dx, 4, "dx")) ||
        (rc = check_ptr(total, 8, "total")) || (rc = check_ptr(pixel_err, 4, "pixel_err", false)) ||
        (rc = check_ptr(frame_err, 8, "frame_err", false)))
        return rc;
    const Geom g = geom_of(scan->geom);
    const NoallocLayout NL = noalloc_layout(g);
    if (NL.total > (size_t)PXST_NOALLOC_SCRATCH_BYTES) {
        set_error("the error pass of this geometry needs %zu bytes of scratch; the fixed array holds %zu",
                  NL.total, (size_t)PXST_NOALLOC_SCRATCH_BYTES);
        return PXST_EUNSUPPORTED;
    }
    char* w = nullptr;
    if ((rc = scratch_address(&w))) return rc;
    Layout L{};
    L.err_part = NL.err_part;
    L.err_pix = NL.err_pix;
    float* refv = (float*)(w + NL.refv);
    float* s2 = (float*)(w + NL.s2);
    if ((rc = launch_prep_reference(g, ref, wsum, refv, nullptr, nullptr, nullptr, nullptr, stream))) return rc;
    if ((rc = launch_sigma2(g, *scan, s2, stream))) return rc;
    return launch_error(g, *scan, refv, s2, u, dx, pixel_err, frame_err, total, w, L, stream);
}

int pxst_regularise_pixel_map(const pxst_geom* geom, const float* u_in, float* u_out, float sigma,
                              int32_t integrate, void* ws, size_t ws_bytes, hipStream_t stream) {
    int rc;
    if ((rc = check_geom(geom))) return rc;
    if ((rc = check_regularise_opts(sigma, integrate))) return rc;
    if ((rc = check_ptr(u_in, 4, "u_in")) || (rc = check_ptr(u_out, 4, "u_out"))) return rc;
    const Geom g = geom_of(*geom);
    const Layout L = make_layout(g, TR_CT_MAX, integrate != 0);
    if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
    return launch_regularise(g, u_in, u_out, sigma, integrate, (char*)ws, L, stream);
}

// A second stream per device (default priority, non-blocking) and three events (fork,
// join, inverted map built), created on first use and kept until the process ends.  The returned lock
// serialises the enqueueing of solves on one device, so that the events' records and
// waits of concurrent callers do not interleave.
namespace {
struct AuxStream {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr, mapped = nullptr;
    std::mutex mu;
};
std::mutex g_aux_mu;
std::map<int, AuxStream*> g_aux;
}  // namespace

static int aux_stream(std::unique_lock<std::mutex>& lk, hipStream_t& s, hipEvent_t& fork, hipEvent_t& join,
                      hipEvent_t& mapped) {
    int dev = 0;
    int rc = check_hip(hipGetDevice(&dev), "device");
    if (rc) return rc;
    AuxStream* x = nullptr;
    {
        std::lock_guard<std::mutex> g(g_aux_mu);
        AuxStream*& slot = g_aux[dev];
        if (!slot) slot = new AuxStream();
        x = slot;
    }
    lk = std::unique_lock<std::mutex>(x->mu);
    if (!x->s) {
        if ((rc = check_hip(hipStreamCreateWithFlags(&x->s, hipStreamNonBlocking), "stream create"))) return rc;
        if ((rc = check_hip(hipEventCreateWithFlags(&x->fork, hipEventDisableTiming), "event create")) ||
            (rc = check_hip(hipEventCreateWithFlags(&x->join, hipEventDisableTiming), "event create")) ||
            (rc = check_hip(hipEventCreateWithFlags(&x->mapped, hipEventDisableTiming), "event create")))
            return rc;
    }
    s = x->s;
    fork = x->fork;
    join = x->join;
    mapped = x->mapped;
    return PXST_OK;
}

int pxst_solve(const pxst_scan* scan, const pxst_solve_opts* opts, float* u, float* dx, float* ref,
               double* wsum, double* err_hist, void* ws, size_t ws_bytes, hipStream_t stream) {
    int rc;
    if ((rc = check_scan(scan))) return rc;
    if (!opts) {
        set_error("options are null");
        return PXST_EINVAL;
    }
    if (opts->n_iter < 0) {
        set_error("n_iter must be >= 0");
        return PXST_EINVAL;
    }
    if ((rc = check_window(opts->pm, PXST_MAX_PM_RADIUS, "pixel-map"))) return rc;
    if (opts->update_dx && (rc = check_window(opts->tr, PXST_MAX_TR_RADIUS, "translation")))
        return rc;
    if ((rc = check_ref_mode(opts->ref_mode))) return rc;
    if ((rc = check_regularise_opts(opts->pm_sigma, opts->pm_integrate))) return rc;
    if ((rc = check_ptr(u, 4, "u")) || (rc = check_ptr(dx, 4, "dx")) ||
        (rc = check_ptr(ref, 4, "ref")) || (rc = check_ptr(wsum, 8, "wsum")) ||
        (rc = check_ptr(err_hist, 8, "err_hist", false)))
        return rc;
    const Geom g = geom_of(scan->geom);
    const Layout L = make_layout(g, tr_ct_of(opts), opts->pm_integrate != 0);
    if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
    char* w = (char*)ws;
    int* sat = (int*)(w + L.sat);
    int* sat_tmp = (int*)(w + L.sat_tmp);
    float* s2 = (float*)(w + L.s2);
    // Iteration k's error pass reads (u, dx) of the iteration and its reference copy
    // only, so it runs on a second stream while iteration k + 1 updates the reference
    // into the other copy; the main stream waits for it before the search of
    // iteration k + 1 overwrites the map (and before returning).  With the translation
    // update on, the next reference update's inverted map (which depends on the map u
    // only) is built on the second stream too, while the translations are searched.
    std::unique_lock<std::mutex> lk;
    hipStream_t es = stream;
    hipEvent_t fork = nullptr, join = nullptr, mapped = nullptr;
    if (opts->n_iter > 0 && (rc = aux_stream(lk, es, fork, join, mapped))) return rc;
    auto refv_of = [&](int k) { return (float*)(w + ((k & 1) ? L.refv2 : L.refv)); };
    if ((rc = launch_sigma2(g, *scan, s2, stream))) return rc;
    if (opts->n_iter > 0 && (rc = launch_pm_setup(g, *scan, w, L, stream))) return rc;
    bool err_pending = false, map_ready = false;
    auto fork_to_aux = [&]() {
        int r = check_hip(hipEventRecord(fork, stream), "event record");
        return r ? r : check_hip(hipStreamWaitEvent(es, fork, 0), "stream wait");
    };
    for (int k = 0; k < opts->n_iter; ++k) {
        float* refv = refv_of(k);
        if (map_ready && (rc = check_hip(hipStreamWaitEvent(stream, mapped, 0), "stream wait"))) return rc;
        if ((rc = launch_update_reference(g, *scan, u, dx, ref, wsum, refv, w, L, stream, opts->ref_mode,
                                          !map_ready)))
            return rc;
        map_ready = false;
        if ((rc = launch_prep_reference(g, nullptr, nullptr, refv, sat, sat_tmp, (float*)(w + L.rowmax),
                                             (int*)(w + L.fscale), stream))) return rc;
        if (err_pending && (rc = check_hip(hipStreamWaitEvent(stream, join, 0), "stream wait"))) return rc;
        err_pending = false;
        if ((rc = launch_pixel_map(g, *scan, refv, sat, dx, u, opts->pm, u, nullptr, nullptr, w, L,
                                   stream)))
            return rc;
        if ((opts->pm_sigma > 0.f || opts->pm_integrate) &&
            (rc = launch_regularise(g, u, u, opts->pm_sigma, opts->pm_integrate, w, L, stream)))
            return rc;
        if (opts->update_dx) {
            if ((rc = fork_to_aux()) || (rc = launch_inverse_map(g, *scan, u, w, L, es)) ||
                (rc = check_hip(hipEventRecord(mapped, es), "event record")))
                return rc;
            map_ready = true;
            if ((rc = launch_translations(g, *scan, refv, u, dx, opts->tr, dx, nullptr, nullptr, w, L, stream)))
                return rc;
        }
        double* tot = err_hist ? err_hist + k : (double*)(w + L.err_pix) + g.N;
        if ((rc = fork_to_aux())) return rc;
        if ((rc = launch_error(g, *scan, refv, s2, u, dx, nullptr, nullptr, tot, w, L, es))) return rc;
        if ((rc = check_hip(hipEventRecord(join, es), "event record"))) return rc;
        err_pending = true;
    }
    if (map_ready && (rc = check_hip(hipStreamWaitEvent(stream, mapped, 0), "stream wait"))) return rc;
    rc = launch_update_reference(g, *scan, u, dx, ref, wsum, refv_of(opts->n_iter), w, L, stream, opts->ref_mode,
                                 !map_ready);
    if (err_pending) {
        const int rj = check_hip(hipStreamWaitEvent(stream, join, 0), "stream wait");
        if (!rc) rc = rj;
    }
    return rc;
}

int pxst_profile_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    return PXST_OK;
}

int pxst_profile_select(const char* families) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_sel.clear();
    g_prof_all = families == nullptr || families[0] == '\0';
    if (g_prof_all) return PXST_OK;
    std::string cur;
    for (const char* c = families;; ++c) {
        if (*c == ',' || *c == '\0') {
            if (!cur.empty()) g_prof_sel.push_back(cur);
            cur.clear();
            if (*c == '\0') break;
        } else if (*c != ' ') {
            cur += *c;
        }
    }
    return PXST_OK;
}

int pxst_profile_read(const char* family, double* total_ms, int64_t* launches, int64_t* work_units) {
    if (!family || !total_ms || !launches) {
        set_error("null argument");
        return PXST_EINVAL;
    }
    hipDeviceSynchronize();   // pending counter copies land before they are read
    std::lock_guard<std::mutex> lk(g_prof_mu);
    *total_ms = 0.0;
    *launches = 0;
    if (work_units) *work_units = 0;
    auto it = g_prof.find(family);
    if (it == g_prof.end()) return PXST_OK;
    Family& f = it->second;
    for (Span& sp : f.spans) {
        float ms = 0.f;
        if (hipEventSynchronize(sp.b) == hipSuccess && hipEventElapsedTime(&ms, sp.a, sp.b) == hipSuccess) {
            *total_ms += ms;
            *launches += 1;
            if (work_units) *work_units += sp.pinned ? (long long)(*sp.pinned) * sp.scale : sp.work;
        }
        f.pool.push_back(sp.a);
        f.pool.push_back(sp.b);
        if (sp.snap >= 0) {
            Snap& sn = g_snaps[sp.snap];
            if (--sn.refs <= 0) sn.busy = false;
        } else if (sp.pinned) {
            f.pinned_pool.push_back(sp.pinned);
        }
    }
    f.spans.clear();
    return PXST_OK;
}

size_t pxst_batch_workspace_bytes(int32_t n_jobs) {
    if (n_jobs < 0) {
        set_error("n_jobs must be >= 0");
        return 0;
    }
    // argument tables of the batched stages: the pixel-map search's, and one table per
    // group of jobs (at most n_jobs groups) for the inverted maps, the splat, the
    // summed-area tables, the translation search and the error, each rounded up to 256
    // bytes
    const size_t n = (size_t)n_jobs;
    const size_t per = sizeof(MapArgs) + sizeof(SplatArgs) + sizeof(SatArgs) + sizeof(TrArgs) + sizeof(ErrArgs);
    return pixel_map_batch_table_bytes(n_jobs) + n * per + 5 * n * 256 + 4096;
}

int pxst_batch_iterate(const pxst_job* jobs, int32_t n_jobs, void* batch_ws, size_t batch_ws_bytes,
                       hipStream_t stream) {
    if (n_jobs < 0 || (n_jobs > 0 && !jobs)) {
        set_error("bad job list");
        return PXST_EINVAL;
    }
    // validate every job before enqueuing anything
    for (int j = 0; j < n_jobs; ++j) {
        const pxst_job& J = jobs[j];
        int rc;
        if ((rc = check_scan(&J.scan))) return rc;
        if (J.iter < 0 || J.iter > J.opts.n_iter) {
            set_error("job %d: iter %d outside 0..n_iter", j, J.iter);
            return PXST_EINVAL;
        }
        if ((rc = check_window(J.opts.pm, PXST_MAX_PM_RADIUS, "pixel-map"))) return rc;
        if (J.opts.update_dx && (rc = check_window(J.opts.tr, PXST_MAX_TR_RADIUS, "translation")))
            return rc;
        if ((rc = check_ref_mode(J.opts.ref_mode))) return rc;
        if ((rc = check_regularise_opts(J.opts.pm_sigma, J.opts.pm_integrate))) return rc;
        if ((rc = check_ptr(J.u, 4, "u")) || (rc = check_ptr(J.dx, 4, "dx")) ||
            (rc = check_ptr(J.ref, 4, "ref")) || (rc = check_ptr(J.wsum, 8, "wsum")) ||
            (rc = check_ptr(J.err_hist, 8, "err_hist", false)))
            return rc;
        const Layout L = make_layout(geom_of(J.scan.geom), tr_ct_of(&J.opts), J.opts.pm_integrate != 0);
        if ((rc = check_ws(J.ws, J.ws_bytes, L.total))) return rc;
    }
    if (n_jobs == 0) return PXST_OK;
    {
        const size_t need = pxst_batch_workspace_bytes(n_jobs);
        int rc;
        if ((rc = check_ws(batch_ws, batch_ws_bytes, need))) return rc;
    }

    std::lock_guard<std::mutex> lk(g_batch_mu);
    if (g_batch_done) hipEventSynchronize(g_batch_done);   // previous tables copied
    if (g_batch_cap < batch_ws_bytes) {
        if (g_batch_host) hipHostFree(g_batch_host);
        g_batch_host = nullptr;
        g_batch_cap = 0;
        if (hipHostMalloc((void**)&g_batch_host, batch_ws_bytes, hipHostMallocDefault) != hipSuccess) {
            g_batch_host = nullptr;
            set_error("cannot allocate %zu bytes of pinned staging memory", batch_ws_bytes);
            return PXST_EHIP;
        }
        g_batch_cap = batch_ws_bytes;
    }
    if (!g_batch_done && hipEventCreateWithFlags(&g_batch_done, hipEventDisableTiming) != hipSuccess) {
        set_error("cannot create an event");
        return PXST_EHIP;
    }
    BatchArena ar;
    ar.host = g_batch_host;
    ar.dev = (char*)batch_ws;
    ar.cap = batch_ws_bytes;
    ar.stream = stream;

    struct JobState {
        Geom g;
        Layout L;
        char* w;
        float* refv;
        bool iterates;
    };
    std::vector<JobState> st(n_jobs);
    for (int j = 0; j < n_jobs; ++j) {
        st[j].g = geom_of(jobs[j].scan.geom);
        st[j].L = make_layout(st[j].g, tr_ct_of(&jobs[j].opts), jobs[j].opts.pm_integrate != 0);
        st[j].w = (char*)jobs[j].ws;
        st[j].refv = (float*)(st[j].w + st[j].L.refv);
        st[j].iterates = jobs[j].iter < jobs[j].opts.n_iter;
    }

    // ---- every argument table, staged on the host before anything is enqueued
    // (1) reference update (exact arithmetic, stored as float32 or rounded to bfloat16):
    // one group per frame-chunking form; the float32-gather arithmetic runs per job
    struct RefGroup {
        std::vector<MapArgs> m;
        std::vector<SplatArgs> sp;
        const MapArgs* dm = nullptr;
        const SplatArgs* ds = nullptr;
    };
    RefGroup rg[2];
    for (int j = 0; j < n_jobs; ++j) {
        const pxst_job& J = jobs[j];
        if (J.opts.ref_mode == PXST_REF_FP32) continue;
        const SplatArgs sa = make_splat_args(st[j].g, J.scan, J.dx, J.ref, J.wsum, st[j].refv, st[j].w, st[j].L);
        RefGroup& G = rg[sa.nchunks > 1 ? 1 : 0];
        G.m.push_back(make_map_args(st[j].g, J.scan, J.u, st[j].w, st[j].L));
        G.sp.push_back(sa);
    }
    for (RefGroup& G : rg)
        if (!G.m.empty()) {
            G.dm = (const MapArgs*)stage_raw(ar, G.m.data(), G.m.size() * sizeof(MapArgs));
            G.ds = (const SplatArgs*)stage_raw(ar, G.sp.data(), G.sp.size() * sizeof(SplatArgs));
        }
    // (2) summed-area tables of the jobs that iterate
    std::vector<SatArgs> sat;
    for (int j = 0; j < n_jobs; ++j)
        if (st[j].iterates) sat.push_back(make_sat_args(st[j].g, st[j].refv, st[j].w, st[j].L));
    const SatArgs* sat_dev =
        sat.empty() ? nullptr : (const SatArgs*)stage_raw(ar, sat.data(), sat.size() * sizeof(SatArgs));
    // (3) pixel-map search
    std::vector<PmJobDesc> pm;
    for (int j = 0; j < n_jobs; ++j) {
        const pxst_job& J = jobs[j];
        if (!st[j].iterates) continue;
        PmJobDesc d;
        d.g = st[j].g;
        d.sc = J.scan;
        d.refv = st[j].refv;
        d.sat = (const int*)(st[j].w + st[j].L.sat);
        d.dx = J.dx;
        d.u_in = J.u;
        d.u_out = J.u;
        d.win = J.opts.pm;
        d.ws = st[j].w;
        d.L = &st[j].L;
        pm.push_back(d);
    }
    std::shared_ptr<PmBatchImpl> pmb;
    int rc = stage_pixel_map_batch(pm.data(), (int)pm.size(), ar, pmb);
    if (rc) return rc;
    // (4) translation search: one group per window
    std::vector<std::vector<TrArgs>> trg;
    for (int j = 0; j < n_jobs; ++j) {
        const pxst_job& J = jobs[j];
        if (!st[j].iterates || !J.opts.update_dx) continue;
        const TrArgs t = make_tr_args(st[j].g, J.scan, st[j].refv, J.u, J.dx, J.opts.tr, J.dx, nullptr, nullptr,
                                      st[j].w, st[j].L);
        size_t k = 0;
        while (k < trg.size() && (trg[k][0].tx != t.tx || trg[k][0].ty != t.ty)) ++k;
        if (k == trg.size()) trg.emplace_back();
        trg[k].push_back(t);
    }
    std::vector<const TrArgs*> trg_dev;
    for (auto& G : trg) trg_dev.push_back((const TrArgs*)stage_raw(ar, G.data(), G.size() * sizeof(TrArgs)));
    // (5) error: one group per reference lookup form (pairs of rows or single rows)
    std::vector<ErrArgs> eg[2];
    for (int j = 0; j < n_jobs; ++j) {
        const pxst_job& J = jobs[j];
        if (!st[j].iterates) continue;
        double* total = J.err_hist ? J.err_hist + J.iter : (double*)(st[j].w + st[j].L.err_pix) + st[j].g.N;
        const ErrArgs e = make_err_args(st[j].g, J.scan, st[j].refv, (const float*)(st[j].w + st[j].L.s2), J.u,
                                        J.dx, nullptr, nullptr, total, st[j].w, st[j].L);
        eg[(e.Rs >= 2 && e.Rf >= 2) ? 1 : 0].push_back(e);
    }
    const ErrArgs* eg_dev[2] = {nullptr, nullptr};
    for (int k = 0; k < 2; ++k)
        if (!eg[k].empty()) eg_dev[k] = (const ErrArgs*)stage_raw(ar, eg[k].data(), eg[k].size() * sizeof(ErrArgs));
    if (ar.overflow) {
        set_error("batch workspace too small for the argument tables");
        return PXST_EWORKSPACE;
    }

    // ---- launches: one copy of all tables, then the stages in order.  Past this point
    // only a failing HIP call returns early, leaving the jobs' states undefined.
    rc = flush_tables(ar);
    if (!rc) rc = check_hip(hipEventRecord(g_batch_done, stream), "event record");
    // variance and search setup once per job
    for (int j = 0; j < n_jobs && !rc; ++j) {
        const pxst_job& J = jobs[j];
        if (J.iter != 0) continue;
        rc = launch_sigma2(st[j].g, J.scan, (float*)(st[j].w + st[j].L.s2), stream);
        if (!rc && J.opts.n_iter > 0) rc = launch_pm_setup(st[j].g, J.scan, st[j].w, st[j].L, stream);
    }
    // (i) reference update of every job
    for (RefGroup& G : rg)
        if (!rc && !G.m.empty())
            rc = launch_reference_jobs(G.m.data(), G.sp.data(), (int)G.m.size(), G.dm, G.ds, stream);
    for (int j = 0; j < n_jobs && !rc; ++j) {
        const pxst_job& J = jobs[j];
        if (J.opts.ref_mode == PXST_REF_BF16)
            rc = launch_round_bf16(st[j].g, J.ref, st[j].refv, stream);
        else if (J.opts.ref_mode == PXST_REF_FP32)
            rc = launch_update_reference(st[j].g, J.scan, J.u, J.dx, J.ref, J.wsum, st[j].refv, st[j].w, st[j].L,
                                         stream, J.opts.ref_mode);
    }
    if (!rc && !sat.empty()) rc = launch_sat_jobs(sat.data(), (int)sat.size(), sat_dev, stream);
    // (ii) pixel-map search of the jobs that iterate
    if (!rc) rc = run_pixel_map_batch(*pmb, stream);
    // (iii) regularisation of the map, translations and (iv) total error
    for (int j = 0; j < n_jobs && !rc; ++j) {
        const pxst_job& J = jobs[j];
        if (st[j].iterates && (J.opts.pm_sigma > 0.f || J.opts.pm_integrate))
            rc = launch_regularise(st[j].g, J.u, J.u, J.opts.pm_sigma, J.opts.pm_integrate, st[j].w, st[j].L,
                                   stream);
    }
    for (size_t k = 0; k < trg.size() && !rc; ++k)
        rc = launch_translations_jobs(trg[k].data(), (int)trg[k].size(), trg_dev[k], stream);
    for (int k = 0; k < 2 && !rc; ++k)
        if (!eg[k].empty()) rc = launch_error_jobs(eg[k].data(), (int)eg[k].size(), eg_dev[k], stream);
    return rc;
}

}  // extern "C"

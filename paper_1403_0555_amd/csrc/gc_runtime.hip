// Host runtime and C ABI of the Gribov-copy enumerator (see include/gribov.h).
//
// A context owns a device, a few HIP streams, an HBM byte budget, a pool of
// device blocks, the loaded orbits and their launches ("jobs").  gc_launch
// admits a job when its bytes fit the free budget (else it waits in FIFO
// order) and enqueues on a stream: reset (fill kernels), the persistent solve
// kernel, finalize (table compaction), and the D2H of the job's counters.  A
// scheduler thread watches the jobs' completion events, frees their working
// memory and admits waiting jobs, so launches that arrive while others run
// overlap on the device.
#include "../../include/gribov.h"
#include "gc_internal.h"
#include "gc_wave.h"

#include <algorithm>
#include <cstdlib>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

// Working memory of gc_launch_static, for callers that cannot allocate: one
// array per GPU, resident from the module load until the process ends.  Host
// code reaches it only through the device address hipGetSymbolAddress
// returns (kept per device), never through this name.
#define GC_STATIC_SCRATCH_BYTES (64ull << 20)
static __device__ __align__(256) unsigned char scratch[GC_STATIC_SCRATCH_BYTES];

namespace {

using Clock = std::chrono::steady_clock;

// Device address of scratch per device ordinal, looked up once per device
// with that device current.
std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;

hipError_t scratch_address(int device, void **out)
{
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return hipSuccess;
    }
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
    *out = p;
    return hipSuccess;
}

double ms_since(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double, std::milli>(b - a).count();
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

uint64_t next_pow2(uint64_t x)
{
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

// ---------------------------------------------------------------------------
// Lattice checks and geometry (Sec. I: periodic lattice; Sec. III: checkerboard)
// ---------------------------------------------------------------------------
constexpr int kMaxV = 4096;
constexpr double kPiD = 3.14159265358979311599796346854;   // fl(pi)

int num_colours(int d, const int *n)
{
    bool all_even = true;
    for (int mu = 0; mu < d; ++mu)
        if (n[mu] % 2) all_even = false;
    if (all_even) return 2;
    int nmin = n[0];
    for (int mu = 1; mu < d; ++mu) nmin = std::min(nmin, n[mu]);
    for (int K = 3; K <= nmin; ++K) {
        bool ok = true;
        for (int mu = 0; mu < d; ++mu)
            if (n[mu] % K) ok = false;
        if (ok) return K;
    }
    return 0;
}

gc_status check_lattice(const gc_lattice *lat, int *K_out, int *V_out)
{
    if (!lat || lat->dim < 1 || lat->dim > 4) return GC_EINVAL;
    int64_t V = 1;
    for (int mu = 0; mu < lat->dim; ++mu) {
        if (lat->extent[mu] < 2 || lat->extent[mu] > 65536) return GC_EINVAL;
        V *= lat->extent[mu];
        if (V > 65536) return GC_EUNSUPPORTED;
    }
    if (lat->antiperiodic >> lat->dim) return GC_EINVAL;
    const int K = num_colours(lat->dim, lat->extent);
    if (K == 0) return GC_EUNSUPPORTED;
    if (K_out) *K_out = K;
    if (V_out) *V_out = (int)V;
    return GC_OK;
}

uint64_t creg_key(int d, int ns, bool mixed) { return ((uint64_t)d << 40) | ((uint64_t)ns << 8) | (mixed ? 1u : 0u); }

int block_for(int V)
{
    if (V <= 128) return 64;
    if (V <= 512) return 128;
    return 256;
}

// ---------------------------------------------------------------------------
// Device memory pool: freed blocks are cached and reused by later requests of
// at most their size (and not more than 25% smaller).  Sizes are rounded to
// 2 MiB granules (powers of two below that).
// ---------------------------------------------------------------------------
struct Pool {
    std::multimap<size_t, void *> free_blocks;
    size_t cached = 0;

    static size_t rounded(size_t bytes)
    {
        const size_t g = size_t(2) << 20;
        if (bytes <= g) return next_pow2(std::max<size_t>(bytes, 4096));
        return (bytes + g - 1) / g * g;
    }
    hipError_t get(size_t bytes, void **p, size_t *got)
    {
        bytes = rounded(bytes);
        auto it = free_blocks.lower_bound(bytes);
        if (it != free_blocks.end() && it->first <= bytes + bytes / 4) {
            *p = it->second;
            *got = it->first;
            cached -= it->first;
            free_blocks.erase(it);
            return hipSuccess;
        }
        *got = bytes;
        return hipMalloc(p, bytes);
    }
    void put(void *p, size_t bytes)
    {
        if (!p) return;
        free_blocks.emplace(bytes, p);
        cached += bytes;
    }
    void drain()
    {
        for (auto &kv : free_blocks) (void)hipFree(kv.second);
        free_blocks.clear();
        cached = 0;
    }
};

// Pinned host blocks for a job's descriptor staging and its result
// counters, reused like the device pool: hipHostMalloc and hipHostFree are
// kept off the launch and release paths (a free waits for the device).
struct PinnedPool {
    std::multimap<size_t, void *> free_blocks;

    hipError_t get(size_t bytes, void **p, size_t *got)
    {
        bytes = std::max<size_t>(next_pow2(bytes), 4096);
        auto it = free_blocks.find(bytes);
        if (it != free_blocks.end()) {
            *p = it->second;
            *got = bytes;
            free_blocks.erase(it);
            return hipSuccess;
        }
        *got = bytes;
        return hipHostMalloc(p, bytes, hipHostMallocDefault);
    }
    void put(void *p, size_t bytes)
    {
        if (p) free_blocks.emplace(bytes, p);
    }
    void drain()
    {
        for (auto &kv : free_blocks) (void)hipHostFree(kv.second);
        free_blocks.clear();
    }
};

struct Orbit;

// An orbit's host copy table in a pinned block of the context's pool, so
// that the device-to-host copy runs at the link's speed: grown on demand,
// kept across launches of the orbit, handed back to the pool (not freed)
// when the orbit is released.
struct HostCopies {
    gc_copy *p = nullptr;
    size_t n = 0, cap_bytes = 0;
    gc_copy *data() { return p; }
    size_t size() const { return n; }
    gc_copy &operator[](size_t i) { return p[i]; }
    gc_copy *begin() { return p; }
    gc_copy *end() { return p + n; }
    const gc_copy *begin() const { return p; }
    const gc_copy *end() const { return p + n; }
    void clear() { n = 0; }
};

// Relax launch groups: orbits with odd extents use the workgroup-per-start
// kernel; orbits with even extents the wavefront-per-start kernel, one launch
// per dimension, layout and slot count (the kernel is specialised on them).
struct Group {
    bool wave = false;
    int d = 0;
    std::vector<int> jobs;           // indices into Job::orbits
    int block = 64, grid = 1, ns = 1, coef_lds = 0, creg = 0, wps = 0;
    int rm = 0;                      // relax mode of the exchange-region kernel (ns > 2)
    int full = 0;                    // GC_RM_FULL_SLOTS for the double-precision kernel, or 0
    size_t lds = 0;
    // mixed precision above two slots per lane: the single-precision phase
    // in its own kernel, before the double-precision one
    int split = 0, grid32 = 1;
    size_t lds32 = 0;
    size_t o_jobs = 0, o_worbs = 0, o_next = 0, o_prefix = 0, o_bounce = 0;
    size_t o_jobs1 = 0;              // first-pass descriptors of a batch-synchronous launch
    uint64_t total = 0;
};

// Kernel variant word of a wavefront-per-start group (gc_launch_wave).
int wave_variant(const Group &g) { return g.coef_lds | (g.creg << 1) | ((g.rm | g.full) << 3); }

// Orbits of one relax group sharing one post-kernel shape (workgroup size by
// V), so that an orbit's per-start arithmetic is the same alone and in a
// batch.
struct PostGroup {
    int block = 64, sp = 1, wreg = 1, grid = 1;
    size_t lds = 0;
    uint64_t total = 0, wstride = 0;
    std::vector<int> jobs;
    int chain = 0;                   // relax group whose orbits these are
    size_t o_jobs = 0, o_prefix = 0, o_next = 0, o_wbuf = 0;
};

// Orbits of one relax group sharing one filter-pass kernel: the
// line-segment Lanczos kernel (fast, seg sites per thread) or the general
// post kernel in its filter mode.
struct FilterGroup {
    bool fast = false;
    int d = 0;                        // lattice dimension (fast kernel: one per dimension)
    int form = 0;                     // fast kernel: gc_lanczos_form (whole lines, array stride)
    int block = 64, seg = 1, sp = 1, wreg = 1, grid = 1;
    size_t lds = 0;
    uint64_t total = 0, wstride = 0;   // total: an upper bound of the copies (the starts)
    std::vector<int> jobs;
    int chain = 0;
    size_t o_jobs = 0, o_next = 0, o_wbuf = 0;
};

// Device memory of one job.
struct JobLayout {
    std::vector<size_t> o_rec, o_table, o_cnt, o_copies, o_ncopies, o_states, o_blk, o_sync, o_theta;
    std::vector<uint64_t> table_cap;
    std::vector<Group> groups;
    std::vector<PostGroup> posts;
    std::vector<FilterGroup> filters;
    size_t total = 0;
};

struct Job {
    std::vector<Orbit *> orbits;     // one for gc_launch, several for a batch
    std::vector<uint64_t> n_starts;
    gc_solve_params p{};
    int state = GC_ORBIT_QUEUED;
    gc_status err = GC_OK;           // why the job ended in GC_ORBIT_ERROR
    bool graph = false;
    size_t bytes = 0;                // budget charge while its memory is held
    void *mem = nullptr;             // working block (results stay in it)
    void *staging = nullptr;         // pinned descriptors + result counters
    size_t staging_bytes = 0;
    int stream = -1;
    hipEvent_t ev_k0 = nullptr, ev_k1 = nullptr, ev_k2 = nullptr, ev_k3 = nullptr, ev_done = nullptr;
    hipGraph_t g = nullptr;
    hipGraphExec_t gx = nullptr;
    JobLayout L;
    Clock::time_point t_submit, t_done;
    std::vector<GcJobDev> jobs;      // host images of the per-orbit job structs
    // pinned host results (inside staging)
    GcCounters *h_cnt = nullptr;               // [n_jobs]
    unsigned long long *h_ncopies = nullptr;   // [n_jobs]
    double solve_ms = 0.0, post_ms = 0.0, filter_ms = 0.0;
    uint64_t total = 0;
    // kernel variants forced for this job (gc_autotune trials), -1 / 0: none
    int force_creg = -1;
    std::vector<double> theta;       // the caller's start angles [n][V] (gc_launch_from), else empty
};

struct Orbit {
    gc_orbit handle = 0;
    gc_lattice lat{};
    int d = 0, V = 0, K = 0;
    uint64_t orbit_index = 0;
    std::vector<double> phi;         // as loaded
    void *tables = nullptr;
    size_t table_bytes = 0;
    GcOrbitDev dev{};
    GcWaveOrbit wdev{};              // colour-split tables (K == 2 only)
    void *wave_tables = nullptr;
    size_t wave_bytes = 0;
    // results of the last launch
    Job *job = nullptr;
    int job_index = 0;               // position inside a batch job
    GcJobDev res{};                  // pointers into the job's block
    bool have_copies = false;
    HostCopies copies;
    bool have_starts = false;
    std::vector<gc_start_record> starts;
    uint64_t paper_count = 0;
    gc_progress last{};
};

}  // namespace

struct gc_ctx {
    int device = 0;
    int n_cu = 0;
    size_t lds_max = 0;
    int creg_override = -1;   // GC_WAVE_CREG: register-held coefficient colours (tuning)
    int wps_override = -1;    // GC_WPS: 1 workgroup per start where available, 0 never (tuning)
    // kernel variants chosen by gc_autotune: relax coefficient colours and
    // layout per (d, slots per lane, precision), post workgroup shape per V
    std::map<uint64_t, int> tune_creg;
    std::string tune_cache;             // file the choices persist in ("" none)
    uint64_t budget = 0, used = 0;
    std::vector<hipStream_t> streams;   // launch streams (the caller's one when given)
    bool own_streams = true;
    std::vector<hipStream_t> aux;       // fork streams for graph capture of batches
    hipStream_t util = nullptr;         // small synchronous helpers (orbit generation, counts)
    unsigned char *scratch = nullptr;   // device address of the static array of gc_launch_static
    std::vector<int> stream_load;
    Pool pool;
    PinnedPool pinned;
    std::vector<hipEvent_t> events, events_nt;   // reusable timing / non-timing events
    std::mutex mu;
    std::condition_variable cv;       // wakes the scheduler
    std::condition_variable done_cv;  // wakes waiters
    std::thread sched;
    bool stop = false;
    bool failed = false;
    std::string err;
    uint64_t next_handle = 1;
    std::map<gc_orbit, std::unique_ptr<Orbit>> orbits;
    std::deque<Job *> queued;
    std::vector<Job *> running;
};

namespace {

gc_status fail(gc_ctx *c, hipError_t e, const char *what)
{
    c->failed = true;
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    c->err = buf;
    return GC_EDEVICE;
}

#define GC_HIP(call)                                       \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return fail(ctx, e_, #call); \
    } while (0)

// Build and upload the geometry tables of an orbit.
gc_status build_orbit(gc_ctx *ctx, Orbit *o)
{
    const int d = o->d, V = o->V;
    const int *n = o->lat.extent;
    int stride[4];
    stride[0] = 1;
    for (int mu = 1; mu < d; ++mu) stride[mu] = stride[mu - 1] * n[mu - 1];
    std::vector<int> coord((size_t)V * d);
    for (int i = 0; i < V; ++i) {
        int r = i;
        for (int mu = 0; mu < d; ++mu) {
            coord[(size_t)i * d + mu] = r % n[mu];
            r /= n[mu];
        }
    }
    std::vector<uint16_t> nbr((size_t)2 * d * V);
    std::vector<int> col(V);
    for (int i = 0; i < V; ++i) {
        int sum = 0;
        for (int mu = 0; mu < d; ++mu) {
            const int x = coord[(size_t)i * d + mu];
            sum += x;
            const int xf = (x + 1) % n[mu], xb = (x + n[mu] - 1) % n[mu];
            nbr[(size_t)mu * V + i] = (uint16_t)(i + (xf - x) * stride[mu]);
            nbr[(size_t)(d + mu) * V + i] = (uint16_t)(i + (xb - x) * stride[mu]);
        }
        col[i] = sum % o->K;
    }
    std::vector<int32_t> coff(o->K + 1, 0);
    std::vector<uint16_t> perm;
    perm.reserve(V);
    for (int c = 0; c < o->K; ++c) {
        coff[c] = (int32_t)perm.size();
        for (int i = 0; i < V; ++i)
            if (col[i] == c) perm.push_back((uint16_t)i);
    }
    coff[o->K] = V;
    // antiperiodic gauge transformations in direction mu are the periodic
    // problem with U -> -U on the links that wrap around mu, i.e. phi + pi
    // there: that angle enters U and the plaquette and line sums of the key
    std::vector<double> pe(o->phi);
    for (int mu = 0; mu < d; ++mu) {
        if (!((o->lat.antiperiodic >> mu) & 1u)) continue;
        for (int i = 0; i < V; ++i)
            if (coord[(size_t)i * d + mu] == n[mu] - 1) pe[(size_t)mu * V + i] += kPiD;
    }
    std::vector<double2> U64((size_t)d * V);
    std::vector<float2> U32((size_t)d * V);
    for (size_t l = 0; l < (size_t)d * V; ++l) {
        U64[l] = make_double2(std::cos(pe[l]), std::sin(pe[l]));
        U32[l] = make_float2((float)U64[l].x, (float)U64[l].y);
    }
    GcOrbitDev &D = o->dev;
    memset(&D, 0, sizeof D);
    D.d = d;
    D.V = V;
    D.K = o->K;
    for (int mu = 0; mu < d; ++mu) D.ext[mu] = n[mu];
    int np = 0;
    for (int mu = 0; mu < d; ++mu)
        for (int nu = mu + 1; nu < d; ++nu) {
            D.plane_mu[np] = mu;
            D.plane_nu[np] = nu;
            ++np;
        }
    D.n_plaq = np * V;
    std::vector<double> phi_plaq((size_t)D.n_plaq);
    const double *phi = pe.data();
    for (int p = 0; p < np; ++p) {
        const int mu = D.plane_mu[p], nu = D.plane_nu[p];
        for (int i = 0; i < V; ++i) {
            const int fm = nbr[(size_t)mu * V + i], fn = nbr[(size_t)nu * V + i];
            double s = phi[(size_t)mu * V + i] + phi[(size_t)nu * V + fm];
            s = s - phi[(size_t)mu * V + fn];
            s = s - phi[(size_t)nu * V + i];
            phi_plaq[(size_t)p * V + i] = s;
        }
    }
    std::vector<double> phi_line;
    std::vector<uint16_t> line_site;
    for (int mu = 0; mu < d; ++mu) {
        D.line_off[mu] = (int32_t)line_site.size();
        for (int i0 = 0; i0 < V; ++i0) {
            if (coord[(size_t)i0 * d + mu] != 0) continue;
            double s = 0.0;
            int i = i0;
            for (int t = 0; t < n[mu]; ++t) {
                s = s + phi[(size_t)mu * V + i];
                i = nbr[(size_t)mu * V + i];
            }
            line_site.push_back((uint16_t)i0);
            phi_line.push_back(s);
        }
    }
    D.line_off[d] = (int32_t)line_site.size();
    D.n_lines = (int32_t)line_site.size();
    D.n_elems = D.n_plaq + D.n_lines;
    D.orbit_index = o->orbit_index;

    // one device block for every table
    size_t off = 0;
    auto place = [&](size_t bytes) { size_t at = off; off = align_up(off + bytes, 256); return at; };
    const size_t o_coff = place(coff.size() * 4), o_perm = place(perm.size() * 2), o_nbr = place(nbr.size() * 2);
    const size_t o_u64 = place(U64.size() * 16), o_u32 = place(U32.size() * 8);
    const size_t o_pp = place(phi_plaq.size() * 8 + 8), o_pl = place(phi_line.size() * 8 + 8);
    const size_t o_ls = place(line_site.size() * 2 + 2);
    std::vector<unsigned char> host(off, 0);
    memcpy(&host[o_coff], coff.data(), coff.size() * 4);
    memcpy(&host[o_perm], perm.data(), perm.size() * 2);
    memcpy(&host[o_nbr], nbr.data(), nbr.size() * 2);
    memcpy(&host[o_u64], U64.data(), U64.size() * 16);
    memcpy(&host[o_u32], U32.data(), U32.size() * 8);
    if (!phi_plaq.empty()) memcpy(&host[o_pp], phi_plaq.data(), phi_plaq.size() * 8);
    memcpy(&host[o_pl], phi_line.data(), phi_line.size() * 8);
    memcpy(&host[o_ls], line_site.data(), line_site.size() * 2);
    void *dev = nullptr;
    size_t got = 0;
    GC_HIP(ctx->pool.get(off, &dev, &got));
    o->tables = dev;
    o->table_bytes = got;
    GC_HIP(hipMemcpy(dev, host.data(), off, hipMemcpyHostToDevice));
    unsigned char *b = (unsigned char *)dev;
    D.coff = (const int32_t *)(b + o_coff);
    D.perm = (const uint16_t *)(b + o_perm);
    D.nbr = (const uint16_t *)(b + o_nbr);
    D.U64 = (const double2 *)(b + o_u64);
    D.U32 = (const float2 *)(b + o_u32);
    D.phi_plaq = (const double *)(b + o_pp);
    D.phi_line = (const double *)(b + o_pl);
    D.line_site = (const uint16_t *)(b + o_ls);
    memset(&o->wdev, 0, sizeof o->wdev);
    if (o->K == 2) {
        // colour-split tables: (c, h) with c the colour, h = i >> 1
        const int half = V / 2;
        std::vector<uint16_t> loc(V);
        std::vector<int> site((size_t)2 * half, -1);
        for (int i = 0; i < V; ++i) {
            loc[i] = (uint16_t)(col[i] * half + (i >> 1));
            site[(size_t)col[i] * half + (i >> 1)] = i;
        }
        std::vector<uint16_t> nb((size_t)2 * half * 8, 0);
        std::vector<double2> c64((size_t)2 * 2 * d * half);
        std::vector<float2> c32((size_t)2 * 2 * d * half);
        const bool scaled = 16 * (size_t)half <= 0xFFFF;
        std::vector<uint16_t> nbo(scaled ? (size_t)2 * half * 8 : 0, 0), nbo32(scaled ? (size_t)2 * half * 8 : 0, 0);
        std::vector<double2> l64((size_t)2 * d * half);
        std::vector<float2> l32((size_t)2 * d * half);
        for (int c = 0; c < 2; ++c)
            for (int h = 0; h < half; ++h) {
                const int i = site[(size_t)c * half + h];
                for (int k = 0; k < 2 * d; ++k) {
                    const int mu = k < d ? k : k - d;
                    const int nsite = k < d ? nbr[(size_t)mu * V + i] : nbr[(size_t)(d + mu) * V + i];
                    nb[((size_t)c * half + h) * 8 + k] = (uint16_t)(nsite >> 1);
                    if (scaled) {
                        nbo[((size_t)c * half + h) * 8 + k] = (uint16_t)(16 * (nsite >> 1));
                        nbo32[((size_t)c * half + h) * 8 + k] = (uint16_t)(8 * (nsite >> 1));
                    }
                    double2 u;
                    if (k < d) {
                        u = U64[(size_t)mu * V + i];
                        l64[((size_t)c * d + mu) * half + h] = u;
                        l32[((size_t)c * d + mu) * half + h] = make_float2((float)u.x, (float)u.y);
                    } else {
                        u = U64[(size_t)mu * V + nsite];
                        u.y = -u.y;
                    }
                    c64[((size_t)c * 2 * d + k) * half + h] = u;
                    c32[((size_t)c * 2 * d + k) * half + h] = make_float2((float)u.x, (float)u.y);
                }
            }
        size_t woff = 0;
        auto wplace = [&](size_t bytes) { size_t at = woff; woff = align_up(woff + bytes, 256); return at; };
        const size_t w_loc = wplace(loc.size() * 2), w_nb = wplace(nb.size() * 2), w_c64 = wplace(c64.size() * 16),
                     w_c32 = wplace(c32.size() * 8),
                     w_nbo = wplace(nbo.size() * 2), w_nbo32 = wplace(nbo32.size() * 2), w_l64 = wplace(l64.size() * 16), w_l32 = wplace(l32.size() * 8);
        std::vector<unsigned char> wh(woff, 0);
        memcpy(&wh[w_loc], loc.data(), loc.size() * 2);
        memcpy(&wh[w_nb], nb.data(), nb.size() * 2);
        memcpy(&wh[w_c64], c64.data(), c64.size() * 16);
        memcpy(&wh[w_c32], c32.data(), c32.size() * 8);
        if (scaled) {
            memcpy(&wh[w_nbo], nbo.data(), nbo.size() * 2);
            memcpy(&wh[w_nbo32], nbo32.data(), nbo32.size() * 2);
        }
        memcpy(&wh[w_l64], l64.data(), l64.size() * 16);
        memcpy(&wh[w_l32], l32.data(), l32.size() * 8);
        void *wdevmem = nullptr;
        GC_HIP(ctx->pool.get(woff, &wdevmem, &got));
        o->wave_tables = wdevmem;
        o->wave_bytes = got;
        GC_HIP(hipMemcpy(wdevmem, wh.data(), woff, hipMemcpyHostToDevice));
        unsigned char *wb = (unsigned char *)wdevmem;
        o->wdev.half = half;
        o->wdev.loc = (const uint16_t *)(wb + w_loc);
        o->wdev.nb = (const uint4 *)(wb + w_nb);
        o->wdev.coef64 = (const double2 *)(wb + w_c64);
        o->wdev.coef32 = (const float2 *)(wb + w_c32);
        o->wdev.nbo = scaled ? (const uint4 *)(wb + w_nbo) : nullptr;
        o->wdev.nbo32 = scaled ? (const uint4 *)(wb + w_nbo32) : nullptr;
        o->wdev.link64 = (const double2 *)(wb + w_l64);
        o->wdev.link32 = (const float2 *)(wb + w_l32);
    }
    return GC_OK;
}

// Device block from the context's pool; on exhaustion the cached blocks are
// returned to the device once and the request retried.  Out of memory is
// GC_ENOMEM (the context stays usable).
gc_status pool_get(gc_ctx *ctx, size_t bytes, void **p, size_t *got)
{
    hipError_t e = ctx->pool.get(bytes, p, got);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
        (void)hipGetLastError();
        ctx->pool.drain();
        e = ctx->pool.get(bytes, p, got);
    }
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
        (void)hipGetLastError();
        *p = nullptr;
        return GC_ENOMEM;
    }
    if (e != hipSuccess) return fail(ctx, e, "hipMalloc");
    return GC_OK;
}

hipEvent_t take_event(gc_ctx *ctx, bool timing)
{
    std::vector<hipEvent_t> &v = timing ? ctx->events : ctx->events_nt;
    if (!v.empty()) {
        hipEvent_t e = v.back();
        v.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, timing ? hipEventDefault : hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

void give_event(gc_ctx *ctx, hipEvent_t &e, bool timing)
{
    if (e) (timing ? ctx->events : ctx->events_nt).push_back(e);
    e = nullptr;
}

// The instantiated slot count of the one-wavefront kernel for ns slots per
// lane (orbits of one bucket share a kernel).
int ns_bucket(int d, int ns)
{
    static const int b1[] = {1, 4, 12, 16}, b2[] = {1, 2, 4, 12, 16}, b3[] = {2, 4, 8, 16}, b4[] = {1, 2, 4, 11, 16};
    const int *b = d == 1 ? b1 : d == 2 ? b2 : d == 3 ? b3 : b4;
    const int nb = d == 1 ? 4 : d == 2 ? 5 : d == 3 ? 4 : 5;
    for (int k = 0; k < nb; ++k)
        if (ns <= b[k]) return b[k];
    return 16;
}

// Layout of a job's device block and its launch groups.  Each orbit runs the
// context's tuned kernel variant for its shape unless the job forces one
// (autotune trials).  Orbits are grouped by relax kernel; each group is one
// chain of launches (relax, post, finalize) that a batch runs concurrently
// with the other chains.
gc_status plan_job(gc_ctx *ctx, Job *job, JobLayout &L)
{
    L = JobLayout{};
    const int nj = (int)job->orbits.size();
    const bool mixed = job->p.precision == GC_MIXED;
    size_t off = 0;
    auto place = [&](size_t bytes) { size_t at = off; off = align_up(off + bytes, 256); return at; };
    for (int j = 0; j < nj; ++j) {
        Orbit *o = job->orbits[j];
        const uint64_t n = job->n_starts[j];
        if (o->V > kMaxV) return GC_EUNSUPPORTED;
        const uint64_t cap = next_pow2(std::max<uint64_t>(2 * n, 64));
        L.table_cap.push_back(cap);
        L.o_rec.push_back(place(sizeof(GcStartRec) * n));
        L.o_table.push_back(place(sizeof(GcEntry) * cap));
        L.o_cnt.push_back(place(sizeof(GcCounters)));
        L.o_copies.push_back(place(sizeof(GcCopyRec) * n));
        L.o_ncopies.push_back(place(sizeof(unsigned long long)));
        L.o_blk.push_back(place(sizeof(uint32_t) * ((cap + 255) / 256)));
        L.o_states.push_back(place(sizeof(double2) * n * (uint64_t)o->V));
        L.o_sync.push_back(job->p.sync_batch ? place(sizeof(uint32_t) * n) : 0);
        L.o_theta.push_back(job->theta.empty() ? 0 : place(sizeof(double) * n * (uint64_t)o->V));
        // two colours: one wavefront per start (GC_WAVES states per
        // workgroup in LDS) up to 128 slots per colour, a workgroup of wps
        // wavefronts per start above; other colourings take the generic
        // workgroup kernel
        const int o_ns = (o->V / 2 + 63) / 64;
        int wps = (o->K == 2) ? gc_wps_for(o_ns) : -1;
        if (wps > 0 && (size_t)(GC_WAVES + 1) * 16 * o->V <= ctx->lds_max) {
            // both layouts fit: one wavefront per start (the exchange-region
            // kernel measured several times faster than a workgroup per
            // start, and it keeps one reduction order for a shape), unless
            // the context forces the workgroup layout
            if (ctx->wps_override <= 0) wps = 0;
        }
        if (wps > 0 && 32 * (size_t)o->V > ctx->lds_max) wps = -1;
        const bool wave = (o->K == 2) && wps >= 0 && (wps > 0 || (size_t)(GC_WAVES + 1) * 16 * o->V <= ctx->lds_max);
        // groups by kernel: dimension, layout and instantiated slot count,
        // or (generic) block size; an orbit's arithmetic does not depend on
        // the other orbits of its group
        const int gd = wave ? o->d : -block_for(o->V);
        const int gw = wave ? std::max(wps, 0) : 0;
        const int gb = (wave && gw == 0) ? ns_bucket(o->d, o_ns) : 0;
        Group *g = nullptr;
        for (Group &x : L.groups)
            if (x.wave == wave && x.d == gd && x.wps == gw && x.ns == gb) g = &x;
        if (!g) {
            L.groups.push_back(Group{});
            g = &L.groups.back();
            g->wave = wave;
            g->d = gd;
            g->wps = gw;
            g->ns = gb;
        }
        g->jobs.push_back(j);
        g->total += n;
    }
    for (Group &g : L.groups) {
        int gV = 0;
        for (int j : g.jobs) gV = std::max(gV, job->orbits[j]->V);
        int per_cu = 0;
        if (g.wave && g.wps > 0) {
            g.block = 64 * g.wps;
            g.lds = 32 * (size_t)gV;   // neighbour table + one state
            hipError_t e = gc_wps_occupancy(g.d, g.wps, g.lds, &per_cu);
            if (e != hipSuccess) return fail(ctx, e, "occupancy");
        } else if (g.wave) {
            g.ns = (gV / 2 + 63) / 64;
            g.block = 64 * gc_wave_starts_per_wg(g.ns);
            g.rm = g.ns > 2 ? gc_wave_relax_mode(job->p.omega, job->p.stop_norm) : 0;
            // every orbit fills all slots of a lane but the last: the
            // double-precision kernel tests only the last slot
            if (g.ns > 2) {
                bool full = true;
                for (int j : g.jobs) full = full && (job->orbits[j]->V / 2 + 63) / 64 == ns_bucket(g.d, g.ns);
                g.full = full ? GC_RM_FULL_SLOTS : 0;
            }
            size_t coef_bytes = 0;
            for (int j : g.jobs) {
                const Orbit *o = job->orbits[j];
                coef_bytes = std::max(coef_bytes, (size_t)2 * o->d * o->V * (mixed ? 24 : 16));
            }
            // neighbour table + states (two-colour regions of 16V, or 8V
            // exchange regions of the register-resident kernel) + links
            // staged in LDS
            const size_t states = g.ns > 2 ? gc_rr_lds_bytes(g.d, ns_bucket(g.d, g.ns), gV)
                                           : (size_t)(GC_WAVES + 1) * 16 * gV;
            // a staged coefficient table only where a lane has at most two
            // slots; above, the links are read through buffer loads
            g.coef_lds = (g.ns <= 2 && coef_bytes + states <= 64 * 1024) ? 1 : 0;
            g.lds = states + (g.coef_lds ? coef_bytes : 0);
            if (g.lds > ctx->lds_max) return GC_EUNSUPPORTED;
            // colour-0 coefficients in registers by default where a lane has
            // at most two slots: the uneven 32-orbit batch runs 1.4-2.2 %
            // faster so than with none, though 4^4 alone is faster with none
            // (44.7 against 49.9 ms per step), which the autotuner finds;
            // GC_WAVE_CREG overrides
            g.creg = std::min(1, gc_wave_creg_max(g.d, g.ns));
            const auto tc = ctx->tune_creg.find(creg_key(g.d, g.ns, mixed));
            if (tc != ctx->tune_creg.end()) g.creg = std::min(tc->second, gc_wave_creg_max(g.d, g.ns));
            if (ctx->creg_override >= 0) g.creg = std::min(ctx->creg_override, gc_wave_creg_max(g.d, g.ns));
            if (job->force_creg >= 0) g.creg = std::min(job->force_creg, gc_wave_creg_max(g.d, g.ns));
            hipError_t e = gc_wave_occupancy(g.d, g.ns, wave_variant(g), g.lds, &per_cu);
            if (e != hipSuccess) return fail(ctx, e, "occupancy");
            if (g.ns > 2 && mixed) {
                g.split = 1;
                g.lds32 = gc_rr32_lds_bytes(g.d, ns_bucket(g.d, g.ns), gV);
                if (g.lds32 > ctx->lds_max) return GC_EUNSUPPORTED;
                int pc32 = 0;
                e = gc_wave32_occupancy(g.d, g.ns, g.rm, g.lds32, &pc32);
                if (e != hipSuccess) return fail(ctx, e, "occupancy");
                pc32 = std::max(pc32, 1);
                g.grid32 = (int)std::min<uint64_t>((uint64_t)pc32 * ctx->n_cu,
                                                   std::max<uint64_t>((g.total + GC_WAVES_RR32 - 1) / GC_WAVES_RR32, 1));
            }
        } else {
            g.block = block_for(gV);
            g.lds = gc_relax_wg_lds_bytes(gV);
            if (g.lds > ctx->lds_max) return GC_EUNSUPPORTED;
            hipError_t e = gc_relax_wg_occupancy(g.block, g.lds, &per_cu);
            if (e != hipSuccess) return fail(ctx, e, "occupancy");
        }
        per_cu = std::max(per_cu, 1);
        const uint64_t per_wg = (g.wave && g.wps == 0) ? (uint64_t)gc_wave_starts_per_wg(g.ns) : 1;
        uint64_t grid = (uint64_t)per_cu * (uint64_t)ctx->n_cu;
        grid = std::min<uint64_t>(grid, std::max<uint64_t>((g.total + per_wg - 1) / per_wg, 1));
        g.grid = (int)grid;
        g.o_jobs = place(sizeof(GcJobDev) * g.jobs.size());
        g.o_jobs1 = job->p.sync_batch ? place(sizeof(GcJobDev) * g.jobs.size()) : 0;
        g.o_worbs = place(sizeof(GcWaveOrbit) * g.jobs.size());
        g.o_next = place(sizeof(unsigned long long) * g.jobs.size());
        g.o_prefix = place(sizeof(uint64_t) * (g.jobs.size() + 1));
        // promotion scratch of the two-region kernels (the register-resident
        // kernel promotes in registers)
        g.o_bounce = (g.wave && (g.wps > 0 || g.ns <= 2)) ? place(sizeof(float2) * (size_t)gV * per_wg * g.grid) : 0;
    }
    // key pass: one workgroup per start, one launch per workgroup shape
    // within each relax group's chain; filter pass: one workgroup per copy,
    // one launch per kernel shape within the chain.  Both shapes depend on
    // the lattice only, so an orbit's results do not depend on tuning or on
    // the other orbits of a batch.
    const int lmax = (int)std::min<uint32_t>(std::max<uint32_t>(job->p.lanczos_max_iter, 1), GC_LMAX);
    for (size_t gi = 0; gi < L.groups.size(); ++gi) {
        for (int j : L.groups[gi].jobs) {
            const Orbit *o = job->orbits[j];
            int block = 0, sp = 0, wreg = 0;
            gc_post_shape(o->V, &block, &sp, &wreg);
            if (block == 0) return GC_EUNSUPPORTED;
            int k = 0;
            while (k < (int)L.posts.size() && !(L.posts[k].chain == (int)gi && L.posts[k].block == block &&
                                                L.posts[k].sp == sp && L.posts[k].wreg == wreg))
                ++k;
            if (k == (int)L.posts.size()) {
                L.posts.push_back(PostGroup{});
                L.posts[k].block = block;
                L.posts[k].sp = sp;
                L.posts[k].wreg = wreg;
                L.posts[k].chain = (int)gi;
            }
            L.posts[k].jobs.push_back(j);
            L.posts[k].total += job->n_starts[j];
            // filter: the line-segment kernel where one is instantiated and
            // fits, else the general kernel with the key pass's shape
            FilterGroup f;
            f.chain = (int)gi;
            int fb = 0, fs = 0;
            if (gc_lanczos_shape(o->d, o->lat.extent, o->V, &fb, &fs) &&
                gc_lanczos_lds_bytes(o->d, o->lat.extent[0], fs, o->V, lmax, fb) <= ctx->lds_max) {
                f.fast = true;
                f.d = o->d;
                f.form = gc_lanczos_form(o->lat.extent[0], fs, o->V, fb);
                f.block = fb;
                f.seg = fs;
            } else {
                f.block = block;
                f.sp = sp;
                f.wreg = wreg;
            }
            int m = 0;
            while (m < (int)L.filters.size() &&
                   !(L.filters[m].chain == f.chain && L.filters[m].fast == f.fast && L.filters[m].d == f.d &&
                     L.filters[m].form == f.form &&
                     L.filters[m].block == f.block && L.filters[m].seg == f.seg && L.filters[m].sp == f.sp &&
                     L.filters[m].wreg == f.wreg))
                ++m;
            if (m == (int)L.filters.size()) L.filters.push_back(f);
            L.filters[m].jobs.push_back(j);
            L.filters[m].total += job->n_starts[j];
        }
    }
    for (PostGroup &pg : L.posts) {
        int pV = 0, pd = 0;
        for (int j : pg.jobs) {
            pV = std::max(pV, job->orbits[j]->V);
            pd = std::max(pd, job->orbits[j]->d);
        }
        pg.lds = gc_post_lds_bytes(pd, pV, 1, lmax);
        if (pg.lds > ctx->lds_max) return GC_EUNSUPPORTED;
        int per_cu = 0;
        hipError_t e = gc_post_occupancy(pg.block, pg.sp, pg.wreg, 1, pg.lds, &per_cu);
        if (e != hipSuccess) return fail(ctx, e, "occupancy");
        per_cu = std::max(per_cu, 1);
        pg.grid = (int)std::min<uint64_t>((uint64_t)per_cu * ctx->n_cu, std::max<uint64_t>(pg.total, 1));
        pg.o_jobs = place(sizeof(GcJobDev) * pg.jobs.size());
        pg.o_prefix = place(sizeof(uint64_t) * (pg.jobs.size() + 1));
        pg.o_next = place(sizeof(unsigned long long));
    }
    for (FilterGroup &fg : L.filters) {
        size_t lds = 0;
        int fV = 0, fd = 0;
        for (int j : fg.jobs) {
            const Orbit *o = job->orbits[j];
            fV = std::max(fV, o->V);
            fd = std::max(fd, o->d);
            lds = std::max(lds, fg.fast ? gc_lanczos_lds_bytes(o->d, o->lat.extent[0], fg.seg, o->V, lmax, fg.block)
                                        : gc_post_lds_bytes(o->d, o->V, 0, lmax));
        }
        if (lds > ctx->lds_max) return GC_EUNSUPPORTED;
        fg.lds = lds;
        int per_cu = 0;
        hipError_t e = fg.fast ? gc_lanczos_occupancy(fg.d, fg.block, fg.seg, fg.form, lds, &per_cu)
                               : gc_post_occupancy(fg.block, fg.sp, fg.wreg, 0, lds, &per_cu);
        if (e != hipSuccess) return fail(ctx, e, "occupancy");
        per_cu = std::max(per_cu, 1);
        fg.grid = (int)std::min<uint64_t>((uint64_t)per_cu * ctx->n_cu, std::max<uint64_t>(fg.total, 1));
        fg.o_jobs = place(sizeof(GcJobDev) * fg.jobs.size());
        fg.o_next = place(sizeof(unsigned long long));
        if (!fg.fast && !fg.wreg) {
            fg.wstride = ((uint64_t)(fd + 3) * fV + 31) & ~(uint64_t)31;
            fg.o_wbuf = place(sizeof(double) * fg.wstride * fg.grid);
        }
    }
    L.total = off;
    return GC_OK;
}

// Return a job's device block, pinned staging, events and graph to the
// context's pools.  Nothing here waits for the device.
void free_job(gc_ctx *ctx, Job *job)
{
    if (job->mem) {
        ctx->pool.put(job->mem, job->bytes);
        job->mem = nullptr;
    }
    if (job->staging) {
        ctx->pinned.put(job->staging, job->staging_bytes);
        job->staging = nullptr;
    }
    give_event(ctx, job->ev_k0, true);
    give_event(ctx, job->ev_k1, true);
    give_event(ctx, job->ev_k2, true);
    give_event(ctx, job->ev_k3, true);
    give_event(ctx, job->ev_done, false);
    if (job->gx) (void)hipGraphExecDestroy(job->gx);
    if (job->g) (void)hipGraphDestroy(job->g);
    job->gx = nullptr;
    job->g = nullptr;
    job->h_cnt = nullptr;
    job->h_ncopies = nullptr;
}

// A job that cannot run: its orbits report GC_ORBIT_ERROR and gc_wait
// returns err.  Its memory goes back to the pools.
void fail_job(gc_ctx *ctx, Job *job, gc_status err)
{
    if (job->mem) ctx->used -= job->bytes;
    free_job(ctx, job);
    job->bytes = 0;
    job->state = GC_ORBIT_ERROR;
    job->err = err;
    for (Orbit *o : job->orbits)
        if (o->job == job) o->last.state = GC_ORBIT_ERROR;
    ctx->done_cv.notify_all();
}

// Host images of a job's per-orbit descriptors, pointing into the block at
// base.
void fill_job_devs(Job *job, unsigned char *base)
{
    const int nj = (int)job->orbits.size();
    const JobLayout &L = job->L;
    job->jobs.assign(nj, GcJobDev{});
    for (int j = 0; j < nj; ++j) {
        Orbit *o = job->orbits[j];
        GcJobDev &J = job->jobs[j];
        memset(&J, 0, sizeof J);
        J.orb = o->dev;
        J.omega = job->p.omega;
        J.eps32 = job->p.eps32;
        J.eps64 = job->p.eps64;
        J.lambda_tol = job->p.lambda_tol;
        J.precision = job->p.precision;
        J.stop_norm = job->p.stop_norm;
        J.check_every = (int32_t)std::max<uint32_t>(job->p.check_every, 1);
        J.lanczos_max = (int32_t)std::min<uint32_t>(std::max<uint32_t>(job->p.lanczos_max_iter, 1), GC_LMAX);
        J.max_sweeps = job->p.max_sweeps;
        J.start_seed = job->p.start_seed;
        J.first_start = job->p.first_start;
        J.n_starts = job->n_starts[j];
        J.rec = (GcStartRec *)(base + L.o_rec[j]);
        J.table = (GcEntry *)(base + L.o_table[j]);
        J.table_mask = L.table_cap[j] - 1;
        J.cnt = (GcCounters *)(base + L.o_cnt[j]);
        J.copies = (GcCopyRec *)(base + L.o_copies[j]);
        J.n_copies = (unsigned long long *)(base + L.o_ncopies[j]);
        J.states = (double2 *)(base + L.o_states[j]);
        J.blk = (uint32_t *)(base + L.o_blk[j]);
        J.sync_batch = job->p.sync_batch;
        J.fixed_sweeps = job->p.sync_batch ? (uint32_t *)(base + L.o_sync[j]) : nullptr;
        J.theta_init = job->theta.empty() ? nullptr : (const double *)(base + L.o_theta[j]);
    }
}

// Descriptor arrays the kernels of a job read, each with its offset in the
// job's block: the fix-up pass's job, the post groups' and relax groups' job
// arrays and start prefixes, the wave tables.
struct Blob {
    size_t dst;
    std::vector<unsigned char> bytes;
};

std::vector<Blob> job_blobs(Job *job)
{
    const JobLayout &L = job->L;
    std::vector<Blob> blobs;
    auto add_blob = [&](size_t dst, const void *src, size_t bytes) {
        blobs.push_back(Blob{dst, std::vector<unsigned char>((const unsigned char *)src, (const unsigned char *)src + bytes)});
    };
    if (!job->theta.empty()) add_blob(L.o_theta[0], job->theta.data(), sizeof(double) * job->theta.size());
    for (const FilterGroup &fg : L.filters) {
        std::vector<GcJobDev> fj;
        for (int j : fg.jobs) fj.push_back(job->jobs[j]);
        add_blob(fg.o_jobs, fj.data(), sizeof(GcJobDev) * fj.size());
    }
    for (const PostGroup &pg : L.posts) {
        std::vector<GcJobDev> pj;
        std::vector<uint64_t> pp(1, 0);
        for (int j : pg.jobs) {
            pj.push_back(job->jobs[j]);
            pp.push_back(pp.back() + job->n_starts[j]);
        }
        add_blob(pg.o_jobs, pj.data(), sizeof(GcJobDev) * pj.size());
        add_blob(pg.o_prefix, pp.data(), sizeof(uint64_t) * pp.size());
    }
    for (const Group &g : L.groups) {
        std::vector<GcJobDev> gj;
        std::vector<GcWaveOrbit> gw;
        std::vector<uint64_t> gp(1, 0);
        for (int j : g.jobs) {
            gj.push_back(job->jobs[j]);
            gw.push_back(job->orbits[j]->wdev);
            gp.push_back(gp.back() + job->n_starts[j]);
        }
        if (job->p.sync_batch) {
            // first pass: every start stops on its own; second pass: fixed counts
            add_blob(g.o_jobs1, gj.data(), sizeof(GcJobDev) * gj.size());
            for (GcJobDev &J : gj) J.flags |= GC_JOB_SYNC2;
        }
        // split mixed launch: the double-precision kernel resumes the
        // promoted states
        if (g.split)
            for (GcJobDev &J : gj) J.flags |= GC_JOB_FROM32;
        add_blob(g.o_jobs, gj.data(), sizeof(GcJobDev) * gj.size());
        add_blob(g.o_worbs, gw.data(), sizeof(GcWaveOrbit) * gw.size());
        add_blob(g.o_prefix, gp.data(), sizeof(uint64_t) * gp.size());
    }
    return blobs;
}

// One chain of a job: the relax group's kernel, its orbits' post passes,
// their table compaction and representative fix-ups, on stream qs.  timed:
// HIP events around the relax and post kernels (single-orbit launches).
hipError_t enqueue_chain(Job *job, unsigned char *base, int gi, hipStream_t qs, bool timed)
{
    const JobLayout &L = job->L;
    const Group &g = L.groups[gi];
    hipError_t e = hipSuccess;
    for (int j : g.jobs) {
        e = gc_launch_reset(&job->jobs[j], 1, qs);
        if (e != hipSuccess) return e;
    }
    e = gc_launch_zero_u64((unsigned long long *)(base + g.o_next), (int)g.jobs.size(), qs);
    if (e != hipSuccess) return e;
    for (const PostGroup &pg : L.posts) {
        if (pg.chain != gi) continue;
        e = gc_launch_zero_u64((unsigned long long *)(base + pg.o_next), 1, qs);
        if (e != hipSuccess) return e;
    }
    for (const FilterGroup &fg : L.filters) {
        if (fg.chain != gi) continue;
        e = gc_launch_zero_u64((unsigned long long *)(base + fg.o_next), 1, qs);
        if (e != hipSuccess) return e;
    }
    if (timed && (e = hipEventRecord(job->ev_k0, qs)) != hipSuccess) return e;
    auto relax = [&](size_t o_jobs) -> hipError_t {
        if (g.wave && g.wps > 0)
            return gc_launch_wps(g.d, g.wps, (const GcJobDev *)(base + o_jobs),
                                 (const GcWaveOrbit *)(base + g.o_worbs), (int)g.jobs.size(),
                                 (unsigned long long *)(base + g.o_next), (float2 *)(base + g.o_bounce), g.grid,
                                 g.lds, qs);
        if (g.wave && g.split) {
            // single precision, then double precision from the promoted states
            hipError_t e2 = gc_launch_wave32(g.d, g.ns, (const GcJobDev *)(base + o_jobs),
                                             (const GcWaveOrbit *)(base + g.o_worbs), (int)g.jobs.size(),
                                             (unsigned long long *)(base + g.o_next), g.rm, g.grid32, g.lds32, qs);
            if (e2 == hipSuccess)
                e2 = gc_launch_zero_u64((unsigned long long *)(base + g.o_next), (int)g.jobs.size(), qs);
            if (e2 != hipSuccess) return e2;
        }
        if (g.wave)
            return gc_launch_wave(g.d, g.ns, (const GcJobDev *)(base + o_jobs),
                                  (const GcWaveOrbit *)(base + g.o_worbs), (int)g.jobs.size(),
                                  (unsigned long long *)(base + g.o_next), wave_variant(g),
                                  (float2 *)(base + g.o_bounce), g.grid, g.lds, qs);
        return gc_launch_relax_wg(g.block, (const GcJobDev *)(base + o_jobs), (int)g.jobs.size(),
                                  (const uint64_t *)(base + g.o_prefix), (unsigned long long *)(base + g.o_next),
                                  g.total, g.grid, g.lds, qs);
    };
    if (job->p.sync_batch) {
        // batch-synchronous stop: a first pass finds every start's own
        // stopping sweep, the second runs each batch to its largest
        if ((e = relax(g.o_jobs1)) != hipSuccess) return e;
        for (int j : g.jobs)
            if ((e = gc_launch_sync(&job->jobs[j], 1, qs)) != hipSuccess) return e;
        e = gc_launch_zero_u64((unsigned long long *)(base + g.o_next), (int)g.jobs.size(), qs);
        if (e != hipSuccess) return e;
    }
    if ((e = relax(g.o_jobs)) != hipSuccess) return e;
    if (timed && (e = hipEventRecord(job->ev_k1, qs)) != hipSuccess) return e;
    // key pass over the starts, then each orbit's table compacted in key
    // order, then the filter pass over the copies
    for (const PostGroup &pg : L.posts) {
        if (pg.chain != gi) continue;
        e = gc_launch_post(pg.block, pg.sp, pg.wreg, 1, (const GcJobDev *)(base + pg.o_jobs), (int)pg.jobs.size(),
                           (const uint64_t *)(base + pg.o_prefix), (unsigned long long *)(base + pg.o_next),
                           pg.total, nullptr, 0, pg.grid, pg.lds, qs);
        if (e != hipSuccess) return e;
    }
    for (int j : g.jobs) {
        e = gc_launch_finalize(&job->jobs[j], 1, qs);
        if (e != hipSuccess) return e;
    }
    if (timed && (e = hipEventRecord(job->ev_k2, qs)) != hipSuccess) return e;
    for (const FilterGroup &fg : L.filters) {
        if (fg.chain != gi) continue;
        if (fg.fast)
            e = gc_launch_lanczos(fg.d, fg.block, fg.seg, fg.form, (const GcJobDev *)(base + fg.o_jobs),
                                  (int)fg.jobs.size(),
                                  (unsigned long long *)(base + fg.o_next), fg.grid, fg.lds, qs);
        else
            e = gc_launch_post(fg.block, fg.sp, fg.wreg, 0, (const GcJobDev *)(base + fg.o_jobs), (int)fg.jobs.size(),
                               nullptr, (unsigned long long *)(base + fg.o_next), 0,
                               fg.wreg ? nullptr : (double *)(base + fg.o_wbuf), fg.wstride, fg.grid, fg.lds, qs);
        if (e != hipSuccess) return e;
    }
    if (timed && (e = hipEventRecord(job->ev_k3, qs)) != hipSuccess) return e;
    return hipSuccess;
}

// Enqueue a job's device work on its stream without waiting for anything.
// Caller holds ctx->mu, has charged nothing yet and has picked an idle
// stream.  A batch (job->graph) is captured once into a HIP graph whose
// relax groups run as concurrent branches; relaunching the same batch
// replays that graph on the same device block.
gc_status start_job(gc_ctx *ctx, Job *job)
{
    hipStream_t s = ctx->streams[job->stream];
    const int nj = (int)job->orbits.size();
    if (job->gx) {
        // replay: the captured graph rewrites its own descriptors and resets
        ctx->used += job->bytes;
        ctx->stream_load[job->stream]++;
        GC_HIP(hipEventRecord(job->ev_k0, s));
        GC_HIP(hipGraphLaunch(job->gx, s));
        GC_HIP(hipEventRecord(job->ev_k1, s));
        GC_HIP(hipEventRecord(job->ev_done, s));
        job->state = GC_ORBIT_RUNNING;
        for (int j = 0; j < nj; ++j) job->orbits[j]->res = job->jobs[j];
        ctx->running.push_back(job);
        return GC_OK;
    }
    JobLayout &L = job->L;
    gc_status st = plan_job(ctx, job, L);
    if (st != GC_OK) return st;
    size_t got = 0;
    st = pool_get(ctx, L.total, &job->mem, &got);
    if (st != GC_OK) return st;
    job->bytes = got;
    ctx->used += job->bytes;
    unsigned char *base = (unsigned char *)job->mem;

    fill_job_devs(job, base);
    job->total = 0;
    for (uint64_t n : job->n_starts) job->total += n;

    // pinned staging: every descriptor array the kernels read, copied to
    // the device block by the stream itself, then the result counters
    struct Piece {
        size_t dst, src, bytes;
    };
    std::vector<Piece> pieces;
    size_t soff = 0;
    auto stage = [&](size_t dst, size_t bytes) {
        pieces.push_back(Piece{dst, soff, bytes});
        soff = align_up(soff + bytes, 64);
        return pieces.back().src;
    };
    const std::vector<Blob> blobs = job_blobs(job);
    for (const Blob &bl : blobs) stage(bl.dst, bl.bytes.size());
    const size_t o_hcnt = soff;
    soff = align_up(soff + sizeof(GcCounters) * nj, 64);
    const size_t o_hnc = soff;
    soff = align_up(soff + sizeof(unsigned long long) * nj, 64);
    {
        hipError_t e = ctx->pinned.get(soff, &job->staging, &job->staging_bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return GC_ENOMEM;
        }
    }
    unsigned char *sb = (unsigned char *)job->staging;
    for (size_t k = 0; k < blobs.size(); ++k) memcpy(sb + pieces[k].src, blobs[k].bytes.data(), blobs[k].bytes.size());
    job->h_cnt = (GcCounters *)(sb + o_hcnt);
    job->h_ncopies = (unsigned long long *)(sb + o_hnc);
    memset(job->h_cnt, 0, sizeof(GcCounters) * nj);
    memset(job->h_ncopies, 0, sizeof(unsigned long long) * nj);

    job->ev_k0 = take_event(ctx, true);
    job->ev_k1 = take_event(ctx, true);
    job->ev_k2 = take_event(ctx, true);
    job->ev_k3 = take_event(ctx, true);
    job->ev_done = take_event(ctx, false);
    if (!job->ev_k0 || !job->ev_k1 || !job->ev_k2 || !job->ev_k3 || !job->ev_done)
        return fail(ctx, hipErrorOutOfMemory, "event");

    const int nchain = (int)L.groups.size();
    const bool fork = job->graph && nchain > 1;
    std::vector<hipEvent_t> fork_ev;
    if (fork) {
        while ((int)ctx->aux.size() < nchain - 1) {
            hipStream_t a = nullptr;
            GC_HIP(hipStreamCreateWithFlags(&a, hipStreamNonBlocking));
            ctx->aux.push_back(a);
        }
        for (int k = 0; k < nchain; ++k) {
            hipEvent_t e = take_event(ctx, false);
            if (!e) return fail(ctx, hipErrorOutOfMemory, "event");
            fork_ev.push_back(e);
        }
    }
    auto enqueue_body = [&](hipStream_t qs) -> hipError_t {
        hipError_t e = hipSuccess;
        for (const Piece &pc : pieces) {
            e = hipMemcpyAsync(base + pc.dst, sb + pc.src, pc.bytes, hipMemcpyHostToDevice, qs);
            if (e != hipSuccess) return e;
        }
        if (!fork) {
            for (int gi = 0; gi < nchain; ++gi) {
                e = enqueue_chain(job, base, gi, qs, !job->graph && nchain == 1);
                if (e != hipSuccess) return e;
            }
        } else {
            if ((e = hipEventRecord(fork_ev[0], qs)) != hipSuccess) return e;
            for (int gi = 1; gi < nchain; ++gi) {
                hipStream_t as = ctx->aux[gi - 1];
                if ((e = hipStreamWaitEvent(as, fork_ev[0], 0)) != hipSuccess) return e;
                if ((e = enqueue_chain(job, base, gi, as, false)) != hipSuccess) return e;
                if ((e = hipEventRecord(fork_ev[gi], as)) != hipSuccess) return e;
            }
            if ((e = enqueue_chain(job, base, 0, qs, false)) != hipSuccess) return e;
            for (int gi = 1; gi < nchain; ++gi)
                if ((e = hipStreamWaitEvent(qs, fork_ev[gi], 0)) != hipSuccess) return e;
        }
        for (int j = 0; j < nj; ++j) {
            e = hipMemcpyAsync(&job->h_cnt[j], job->jobs[j].cnt, sizeof(GcCounters), hipMemcpyDeviceToHost, qs);
            if (e != hipSuccess) return e;
            e = hipMemcpyAsync(&job->h_ncopies[j], job->jobs[j].n_copies, sizeof(unsigned long long),
                               hipMemcpyDeviceToHost, qs);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    if (job->graph) {
        GC_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        hipError_t e = enqueue_body(s);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(s, &g);
        for (hipEvent_t &fe : fork_ev) give_event(ctx, fe, false);
        if (e != hipSuccess) return fail(ctx, e, "batch capture");
        if (e2 != hipSuccess) return fail(ctx, e2, "hipStreamEndCapture");
        job->g = g;
        GC_HIP(hipGraphInstantiate(&job->gx, g, nullptr, nullptr, 0));
        GC_HIP(hipEventRecord(job->ev_k0, s));
        GC_HIP(hipGraphLaunch(job->gx, s));
        GC_HIP(hipEventRecord(job->ev_k1, s));
    } else {
        hipError_t e = enqueue_body(s);
        if (e != hipSuccess) return fail(ctx, e, "launch");
    }
    GC_HIP(hipEventRecord(job->ev_done, s));
    ctx->stream_load[job->stream]++;
    job->state = GC_ORBIT_RUNNING;
    for (int j = 0; j < nj; ++j) job->orbits[j]->res = job->jobs[j];
    ctx->running.push_back(job);
    return GC_OK;
}

// Budget charge of a queued job (computed without allocating).
gc_status job_bytes(gc_ctx *ctx, Job *job, size_t *bytes)
{
    if (job->gx) {
        *bytes = job->bytes;
        return GC_OK;
    }
    JobLayout L;
    gc_status st = plan_job(ctx, job, L);
    if (st != GC_OK) return st;
    *bytes = Pool::rounded(L.total);
    return GC_OK;
}

int idle_stream(gc_ctx *ctx)
{
    for (int k = 0; k < (int)ctx->stream_load.size(); ++k)
        if (ctx->stream_load[k] == 0) return k;
    return -1;
}

// Start queued jobs in arrival order while their bytes fit the budget
// (device memory held by running jobs and unreleased results counts) and a
// stream is idle.  Never waits for the device.
void admit_locked(gc_ctx *ctx)
{
    while (!ctx->queued.empty() && !ctx->failed) {
        Job *job = ctx->queued.front();
        size_t need = 0;
        gc_status st = job_bytes(ctx, job, &need);
        if (st != GC_OK) {
            ctx->queued.pop_front();
            fail_job(ctx, job, st);
            continue;
        }
        if (ctx->used + need > ctx->budget) break;
        const int si = idle_stream(ctx);
        if (si < 0) break;
        ctx->queued.pop_front();
        job->stream = si;
        st = start_job(ctx, job);
        if (st != GC_OK) fail_job(ctx, job, st);
        else ctx->cv.notify_all();   // the scheduler watches running jobs
    }
}

// A finished job: its counters are on the host; the results stay in its
// block (and count against the budget) until the orbits are released or
// relaunched.
void complete_locked(gc_ctx *ctx, Job *job)
{
    job->t_done = Clock::now();
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, job->ev_k0, job->ev_k1) == hipSuccess) job->solve_ms = ms;
    if (!job->graph && hipEventElapsedTime(&ms, job->ev_k1, job->ev_k2) == hipSuccess) job->post_ms = ms;
    if (!job->graph && hipEventElapsedTime(&ms, job->ev_k2, job->ev_k3) == hipSuccess) job->filter_ms = ms;
    job->state = GC_ORBIT_DONE;
    ctx->stream_load[job->stream]--;
    for (size_t j = 0; j < job->orbits.size(); ++j) {
        Orbit *o = job->orbits[j];
        if (o->job != job) continue;
        gc_progress &P = o->last;
        const GcCounters &c = job->h_cnt[j];
        P.state = GC_ORBIT_DONE;
        P.n_starts = job->n_starts[j];
        P.starts_done = c.starts_done;
        P.converged = c.converged;
        P.nonconverged = c.nonconverged;
        P.distinct = job->h_ncopies[j];
        P.sweeps_total = c.sweeps_total;
        P.site_updates = c.sweeps_total * (uint64_t)o->V;
        P.lanczos_runs = c.lanczos_runs;
        P.submit_to_done_ms = ms_since(job->t_submit, job->t_done);
        P.device_ms = job->solve_ms;
        P.post_ms = job->post_ms;
        P.filter_ms = job->filter_ms;
        if (c.errors) {
            ctx->failed = true;
            ctx->err = "copy table insert failed (table full or spin limit)";
        }
    }
}

void scheduler_main(gc_ctx *ctx)
{
    (void)hipSetDevice(ctx->device);
    std::unique_lock<std::mutex> lk(ctx->mu);
    while (!ctx->stop) {
        if (ctx->running.empty()) {
            ctx->cv.wait(lk);
            continue;
        }
        bool changed = false;
        for (size_t k = 0; k < ctx->running.size();) {
            Job *job = ctx->running[k];
            hipError_t q = hipEventQuery(job->ev_done);
            if (q == hipSuccess) {
                complete_locked(ctx, job);
                ctx->running.erase(ctx->running.begin() + k);
                changed = true;
            } else if (q != hipErrorNotReady) {
                fail(ctx, q, "kernel");
                job->state = GC_ORBIT_ERROR;
                job->err = GC_EDEVICE;
                ctx->running.erase(ctx->running.begin() + k);
                changed = true;
            } else {
                ++k;
            }
        }
        if (changed) {
            admit_locked(ctx);
            ctx->done_cv.notify_all();
        }
        ctx->cv.wait_for(lk, std::chrono::microseconds(100));
    }
}

Orbit *find_orbit(gc_ctx *ctx, gc_orbit h)
{
    auto it = ctx->orbits.find(h);
    return it == ctx->orbits.end() ? nullptr : it->second.get();
}

// Release the results a finished job keeps for one orbit; the job's block is
// returned to the pool (and stops counting against the budget) once no orbit
// refers to it.
void drop_results_locked(gc_ctx *ctx, Orbit *o)
{
    Job *job = o->job;
    if (!job) return;
    o->job = nullptr;
    o->have_copies = false;
    o->have_starts = false;
    o->copies.clear();
    o->starts.clear();
    bool still_used = false;
    for (auto &kv : ctx->orbits)
        if (kv.second->job == job) still_used = true;
    if (!still_used) {
        if (job->mem) ctx->used -= job->bytes;
        free_job(ctx, job);
        delete job;
    }
}

gc_status wait_locked(gc_ctx *ctx, std::unique_lock<std::mutex> &lk, Orbit *o, int64_t timeout_ms)
{
    Job *job = o->job;
    if (!job) return GC_ESTATE;
    // a queued job with nothing running waits for memory that only
    // gc_release (or another launch replacing results) can free
    auto stalled = [&] { return job->state == GC_ORBIT_QUEUED && ctx->running.empty(); };
    auto pred = [&] {
        return ctx->failed || job->state == GC_ORBIT_DONE || job->state == GC_ORBIT_ERROR || stalled();
    };
    if (timeout_ms < 0) {
        ctx->done_cv.wait(lk, pred);
    } else if (!ctx->done_cv.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred)) {
        return GC_ETIMEOUT;
    }
    if (ctx->failed) return GC_EDEVICE;
    if (job->state == GC_ORBIT_ERROR) return job->err != GC_OK ? job->err : GC_EDEVICE;
    if (stalled()) return GC_ENOMEM;
    return GC_OK;
}

void fill_defaults(gc_solve_params *p)
{
    memset(p, 0, sizeof *p);
    p->omega = 1.0;
    p->eps32 = 1e-6;
    p->eps64 = 1e-14;
    p->lambda_tol = 1e-6;
    p->precision = GC_FP64;
    p->stop_norm = GC_MEAN_SQ;
    p->check_every = 1;
    p->lanczos_max_iter = 300;
    p->max_sweeps = 100000;
    p->start_seed = 0;
    p->first_start = 0;
    p->sync_batch = 0;
}

gc_status check_params(const gc_solve_params *p)
{
    if (!(p->omega > 0.0 && p->omega < 2.0)) return GC_EINVAL;
    if (!(p->eps64 > 0.0) || !(p->eps32 > 0.0) || !std::isfinite(p->eps64) || !std::isfinite(p->eps32)) return GC_EINVAL;
    if (p->precision != GC_FP64 && p->precision != GC_MIXED) return GC_EINVAL;
    if (p->stop_norm != GC_MEAN_SQ && p->stop_norm != GC_MAX_ABS) return GC_EINVAL;
    if (p->max_sweeps < 1 || p->max_sweeps > 0xFFFFFFFFull) return GC_EINVAL;
    if (!(p->lambda_tol >= 0.0)) return GC_EINVAL;
    if (p->sync_batch && p->precision != GC_FP64) return GC_EINVAL;
    return GC_OK;
}

gc_status new_orbit(gc_ctx *ctx, const gc_lattice *lat, std::vector<double> &&phi, uint64_t orbit_index,
                    gc_orbit *out)
{
    int K = 0, V = 0;
    gc_status st = check_lattice(lat, &K, &V);
    if (st != GC_OK) return st;
    if (V > kMaxV || gc_relax_wg_lds_bytes(V) > ctx->lds_max) return GC_EUNSUPPORTED;
    auto o = std::make_unique<Orbit>();
    o->lat = *lat;
    o->d = lat->dim;
    o->V = V;
    o->K = K;
    o->orbit_index = orbit_index;
    o->phi = std::move(phi);
    st = build_orbit(ctx, o.get());
    if (st != GC_OK) {
        if (o->tables) ctx->pool.put(o->tables, o->table_bytes);
        if (o->wave_tables) ctx->pool.put(o->wave_tables, o->wave_bytes);
        return st;
    }
    ctx->used += o->table_bytes + o->wave_bytes;
    o->handle = ctx->next_handle++;
    *out = o->handle;
    ctx->orbits[o->handle] = std::move(o);
    return GC_OK;
}

bool same_params(const gc_solve_params &a, const gc_solve_params &b) { return memcmp(&a, &b, sizeof a) == 0; }

// A batch relaunched with the same orbits, start counts and parameters
// reuses the previous launch's device block and captured graph (the replay
// overwrites the previous results, which the relaunch replaces anyway).
Job *reusable_graph_locked(gc_ctx *ctx, Job *job)
{
    if (!job->graph || job->orbits.empty()) return nullptr;
    Job *prev = job->orbits[0]->job;
    if (!prev || !prev->graph || !prev->gx || prev->state != GC_ORBIT_DONE) return nullptr;
    if (prev->orbits != job->orbits || prev->n_starts != job->n_starts || !same_params(prev->p, job->p)) return nullptr;
    for (Orbit *o : job->orbits)
        if (o->job != prev) return nullptr;
    return prev;
}

gc_status enqueue_locked(gc_ctx *ctx, Job *job)
{
    job->t_submit = Clock::now();
    Job *prev = reusable_graph_locked(ctx, job);
    if (prev) {
        // take over the block, staging, events and graph of the previous launch
        ctx->used -= prev->bytes;
        job->bytes = prev->bytes;
        job->mem = prev->mem;
        job->staging = prev->staging;
        job->staging_bytes = prev->staging_bytes;
        job->ev_k0 = prev->ev_k0;
        job->ev_k1 = prev->ev_k1;
        job->ev_k2 = prev->ev_k2;
        job->ev_k3 = prev->ev_k3;
        job->ev_done = prev->ev_done;
        job->g = prev->g;
        job->gx = prev->gx;
        job->L = prev->L;
        job->jobs = prev->jobs;
        job->h_cnt = prev->h_cnt;
        job->h_ncopies = prev->h_ncopies;
        job->total = prev->total;
        prev->mem = prev->staging = nullptr;
        prev->ev_k0 = prev->ev_k1 = prev->ev_k2 = prev->ev_k3 = prev->ev_done = nullptr;
        prev->g = nullptr;
        prev->gx = nullptr;
        prev->bytes = 0;
    } else {
        size_t need = 0;
        gc_status st = job_bytes(ctx, job, &need);
        if (st != GC_OK) return st;
        if (need > ctx->budget) return GC_ENOMEM;
    }
    for (size_t j = 0; j < job->orbits.size(); ++j) {
        Orbit *o = job->orbits[j];
        drop_results_locked(ctx, o);
        o->job = job;
        o->job_index = (int)j;
        memset(&o->last, 0, sizeof o->last);
        o->last.state = GC_ORBIT_QUEUED;
        o->last.n_starts = job->n_starts[j];
    }
    ctx->queued.push_back(job);
    admit_locked(ctx);
    ctx->cv.notify_all();
    return GC_OK;
}

gc_status ensure_copies_locked(gc_ctx *ctx, Orbit *o)
{
    if (o->have_copies) return GC_OK;
    Job *job = o->job;
    const uint64_t n = job->h_ncopies[o->job_index];
    static_assert(sizeof(GcCopyRec) == sizeof(gc_copy), "copy layout");
    // the copies come in table order, which is key_hi order except where
    // linear probing displaced an entry (past its successors, or around the
    // end of the table): an insertion pass finishes the sort by key
    if (n * sizeof(gc_copy) > o->copies.cap_bytes) {
        // a larger pinned block first, then the old one back to the pool
        void *blk = nullptr;
        size_t got = 0;
        if (ctx->pinned.get(n * sizeof(gc_copy), &blk, &got) != hipSuccess) {
            (void)hipGetLastError();
            ctx->err = "no pinned host memory for the copy table (" + std::to_string(n) + " copies)";
            return GC_ENOMEM;
        }
        ctx->pinned.put(o->copies.p, o->copies.cap_bytes);
        o->copies.p = (gc_copy *)blk;
        o->copies.cap_bytes = got;
    }
    o->copies.n = n;
    if (n) GC_HIP(hipMemcpy(o->copies.data(), o->res.copies, n * sizeof(gc_copy), hipMemcpyDeviceToHost));
    auto less = [](const gc_copy &a, const gc_copy &b) {
        return a.key_hi != b.key_hi ? a.key_hi < b.key_hi : a.key_lo < b.key_lo;
    };
    for (uint64_t k = 1; k < n; ++k) {
        if (!less(o->copies[k], o->copies[k - 1])) continue;
        const gc_copy v = o->copies[k];
        uint64_t m = k;
        while (m > 0 && less(v, o->copies[m - 1])) {
            o->copies[m] = o->copies[m - 1];
            --m;
        }
        o->copies[m] = v;
    }
    uint64_t inr = 0, sad = 0, sng = 0, col = 0, inr_hits = 0, lits = 0;
    for (const gc_copy &c : o->copies) {
        if (c.flags & GC_FLAG_IN_REGION) {
            ++inr;
            inr_hits += c.hits;
        }
        if (c.flags & GC_FLAG_SADDLE) ++sad;
        if (c.flags & GC_FLAG_SINGULAR) ++sng;
        if (c.flags & GC_FLAG_COLLISION) ++col;
        lits += c.lanczos_iters;
    }
    o->last.in_region = inr;
    o->last.in_region_hits = inr_hits;
    o->last.lanczos_iters = lits;
    o->last.saddles = sad;
    o->last.singular = sng;
    o->last.collisions = col;
    o->have_copies = true;
    return GC_OK;
}

gc_status ensure_starts_locked(gc_ctx *ctx, Orbit *o)
{
    if (o->have_starts) return GC_OK;
    const uint64_t n = o->job->n_starts[o->job_index];
    o->starts.resize(n);
    static_assert(sizeof(GcStartRec) == sizeof(gc_start_record), "record layout");
    if (n) GC_HIP(hipMemcpy(o->starts.data(), o->res.rec, n * sizeof(gc_start_record), hipMemcpyDeviceToHost));
    std::vector<uint32_t> xs;
    xs.reserve(n);
    for (const gc_start_record &r : o->starts)
        if (r.status == GC_START_CONVERGED) xs.push_back(r.paper_X);
    std::sort(xs.begin(), xs.end());
    o->paper_count = (uint64_t)(std::unique(xs.begin(), xs.end()) - xs.begin());
    o->last.paper_count = o->paper_count;
    o->have_starts = true;
    return GC_OK;
}

// Create and enqueue a job (caller holds ctx->mu).  force: kernel variants
// of an autotune trial, or NULL.
gc_status launch_locked(gc_ctx *ctx, const std::vector<Orbit *> &orbits, const std::vector<uint64_t> &n_starts,
                        const gc_solve_params &p, bool graph, const Job *force)
{
    for (Orbit *o : orbits)
        if (o->job && (o->job->state == GC_ORBIT_QUEUED || o->job->state == GC_ORBIT_RUNNING)) return GC_EBUSY;
    Job *job = new Job;
    job->orbits = orbits;
    job->n_starts = n_starts;
    job->p = p;
    job->graph = graph;
    if (force) job->force_creg = force->force_creg;
    gc_status st = enqueue_locked(ctx, job);
    if (st != GC_OK) delete job;
    return st;
}

// Tuning cache: one line per choice, "creg <key> <value>".
void load_tune_cache(gc_ctx *ctx)
{
    FILE *f = fopen(ctx->tune_cache.c_str(), "r");
    if (!f) return;
    char kind[16];
    unsigned long long k = 0;
    int a = 0;
    while (fscanf(f, "%15s %llu %d", kind, &k, &a) == 3) {
        if (!strcmp(kind, "creg")) ctx->tune_creg[(uint64_t)k] = a;
        else if (strcmp(kind, "wps")) break;   // layout choices of older caches: no longer tuned
    }
    fclose(f);
}

void save_tune_cache(gc_ctx *ctx)
{
    if (ctx->tune_cache.empty()) return;
    const std::string tmp = ctx->tune_cache + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return;
    for (auto &kv : ctx->tune_creg) fprintf(f, "creg %llu %d\n", (unsigned long long)kv.first, kv.second);
    fclose(f);
    (void)rename(tmp.c_str(), ctx->tune_cache.c_str());
}

// theta_i - theta_{V-1} of one start of the orbit's DONE launch.
gc_status start_state_locked(gc_ctx *ctx, Orbit *o, uint64_t start_id, double *theta_out)
{
    const gc_solve_params &p = o->job->p;
    const uint64_t n = o->job->n_starts[o->job_index];
    if (start_id < p.first_start || start_id - p.first_start >= n) return GC_EINVAL;
    const int V = o->V;
    std::vector<double2> g(V);
    GC_HIP(hipMemcpy(g.data(), o->res.states + (start_id - p.first_start) * (uint64_t)V, sizeof(double2) * V,
                     hipMemcpyDeviceToHost));
    // theta_i - theta_{V-1} = arg(g_i conj(g_{V-1})), exactly 0 at the last site
    const double2 gl = g[V - 1];
    for (int i = 0; i < V; ++i) {
        const double im = g[i].y * gl.x - g[i].x * gl.y;
        const double re = g[i].x * gl.x + g[i].y * gl.y;
        theta_out[i] = std::atan2(im, re);
    }
    return GC_OK;
}

#define GC_ENTER(ctx)                                  \
    if (!(ctx)) return GC_EINVAL;                      \
    std::unique_lock<std::mutex> lk((ctx)->mu);        \
    if ((ctx)->failed) return GC_EDEVICE;              \
    (void)hipSetDevice((ctx)->device)

}  // namespace

extern "C" {

const char *gc_version(void) { return "0.1.0"; }

const char *gc_status_str(gc_status s)
{
    switch (s) {
    case GC_OK: return "ok";
    case GC_EINVAL: return "invalid argument";
    case GC_ENOMEM: return "request exceeds the HBM budget";
    case GC_EUNSUPPORTED: return "unsupported lattice";
    case GC_EDEVICE: return "device error";
    case GC_EBUSY: return "orbit busy";
    case GC_ETIMEOUT: return "timeout";
    case GC_ENOTFOUND: return "not found";
    case GC_ESTATE: return "invalid state";
    default: return "unknown status";
    }
}

gc_status gc_lattice_check(const gc_lattice *lat, int32_t *n_colours)
{
    int K = 0, V = 0;
    gc_status st = check_lattice(lat, &K, &V);
    if (st == GC_OK && V > kMaxV) st = GC_EUNSUPPORTED;
    if (st == GC_OK && n_colours) *n_colours = K;
    return st;
}

gc_status gc_solve_params_default(gc_solve_params *p)
{
    if (!p) return GC_EINVAL;
    fill_defaults(p);
    return GC_OK;
}

gc_status gc_create(const gc_ctx_params *params, gc_ctx **out)
{
    if (!out) return GC_EINVAL;
    *out = nullptr;
    gc_ctx_params P{};
    if (params) P = *params;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return GC_EDEVICE;
    if (P.device < 0 || P.device >= ndev) return GC_EINVAL;
    if (hipSetDevice(P.device) != hipSuccess) return GC_EDEVICE;
    auto ctx = std::make_unique<gc_ctx>();
    ctx->device = P.device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, P.device) != hipSuccess) return GC_EDEVICE;
    ctx->n_cu = prop.multiProcessorCount;
    ctx->lds_max = prop.sharedMemPerBlock;
    if (const char *v = getenv("GC_WAVE_CREG")) ctx->creg_override = atoi(v);
    if (const char *v = getenv("GC_WPS")) ctx->wps_override = atoi(v) != 0 ? 1 : 0;
    ctx->budget = P.hbm_budget_bytes ? P.hbm_budget_bytes : (64ull << 30);
    if (P.hip_stream) {
        ctx->streams.push_back((hipStream_t)P.hip_stream);
        ctx->stream_load.push_back(0);
        ctx->own_streams = false;
    } else {
        const int ns = P.n_streams > 0 ? std::min(P.n_streams, 16) : 4;
        for (int k = 0; k < ns; ++k) {
            hipStream_t s;
            if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return GC_EDEVICE;
            ctx->streams.push_back(s);
            ctx->stream_load.push_back(0);
        }
    }
    if (hipStreamCreateWithFlags(&ctx->util, hipStreamNonBlocking) != hipSuccess) return GC_EDEVICE;
    {
        void *sp = nullptr;
        if (scratch_address(P.device, &sp) != hipSuccess) return GC_EDEVICE;
        ctx->scratch = (unsigned char *)sp;
    }
    if (P.tune_cache) {
        ctx->tune_cache = P.tune_cache;
        load_tune_cache(ctx.get());
    }
    gc_ctx *raw = ctx.release();
    raw->sched = std::thread(scheduler_main, raw);
    *out = raw;
    return GC_OK;
}

gc_status gc_destroy(gc_ctx *ctx)
{
    if (!ctx) return GC_EINVAL;
    {
        std::unique_lock<std::mutex> lk(ctx->mu);
        (void)hipSetDevice(ctx->device);
        for (hipStream_t s : ctx->streams) (void)hipStreamSynchronize(s);
        (void)hipStreamSynchronize(ctx->util);
        ctx->stop = true;
        ctx->cv.notify_all();
    }
    ctx->sched.join();
    (void)hipSetDevice(ctx->device);
    std::vector<Job *> jobs;
    for (auto &kv : ctx->orbits)
        if (kv.second->job && std::find(jobs.begin(), jobs.end(), kv.second->job) == jobs.end())
            jobs.push_back(kv.second->job);
    for (Job *j : ctx->queued)
        if (std::find(jobs.begin(), jobs.end(), j) == jobs.end()) jobs.push_back(j);
    for (Job *j : jobs) {
        free_job(ctx, j);
        delete j;
    }
    for (auto &kv : ctx->orbits) {
        ctx->pool.put(kv.second->tables, kv.second->table_bytes);
        ctx->pool.put(kv.second->wave_tables, kv.second->wave_bytes);
        ctx->pinned.put(kv.second->copies.p, kv.second->copies.cap_bytes);
        kv.second->copies = HostCopies{};
    }
    ctx->pool.drain();
    ctx->pinned.drain();
    for (hipEvent_t e : ctx->events) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->events_nt) (void)hipEventDestroy(e);
    if (ctx->own_streams)
        for (hipStream_t s : ctx->streams) (void)hipStreamDestroy(s);
    for (hipStream_t s : ctx->aux) (void)hipStreamDestroy(s);
    (void)hipStreamDestroy(ctx->util);
    delete ctx;
    return GC_OK;
}

gc_status gc_orbit_load(gc_ctx *ctx, const gc_lattice *lat, const double *phi, uint64_t orbit_index, gc_orbit *out)
{
    if (!lat || !phi || !out) return GC_EINVAL;
    int K = 0, V = 0;
    gc_status st = check_lattice(lat, &K, &V);
    if (st != GC_OK) return st;
    const size_t n = (size_t)lat->dim * V;
    for (size_t l = 0; l < n; ++l)
        if (!std::isfinite(phi[l])) return GC_EINVAL;
    GC_ENTER(ctx);
    std::vector<double> v(phi, phi + n);
    return new_orbit(ctx, lat, std::move(v), orbit_index, out);
}

gc_status gc_orbit_random(gc_ctx *ctx, const gc_lattice *lat, uint64_t seed, uint64_t orbit_index, gc_orbit *out)
{
    if (!lat || !out) return GC_EINVAL;
    int K = 0, V = 0;
    gc_status st = check_lattice(lat, &K, &V);
    if (st != GC_OK) return st;
    GC_ENTER(ctx);
    const int64_t n = (int64_t)lat->dim * V;
    void *blk = nullptr;
    size_t got = 0;
    st = pool_get(ctx, sizeof(double) * n, &blk, &got);
    if (st != GC_OK) return st;
    hipStream_t s = ctx->util;
    hipError_t e = gc_launch_orbit_random((double *)blk, n, seed, orbit_index, s);
    std::vector<double> v(n);
    if (e == hipSuccess) e = hipMemcpyAsync(v.data(), blk, sizeof(double) * n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    ctx->pool.put(blk, got);
    if (e != hipSuccess) return fail(ctx, e, "orbit_random");
    return new_orbit(ctx, lat, std::move(v), orbit_index, out);
}

gc_status gc_orbit_load_su2(gc_ctx *ctx, const gc_lattice *lat, const double *links, uint64_t orbit_index,
                            const gc_mag_params *mp, gc_mag_info *info, gc_orbit *out)
{
    if (!lat || !links || !out) return GC_EINVAL;
    int K = 0, V = 0;
    gc_status st = check_lattice(lat, &K, &V);
    if (st != GC_OK) return st;
    const int d = lat->dim;
    // the checkerboard of even extents, periodic gauge transformations, and
    // the transformations of a configuration held in LDS (32 V bytes)
    for (int mu = 0; mu < d; ++mu)
        if (lat->extent[mu] % 2) return GC_EUNSUPPORTED;
    if (lat->antiperiodic || V > 4096) return GC_EUNSUPPORTED;
    const double eps = mp ? mp->eps : 1e-20;
    const uint64_t cap = mp ? mp->max_sweeps : 100000;
    // at most 10^6 sweeps: about 20 s for the largest supported lattice
    if (!(eps >= 0.0) || !std::isfinite(eps) || cap < 1 || cap > 1000000) return GC_EINVAL;
    const size_t nl = (size_t)d * V;
    for (size_t l = 0; l < nl; ++l) {
        const double *q = links + 4 * l;
        if (!std::isfinite(q[0]) || !std::isfinite(q[1]) || !std::isfinite(q[2]) || !std::isfinite(q[3]))
            return GC_EINVAL;
        if (std::fabs(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3] - 1.0) > 1e-10) return GC_EINVAL;
    }
    // periodic neighbours (x_0 fastest) and the sites of each colour
    std::vector<int> nbr((size_t)2 * d * V), csite;
    csite.reserve(V);
    int stride[4] = {1, 1, 1, 1};
    for (int mu = 1; mu < d; ++mu) stride[mu] = stride[mu - 1] * lat->extent[mu - 1];
    for (int c = 0; c < 2; ++c)
        for (int i = 0; i < V; ++i) {
            int par = 0;
            for (int mu = 0; mu < d; ++mu) par += (i / stride[mu]) % lat->extent[mu];
            if (par % 2 == c) csite.push_back(i);
        }
    for (int mu = 0; mu < d; ++mu)
        for (int i = 0; i < V; ++i) {
            const int n = lat->extent[mu], x = (i / stride[mu]) % n;
            nbr[(size_t)mu * V + i] = i + (((x + 1) % n) - x) * stride[mu];
            nbr[(size_t)(d + mu) * V + i] = i + (((x + n - 1) % n) - x) * stride[mu];
        }
    GC_ENTER(ctx);
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t o_links = 0, o_nbr = al(o_links + 32 * nl), o_cs = al(o_nbr + 4 * nbr.size()),
                 o_phi = al(o_cs + 4 * csite.size()), o_out = al(o_phi + 8 * nl), total = al(o_out + sizeof(GcMagOut));
    void *blk = nullptr;
    size_t got = 0;
    st = pool_get(ctx, total, &blk, &got);
    if (st != GC_OK) return st;
    unsigned char *b = (unsigned char *)blk;
    hipStream_t s = ctx->util;
    std::vector<double> phi(nl);
    GcMagOut mo{};
    // the reduction takes milliseconds: the context stays available meanwhile
    lk.unlock();
    hipError_t e = hipMemcpyAsync(b + o_links, links, 32 * nl, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(b + o_nbr, nbr.data(), 4 * nbr.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(b + o_cs, csite.data(), 4 * csite.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = gc_launch_mag((const double *)(b + o_links), (const int *)(b + o_nbr), (const int *)(b + o_cs), d, V, eps,
                          cap, (double *)(b + o_phi), (GcMagOut *)(b + o_out), s);
    if (e == hipSuccess) e = hipMemcpyAsync(phi.data(), b + o_phi, 8 * nl, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&mo, b + o_out, sizeof mo, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    lk.lock();
    ctx->pool.put(blk, got);
    if (e != hipSuccess) return fail(ctx, e, "maximal Abelian reduction");
    if (ctx->failed) return GC_EDEVICE;
    if (info) {
        info->sweeps = mo.sweeps;
        info->R = mo.R;
        info->converged = mo.converged;
    }
    return new_orbit(ctx, lat, std::move(phi), orbit_index, out);
}

gc_status gc_orbit_angles(gc_ctx *ctx, gc_orbit orbit, double *phi_out)
{
    if (!phi_out) return GC_EINVAL;
    GC_ENTER(ctx);
    Orbit *o = find_orbit(ctx, orbit);
    if (!o) return GC_EINVAL;
    memcpy(phi_out, o->phi.data(), o->phi.size() * sizeof(double));
    return GC_OK;
}

gc_status gc_launch(gc_ctx *ctx, gc_orbit orbit, uint64_t n_starts, const gc_solve_params *params)
{
    gc_solve_params p;
    if (params) p = *params; else fill_defaults(&p);
    gc_status st = check_params(&p);
    if (st != GC_OK) return st;
    if (n_starts == 0 || n_starts > (1ull << 32)) return GC_EINVAL;
    GC_ENTER(ctx);
    Orbit *o = find_orbit(ctx, orbit);
    if (!o) return GC_EINVAL;
    return launch_locked(ctx, {o}, {n_starts}, p, false, nullptr);
}

gc_status gc_launch_from(gc_ctx *ctx, gc_orbit orbit, uint64_t n_starts, const double *theta,
                         const gc_solve_params *params)
{
    gc_solve_params p;
    if (params) p = *params; else fill_defaults(&p);
    gc_status st = check_params(&p);
    if (st != GC_OK) return st;
    if (n_starts == 0 || n_starts > (1ull << 32) || !theta) return GC_EINVAL;
    GC_ENTER(ctx);
    Orbit *o = find_orbit(ctx, orbit);
    if (!o) return GC_EINVAL;
    const size_t n = (size_t)n_starts * (size_t)o->V;
    for (size_t k = 0; k < n; ++k)
        if (!std::isfinite(theta[k])) return GC_EINVAL;
    for (Orbit *x : {o})
        if (x->job && (x->job->state == GC_ORBIT_QUEUED || x->job->state == GC_ORBIT_RUNNING)) return GC_EBUSY;
    Job *job = new Job;
    job->orbits.push_back(o);
    job->n_starts.push_back(n_starts);
    job->p = p;
    job->theta.assign(theta, theta + n);
    st = enqueue_locked(ctx, job);
    if (st != GC_OK) delete job;
    return st;
}

gc_status gc_histogram(gc_ctx *ctx, int32_t n_orbits, const gc_orbit *orbits, int32_t quantity, int32_t weight,
                       uint32_t require_flags, double lo, double hi, int32_t n_bins, uint64_t *counts)
{
    if (n_orbits < 1 || !orbits || !counts || n_bins < 1 || n_bins > (1 << 24) || !(hi > lo) ||
        !std::isfinite(lo) || !std::isfinite(hi) || (quantity != GC_HIST_X && quantity != GC_HIST_REL) ||
        (weight != GC_HIST_COPIES && weight != GC_HIST_STARTS))
        return GC_EINVAL;
    GC_ENTER(ctx);
    std::vector<Orbit *> os;
    for (int32_t k = 0; k < n_orbits; ++k) {
        Orbit *o = find_orbit(ctx, orbits[k]);
        if (!o) return GC_EINVAL;
        if (!o->job || o->job->state != GC_ORBIT_DONE) return GC_ESTATE;
        os.push_back(o);
    }
    const size_t per = (size_t)n_bins + 2;
    void *blk = nullptr;
    size_t got = 0;
    gc_status st = pool_get(ctx, sizeof(unsigned long long) * (per * n_orbits + n_orbits), &blk, &got);
    if (st != GC_OK) return st;
    unsigned long long *cnt = (unsigned long long *)blk, *fmin = cnt + per * n_orbits;
    hipStream_t s = ctx->util;
    hipError_t e = gc_launch_zero_u64(cnt, (int)(per * n_orbits), s);
    const unsigned long long inf_bits = ~0ULL;
    for (int32_t k = 0; k < n_orbits && e == hipSuccess; ++k) {
        e = gc_launch_store(fmin + k, &inf_bits, sizeof inf_bits, s);
        if (e != hipSuccess) break;
        const Orbit *o = os[k];
        e = gc_launch_histogram(o->res.copies, o->res.n_copies, (double)o->d * (double)o->V, quantity,
                                weight == GC_HIST_STARTS, require_flags, lo, hi, n_bins, cnt + per * k, fmin + k, s);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(counts, cnt, sizeof(unsigned long long) * per * n_orbits, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    ctx->pool.put(blk, got);
    if (e != hipSuccess) return fail(ctx, e, "gc_histogram");
    return GC_OK;
}

gc_status gc_launch_batch(gc_ctx *ctx, int32_t n_orbits, const gc_orbit *orbits, const uint64_t *n_starts,
                          const gc_solve_params *params)
{
    if (n_orbits < 1 || n_orbits > 256 || !orbits || !n_starts) return GC_EINVAL;
    gc_solve_params p;
    if (params) p = *params; else fill_defaults(&p);
    gc_status st = check_params(&p);
    if (st != GC_OK) return st;
    GC_ENTER(ctx);
    std::vector<Orbit *> os;
    std::vector<uint64_t> ns;
    for (int k = 0; k < n_orbits; ++k) {
        Orbit *o = find_orbit(ctx, orbits[k]);
        if (!o || n_starts[k] == 0 || n_starts[k] > (1ull << 32)) return GC_EINVAL;
        if (std::find(os.begin(), os.end(), o) != os.end()) return GC_EINVAL;
        os.push_back(o);
        ns.push_back(n_starts[k]);
    }
    return launch_locked(ctx, os, ns, p, true, nullptr);
}

gc_status gc_poll(gc_ctx *ctx, gc_orbit orbit, gc_progress *out)
{
    if (!out) return GC_EINVAL;
    GC_ENTER(ctx);
    Orbit *o = find_orbit(ctx, orbit);
    if (!o) return GC_EINVAL;
    if (!o->job) {
        memset(out, 0, sizeof *out);
        out->state = GC_ORBIT_IDLE;
        return GC_OK;
    }
    if (o->job->state == GC_ORBIT_DONE) {
        gc_status st = ensure_copies_locked(ctx, o);
        if (st != GC_OK) return st;
    } else {
        o->last.state = o->job->state;
    }
    *out = o->last;
    return GC_OK;
}

gc_status gc_wait(gc_ctx *ctx, gc_orbit orbit, int64_t timeout_ms)
{
    GC_ENTER(ctx);
    Orbit *o = find_orbit(ctx, orbit);
    if (!o) return GC_EINVAL;
    return wait_locked(ctx, lk, o, timeout_ms);
}

gc_status gc_saturation(gc_ctx *ctx, gc_orbit orbit, int32_t n_points, const uint64_t *sample_sizes,
                        int32_t in_region_only, uint64_t *distinct_out)
{
    if (n_points < 0 || (n_points > 0 && (!sample_sizes || !distinct_out))) return GC_EINVAL;
    GC_ENTER(ctx);
    Orbit *o = find_orbit(ctx, orbit);
    if (!o) return GC_EINVAL;
    if (!o->job || o->job->state != GC_ORBIT_DONE) return GC_ESTATE;
    gc_status st = ensure_copies_locked(ctx, o);
    if (st != GC_OK) return st;
    // a copy is found within the first N starts of the launch iff the lowest
    // start id reaching it is below first_start + N
    const uint64_t base = o->job->p.first_start;
    std::vector<uint64_t> first;
    first.reserve(o->copies.size());
    for (const gc_copy &c : o->copies)
        if (!in_region_only || (c.flags & GC_FLAG_IN_REGION)) first.push_back(c.first_start - base);
    std::sort(first.begin(), first.end());
    for (int32_t k = 0; k < n_points; ++k)
        distinct_out[k] = (uint64_t)(std::lower_bound(first.begin(), first.end(), sample_sizes[k]) - first.begin());
    return GC_OK;
}

gc_status gc_paper_saturation(gc_ctx *ctx, gc_orbit orbit, int32_t n_points, const uint64_t *sample_sizes,
                              uint64_t *distinct_out)
{
    if (n_points < 0 || (n_points > 0 && (!sample_sizes || !distinct_out))) return GC_EINVAL;
    for (int32_t k = 1; k < n_points; ++k)
        if (sample_sizes[k] < sample_sizes[k - 1]) return GC_EINVAL;
    GC_ENTER(ctx);
    Orbit *o = find_orbit(ctx, orbit);
    if (!o) return GC_EINVAL;
    if (!o->job || o->job->state != GC_ORBIT_DONE) return GC_ESTATE;
    if (n_points == 0) return GC_OK;
    const uint64_t n = o->job->n_starts[o->job_index];
    // [GC_PAPER_VALUES / 64] bitmap words, the running count, one snapshot per point
    const size_t words = GC_PAPER_VALUES / 64;
    void *blk = nullptr;
    size_t got = 0;
    gc_status st = pool_get(ctx, sizeof(unsigned long long) * (words + 1 + (size_t)n_points), &blk, &got);
    if (st != GC_OK) return st;
    unsigned long long *buf = (unsigned long long *)blk;
    unsigned long long *count = buf + words, *snap = count + 1;
    std::vector<unsigned long long> host(n_points);
    hipStream_t s = ctx->util;
    hipError_t e = gc_launch_zero_u64(buf, (int)(words + 1), s);
    uint64_t done = 0;
    for (int32_t k = 0; k < n_points && e == hipSuccess; ++k) {
        const uint64_t upto = std::min<uint64_t>(sample_sizes[k], n);
        e = gc_launch_paper_mark((const GcStartRec *)o->res.rec, done, upto, (uint32_t *)buf, count, s);
        done = std::max(done, upto);
        if (e == hipSuccess) e = hipMemcpyAsync(snap + k, count, sizeof *count, hipMemcpyDeviceToDevice, s);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(host.data(), snap, sizeof(unsigned long long) * n_points, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    ctx->pool.put(blk, got);
    if (e != hipSuccess) return fail(ctx, e, "gc_paper_saturation");
    for (int32_t k = 0; k < n_points; ++k) distinct_out[k] = host[k];
    return GC_OK;
}

gc_status gc_fetch(gc_ctx *ctx, gc_orbit orbit, uint64_t offset, uint64_t cap, gc_copy *out, uint64_t *n_written,
                   uint64_t *n_total)
{
    if (cap && !out) return GC_EINVAL;
    GC_ENTER(ctx);
    Orbit *o = find_orbit(ctx, orbit);
    if (!o) return GC_EINVAL;
    if (!o->job || o->job->state != GC_ORBIT_DONE) return GC_ESTATE;
    gc_status st = ensure_copies_locked(ctx, o);
    if (st != GC_OK) return st;
    const uint64_t n = o->copies.size();
    const uint64_t w = offset < n ? std::min(cap, n - offset) : 0;
    if (w) memcpy(out, o->copies.data() + offset, w * sizeof(gc_copy));
    if (n_written) *n_written = w;
    if (n_total) *n_total = n;
    return GC_OK;
}

gc_status gc_fetch_starts(gc_ctx *ctx, gc_orbit orbit, uint64_t offset, uint64_t cap, gc_start_record *out,
                          uint64_t *n_written)
{
    if (cap && !out) return GC_EINVAL;
    GC_ENTER(ctx);
    Orbit *o = find_orbit(ctx, orbit);
    if (!o) return GC_EINVAL;
    if (!o->job || o->job->state != GC_ORBIT_DONE) return GC_ESTATE;
    gc_status st = ensure_starts_locked(ctx, o);
    if (st != GC_OK) return st;
    const uint64_t n = o->starts.size();
    const uint64_t w = offset < n ? std::min(cap, n - offset) : 0;
    if (w) memcpy(out, o->starts.data() + offset, w * sizeof(gc_start_record));
    if (n_written) *n_written = w;
    return GC_OK;
}

gc_status gc_fetch_start_state(gc_ctx *ctx, gc_orbit orbit, uint64_t start_id, double *theta_out)
{
    if (!theta_out) return GC_EINVAL;
    GC_ENTER(ctx);
    Orbit *o = find_orbit(ctx, orbit);
    if (!o) return GC_EINVAL;
    if (!o->job || o->job->state != GC_ORBIT_DONE) return GC_ESTATE;
    return start_state_locked(ctx, o, start_id, theta_out);
}

gc_status gc_fetch_state(gc_ctx *ctx, gc_orbit orbit, uint64_t key_hi, uint64_t key_lo, double *theta_out)
{
    if (!theta_out) return GC_EINVAL;
    GC_ENTER(ctx);
    Orbit *o = find_orbit(ctx, orbit);
    if (!o) return GC_EINVAL;
    if (!o->job || o->job->state != GC_ORBIT_DONE) return GC_ESTATE;
    gc_status st = ensure_copies_locked(ctx, o);
    if (st != GC_OK) return st;
    // the copies are sorted by key
    auto it = std::lower_bound(o->copies.begin(), o->copies.end(), std::make_pair(key_hi, key_lo),
                               [](const gc_copy &c, const std::pair<uint64_t, uint64_t> &k) {
                                   return c.key_hi != k.first ? c.key_hi < k.first : c.key_lo < k.second;
                               });
    if (it == o->copies.end() || it->key_hi != key_hi || it->key_lo != key_lo) return GC_ENOTFOUND;
    return start_state_locked(ctx, o, it->rep_start, theta_out);
}

gc_status gc_release(gc_ctx *ctx, gc_orbit orbit)
{
    GC_ENTER(ctx);
    Orbit *o = find_orbit(ctx, orbit);
    if (!o) return GC_EINVAL;
    if (o->job && (o->job->state == GC_ORBIT_QUEUED || o->job->state == GC_ORBIT_RUNNING)) {
        gc_status st = wait_locked(ctx, lk, o, -1);
        if (st != GC_OK && st != GC_ENOMEM) return st;
        if (st == GC_ENOMEM) {
            // still queued: withdraw it
            Job *job = o->job;
            ctx->queued.erase(std::remove(ctx->queued.begin(), ctx->queued.end(), job), ctx->queued.end());
            fail_job(ctx, job, GC_ENOMEM);
        }
    }
    drop_results_locked(ctx, o);
    // the tables go back to the pools: no free (which waits for the device)
    ctx->pinned.put(o->copies.p, o->copies.cap_bytes);
    o->copies = HostCopies{};
    ctx->pool.put(o->tables, o->table_bytes);
    ctx->pool.put(o->wave_tables, o->wave_bytes);
    ctx->used -= o->table_bytes + o->wave_bytes;
    ctx->orbits.erase(orbit);
    admit_locked(ctx);
    ctx->done_cv.notify_all();
    return GC_OK;
}

gc_status gc_last_error(gc_ctx *ctx, char *buf, size_t cap)
{
    if (!ctx || (!buf && cap)) return GC_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (cap) {
        snprintf(buf, cap, "%s", ctx->err.c_str());
    }
    return GC_OK;
}

gc_status gc_launch_bytes(gc_ctx *ctx, gc_orbit orbit, uint64_t n_starts, const gc_solve_params *params,
                          uint64_t *bytes)
{
    if (!bytes || n_starts == 0) return GC_EINVAL;
    gc_solve_params p;
    if (params) p = *params; else fill_defaults(&p);
    GC_ENTER(ctx);
    Orbit *o = find_orbit(ctx, orbit);
    if (!o) return GC_EINVAL;
    Job tmp;
    tmp.orbits.push_back(o);
    tmp.n_starts.push_back(n_starts);
    tmp.p = p;
    size_t b = 0;
    gc_status st = job_bytes(ctx, &tmp, &b);
    if (st != GC_OK) return st;
    *bytes = b;
    return GC_OK;
}

gc_status gc_memory_info(gc_ctx *ctx, uint64_t *budget, uint64_t *in_use, uint64_t *queued)
{
    GC_ENTER(ctx);
    if (budget) *budget = ctx->budget;
    if (in_use) *in_use = ctx->used;
    if (queued) *queued = ctx->queued.size();
    return GC_OK;
}

gc_status gc_autotune(gc_ctx *ctx, gc_orbit orbit, uint64_t n_starts, const gc_solve_params *params,
                      gc_tune_result *out)
{
    if (!ctx || n_starts == 0 || n_starts > (1ull << 32)) return GC_EINVAL;
    gc_solve_params p;
    if (params) p = *params; else fill_defaults(&p);
    gc_status st = check_params(&p);
    if (st != GC_OK) return st;
    int d = 0, V = 0, K = 0;
    {
        GC_ENTER(ctx);
        Orbit *o = find_orbit(ctx, orbit);
        if (!o) return GC_EINVAL;
        if (o->job && (o->job->state == GC_ORBIT_QUEUED || o->job->state == GC_ORBIT_RUNNING)) return GC_EBUSY;
        d = o->dev.d;
        V = o->V;
        K = o->dev.K;
    }
    const bool mixed = p.precision == GC_MIXED;
    // one measured launch with the given variant forced on that launch only
    // (launches of other orbits meanwhile use the context's choices)
    auto trial = [&](int creg, double *relax_ms, double *post_ms) -> gc_status {
        Job force;
        force.force_creg = creg;
        gc_status s2;
        {
            std::unique_lock<std::mutex> lk(ctx->mu);
            if (ctx->failed) return GC_EDEVICE;
            Orbit *o = find_orbit(ctx, orbit);
            if (!o) return GC_EINVAL;
            s2 = launch_locked(ctx, {o}, {n_starts}, p, false, &force);
            if (s2 == GC_OK) s2 = wait_locked(ctx, lk, o, -1);
            if (s2 == GC_OK) {
                *relax_ms = o->job->solve_ms;
                *post_ms = o->job->post_ms + o->job->filter_ms;
            }
        }
        return s2;
    };
    gc_tune_result r{};
    const bool wave = (K == 2) && (size_t)(GC_WAVES + 1) * 16 * V <= ctx->lds_max;
    const int ns = (V / 2 + 63) / 64;
    const int cmax = wave ? gc_wave_creg_max(d, ns) : 0;
    double rm = 0, pm = 0;
    st = trial(-1, &rm, &pm);   // warm-up: code objects, pool
    if (st != GC_OK) return st;
    double best_r = INFINITY;
    // relax: register-coefficient colours 0..cmax of the one-wavefront
    // layout (the workgroup layout has no such variants), best of two each
    int best_c = 0;
    {
        double bc = INFINITY;
        for (int c = 0; c <= cmax; ++c) {
            double t = INFINITY;
            for (int rep = 0; rep < 2; ++rep) {
                st = trial(c, &rm, &pm);
                if (st != GC_OK) return st;
                t = std::min(t, rm);
            }
            if (t < bc) { bc = t; best_c = c; }
        }
        best_r = bc;
    }
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        if (wave) ctx->tune_creg[creg_key(d, ns, mixed)] = best_c;
        save_tune_cache(ctx);
    }
    // the filter's shape depends on the lattice only: reported, not tuned
    int fb = 0, fs = 0, db = 0, dsp = 0, dw = 0;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        Orbit *o = find_orbit(ctx, orbit);
        if (o && gc_lanczos_shape(o->d, o->lat.extent, o->V, &fb, &fs)) {
            db = fb;
            dsp = fs;
        } else {
            gc_post_shape(V, &db, &dsp, &dw);
        }
    }
    r.relax_variant = best_c;
    r.relax_ms = best_r;
    r.post_block = db;
    r.post_sites_per_thread = dsp;
    r.post_ms = pm;
    if (out) *out = r;
    return GC_OK;
}

gc_status gc_launch_static(gc_ctx *ctx, gc_orbit orbit, uint64_t n_starts, const gc_solve_params *params,
                           void *hip_stream, gc_copy *copies_dev, uint64_t copies_cap, uint64_t *n_copies_dev,
                           uint64_t *counters_dev)
{
    gc_solve_params p;
    if (params) p = *params; else fill_defaults(&p);
    gc_status st = check_params(&p);
    if (st != GC_OK) return st;
    if (n_starts == 0 || n_starts > (1ull << 32) || !copies_dev || !n_copies_dev || copies_cap < n_starts)
        return GC_EINVAL;
    GC_ENTER(ctx);
    Orbit *o = find_orbit(ctx, orbit);
    if (!o) return GC_EINVAL;
    if (!ctx->scratch) return GC_EUNSUPPORTED;
    // nothing of this job outlives the call: descriptors go to the static
    // array through kernel arguments, results to the caller's buffers
    Job job;
    job.orbits.push_back(o);
    job.n_starts.push_back(n_starts);
    job.p = p;
    st = plan_job(ctx, &job, job.L);
    if (st != GC_OK) return st;
    if (job.L.total > GC_STATIC_SCRATCH_BYTES) {
        char buf[160];
        snprintf(buf, sizeof buf, "gc_launch_static: %llu starts need %llu bytes, the static array holds %llu",
                 (unsigned long long)n_starts, (unsigned long long)job.L.total,
                 (unsigned long long)GC_STATIC_SCRATCH_BYTES);
        ctx->err = buf;
        return GC_ENOMEM;
    }
    unsigned char *base = ctx->scratch;
    fill_job_devs(&job, base);
    GcJobDev &J = job.jobs[0];
    J.copies = (GcCopyRec *)copies_dev;
    J.n_copies = (unsigned long long *)n_copies_dev;
    if (counters_dev) J.cnt = (GcCounters *)counters_dev;
    hipStream_t s = (hipStream_t)hip_stream;
    for (const Blob &bl : job_blobs(&job))
        GC_HIP(gc_launch_store(base + bl.dst, bl.bytes.data(), bl.bytes.size(), s));
    for (int gi = 0; gi < (int)job.L.groups.size(); ++gi) GC_HIP(enqueue_chain(&job, base, gi, s, false));
    return GC_OK;
}

gc_status gc_kernel_time_ms(gc_ctx *ctx, gc_orbit orbit, double *solve_ms)
{
    if (!solve_ms) return GC_EINVAL;
    GC_ENTER(ctx);
    Orbit *o = find_orbit(ctx, orbit);
    if (!o) return GC_EINVAL;
    if (!o->job || o->job->state != GC_ORBIT_DONE) return GC_ESTATE;
    *solve_ms = o->job->solve_ms;
    return GC_OK;
}

}  // extern "C"

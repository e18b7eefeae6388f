// api.cpp -- the extern "C" boundary of libpsp (declared in include/psp.h):
// argument checks, status/error reporting, plan handles, workspace layout and
// kernel launches.  All arithmetic of the method runs in the HIP kernels.
#include "psp.h"

#include <hip/hip_runtime.h>

#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <memory>
#include <map>
#include <sstream>
#include <mutex>
#include <tuple>
#include <new>
#include <string>
#include <vector>

#include "common.h"
#include "plan.h"
#include "sparse.h"

#include "dense.h"
#include "powerflow.h"
#include "estimate.h"
#include "adapt.h"

using namespace psp;

namespace {

thread_local std::string g_err;

psp_status fail(psp_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

psp_status hip_fail(hipError_t e, const char* where) {
    return fail(PSP_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(call, where)                       \
    do {                                           \
        hipError_t e_ = (call);                    \
        if (e_ != hipSuccess) return hip_fail(e_, where); \
    } while (0)

constexpr int64_t kAlign = 256;
constexpr int32_t kDenseMaxN = 4096;   // largest n of the dense path
int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

int device_cus() {
    static int cus = 0;
    static std::once_flag once;
    std::call_once(once, [] {
        int dev = 0;
        hipDeviceProp_t p;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess) cus = p.multiProcessorCount;
        if (cus <= 0) cus = 256;
    });
    return cus;
}

}  // namespace

struct psp_plan_s {
    Symbolic sym;
    std::mutex mu;
    // Device metadata: built on the host as one image (image.h), copied by
    // psp_plan_upload into caller-owned device memory; the pointers below are
    // relocated into that copy.  The library never frees it.
    PlanImage img;
    bool imaged = false;
    int device = -1;                   // device of the uploaded copy (-1: not uploaded)
    const void* d_image = nullptr;
    const int32_t* d_dst = nullptr;    // dense slot offset (column-major, ld = d_dst_ld) of each CSR entry
    int32_t d_dst_ld = 0;
    const int32_t* d_perm = nullptr;
    const int32_t* d_rows = nullptr;   // original row of each CSR entry
    const int32_t* d_cols = nullptr;
    const int32_t* d_rowptr = nullptr; // user CSR row pointers
    SparseDevice sp;                   // sparse-path arrays
    uint64_t hash = 0;                 // FNV-1a of the pattern (key of the tuning cache file)
    std::map<std::tuple<int32_t, int32_t, int32_t>, psp_tune_choice_t> tuned;   // (batch, K, nrhs) -> choice
};

struct psp_factors_s {
    psp_plan plan;
    int32_t path, batch, K, nrhs_cap;
    EpsSet es;
    char* ws;
    size_t ws_bytes;
    int32_t* info;
    // dense layout
    int32_t n_pad, ld;
    int64_t slot_stride;   // doubles
    int64_t off_slots, off_tmp;
};

namespace {

struct DenseLayout {
    int32_t n_pad, ld;
    int64_t slot_stride;      // doubles per slot
    int64_t nslots;
    int64_t off_slots, off_xk, off_tmp, total;
};

DenseLayout dense_layout(const Symbolic& s, int32_t batch, int32_t K, int32_t nrhs, int32_t keep) {
    DenseLayout L{};
    const int nb = dense_panel();
    L.n_pad = (s.n + nb - 1) / nb * nb;
    L.ld = L.n_pad;
    const int64_t ntasks = (int64_t)batch * K;
    if (keep) {
        L.slot_stride = align_up((int64_t)L.ld * L.n_pad, kAlign / 8);
        L.nslots = ntasks;
    } else {
        L.slot_stride = align_up((int64_t)L.ld * (L.n_pad + nrhs), kAlign / 8);
        L.nslots = std::min<int64_t>(ntasks, 2LL * device_cus());
    }
    L.off_slots = 0;
    int64_t off = align_up(L.nslots * L.slot_stride * 8, kAlign);
    L.off_xk = off;
    if (!keep) off = align_up(off + ntasks * (int64_t)s.n * nrhs * 8, kAlign);
    L.off_tmp = off;
    if (keep) off = align_up(off + ntasks * (int64_t)L.ld * nrhs * 8, kAlign);
    L.total = off;
    return L;
}

// Builds the plan's device image on the host (once).
void build_image(psp_plan p) {
    std::lock_guard<std::mutex> g(p->mu);
    if (p->imaged) return;
    const Symbolic& s = p->sym;
    PlanImage& img = p->img;
    std::vector<int32_t> rows(s.nnz);
    for (int32_t i = 0; i < s.n; ++i)
        for (int32_t e = s.row_ptr[i]; e < s.row_ptr[i + 1]; ++e) rows[e] = i;
    img.bind(&p->d_perm, img.put(s.perm));
    img.bind(&p->d_rows, img.put(rows));
    img.bind(&p->d_cols, img.put(s.col_idx));
    img.bind(&p->d_rowptr, img.put(s.row_ptr));
    // dense slot offsets, for the dense path's padded leading dimension
    const int nb = dense_panel();
    const int32_t ld = (s.n + nb - 1) / nb * nb;
    if (s.n <= kDenseMaxN) {
        std::vector<int32_t> dst(s.nnz);
        for (int32_t i = 0; i < s.n; ++i)
            for (int32_t e = s.row_ptr[i]; e < s.row_ptr[i + 1]; ++e)
                dst[e] = (int32_t)((int64_t)s.iperm[s.col_idx[e]] * ld + s.iperm[i]);
        img.bind(&p->d_dst, img.put(dst));
        p->d_dst_ld = ld;
    }
    sparse_image(s, img, p->sp);
    p->imaged = true;
}

// Numeric calls need the image on the current device.
psp_status require_upload(psp_plan p) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    std::lock_guard<std::mutex> g(p->mu);
    if (p->device < 0 || !p->d_image) return fail(PSP_E_STATE, "plan is not uploaded: call psp_plan_upload first");
    if (p->device != dev) return fail(PSP_E_STATE, "plan was uploaded to another device");
    return PSP_OK;
}

psp_status make_eps(int32_t K, const double* eps, EpsSet& es) {
    if (K < 1 || K > kMaxK) return fail(PSP_E_INVALID, "K must be in 1.." + std::to_string(kMaxK));
    if (!eps) return fail(PSP_E_INVALID, "eps must not be NULL");
    es.K = K;
    const psp_status st = psp_weights(K, eps, es.c);
    if (st != PSP_OK) return st;
    for (int k = 0; k < K; ++k) es.eps[k] = eps[k];
    return PSP_OK;
}

// Path id -> (base path, sparse execution or -1).
struct PathSel {
    int32_t base;
    int forced;
};

PathSel split_path(int32_t path) {
    switch (path) {
        case PSP_PATH_DENSE: return {PSP_PATH_DENSE, -1};
        case PSP_PATH_SPARSE: return {PSP_PATH_SPARSE, -1};
        case PSP_PATH_SPARSE_BATCHED: return {PSP_PATH_SPARSE, kVarBatched};
        case PSP_PATH_SPARSE_LDS: return {PSP_PATH_SPARSE, kVarLds};
        case PSP_PATH_SPARSE_LEVELS: return {PSP_PATH_SPARSE, kVarGlobal};
        case PSP_PATH_SPARSE_GROUPED: return {PSP_PATH_SPARSE, kVarGrouped};
        case PSP_PATH_SPARSE_STEPS: return {PSP_PATH_SPARSE, kVarSteps};
        case PSP_PATH_SPARSE_TAIL: return {PSP_PATH_SPARSE, kVarTail};
        default: return {-1, -1};
    }
}

int32_t heuristic_path(const Symbolic& s) { return (s.n <= 128) ? PSP_PATH_DENSE : PSP_PATH_SPARSE; }

psp_status check_prior_hip() {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "error left by earlier device work");
    return PSP_OK;
}

// ---- tuning cache: the tuner's choices, persisted to a text file (one line per
// (device, pattern, batch, K, nrhs)) so that a later process finds them without tuning again.
// File: $PSP_TUNE_CACHE, else $HOME/.cache/psp/tune.txt; PSP_TUNE_CACHE set but empty disables it.
std::mutex g_cache_mu;
bool g_cache_loaded = false;
std::map<std::string, psp_tune_choice_t> g_cache;

std::string cache_path() {
    if (const char* e = std::getenv("PSP_TUNE_CACHE")) return e;
    const char* h = std::getenv("HOME");
    return h && *h ? std::string(h) + "/.cache/psp/tune.txt" : std::string();
}

std::string cache_key(psp_plan p, int32_t batch, int32_t K, int32_t nrhs) {
    char buf[160];
    std::snprintf(buf, sizeof(buf), "v2|gfx950|n=%d|nnz=%d|h=%016llx|batch=%d|K=%d|nrhs=%d", p->sym.n, p->sym.nnz,
                  (unsigned long long)p->hash, batch, K, nrhs);
    return buf;
}

void cache_load_locked() {
    if (g_cache_loaded) return;
    g_cache_loaded = true;
    const std::string path = cache_path();
    if (path.empty()) return;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string key;
        psp_tune_choice_t c{};
        if (is >> key >> c.path >> c.steps_mode >> c.steps_wgcu >> c.ring >> c.tail_cols >> c.tail_il >> c.tail_lu >> c.ms) {
            c.source = 2;
            g_cache[key] = c;
        }
    }
}

void cache_store(const std::string& key, const psp_tune_choice_t& c) {
    std::lock_guard<std::mutex> g(g_cache_mu);
    cache_load_locked();
    g_cache[key] = c;
    const std::string path = cache_path();
    if (path.empty()) return;
    const size_t slash = path.find_last_of('/');
    if (slash != std::string::npos) {
        // create the directory and its parent when missing (errors surface as a failed open below)
        const std::string dir = path.substr(0, slash);
        const size_t up = dir.find_last_of('/');
        if (up != std::string::npos && up > 0) ::mkdir(dir.substr(0, up).c_str(), 0755);
        ::mkdir(dir.c_str(), 0755);
    }
    const std::string tmp = path + ".tmp" + std::to_string((long long)::getpid());
    {
        std::ofstream f(tmp);
        if (!f) return;
        for (const auto& kv : g_cache)
            f << kv.first << ' ' << kv.second.path << ' ' << kv.second.steps_mode << ' ' << kv.second.steps_wgcu << ' '
              << kv.second.ring << ' ' << kv.second.tail_cols << ' ' << kv.second.tail_il << ' ' << kv.second.tail_lu << ' '
              << kv.second.ms << '\n';
    }
    std::rename(tmp.c_str(), path.c_str());
}

psp_tune_choice_t default_choice(int32_t path) {
    psp_tune_choice_t c{};
    const Knobs kn;
    c.path = path;
    c.steps_mode = kn.steps_mode;
    c.steps_wgcu = kn.steps_wgcu;
    c.ring = kn.ring;
    c.tail_cols = kn.tail_cols;
    c.tail_il = kn.tail_il;
    c.tail_lu = kn.tail_lu;
    c.ms = -1.0f;
    c.source = 0;
    return c;
}

Knobs knobs_of(const psp_tune_choice_t& c) {
    Knobs kn;
    kn.steps_mode = c.steps_mode;
    kn.steps_wgcu = c.steps_wgcu;
    kn.ring = c.ring;
    kn.tail_cols = c.tail_cols;
    kn.tail_il = c.tail_il;
    kn.tail_lu = c.tail_lu;
    return kn;
}

// The choice for this call: an explicit path with the default launch choices, or for AUTO the
// tuner's choice (this process, else the cache file), else the size heuristic.
psp_tune_choice_t resolve_choice(psp_plan p, int32_t path, int32_t batch, int32_t K, int32_t nrhs) {
    if (path != PSP_PATH_AUTO) return default_choice(path);
    const auto key = std::make_tuple(batch, K, nrhs);
    {
        std::lock_guard<std::mutex> g(p->mu);
        auto it = p->tuned.find(key);
        if (it != p->tuned.end()) return it->second;
    }
    psp_tune_choice_t c = default_choice(heuristic_path(p->sym));
    {
        std::lock_guard<std::mutex> g(g_cache_mu);
        cache_load_locked();
        auto it = g_cache.find(cache_key(p, batch, K, nrhs));
        if (it == g_cache.end()) return c;
        c = it->second;
        c.source = 2;
    }
    std::lock_guard<std::mutex> g(p->mu);
    p->tuned[key] = c;
    return c;
}

int32_t resolve_path(psp_plan p, int32_t path, int32_t batch, int32_t K, int32_t nrhs) {
    return resolve_choice(p, path, batch, K, nrhs).path;
}

size_t path_workspace(const Symbolic& s, int32_t path, int32_t batch, int32_t K, int32_t nrhs, int32_t keep) {
    const PathSel ps = split_path(path);
    if (ps.base == PSP_PATH_DENSE) return (size_t)dense_layout(s, batch, K, nrhs, keep).total;
    if (ps.base == PSP_PATH_SPARSE) return sparse_workspace_bytes(s, batch, K, nrhs, keep, ps.forced);
    return 0;
}

}  // namespace

extern "C" {

const char* psp_last_error(void) { return g_err.c_str(); }

int32_t psp_version(void) { return 200; }

psp_status psp_weights(int32_t K, const double* eps, double* c) {
    if (K < 1 || !eps || !c) return fail(PSP_E_INVALID, "psp_weights: K >= 1 and non-NULL arrays required");
    for (int k = 0; k < K; ++k) {
        if (!std::isfinite(eps[k]) || eps[k] == 0.0) return fail(PSP_E_EPS, "perturbation nodes must be finite and nonzero");
        for (int l = 0; l < k; ++l)
            if (eps[l] == eps[k]) return fail(PSP_E_EPS, "perturbation nodes must be distinct");
    }
    // Lagrange basis at zero: prod over l != k of eps_l / (eps_l - eps_k), in ascending l.
    for (int k = 0; k < K; ++k) {
        double w = 1.0;
        for (int l = 0; l < K; ++l)
            if (l != k) w = w * (eps[l] / (eps[l] - eps[k]));
        c[k] = w;
    }
    return PSP_OK;
}

psp_status psp_plan_create(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, uint32_t flags, psp_plan* out) {
    if (!out) return fail(PSP_E_INVALID, "out must not be NULL");
    *out = nullptr;
    const std::string why = validate_csr(n, row_ptr, col_idx);
    if (!why.empty()) return fail(PSP_E_INVALID, "psp_plan_create: " + why);
    if (flags & ~1u) return fail(PSP_E_INVALID, "psp_plan_create: unknown flag bits");
    try {
        auto p = std::make_unique<psp_plan_s>();
        analyse(n, row_ptr, col_idx, (flags & PSP_ORDER_NATURAL) != 0, p->sym);
        uint64_t h = 1469598103934665603ULL;
        auto mix = [&](uint32_t v) {
            for (int b = 0; b < 4; ++b) {
                h ^= (v >> (8 * b)) & 0xFF;
                h *= 1099511628211ULL;
            }
        };
        mix((uint32_t)n);
        mix(flags);
        for (int32_t i = 0; i <= n; ++i) mix((uint32_t)row_ptr[i]);
        for (int32_t e = 0; e < row_ptr[n]; ++e) mix((uint32_t)col_idx[e]);
        p->hash = h;
        *out = p.release();
    } catch (const std::bad_alloc&) {
        return fail(PSP_E_NOMEM, "psp_plan_create: host allocation failed");
    }
    return PSP_OK;
}

psp_status psp_plan_info(psp_plan p, psp_plan_info_t* o) {
    if (!p || !o) return fail(PSP_E_INVALID, "psp_plan_info: NULL argument");
    const Symbolic& s = p->sym;
    o->n = s.n;
    o->nnz = s.nnz;
    o->nnz_l = s.l_ptr[s.n];
    o->ndense = s.ndense;
    for (int t = 0; t < 3; ++t) o->nlev[t] = (int32_t)s.lev_ptr[t].size() - 1;
    o->flops_dense_factor = s.flops_dense;
    o->flops_sparse_factor = s.flops_sparse;
    try {
        build_image(p);
    } catch (const std::bad_alloc&) {
        return fail(PSP_E_NOMEM, "psp_plan_info: host allocation failed");
    }
    o->steps = p->sp.st.nsteps;
    o->steps_packed = p->sp.st.packed;
    o->steps_lds_bytes = steps_lds_bytes(p->sp);
    o->steps_per_cu = steps_ready(p->sp) ? steps_per_cu(p->sp) : 0;
    o->device_bytes = (int64_t)std::max<size_t>(p->img.bytes(), 256);
    o->tail_n = s.tail_n;
    o->tail_fac_levels = s.tail_n ? s.fac_lev_sp : 0;
    o->tail_tiles = p->sp.idx.tail_tiles;
    o->tail_mfma = p->sp.h_tail_pairs / 4;
    return PSP_OK;
}

psp_status psp_plan_export(psp_plan p, int32_t* perm, int32_t* iperm, int32_t* parent, int32_t* l_ptr,
                           int32_t* l_idx, int32_t* lev_ptr[3], int32_t* lev_idx[3]) {
    if (!p) return fail(PSP_E_INVALID, "psp_plan_export: NULL plan");
    const Symbolic& s = p->sym;
    auto cp = [](int32_t* dst, const std::vector<int32_t>& v) { if (dst && !v.empty()) std::memcpy(dst, v.data(), v.size() * 4); };
    cp(perm, s.perm);
    cp(iperm, s.iperm);
    cp(parent, s.parent);
    cp(l_ptr, s.l_ptr);
    cp(l_idx, s.l_idx);
    for (int t = 0; t < 3; ++t) {
        if (lev_ptr) cp(lev_ptr[t], s.lev_ptr[t]);
        if (lev_idx) cp(lev_idx[t], s.lev_idx[t]);
    }
    return PSP_OK;
}

void psp_plan_destroy(psp_plan p) { delete p; }

size_t psp_plan_device_bytes(psp_plan p) {
    if (!p) return 0;
    try {
        build_image(p);
    } catch (const std::bad_alloc&) {
        return 0;
    }
    return std::max<size_t>(p->img.bytes(), 256);
}

psp_status psp_plan_upload(psp_plan p, void* dev, size_t dev_bytes, void* stream) {
    if (!p || !dev) return fail(PSP_E_INVALID, "psp_plan_upload: NULL argument");
    if (((uintptr_t)dev & 255) != 0) return fail(PSP_E_INVALID, "psp_plan_upload: device buffer must be 256-byte aligned");
    const size_t need = psp_plan_device_bytes(p);
    if (need == 0) return fail(PSP_E_NOMEM, "psp_plan_upload: host allocation failed");
    if (dev_bytes < need) return fail(PSP_E_NOMEM, "psp_plan_upload: device buffer too small: need " + std::to_string(need) + " bytes");
    if (psp_status st = check_prior_hip()) return st;
    int devid = 0;
    HIP_TRY(hipGetDevice(&devid), "hipGetDevice");
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, devid), "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(PSP_E_UNSUPPORTED, std::string("libpsp is built for gfx950, device is ") + prop.gcnArchName);
    const hipStream_t st = (hipStream_t)stream;
    std::lock_guard<std::mutex> g(p->mu);
    HIP_TRY(hipMemcpyAsync(dev, p->img.words.data(), p->img.bytes(), hipMemcpyHostToDevice, st), "hipMemcpyAsync(plan)");
    HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize(plan)");
    p->img.apply(dev);
    p->d_image = dev;
    p->device = devid;
    // one-off kernel attributes, here rather than inside a numeric call that may be captured
    HIP_TRY(sparse_kernel_attrs(), "kernel attributes");
    HIP_TRY(steps_kernel_attrs(), "kernel attributes");
    HIP_TRY(dense_kernel_attrs(), "kernel attributes");
    return PSP_OK;
}

size_t psp_workspace_bytes(psp_plan p, int32_t path, int32_t batch, int32_t K, int32_t nrhs, int32_t keep) {
    if (!p || batch < 1 || K < 1 || nrhs < 0) return 0;
    if (path == PSP_PATH_AUTO) {
        size_t m = 0;
        for (int32_t c = PSP_PATH_DENSE; c <= PSP_PATH_SPARSE_TAIL; ++c)
            if (c != PSP_PATH_DENSE || p->sym.n <= kDenseMaxN) m = std::max(m, path_workspace(p->sym, c, batch, K, nrhs, keep));
        return m;
    }
    return path_workspace(p->sym, path, batch, K, nrhs, keep);
}

}  // extern "C"

namespace {

// psp_solve_batched with the path and launch choices given (path != AUTO).
psp_status solve_choice(psp_plan p, const psp_tune_choice_t& ch, int32_t batch, const double* values, int32_t K,
                        const double* eps, const double* d, int32_t nrhs, const double* B, double* X, int32_t* info,
                        void* ws, size_t ws_bytes, void* stream) {
    if (!p || batch < 1 || !values || !B || !X || !info || !ws) return fail(PSP_E_INVALID, "psp_solve_batched: NULL argument or batch < 1");
    if (nrhs < 1 || nrhs > 64) return fail(PSP_E_INVALID, "psp_solve_batched: nrhs must be in 1..64");
    EpsSet es;
    if (psp_status st = make_eps(K, eps, es)) return st;
    if (psp_status st = check_prior_hip()) return st;
    const Symbolic& s = p->sym;
    const hipStream_t st = (hipStream_t)stream;
    const PathSel ps = split_path(ch.path);
    const Knobs kn = knobs_of(ch);
    if (ps.base == PSP_PATH_DENSE) {
        if (s.n > kDenseMaxN) return fail(PSP_E_UNSUPPORTED, "dense path supports n <= 4096");
        const DenseLayout L = dense_layout(s, batch, K, nrhs, 0);
        if (ws_bytes < (size_t)L.total) return fail(PSP_E_NOMEM, "workspace too small: need " + std::to_string(L.total) + " bytes");
        if (psp_status r = require_upload(p)) return r;
        char* w = (char*)ws;
        DenseArgs a{};
        a.n = s.n; a.n_pad = L.n_pad; a.ld = L.ld; a.nrhs = nrhs; a.nnz = s.nnz; a.batch = batch;
        a.dst = p->d_dst; a.perm = p->d_perm; a.values = values; a.dvec = d; a.B = B;
        a.Xk = (double*)(w + L.off_xk); a.info = info; a.slots = (double*)(w + L.off_slots);
        a.slot_stride = L.slot_stride; a.ntasks = batch * K; a.keep = 0;
        int occ = 1;
        if (dense_occupancy(&occ) != hipSuccess || occ < 1) occ = 1;
        const int64_t resident = std::min<int64_t>(L.nslots, (int64_t)occ * device_cus());
        // Enough Jacobians to fill the GPU: one task per Jacobian, combine fused.
        a.per_jacobian = batch >= resident ? 1 : 0;
        a.X = X;
        const int64_t tasks = a.per_jacobian ? batch : a.ntasks;
        const int grid = (int)std::min<int64_t>(tasks, resident);
        HIP_TRY(launch_dense_factor_solve(a, es, grid, st), "dense factor/solve launch");
        if (!a.per_jacobian) HIP_TRY(launch_combine((int64_t)s.n * nrhs, batch, es, a.Xk, X, st), "combine launch");
        return PSP_OK;
    }
    if (ps.base == PSP_PATH_SPARSE) {
        if (sparse_variant(s, (int64_t)batch * K, nrhs, ps.forced) < 0)
            return fail(PSP_E_UNSUPPORTED, "this sparse execution cannot run the plan (update lists or LDS size)");
        const size_t need = sparse_workspace_bytes(s, batch, K, nrhs, 0, ps.forced);
        if (ws_bytes < need) return fail(PSP_E_NOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
        if (psp_status r = require_upload(p)) return r;
        if (ps.forced == kVarSteps && !steps_ready(p->sp))
            return fail(PSP_E_UNSUPPORTED, "this sparse execution cannot run the plan (step schedule does not fit in LDS)");
        HIP_TRY(sparse_solve_batched(s, p->sp, batch, values, es, d, nrhs, B, X, info, ws, st, ps.forced, kn),
                "sparse launch");
        return PSP_OK;
    }
    return fail(PSP_E_INVALID, "unknown path");
}

}  // namespace

extern "C" {

psp_status psp_solve_batched(psp_plan p, int32_t path, int32_t batch, const double* values, int32_t K,
                             const double* eps, const double* d, int32_t nrhs, const double* B, double* X,
                             int32_t* info, void* ws, size_t ws_bytes, void* stream) {
    if (!p) return fail(PSP_E_INVALID, "psp_solve_batched: NULL plan");
    return solve_choice(p, resolve_choice(p, path, batch, K, nrhs), batch, values, K, eps, d, nrhs, B, X, info, ws,
                        ws_bytes, stream);
}

psp_status psp_tune_choice(psp_plan p, int32_t batch, int32_t K, int32_t nrhs, psp_tune_choice_t* out) {
    if (!p || !out) return fail(PSP_E_INVALID, "psp_tune_choice: NULL argument");
    *out = resolve_choice(p, PSP_PATH_AUTO, batch, K, nrhs);
    return PSP_OK;
}

psp_status psp_set_tune_choice(psp_plan p, int32_t batch, int32_t K, int32_t nrhs, const psp_tune_choice_t* c) {
    if (!p || !c) return fail(PSP_E_INVALID, "psp_set_tune_choice: NULL argument");
    if (split_path(c->path).base < 0) return fail(PSP_E_INVALID, "psp_set_tune_choice: unknown path");
    if (c->steps_mode < -1 || c->steps_mode > 1 || c->steps_wgcu < 0 || c->steps_wgcu > 1 ||
        (c->ring != 7 && c->ring != 4) || (c->tail_cols != 16 && c->tail_cols != 4 && c->tail_cols != 1) ||
        c->tail_il < -1 || c->tail_il > 1 || c->tail_lu < 0 || c->tail_lu > 1)
        return fail(PSP_E_INVALID, "psp_set_tune_choice: a launch choice is out of range");
    psp_tune_choice_t v = *c;
    v.source = 1;
    std::lock_guard<std::mutex> g(p->mu);
    p->tuned[std::make_tuple(batch, K, nrhs)] = v;
    return PSP_OK;
}

psp_status psp_solve_batched_noalloc(psp_plan p, int32_t batch, const double* values, int32_t K, const double* eps,
                                     const double* d, const double* B, double* X, int32_t* info, void* stream) {
    if (!p || batch < 1 || !values || !B || !X || !info)
        return fail(PSP_E_INVALID, "psp_solve_batched_noalloc: NULL argument or batch < 1");
    EpsSet es;
    if (psp_status st = make_eps(K, eps, es)) return st;
    if (psp_status st = check_prior_hip()) return st;
    if (psp_status r = require_upload(p)) return r;
    if (!steps_ready(p->sp))
        return fail(PSP_E_UNSUPPORTED, "psp_solve_batched_noalloc: the plan has no step schedule (it does not fit in LDS)");
    const Symbolic& s = p->sym;
    const bool per_jacobian = steps_per_jacobian(p->sp, batch);
    const size_t need = per_jacobian ? 0 : (size_t)batch * K * s.n * sizeof(double);
    if (need > noalloc_scratch_bytes())
        return fail(PSP_E_UNSUPPORTED, "psp_solve_batched_noalloc: needs " + std::to_string(need) +
                                           " bytes of scratch, the library's static scratch holds " +
                                           std::to_string(noalloc_scratch_bytes()));
    void* scratch = nullptr;
    HIP_TRY(noalloc_scratch(&scratch), "hipGetSymbolAddress(scratch)");
    HIP_TRY(steps_solve(p->sp, s.n, s.nnz, batch, values, es, d, B, X, info, (double*)scratch, (hipStream_t)stream),
            "step-kernel launch");
    return PSP_OK;
}

namespace {
// Which path runs the adaptive call: the step schedule, else the dense-trailing-block path (0: none).
int adaptive_path(psp_plan p) {
    try {
        build_image(p);
    } catch (const std::bad_alloc&) {
        return 0;
    }
    if (steps_ready(p->sp)) return PSP_PATH_SPARSE_STEPS;
    if (sparse_tail_adaptive_ok(p->sym, p->sp)) return PSP_PATH_SPARSE_TAIL;
    return 0;
}
}  // namespace

size_t psp_solve_adaptive_workspace_bytes(psp_plan p, int32_t batch, int32_t K) {
    if (!p || batch < 1 || K < 1 || K > kMaxK) return 0;
    const size_t base =
        (size_t)(align_up((int64_t)batch * K * p->sym.n * 8, kAlign) + align_up((int64_t)batch * 4, kAlign) + kAlign);
    if (adaptive_path(p) == PSP_PATH_SPARSE_TAIL)
        return base + (size_t)align_up((int64_t)sparse_tail_run_bytes(p->sym, batch, K), kAlign);
    return base;
}

psp_status psp_solve_adaptive(psp_plan p, int32_t batch, const double* values, int32_t K, const double* eps,
                              const double* d, double tol, const double* B, double* X, int32_t* info, double* est,
                              double* scale, void* ws, size_t ws_bytes, void* stream) {
    if (!p || batch < 1 || !values || !B || !X || !info || !est || !scale || !ws)
        return fail(PSP_E_INVALID, "psp_solve_adaptive: NULL argument or batch < 1");
    if (K < 3) return fail(PSP_E_INVALID, "psp_solve_adaptive: the error estimate needs K >= 3 nodes");
    if (!std::isfinite(tol) || tol < 0.0) return fail(PSP_E_INVALID, "psp_solve_adaptive: tol must be finite and >= 0");
    EpsSet es;
    if (psp_status st = make_eps(K, eps, es)) return st;
    if (psp_status st = check_prior_hip()) return st;
    if (psp_status r = require_upload(p)) return r;
    const int path = adaptive_path(p);
    if (path == 0)
        return fail(PSP_E_UNSUPPORTED,
                    "psp_solve_adaptive: the plan has neither a step schedule nor a dense trailing block path");
    const size_t need = psp_solve_adaptive_workspace_bytes(p, batch, K);
    if (ws_bytes < need) return fail(PSP_E_NOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
    if (((uintptr_t)ws & 255) != 0) return fail(PSP_E_INVALID, "psp_solve_adaptive: workspace must be 256-byte aligned");
    const Symbolic& s = p->sym;
    const hipStream_t st = (hipStream_t)stream;
    // divided-difference weights over nodes 0..j (ascending-l products, one reciprocal), the node
    // product and the rounding coefficient of the scale rule
    AdaptConst c{};
    for (int which = 0; which < 2; ++which) {
        const int j = K - 1 - which;
        double* w = which == 0 ? c.w1 : c.w2;
        for (int k = 0; k <= j; ++k) {
            double prod = 1.0;
            for (int l = 0; l <= j; ++l)
                if (l != k) prod = prod * (eps[k] - eps[l]);
            w[k] = 1.0 / prod;
        }
    }
    double emax = 0.0;
    c.P = 1.0;
    for (int k = 0; k < K; ++k) {
        c.c[k] = es.c[k];
        const double a = std::fabs(eps[k]);
        emax = std::max(emax, a);
        c.P = c.P * a;
    }
    c.b = (50.0 * 0x1p-53) / emax;
    char* w = (char*)ws;
    double* Xk = (double*)w;
    int32_t* list = (int32_t*)(w + align_up((int64_t)batch * K * s.n * 8, kAlign));
    int32_t* count = (int32_t*)((char*)list + align_up((int64_t)batch * 4, kAlign));
    if (path == PSP_PATH_SPARSE_TAIL) {
        // the first solve writes the per-system solutions; the second solves every Jacobian again
        // at its node scale (1 for those that passed: the same bits), the error test re-estimates
        // the rescaled ones
        void* tws = (char*)count + kAlign;
        const psp_tune_choice_t ch = resolve_choice(p, PSP_PATH_SPARSE_TAIL, batch, K, 1);
        const Knobs kn = knobs_of(ch);
        HIP_TRY(launch_adapt_reset(count, st), "adapt reset launch");
        HIP_TRY(sparse_tail_run(s, p->sp, batch, values, es, d, B, X, info, Xk, nullptr, tws, st, kn),
                "dense-block path launch");
        AdaptArgs a{};
        a.n = s.n; a.K = K; a.batch = batch; a.pass = 1; a.combine = 0; a.tol = tol;
        a.Xk = Xk; a.X = X; a.est = est; a.scale = scale; a.list = list; a.count = count;
        HIP_TRY(launch_adapt(a, c, st), "error-test launch");
        HIP_TRY(sparse_tail_run(s, p->sp, batch, values, es, d, B, X, info, Xk, scale, tws, st, kn),
                "dense-block path launch (rescaled nodes)");
        a.pass = 2;
        HIP_TRY(launch_adapt(a, c, st), "error-test launch (rescaled nodes)");
        return PSP_OK;
    }
    const bool per_jacobian = steps_per_jacobian(p->sp, batch);
    HIP_TRY(launch_adapt_reset(count, st), "adapt reset launch");
    HIP_TRY(steps_run(p->sp, s.nnz, batch, values, es, d, B, X, Xk, info, per_jacobian, st, true), "step-kernel launch");
    AdaptArgs a{};
    a.n = s.n; a.K = K; a.batch = batch; a.pass = 1; a.combine = per_jacobian ? 0 : 1; a.tol = tol;
    a.Xk = Xk; a.X = X; a.est = est; a.scale = scale; a.list = list; a.count = count;
    HIP_TRY(launch_adapt(a, c, st), "error-test launch");
    HIP_TRY(steps_run_list(p->sp, s.nnz, batch, values, es, d, B, Xk, info, list, count, scale, st),
            "step-kernel launch (rescaled nodes)");
    a.pass = 2;
    a.combine = 1;
    HIP_TRY(launch_adapt(a, c, st), "error-test launch (rescaled nodes)");
    return PSP_OK;
}

psp_status psp_tune(psp_plan p, int32_t batch, const double* values, int32_t K, const double* eps, const double* d,
                    int32_t nrhs, const double* B, double* X, int32_t* info, void* ws, size_t ws_bytes, void* stream,
                    int32_t* chosen, float* ms) {
    if (!p) return fail(PSP_E_INVALID, "psp_tune: NULL plan");
    const hipStream_t st = (hipStream_t)stream;
    if (ms)
        for (int c = 0; c <= PSP_PATH_SPARSE_TAIL; ++c) ms[c] = -1.0f;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
    HIP_TRY(hipEventCreate(&e1), "hipEventCreate");
    psp_tune_choice_t best{};
    bool have = false;
    psp_status last = PSP_OK;
    for (int32_t c = PSP_PATH_DENSE; c <= PSP_PATH_SPARSE_TAIL && last == PSP_OK; ++c) {
        if (c == PSP_PATH_SPARSE) continue;   // its executions are tried one by one
        if (path_workspace(p->sym, c, batch, K, nrhs, 0) > ws_bytes) continue;
        // the launch choices searched on this path
        std::vector<psp_tune_choice_t> cand;
        const psp_tune_choice_t base = default_choice(c);
        if (c == PSP_PATH_SPARSE_STEPS) {
            const bool two = steps_ready(p->sp) && steps_per_cu(p->sp) == 2;
            for (int mode = 0; mode <= 1; ++mode)
                for (int wgcu = 0; wgcu <= (two ? 1 : 0); ++wgcu)
                    for (int ring : {7, 4}) {
                        psp_tune_choice_t v = base;
                        v.steps_mode = mode;
                        v.steps_wgcu = wgcu;
                        v.ring = ring;
                        cand.push_back(v);
                    }
        } else if (c == PSP_PATH_SPARSE_TAIL) {
            for (int cols : {16, 4, 1})
                for (int il : {1, 0})
                    for (int lu : {1, 0}) {
                        if (il && cols != 16) continue;
                        psp_tune_choice_t v = base;
                        v.tail_cols = cols;
                        v.tail_il = il;
                        v.tail_lu = lu;
                        cand.push_back(v);
                    }
        } else {
            cand.push_back(base);
        }
        for (const psp_tune_choice_t& v : cand) {
            psp_status r = solve_choice(p, v, batch, values, K, eps, d, nrhs, B, X, info, ws, ws_bytes, stream);
            if (r == PSP_E_UNSUPPORTED) break;
            if (r != PSP_OK) { last = r; break; }
            HIP_TRY(hipEventRecord(e0, st), "hipEventRecord");
            for (int rep = 0; rep < 3 && r == PSP_OK; ++rep)
                r = solve_choice(p, v, batch, values, K, eps, d, nrhs, B, X, info, ws, ws_bytes, stream);
            if (r != PSP_OK) { last = r; break; }
            HIP_TRY(hipEventRecord(e1, st), "hipEventRecord");
            HIP_TRY(hipEventSynchronize(e1), "hipEventSynchronize");
            float t = 0.0f;
            HIP_TRY(hipEventElapsedTime(&t, e0, e1), "hipEventElapsedTime");
            t /= 3.0f;
            if (ms && (ms[c] < 0.0f || t < ms[c])) ms[c] = t;
            if (!have || t < best.ms) {
                best = v;
                best.ms = t;
                have = true;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (last != PSP_OK) return last;
    if (!have) return fail(PSP_E_UNSUPPORTED, "psp_tune: no path fits the workspace");
    best.source = 1;
    {
        std::lock_guard<std::mutex> g(p->mu);
        p->tuned[std::make_tuple(batch, K, nrhs)] = best;
    }
    cache_store(cache_key(p, batch, K, nrhs), best);
    if (chosen) *chosen = best.path;
    // leave X / info from the chosen path
    return solve_choice(p, best, batch, values, K, eps, d, nrhs, B, X, info, ws, ws_bytes, stream);
}

psp_status psp_factor(psp_plan p, int32_t path, int32_t batch, const double* values, int32_t K, const double* eps,
                      const double* d, int32_t* info, void* ws, size_t ws_bytes, void* stream, psp_factors* out) {
    if (!out) return fail(PSP_E_INVALID, "out must not be NULL");
    *out = nullptr;
    if (!p || batch < 1 || !values || !info || !ws) return fail(PSP_E_INVALID, "psp_factor: NULL argument or batch < 1");
    EpsSet es;
    if (psp_status st = make_eps(K, eps, es)) return st;
    if (psp_status st = check_prior_hip()) return st;
    const Symbolic& s = p->sym;
    int32_t pth = split_path(path == PSP_PATH_AUTO ? heuristic_path(s) : path).base;
    if (pth < 0) return fail(PSP_E_INVALID, "unknown path");
    const hipStream_t st = (hipStream_t)stream;
    auto f = std::make_unique<psp_factors_s>();
    f->plan = p; f->path = pth; f->batch = batch; f->K = K; f->es = es;
    f->ws = (char*)ws; f->ws_bytes = ws_bytes; f->info = info;
    if (pth == PSP_PATH_DENSE) {
        if (s.n > kDenseMaxN) return fail(PSP_E_UNSUPPORTED, "dense path supports n <= 4096");
        // the nrhs capacity is whatever the workspace holds beyond the factors
        const DenseLayout L0 = dense_layout(s, batch, K, 0, 1);
        if (ws_bytes < (size_t)L0.total) return fail(PSP_E_NOMEM, "workspace too small for the factors");
        const int64_t per_rhs = (int64_t)batch * K * L0.ld * 8;
        f->nrhs_cap = (int32_t)std::min<int64_t>(64, ((int64_t)ws_bytes - L0.off_tmp) / per_rhs);
        if (psp_status r = require_upload(p)) return r;
        f->n_pad = L0.n_pad; f->ld = L0.ld; f->slot_stride = L0.slot_stride;
        f->off_slots = L0.off_slots; f->off_tmp = L0.off_tmp;
        DenseArgs a{};
        a.n = s.n; a.n_pad = L0.n_pad; a.ld = L0.ld; a.nrhs = 0; a.nnz = s.nnz; a.batch = batch;
        a.dst = p->d_dst; a.perm = p->d_perm; a.values = values; a.dvec = d; a.B = nullptr; a.Xk = nullptr;
        a.info = info; a.slots = (double*)(f->ws + L0.off_slots); a.slot_stride = L0.slot_stride;
        a.ntasks = batch * K; a.keep = 1;
        int occ = 1;
        if (dense_occupancy(&occ) != hipSuccess || occ < 1) occ = 1;
        const int grid = (int)std::min<int64_t>((int64_t)a.ntasks, (int64_t)occ * device_cus());
        HIP_TRY(launch_dense_factor_solve(a, es, grid, st), "dense factor launch");
    } else if (pth == PSP_PATH_SPARSE) {
        const size_t need0 = sparse_workspace_bytes(s, batch, K, 0, 1);
        if (ws_bytes < need0) return fail(PSP_E_NOMEM, "workspace too small for the factors");
        if (psp_status r = require_upload(p)) return r;
        f->nrhs_cap = sparse_nrhs_capacity(s, batch, K, ws_bytes);
        HIP_TRY(sparse_factor(s, p->sp, batch, values, es, d, info, ws, st), "sparse factor launch");
    } else {
        return fail(PSP_E_INVALID, "unknown path");
    }
    *out = f.release();
    return PSP_OK;
}

psp_status psp_solve(psp_factors f, int32_t nrhs, const double* B, double* Xk, int32_t transpose, void* stream) {
    if (!f || !B || !Xk) return fail(PSP_E_INVALID, "psp_solve: NULL argument");
    if (nrhs < 1 || nrhs > f->nrhs_cap) return fail(PSP_E_INVALID, "psp_solve: nrhs outside 1..capacity of the workspace");
    const Symbolic& s = f->plan->sym;
    const hipStream_t st = (hipStream_t)stream;
    if (f->path == PSP_PATH_DENSE) {
        DenseSolveArgs a{};
        a.n = s.n; a.n_pad = f->n_pad; a.ld = f->ld; a.nrhs = nrhs; a.K = f->K; a.ntasks = f->batch * f->K;
        a.trans = transpose ? 1 : 0; a.perm = f->plan->d_perm; a.slots = (const double*)(f->ws + f->off_slots);
        a.slot_stride = f->slot_stride; a.B = B; a.Xk = Xk; a.info = f->info; a.tmp = (double*)(f->ws + f->off_tmp);
        const int grid = std::min(a.ntasks, 2 * device_cus());
        HIP_TRY(launch_dense_solve(a, grid, st), "dense solve launch");
        return PSP_OK;
    }
    HIP_TRY(sparse_solve(s, f->plan->sp, f->batch, f->es, nrhs, B, Xk, transpose, f->info, f->ws, st), "sparse solve launch");
    return PSP_OK;
}

psp_status psp_combine(psp_factors f, int32_t nrhs, const double* Xk, double* X, void* stream) {
    if (!f || !Xk || !X || nrhs < 1) return fail(PSP_E_INVALID, "psp_combine: bad argument");
    HIP_TRY(launch_combine((int64_t)f->plan->sym.n * nrhs, f->batch, f->es, Xk, X, (hipStream_t)stream), "combine launch");
    return PSP_OK;
}

psp_status psp_grad_values(psp_factors f, int32_t nrhs, const double* Lamk, const double* Xk, double* gA, void* stream) {
    if (!f || !Lamk || !Xk || !gA || nrhs < 1) return fail(PSP_E_INVALID, "psp_grad_values: bad argument");
    const Symbolic& s = f->plan->sym;
    HIP_TRY(launch_grad_values(s.n, s.nnz, f->batch, nrhs, f->es, f->plan->d_rows, f->plan->d_cols, Lamk, Xk, gA,
                               (hipStream_t)stream),
            "gradient launch");
    return PSP_OK;
}

psp_status psp_residual(psp_plan p, int32_t batch, const double* values, int32_t nrhs, const double* B,
                        const double* X, double* R, double* rnorm, double* bnorm, void* stream) {
    if (!p || batch < 1 || nrhs < 1 || !values || !B || !X || !rnorm)
        return fail(PSP_E_INVALID, "psp_residual: NULL argument, batch < 1 or nrhs < 1");
    if ((int64_t)batch * nrhs > INT32_MAX) return fail(PSP_E_INVALID, "psp_residual: batch * nrhs too large");
    if (!R && p->sym.n > kResLds)
        return fail(PSP_E_UNSUPPORTED, "psp_residual: n > " + std::to_string(kResLds) + " needs the R output");
    if (psp_status st = check_prior_hip()) return st;
    if (psp_status r = require_upload(p)) return r;
    const Symbolic& s = p->sym;
    ResArgs a{};
    a.n = s.n; a.nnz = s.nnz; a.batch = batch; a.nrhs = nrhs;
    a.rowptr = p->d_rowptr; a.cols = p->d_cols; a.values = values; a.B = B; a.X = X;
    a.R = R; a.rnorm = rnorm; a.bnorm = bnorm;
    HIP_TRY(launch_residual(a, (hipStream_t)stream), "residual launch");
    return PSP_OK;
}

psp_status psp_factors_release(psp_factors f) {
    delete f;
    return PSP_OK;
}

}  // extern "C"

namespace {

struct RhoLayout {
    bool refactor;   // factor and solve afresh each step (step kernel) instead of keeping the factors
    int64_t fac_bytes, off_B, off_X, off_v, off_acc, off_info, total;
};

RhoLayout rho_layout(psp_plan p, int32_t batch) {
    const int64_t n = p->sym.n;
    RhoLayout L{};
    // When the step schedule fits, one fused factor-and-solve per step (~0.25 ms for 512
    // Jacobians at n = 601) is far cheaper than a solve with kept factors on the per-level
    // path (~6 ms); both give the same bits.
    L.refactor = steps_fit(p->sym, 1);
    L.fac_bytes = (int64_t)psp_workspace_bytes(p, PSP_PATH_SPARSE, batch, 1, 1, L.refactor ? 0 : 1);
    int64_t off = align_up(L.fac_bytes, kAlign);
    L.off_B = off;
    off = align_up(off + (int64_t)batch * n * 8, kAlign);
    L.off_X = off;
    off = align_up(off + (int64_t)batch * n * 8, kAlign);
    L.off_v = off;
    off = align_up(off + (int64_t)batch * n * 8, kAlign);
    L.off_acc = off;
    off = align_up(off + (int64_t)batch * 8, kAlign);
    L.off_info = off;
    L.total = align_up(off + (int64_t)batch * 4, kAlign);
    return L;
}

}  // namespace

extern "C" {

size_t psp_estimate_rho_workspace_bytes(psp_plan p, int32_t batch) {
    if (!p || batch < 1) return 0;
    return (size_t)rho_layout(p, batch).total;
}

psp_status psp_estimate_rho(psp_plan p, int32_t batch, const double* values, const double* d, double probe,
                            int32_t iters, const double* v0, double* rho, void* ws, size_t ws_bytes, void* stream) {
    if (!p || batch < 1 || !values || !v0 || !rho || !ws)
        return fail(PSP_E_INVALID, "psp_estimate_rho: NULL argument or batch < 1");
    if (iters < 1 || iters > 100000) return fail(PSP_E_INVALID, "psp_estimate_rho: iters must be in 1..100000");
    const RhoLayout L = rho_layout(p, batch);
    if (ws_bytes < (size_t)L.total) return fail(PSP_E_NOMEM, "workspace too small: need " + std::to_string(L.total) + " bytes");
    char* w = (char*)ws;
    int32_t* info = (int32_t*)(w + L.off_info);
    psp_factors f = nullptr;
    if (!L.refactor) {
        if (psp_status st = psp_factor(p, PSP_PATH_SPARSE, batch, values, 1, &probe, d, info, ws, (size_t)L.fac_bytes,
                                       stream, &f))
            return st;
    } else if (!(probe != 0.0) || !std::isfinite(probe)) {
        return fail(PSP_E_EPS, "psp_estimate_rho: probe must be nonzero and finite");
    }
    std::unique_ptr<psp_factors_s> hold(f);
    const hipStream_t st = (hipStream_t)stream;
    RhoArgs a{};
    a.n = p->sym.n; a.batch = batch; a.d = d;
    a.v = (double*)(w + L.off_v); a.B = (double*)(w + L.off_B); a.acc = (double*)(w + L.off_acc); a.rho = rho;
    const int32_t half = iters / 2;
    a.inv_count = 1.0 / (double)(iters - half);
    a.mode = 0;
    a.src = v0;
    HIP_TRY(launch_rho_step(a, st), "rho launch");
    double* X = (double*)(w + L.off_X);
    for (int32_t it = 0; it < iters; ++it) {
        if (L.refactor) {
            if (psp_status r = psp_solve_batched(p, PSP_PATH_SPARSE, batch, values, 1, &probe, d, 1, a.B, X, info, ws,
                                                 (size_t)L.fac_bytes, stream))
                return r;
        } else if (psp_status r = psp_solve(f, 1, a.B, X, 0, stream)) {
            return r;
        }
        a.src = X;
        a.mode = it < half ? 1 : (it == iters - 1 ? 3 : 2);
        HIP_TRY(launch_rho_step(a, st), "rho launch");
    }
    return PSP_OK;
}

}  // extern "C"

struct psp_pf_s {
    psp_plan plan = nullptr;
    int32_t N = 0, ny = 0, pos_ref = 0;
    int device = -1;
    // network arrays in the caller's device buffer (psp_pf_device_bytes)
    const int32_t *d_yptr = nullptr, *d_ycol = nullptr, *d_pv = nullptr, *d_poslam = nullptr;
    const double *d_g = nullptr, *d_b = nullptr;
    const int4* d_pos = nullptr;
    std::vector<int32_t> h_status, h_idx;   // host copies: statuses, running scenarios
};

namespace {

// Byte offsets of the network arrays in the caller's buffer.
struct PfNetLayout {
    int64_t yptr, ycol, pv, poslam, pos, g, b, total;
};

PfNetLayout pf_net_layout(int64_t N, int64_t ny) {
    PfNetLayout L{};
    int64_t off = 0;
    auto take = [&](int64_t bytes) { const int64_t o = off; off = align_up(off + std::max<int64_t>(bytes, 1), kAlign); return o; };
    L.yptr = take(4 * (N + 1));
    L.ycol = take(4 * ny);
    L.pv = take(4 * N);
    L.poslam = take(4 * N);
    L.pos = take(16 * ny);
    L.g = take(8 * ny);
    L.b = take(8 * ny);
    L.total = off;
    return L;
}

struct PfLayout {
    int64_t off_F, off_J, off_dx, off_info, off_idx, total;
    size_t solve_bytes;
};

PfLayout pf_layout(psp_pf pf, int32_t path, int32_t batch, int32_t K) {
    const Symbolic& s = pf->plan->sym;
    PfLayout L{};
    L.solve_bytes = psp_workspace_bytes(pf->plan, path, batch, K, 1, 0);
    int64_t off = align_up((int64_t)L.solve_bytes, kAlign);
    L.off_F = off;
    off = align_up(off + (int64_t)batch * s.n * 8, kAlign);
    L.off_J = off;
    off = align_up(off + (int64_t)batch * s.nnz * 8, kAlign);
    L.off_dx = off;
    off = align_up(off + (int64_t)batch * s.n * 8, kAlign);
    L.off_info = off;
    off = align_up(off + (int64_t)batch * K * 4, kAlign);
    L.off_idx = off;
    L.total = align_up(off + (int64_t)batch * 4, kAlign);
    return L;
}

PfArgs pf_args(psp_pf pf, int32_t batch, const double* x, const double* spec, const double* part, double* F,
               double* J, double* fnorm) {
    PfArgs a{};
    a.N = pf->N; a.n = 2 * pf->N + 1; a.nnz = pf->plan->sym.nnz; a.batch = batch;
    a.yptr = pf->d_yptr; a.ycol = pf->d_ycol; a.g = pf->d_g; a.b = pf->d_b; a.pv = pf->d_pv;
    a.pos = pf->d_pos; a.pos_lam = pf->d_poslam; a.pos_ref = pf->pos_ref;
    a.x = x; a.spec = spec; a.part = part; a.F = F; a.J = J; a.fnorm = fnorm;
    return a;
}

psp_status pf_device_check(psp_pf pf) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev != pf->device) return fail(PSP_E_STATE, "power-flow handle was created on another device");
    return PSP_OK;
}

}  // namespace

extern "C" {

size_t psp_pf_device_bytes(int32_t nbus, int32_t nnz_y) {
    if (nbus < 1 || nnz_y < 0) return 0;
    return (size_t)pf_net_layout(nbus, nnz_y).total;
}

psp_status psp_pf_create(psp_plan plan, int32_t nbus, const int32_t* yp, const int32_t* yc, const double* g,
                         const double* b, const int32_t* pv, void* dev, size_t dev_bytes, void* stream, psp_pf* out) {
    if (!out) return fail(PSP_E_INVALID, "out must not be NULL");
    *out = nullptr;
    if (!plan || nbus < 1 || !yp || !yc || !g || !b || !pv || !dev)
        return fail(PSP_E_INVALID, "psp_pf_create: NULL argument or nbus < 1");
    if (((uintptr_t)dev & 255) != 0) return fail(PSP_E_INVALID, "psp_pf_create: device buffer must be 256-byte aligned");
    const Symbolic& s = plan->sym;
    if ((int64_t)s.n != 2LL * nbus + 1) return fail(PSP_E_INVALID, "psp_pf_create: plan order must be 2*nbus + 1");
    const std::string why = validate_csr(nbus, yp, yc);
    if (!why.empty()) return fail(PSP_E_INVALID, "psp_pf_create: admittance matrix: " + why);
    const int32_t N = nbus, ny = yp[N];
    const PfNetLayout NL = pf_net_layout(N, ny);
    if (dev_bytes < (size_t)NL.total)
        return fail(PSP_E_NOMEM, "psp_pf_create: device buffer too small: need " + std::to_string(NL.total) + " bytes");
    for (int32_t e = 0; e < ny; ++e)
        if (!std::isfinite(g[e]) || !std::isfinite(b[e]))
            return fail(PSP_E_INVALID, "psp_pf_create: non-finite admittance");
    for (int32_t i = 0; i < N; ++i) {
        bool diag = false;
        for (int32_t e = yp[i]; e < yp[i + 1]; ++e) diag |= yc[e] == i;
        if (!diag) return fail(PSP_E_INVALID, "psp_pf_create: admittance row without a diagonal entry");
    }
    if ((int64_t)s.nnz != 4LL * ny + N + 1)
        return fail(PSP_E_INVALID, "psp_pf_create: plan pattern is not the power-flow Jacobian pattern of this network");
    auto find = [&](int32_t r, int32_t c) -> int32_t {
        const int32_t* lo = s.col_idx.data() + s.row_ptr[r];
        const int32_t* hi = s.col_idx.data() + s.row_ptr[r + 1];
        const int32_t* it = std::lower_bound(lo, hi, c);
        return (it != hi && *it == c) ? (int32_t)(it - s.col_idx.data()) : -1;
    };
    std::vector<int4> pos(std::max(ny, 1));
    std::vector<int32_t> poslam(N);
    for (int32_t i = 0; i < N; ++i) {
        for (int32_t e = yp[i]; e < yp[i + 1]; ++e) {
            const int32_t j = yc[e];
            pos[e] = make_int4(find(i, j), find(i, N + j), find(N + i, j), find(N + i, N + j));
            if (pos[e].x < 0 || pos[e].y < 0 || pos[e].z < 0 || pos[e].w < 0)
                return fail(PSP_E_INVALID, "psp_pf_create: plan pattern lacks a Jacobian entry of this network");
        }
        poslam[i] = find(i, 2 * N);
        if (poslam[i] < 0) return fail(PSP_E_INVALID, "psp_pf_create: plan pattern lacks the lambda column");
    }
    const int32_t pref = find(2 * N, 0);
    if (pref < 0) return fail(PSP_E_INVALID, "psp_pf_create: plan pattern lacks the angle-reference entry");
    if (psp_status st = check_prior_hip()) return st;
    if (psp_status r = require_upload(plan)) return r;   // also checks the device
    // one host image of the network arrays, copied with one transfer
    std::vector<char> host((size_t)NL.total, 0);
    std::memcpy(host.data() + NL.yptr, yp, 4 * (size_t)(N + 1));
    std::memcpy(host.data() + NL.ycol, yc, 4 * (size_t)ny);
    std::memcpy(host.data() + NL.pv, pv, 4 * (size_t)N);
    std::memcpy(host.data() + NL.poslam, poslam.data(), 4 * (size_t)N);
    std::memcpy(host.data() + NL.pos, pos.data(), 16 * (size_t)ny);
    std::memcpy(host.data() + NL.g, g, 8 * (size_t)ny);
    std::memcpy(host.data() + NL.b, b, 8 * (size_t)ny);
    const hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(dev, host.data(), host.size(), hipMemcpyHostToDevice, st), "hipMemcpyAsync(power flow)");
    HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize(power flow)");
    auto pf = std::make_unique<psp_pf_s>();
    pf->plan = plan; pf->N = N; pf->ny = ny; pf->pos_ref = pref;
    HIP_TRY(hipGetDevice(&pf->device), "hipGetDevice");
    const char* base = (const char*)dev;
    pf->d_yptr = (const int32_t*)(base + NL.yptr);
    pf->d_ycol = (const int32_t*)(base + NL.ycol);
    pf->d_pv = (const int32_t*)(base + NL.pv);
    pf->d_poslam = (const int32_t*)(base + NL.poslam);
    pf->d_pos = (const int4*)(base + NL.pos);
    pf->d_g = (const double*)(base + NL.g);
    pf->d_b = (const double*)(base + NL.b);
    *out = pf.release();
    return PSP_OK;
}

void psp_pf_destroy(psp_pf pf) { delete pf; }

psp_status psp_pf_eval(psp_pf pf, int32_t batch, const double* x, const double* spec, const double* part, double* F,
                       double* J, double* fnorm, void* stream) {
    if (!pf || batch < 1 || !x || !spec || !part || !F) return fail(PSP_E_INVALID, "psp_pf_eval: NULL argument or batch < 1");
    if (psp_status st = check_prior_hip()) return st;
    if (psp_status st = pf_device_check(pf)) return st;
    HIP_TRY(launch_pf_eval(pf_args(pf, batch, x, spec, part, F, J, fnorm), (hipStream_t)stream), "power-flow launch");
    return PSP_OK;
}

size_t psp_pf_workspace_bytes(psp_pf pf, int32_t path, int32_t batch, int32_t K) {
    if (!pf || batch < 1 || K < 1) return 0;
    return (size_t)pf_layout(pf, path, batch, K).total;
}

psp_status psp_pf_newton(psp_pf pf, int32_t path, int32_t batch, int32_t K, const double* eps, const double* d,
                         double* x, const double* spec, const double* part, double tol, int32_t max_iter,
                         int32_t* iters, int32_t* status, double* fnorm, void* ws, size_t ws_bytes, void* stream) {
    if (!pf || batch < 1 || !x || !spec || !part || !iters || !status || !fnorm || !ws)
        return fail(PSP_E_INVALID, "psp_pf_newton: NULL argument or batch < 1");
    if (max_iter < 0 || !(tol >= 0.0) || !std::isfinite(tol))
        return fail(PSP_E_INVALID, "psp_pf_newton: max_iter < 0 or tol negative / not finite");
    EpsSet es;
    if (psp_status st = make_eps(K, eps, es)) return st;
    if (psp_status st = check_prior_hip()) return st;
    if (psp_status st = pf_device_check(pf)) return st;
    if (split_path(path).base < 0 && path != PSP_PATH_AUTO) return fail(PSP_E_INVALID, "unknown path");
    const PfLayout L = pf_layout(pf, path, batch, K);
    if (ws_bytes < (size_t)L.total) return fail(PSP_E_NOMEM, "workspace too small: need " + std::to_string(L.total) + " bytes");
    try {
        if ((int32_t)pf->h_status.size() < batch) {
            pf->h_status.resize(batch);
            pf->h_idx.resize(batch);
        }
    } catch (const std::bad_alloc&) {
        return fail(PSP_E_NOMEM, "psp_pf_newton: host allocation failed");
    }
    int32_t* h_status = pf->h_status.data();
    int32_t* h_idx = pf->h_idx.data();
    char* w = (char*)ws;
    double* F = (double*)(w + L.off_F);
    double* J = (double*)(w + L.off_J);
    double* dx = (double*)(w + L.off_dx);
    int32_t* info = (int32_t*)(w + L.off_info);
    int32_t* idx = (int32_t*)(w + L.off_idx);
    const hipStream_t st = (hipStream_t)stream;
    HIP_TRY(launch_pf_status(batch, status, iters, 0, st), "power-flow status launch");
    // Each iteration works on the scenarios that were running after the previous
    // evaluation (all at first): evaluate them into rows 0..m-1, and if any is
    // still running, solve those m systems and update.  A scenario that converges
    // at this evaluation is solved once more but not updated (its status changed).
    int32_t m = batch;
    for (int32_t r = 0; r < batch; ++r) h_idx[r] = r;
    for (int32_t it = 0;; ++it) {
        HIP_TRY(hipMemcpyAsync(idx, h_idx, sizeof(int32_t) * m, hipMemcpyHostToDevice, st), "hipMemcpyAsync(idx)");
        PfArgs a = pf_args(pf, m, x, spec, part, F, J, fnorm);
        a.idx = idx;
        a.status = status;
        a.tol = tol;
        HIP_TRY(launch_pf_eval(a, st), "power-flow launch");
        HIP_TRY(hipMemcpyAsync(h_status, status, sizeof(int32_t) * batch, hipMemcpyDeviceToHost, st),
                "hipMemcpyAsync(status)");
        HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
        const bool running = std::any_of(h_status, h_status + batch, [](int32_t v) { return v == kPfRunning; });
        if (!running || it == max_iter) break;
        if (psp_status r = psp_solve_batched(pf->plan, path, m, J, K, eps, d, 1, F, dx, info, ws, L.solve_bytes, stream))
            return r;
        HIP_TRY(launch_pf_update(m, 2 * pf->N + 1, K, idx, x, dx, info, status, iters, st), "power-flow update launch");
        // the idx copy above has completed (the stream was synchronised), so the list can be rebuilt
        m = 0;
        for (int32_t r = 0; r < batch; ++r)
            if (h_status[r] == kPfRunning) h_idx[m++] = r;
    }
    HIP_TRY(launch_pf_status(batch, status, iters, 1, st), "power-flow status launch");
    return PSP_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- groups
struct psp_group_s {
    std::vector<psp_group_shape_t> items;   // path resolved at creation
    std::vector<psp_tune_choice_t> choice;  // with its launch choices
    std::vector<size_t> ws_off, ws_len;     // each item's slice of the workspace
    std::vector<size_t> ad_off, ad_len;     // the same for the adaptive run (psp_solve_adaptive per item)
    size_t ad_total = 0;
    std::vector<int32_t> order, lane;       // LPT order; stream lane of each item (0: the caller's)
    size_t ws_total = 0;
    int32_t K = 0, nrhs = 0, nlanes = 1, device = -1;
    std::vector<double> eps;
    hipStream_t streams[4] = {};            // lanes 1..nlanes-1 (lane 0 is the caller's stream)
    hipEvent_t fork = nullptr, join[4] = {};
    ~psp_group_s() {
        int cur = 0;
        (void)hipGetDevice(&cur);
        if (device >= 0) (void)hipSetDevice(device);
        for (int l = 1; l < nlanes; ++l) {
            if (join[l]) (void)hipEventDestroy(join[l]);
            if (streams[l]) (void)hipStreamDestroy(streams[l]);
        }
        if (fork) (void)hipEventDestroy(fork);
        if (device >= 0) (void)hipSetDevice(cur);
    }
};

namespace {

constexpr int kGroupLanes = 4;   // the caller's stream and three more (GPU_MAX_HW_QUEUES is 4)

// Relative cost of an item for the longest-first ordering: sparse flops of one
// factorisation plus the substitutions, times the systems of the item.
double item_cost(const psp_group_shape_t& it, int32_t K, int32_t nrhs) {
    const Symbolic& s = it.plan->sym;
    const double per = (double)s.flops_sparse + 4.0 * (double)s.l_ptr[s.n] * nrhs + 64.0 * s.n;
    return per * it.batch * K;
}

// outs != NULL: every item through psp_solve_adaptive (error test + rescale) instead of its path.
psp_status group_enqueue(psp_group g, const psp_group_task_t* tasks, char* ws, hipStream_t st,
                         const psp_group_adapt_t* outs = nullptr, double tol = 0.0) {
    const bool forked = g->nlanes > 1;
    if (forked) {
        HIP_TRY(hipEventRecord(g->fork, st), "hipEventRecord(fork)");
        for (int l = 1; l < g->nlanes; ++l) HIP_TRY(hipStreamWaitEvent(g->streams[l], g->fork, 0), "hipStreamWaitEvent");
    }
    psp_status bad = PSP_OK;
    for (int32_t i : g->order) {
        const psp_group_shape_t& it = g->items[i];
        const psp_group_task_t& t = tasks[i];
        const hipStream_t ls = g->lane[i] == 0 ? st : g->streams[g->lane[i]];
        if (outs)
            bad = psp_solve_adaptive(it.plan, it.batch, t.values, g->K, g->eps.data(), t.d, tol, t.B, t.X, t.info,
                                     outs[i].est, outs[i].scale, ws + g->ad_off[i], g->ad_len[i], (void*)ls);
        else
            bad = solve_choice(it.plan, g->choice[i], it.batch, t.values, g->K, g->eps.data(), t.d, g->nrhs, t.B, t.X,
                               t.info, ws + g->ws_off[i], g->ws_len[i], (void*)ls);
        if (bad != PSP_OK) {
            g_err = "group item " + std::to_string(i) + ": " + g_err;
            break;
        }
    }
    // join every lane back into the caller's stream, also after a failure
    if (forked)
        for (int l = 1; l < g->nlanes; ++l) {
            HIP_TRY(hipEventRecord(g->join[l], g->streams[l]), "hipEventRecord(join)");
            HIP_TRY(hipStreamWaitEvent(st, g->join[l], 0), "hipStreamWaitEvent");
        }
    return bad;
}

psp_status group_check(psp_group g, const psp_group_task_t* tasks, void* ws, size_t ws_bytes,
                       const psp_group_adapt_t* outs = nullptr, bool adaptive = false) {
    if (!g || !tasks || !ws) return fail(PSP_E_INVALID, "psp_group: NULL argument");
    const size_t need = adaptive ? g->ad_total : g->ws_total;
    if (ws_bytes < need) return fail(PSP_E_NOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
    if (adaptive) {
        if (!outs) return fail(PSP_E_INVALID, "psp_group: NULL outputs");
        if (g->nrhs != 1 || g->K < 3)
            return fail(PSP_E_INVALID, "psp_group adaptive: needs nrhs = 1 and K >= 3 nodes");
        for (size_t i = 0; i < g->items.size(); ++i) {
            if (!outs[i].est || !outs[i].scale)
                return fail(PSP_E_INVALID, "psp_group: item " + std::to_string(i) + " has a NULL est or scale");
            if (g->ad_len[i] == 0)
                return fail(PSP_E_UNSUPPORTED, "psp_group adaptive: item " + std::to_string(i) +
                                                   " has neither a step schedule nor a dense trailing block path");
        }
    }
    if (((uintptr_t)ws & 255) != 0) return fail(PSP_E_INVALID, "psp_group: workspace must be 256-byte aligned");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev != g->device) return fail(PSP_E_STATE, "group was created on another device");
    for (size_t i = 0; i < g->items.size(); ++i)
        if (!tasks[i].values || !tasks[i].B || !tasks[i].X || !tasks[i].info)
            return fail(PSP_E_INVALID, "psp_group: task " + std::to_string(i) + " has a NULL pointer");
    return PSP_OK;
}

}  // namespace

extern "C" {

psp_status psp_group_create(int32_t nitems, const psp_group_shape_t* shapes, int32_t K, const double* eps, int32_t nrhs,
                            psp_group* out) {
    if (!out) return fail(PSP_E_INVALID, "out must not be NULL");
    *out = nullptr;
    if (nitems < 1 || !shapes) return fail(PSP_E_INVALID, "psp_group_create: no items");
    if (nrhs < 1 || nrhs > 64) return fail(PSP_E_INVALID, "psp_group_create: nrhs must be in 1..64");
    EpsSet es;
    if (psp_status st = make_eps(K, eps, es)) return st;
    for (int32_t i = 0; i < nitems; ++i)
        if (!shapes[i].plan || shapes[i].batch < 1)
            return fail(PSP_E_INVALID, "psp_group_create: item " + std::to_string(i) + " has no plan or batch < 1");
    auto g = std::make_unique<psp_group_s>();
    HIP_TRY(hipGetDevice(&g->device), "hipGetDevice");
    g->K = K;
    g->nrhs = nrhs;
    g->eps.assign(eps, eps + K);
    std::vector<double> cost(nitems);
    for (int32_t i = 0; i < nitems; ++i) {
        psp_group_shape_t it = shapes[i];
        if (psp_status r = require_upload(it.plan)) return fail(r, "psp_group_create: item " + std::to_string(i) + ": " + g_err);
        const psp_tune_choice_t ch = resolve_choice(it.plan, it.path, it.batch, K, nrhs);
        it.path = ch.path;
        if (split_path(it.path).base < 0) return fail(PSP_E_INVALID, "psp_group_create: unknown path");
        g->choice.push_back(ch);
        const size_t w = psp_workspace_bytes(it.plan, it.path, it.batch, K, nrhs, 0);
        if (w == 0) return fail(PSP_E_INVALID, "psp_group_create: item " + std::to_string(i) + " cannot run on its path");
        g->items.push_back(it);
        g->ws_off.push_back(g->ws_total);
        g->ws_len.push_back(w);
        g->ws_total += (size_t)align_up((int64_t)w, kAlign);
        const size_t wa = (nrhs == 1 && K >= 3) ? psp_solve_adaptive_workspace_bytes(it.plan, it.batch, K) : 0;
        g->ad_off.push_back(g->ad_total);
        g->ad_len.push_back(wa);
        g->ad_total += (size_t)align_up((int64_t)wa, kAlign);
        cost[i] = item_cost(it, K, nrhs);
    }
    // longest item first, each to the least-loaded lane
    g->order.resize(nitems);
    for (int32_t i = 0; i < nitems; ++i) g->order[i] = i;
    std::stable_sort(g->order.begin(), g->order.end(), [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
    g->nlanes = std::min<int32_t>(kGroupLanes, nitems);
    std::vector<double> load(g->nlanes, 0.0);
    g->lane.assign(nitems, 0);
    for (int32_t i : g->order) {
        const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        g->lane[i] = l;
        load[l] += cost[i];
    }
    if (g->nlanes > 1) {
        HIP_TRY(hipEventCreateWithFlags(&g->fork, hipEventDisableTiming), "hipEventCreate");
        for (int l = 1; l < g->nlanes; ++l) {
            HIP_TRY(hipStreamCreateWithFlags(&g->streams[l], hipStreamNonBlocking), "hipStreamCreate");
            HIP_TRY(hipEventCreateWithFlags(&g->join[l], hipEventDisableTiming), "hipEventCreate");
        }
    }
    *out = g.release();
    return PSP_OK;
}

size_t psp_group_workspace_bytes(psp_group g) { return g ? std::max<size_t>(g->ws_total, 256) : 0; }

size_t psp_group_adaptive_workspace_bytes(psp_group g) { return g ? std::max<size_t>(g->ad_total, 256) : 0; }

psp_status psp_group_run(psp_group g, const psp_group_task_t* tasks, void* ws, size_t ws_bytes, void* stream) {
    if (psp_status r = group_check(g, tasks, ws, ws_bytes)) return r;
    if (psp_status st = check_prior_hip()) return st;
    return group_enqueue(g, tasks, (char*)ws, (hipStream_t)stream);
}

psp_status psp_group_run_adaptive(psp_group g, const psp_group_task_t* tasks, const psp_group_adapt_t* outs, double tol,
                                  void* ws, size_t ws_bytes, void* stream) {
    if (psp_status r = group_check(g, tasks, ws, ws_bytes, outs, true)) return r;
    if (!std::isfinite(tol) || tol < 0.0) return fail(PSP_E_INVALID, "psp_group adaptive: tol must be finite and >= 0");
    if (psp_status st = check_prior_hip()) return st;
    return group_enqueue(g, tasks, (char*)ws, (hipStream_t)stream, outs, tol);
}

psp_status group_capture(psp_group g, const psp_group_task_t* tasks, void* ws, size_t ws_bytes, void* stream,
                         void** graph_exec, const psp_group_adapt_t* outs, double tol);

psp_status psp_group_capture_adaptive(psp_group g, const psp_group_task_t* tasks, const psp_group_adapt_t* outs,
                                      double tol, void* ws, size_t ws_bytes, void* stream, void** graph_exec) {
    if (!graph_exec) return fail(PSP_E_INVALID, "psp_group_capture: NULL output");
    *graph_exec = nullptr;
    if (psp_status r = group_check(g, tasks, ws, ws_bytes, outs, true)) return r;
    if (!std::isfinite(tol) || tol < 0.0) return fail(PSP_E_INVALID, "psp_group adaptive: tol must be finite and >= 0");
    return group_capture(g, tasks, ws, ws_bytes, stream, graph_exec, outs, tol);
}

psp_status psp_group_capture(psp_group g, const psp_group_task_t* tasks, void* ws, size_t ws_bytes, void* stream,
                             void** graph_exec) {
    if (!graph_exec) return fail(PSP_E_INVALID, "psp_group_capture: NULL output");
    *graph_exec = nullptr;
    if (psp_status r = group_check(g, tasks, ws, ws_bytes)) return r;
    return group_capture(g, tasks, ws, ws_bytes, stream, graph_exec, nullptr, 0.0);
}

psp_status group_capture(psp_group g, const psp_group_task_t* tasks, void* ws, size_t ws_bytes, void* stream,
                         void** graph_exec, const psp_group_adapt_t* outs, double tol) {
    (void)ws_bytes;
    if (psp_status st = check_prior_hip()) return st;
    const hipStream_t st = (hipStream_t)stream;
    if (st == nullptr)
        return fail(PSP_E_INVALID, "psp_group_capture: the null (default) stream cannot be captured; pass a created stream");
    HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    const psp_status r = group_enqueue(g, tasks, (char*)ws, st, outs, tol);
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(st, &graph);
    if (r != PSP_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return r;
    }
    if (ee != hipSuccess) return hip_fail(ee, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return hip_fail(ei, "hipGraphInstantiate");
    *graph_exec = (void*)exec;
    return PSP_OK;
}

psp_status psp_graph_launch(void* graph_exec, void* stream) {
    if (!graph_exec) return fail(PSP_E_INVALID, "psp_graph_launch: NULL graph");
    HIP_TRY(hipGraphLaunch((hipGraphExec_t)graph_exec, (hipStream_t)stream), "hipGraphLaunch");
    return PSP_OK;
}

void psp_graph_destroy(void* graph_exec) {
    if (graph_exec) (void)hipGraphExecDestroy((hipGraphExec_t)graph_exec);
}

void psp_group_destroy(psp_group g) { delete g; }

}  // extern "C"

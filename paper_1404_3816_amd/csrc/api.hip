// Host side of the C ABI declared in include/hikf.h.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "hikf_internal.h"

namespace hikf {

Layout make_layout(const Geometry &g) {
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    const size_t m = size_t(g.m), p = size_t(g.p), tq = g.fmm_prec == HIKF_FMM_F64 ? 8 : 4;
    L.C = take(m * p * 8);
    L.CQ = take(m * p * tq);
    L.xhat = take(m * 8);
    L.var = take(m * 8);
    L.sinv = take(p * p * 8);
    L.xbuf = take(size_t(g.pp) * g.pp * 8);
    L.G = take(p * p * 8);
    L.hvec = take(p * 8);
    L.nu = take(p * 8);
    L.partial = take(p * size_t(g.cpr) * (p + 1) * 8);
    L.rowptr = take((p + 1) * 8);
    L.col = take(size_t(g.nnz) * 4);
    L.val = take(size_t(g.nnz) * 8);
    L.rdiag = take(p * 8);
    L.status = take(kNumStatus * 4);
    L.minpiv = take(8);
    L.steps = take(8);
    L.negvar = take(8);
    L.GQ = take(p * p * 8);
    L.Gn = take(p * p * 8);
    L.hpart = take(size_t(g.pp / 32) * p * 8);
    L.histC = take(size_t(g.history) * m * p * 8);
    L.histS = take(size_t(g.history) * p * p * 8);
    L.ybuf = take(p * 8);
    L.psA = take(size_t(g.pp) * g.pp * 8);
    L.pivs = take(size_t(g.pp / 32) * 8);
    L.Gg = take(p * p * 8);
    L.hg = take(p * 8);
    L.drift = take(3 * 8);
    L.hash = take(8);
    L.resident_bytes = off;

    off = 0;
    if (g.sparse) {
        // counting sort of the nonzeros by leaf: cursors, offsets, placed
        // nonzero indices, then per bucket (ray * 64 + point, value)
        const size_t leaves = size_t(g.boxes(g.depth)), nz = size_t(g.nnz);
        L.bcur = take(leaves * 4);
        L.boff = take((leaves + 1) * 4);
        L.btmp = take(nz * 4);
        L.bkey = take(nz * 4);
        L.bval = take(nz * tq);
    } else {
        L.W = take(size_t(g.mpad) * p * tq);
    }
    L.knear = take(size_t(g.dim == 2 ? 9 : 27) * kLeafPts * kLeafPts * tq);
    if (g.psd_guard) L.psw = take(3 * p * p * 8);
    if (g.far) {
        const size_t r = size_t(g.r);
        L.sleaf = take(r * kLeafPts * tq);
        L.schild = take((size_t(1) << g.dim) * r * r * tq);
        L.m2l = take(size_t(g.depth - 1) * g.noff() * r * r * tq);
        size_t ml_bytes = 0;
        for (int lev = 2; lev <= g.depth; ++lev) {
            L.ML_level[lev] = take(size_t(g.boxes(lev)) * r * p * tq);
        }
        ml_bytes = off - L.ML_level[2];
        L.L_base = take(ml_bytes);
    }
    if (g.far && g.m2l_eps > 0.0) {
        // low-rank M2L: Gram matrices and bases per level (FP64), the
        // per-slot products W, the compressed operators and the compress /
        // expand operators (pass precision), compressed M and L of a level
        const size_t r = size_t(g.r), rr = r * r, nlev = size_t(g.depth - 1);
        L.lrA = take(nlev * rr * 8);
        L.lrU = take(nlev * rr * 8);
        L.lrW = take(size_t(g.noff()) * rr * 8);
        L.lrC = take(nlev * g.noff() * rr * tq);
        L.lrUt = take(nlev * rr * tq);
        L.lrUe = take(nlev * rr * tq);
        L.lrM = take(size_t(g.boxes(g.depth)) * r * p * tq);
        L.lrL = take(size_t(g.boxes(g.depth)) * r * p * tq);
    }
    if (g.fmm_prec == HIKF_FMM_BF16X3 || g.fmm_prec == HIKF_FMM_BF16) {
        // BF16 hi / lo operands: W per leaf as [column][point], multipoles per
        // box as [column][node], M2L tables as [target node][source node],
        // node counts padded to kr32 = 32 ceil(r / 32)
        const size_t leaves = size_t(g.boxes(g.depth));
        if (!g.sparse) L.Wsplit = take(2 * leaves * p * kLeafPts * 2);
        if (g.far) {
            const size_t kr = size_t(g.kr32()), rt = size_t(g.r + 15) / 16 * 16;
            L.Tsplit = take(2 * size_t(g.depth - 1) * g.noff() * rt * kr * 2);
            for (int lev = 2; lev <= g.depth; ++lev)
                L.MS_level[lev] = take(2 * size_t(g.boxes(lev)) * p * kr * 2);
        }
    }
    L.scratch_bytes = off > 0 ? off : 256;
    return L;
}

hipError_t Timing::create() {
    // events are created on first use of a (phase, slot) pair
    on = true;
    return hipSuccess;
}

void Timing::destroy() {
    for (int ph = 0; ph < HIKF_NUM_PHASES; ++ph)
        for (int k = 0; k < kRing; ++k)
            for (int b = 0; b < 2; ++b)
                if (ev[ph][k][b]) {
                    (void)hipEventDestroy(ev[ph][k][b]);
                    ev[ph][k][b] = nullptr;
                }
    on = false;
}

hipError_t Timing::drain(int ph, int slot) {
    if (!pending[ph][slot]) return hipSuccess;
    hipError_t e = hipEventSynchronize(ev[ph][slot][1]);
    if (e != hipSuccess) return e;
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, ev[ph][slot][0], ev[ph][slot][1]);
    if (e != hipSuccess) return e;
    total_ms[ph] += ms;
    count[ph] += 1;
    pending[ph][slot] = false;
    return hipSuccess;
}

void Timing::begin(int ph, hipStream_t s) {
    const int slot = next[ph];
    cur[ph] = -1;
    if (drain(ph, slot) != hipSuccess) return;
    for (int b = 0; b < 2; ++b)
        if (!ev[ph][slot][b] && hipEventCreate(&ev[ph][slot][b]) != hipSuccess) return;
    if (hipEventRecord(ev[ph][slot][0], s) == hipSuccess) cur[ph] = slot;
}

void Timing::end(int ph, hipStream_t s) {
    const int slot = cur[ph];
    if (slot < 0) return;                          // begin() could not record
    if (hipEventRecord(ev[ph][slot][1], s) != hipSuccess) return;
    pending[ph][slot] = true;
    next[ph] = (slot + 1) % kRing;
}

hipError_t Timing::collect() {
    for (int ph = 0; ph < HIKF_NUM_PHASES; ++ph)
        for (int k = 0; k < kRing; ++k) {
            hipError_t e = drain(ph, k);
            if (e != hipSuccess) return e;
        }
    return hipSuccess;
}

}  // namespace hikf

namespace {

using hikf::Geometry;

// Internal streams of hikf_step_batch, one set per device, created on first
// use and kept until the process ends (default priority, non-blocking).
constexpr int kPool = 4;
struct StreamPool {
    hipStream_t s[kPool] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kPool] = {};
    std::mutex mu;
};

StreamPool *stream_pool() {
    static std::mutex mu;
    static std::map<int, StreamPool *> pools;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    auto it = pools.find(dev);
    if (it != pools.end()) return it->second;
    StreamPool *p = new (std::nothrow) StreamPool();
    if (!p) return nullptr;
    bool ok = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming) == hipSuccess;
    for (int k = 0; ok && k < kPool; ++k)
        ok = hipStreamCreateWithFlags(&p->s[k], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&p->join[k], hipEventDisableTiming) == hipSuccess;
    if (!ok) return nullptr;                      // fall back to one stream
    pools[dev] = p;
    return p;
}

// Built-in row-pass variant (rowpass.h) when neither the options nor a
// tuning cache choose one.
constexpr int kDefaultRowpassVariant = 0;

// The row-pass variant a tuning cache records for (p, C_Q type): the entry
// with the same p and type whose m is nearest (in log scale) to this m, or
// -1.  The cache is the JSON file the package's tuner writes:
//   {"rowpass": [{"p": 256, "cq": "f32", "m": 1048576, "variant": 1, ...}, ...], ...}
// Only that array is read; unknown keys are skipped.
int cached_rowpass_variant(const char *path, int p, bool cq64, int64_t m) {
    if (!path) return -1;
    FILE *fp = fopen(path, "rb");
    if (!fp) return -1;
    std::string txt;
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof(buf), fp)) > 0 && txt.size() < (size_t(1) << 24))
        txt.append(buf, n);
    fclose(fp);
    size_t pos = txt.find("\"rowpass\"");
    if (pos == std::string::npos) return -1;
    pos = txt.find('[', pos);
    if (pos == std::string::npos) return -1;
    // the top-level objects of that array (brackets inside strings do not
    // occur in this file's format)
    std::vector<std::string> objs;
    {
        int depth = 0;
        size_t start = 0;
        for (size_t i = pos + 1; i < txt.size(); ++i) {
            const char ch = txt[i];
            if (ch == '{' || ch == '[') {
                if (depth == 0 && ch == '{') start = i;
                ++depth;
            } else if (ch == '}' || ch == ']') {
                if (depth == 0) break;            // end of the rowpass array
                --depth;
                if (depth == 0 && ch == '}') objs.push_back(txt.substr(start, i - start + 1));
            }
        }
    }
    // value of "key" inside the object text obj (number or quoted string)
    auto field = [](const std::string &obj, const char *key, std::string *out) {
        const std::string k = std::string("\"") + key + "\"";
        size_t i = obj.find(k);
        if (i == std::string::npos) return false;
        i = obj.find(':', i + k.size());
        if (i == std::string::npos) return false;
        ++i;
        while (i < obj.size() && (obj[i] == ' ' || obj[i] == '\t' || obj[i] == '\n' || obj[i] == '\r')) ++i;
        size_t j = i;
        if (j < obj.size() && obj[j] == '"') {
            const size_t e = obj.find('"', j + 1);
            if (e == std::string::npos) return false;
            *out = obj.substr(j + 1, e - j - 1);
            return true;
        }
        while (j < obj.size() && obj[j] != ',' && obj[j] != '}') ++j;
        *out = obj.substr(i, j - i);
        return true;
    };
    int best = -1;
    double best_d = 1e300;
    for (const std::string &obj : objs) {
        std::string vp, vcq, vm, vv;
        if (!field(obj, "p", &vp) || !field(obj, "cq", &vcq) || !field(obj, "m", &vm) ||
            !field(obj, "variant", &vv))
            continue;
        char *ep = nullptr;
        const long ep_p = strtol(vp.c_str(), &ep, 10);
        const double em = strtod(vm.c_str(), nullptr);
        const long ev = strtol(vv.c_str(), nullptr, 10);
        if (ep_p != p || vcq != (cq64 ? "f64" : "f32") || ev < 0 || ev > 7 || !(em > 0)) continue;
        const double d = fabs(log(em / double(m)));
        if (d < best_d) {
            best_d = d;
            best = int(ev);
        }
    }
    return best;
}

// The row-pass variant hikf_init uses: the forced one, else the tuning
// cache's, else the built-in default.
int resolve_rowpass_variant(const Geometry &g, const hikf_options *op) {
    if (op->rowpass_variant > 0) return op->rowpass_variant - 1;
    const int v = cached_rowpass_variant(op->tune_cache, g.p, g.fmm_prec == HIKF_FMM_F64, g.m);
    return v >= 0 ? v : kDefaultRowpassVariant;
}

hikf_status build_geometry(const hikf_problem *pr, const hikf_options *op, Geometry *g) {
    if (!pr || !op || !g) return HIKF_E_INVALID;
    if (pr->dim != 2 && pr->dim != 3) return HIKF_E_INVALID;
    if (pr->n < 1 || pr->p < 1 || pr->nnz < 0) return HIKF_E_INVALID;
    if (op->n_c < 1 || op->n_c > 8) return HIKF_E_INVALID;
    if (op->fmm_precision < HIKF_FMM_F32 || op->fmm_precision > HIKF_FMM_BF16) return HIKF_E_INVALID;
    if (pr->kernel_family != HIKF_KERNEL_POWEXP && pr->kernel_family != HIKF_KERNEL_TEST_R2)
        return HIKF_E_INVALID;
    if (!(pr->theta > 0.0) || !std::isfinite(pr->theta)) return HIKF_E_INVALID;
    if (pr->kernel_family == HIKF_KERNEL_POWEXP) {
        if (!(pr->ell > 0.0) || !std::isfinite(pr->ell)) return HIKF_E_INVALID;
        if (!(pr->gamma > 0.0 && pr->gamma <= 2.0)) return HIKF_E_INVALID;
    }
    if (pr->prior_kind != HIKF_PRIOR_ZERO && pr->prior_kind != HIKF_PRIOR_SCALED_I &&
        pr->prior_kind != HIKF_PRIOR_KERNEL)
        return HIKF_E_INVALID;
    if (pr->prior_kind == HIKF_PRIOR_SCALED_I && !(pr->alpha >= 0.0 && std::isfinite(pr->alpha)))
        return HIKF_E_INVALID;
    if (!pr->h_rowptr_dev || !pr->r_diag_dev || (pr->nnz > 0 && (!pr->h_col_dev || !pr->h_val_dev)))
        return HIKF_E_INVALID;
    g->dim = pr->dim;
    g->n = pr->n;
    g->ls = pr->dim == 2 ? 8 : 4;
    // the tree covers npad = ls * 2^D >= n cells per axis; cells beyond n
    // are padding with zero weight (their rows are never produced)
    if (pr->n > (1 << 20)) return HIKF_E_UNSUPPORTED;
    int D = 0;
    while ((g->ls << D) < pr->n) ++D;
    g->depth = D;
    g->npad = g->ls << D;
    g->m = int64_t(pr->n) * pr->n * (pr->dim == 3 ? pr->n : 1);
    g->mpad = int64_t(g->npad) * g->npad * (pr->dim == 3 ? g->npad : 1);
    if (g->mpad >= (int64_t(1) << 31)) return HIKF_E_UNSUPPORTED;
    if (pr->p % 16 != 0 || pr->p > hikf::kMaxP) return HIKF_E_UNSUPPORTED;
    g->p = pr->p;
    g->pp = (pr->p + 31) / 32 * 32;
    g->nnz = pr->nnz;
    g->nc = op->n_c;
    g->r = op->n_c * op->n_c * (pr->dim == 3 ? op->n_c : 1);
    if (g->r > hikf::kMaxR) return HIKF_E_UNSUPPORTED;
    g->direct = op->direct != 0;
    g->far = !g->direct && D >= 2;
    g->sparse = op->sparse != 0 && !g->direct;
    if (g->sparse && pr->nnz >= (int64_t(1) << 31)) return HIKF_E_UNSUPPORTED;   // int bucket slots
    g->fmm_prec = op->fmm_precision;
    g->prior = pr->prior_kind;
    if (op->history < 0 || op->history > 1000000) return HIKF_E_INVALID;
    if (op->rowpass_variant < 0 || op->rowpass_variant > 8) return HIKF_E_INVALID;
    if (op->psd_guard != 0 && op->psd_guard != 1) return HIKF_E_INVALID;
    g->psd_guard = op->psd_guard == 1;
    if (!(op->m2l_eps >= 0.0 && op->m2l_eps < 1.0)) return HIKF_E_INVALID;
    g->m2l_eps = op->m2l_eps;
    g->rp_variant = op->rowpass_variant > 0 ? op->rowpass_variant - 1 : kDefaultRowpassVariant;
    g->history = op->history;
    g->alpha = pr->alpha;
    g->kp.family = pr->kernel_family;
    g->kp.theta = pr->theta;
    g->kp.ell = pr->kernel_family == HIKF_KERNEL_POWEXP ? pr->ell : 1.0;
    g->kp.gamma = pr->kernel_family == HIKF_KERNEL_POWEXP ? pr->gamma : 1.0;
    int64_t per_ray = (pr->nnz + pr->p - 1) / pr->p;
    int64_t cpr = (per_ray + 63) / 64;
    g->cpr = int(cpr < 1 ? 1 : (cpr > 1024 ? 1024 : cpr));
    return HIKF_OK;
}

// Covariance queries: Q v runs through the filter's tree with 16 columns
// (FP32 for the BF16 modes); the scratch holds that FMM's workspace, its
// m x 16 result, the per-step chunk sums of C_s^T v and the vectors w_s.
struct QueryPlan {
    Geometry g;
    hikf::Layout lay;
    int nchunk;
    size_t off_qv, off_part, off_w, bytes;
};

QueryPlan query_plan(const Geometry &g0) {
    QueryPlan q;
    q.g = g0;
    q.g.p = 16;
    q.g.pp = 32;
    q.g.nnz = 0;
    q.g.history = 0;
    q.g.sparse = false;           // Q v runs on a dense first column
    q.g.psd_guard = false;
    q.g.m2l_eps = 0.0;
    if (q.g.fmm_prec == HIKF_FMM_BF16X3 || q.g.fmm_prec == HIKF_FMM_BF16) q.g.fmm_prec = HIKF_FMM_F32;
    q.lay = hikf::make_layout(q.g);
    const size_t tq = q.g.fmm_prec == HIKF_FMM_F64 ? 8 : 4;
    int64_t nc = (g0.m + 2047) / 2048;
    q.nchunk = int(nc < 1 ? 1 : (nc > 256 ? 256 : nc));
    size_t off = hikf::align256(q.lay.scratch_bytes);
    q.off_qv = off;
    off = hikf::align256(off + size_t(g0.m) * 16 * tq);
    q.off_part = off;
    off = hikf::align256(off + size_t(g0.history) * q.nchunk * g0.p * 8);
    q.off_w = off;
    off = hikf::align256(off + size_t(g0.history) * g0.p * 8);
    q.bytes = off;
    return q;
}

hikf_status set_err(hikf_filter *f, hikf_status st, const char *what, hipError_t e);

// P_t v for hikf_cov_apply and hikf_cov_apply_noalloc: the FMM product Q v
// and the history terms, with every workspace array inside `scr`.
hikf_status cov_apply_run(hikf_filter *f, const QueryPlan &q, const double *v_dev,
                          double *out_dev, char *scr, void *stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    f->last_stream = s;
    long long t = 0;
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipMemcpy(&t, f->res + f->lay.steps, 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return set_err(f, HIKF_E_DEVICE, "query sync", e);
    if (t > f->g.history) return HIKF_E_UNSUPPORTED;
    e = hikf::launch_fmm_apply(q.g, q.lay, scr, v_dev, scr + q.off_qv, s);
    if (e == hipSuccess)
        e = hikf::launch_cov_tail(f->g, f->lay, f->res, int(t), v_dev, scr + q.off_qv, 16,
                                  reinterpret_cast<double *>(scr + q.off_part), q.nchunk,
                                  reinterpret_cast<double *>(scr + q.off_w), out_dev, s);
    if (e != hipSuccess) return set_err(f, HIKF_E_DEVICE, "cov apply", e);
    return HIKF_OK;
}

void pair_counts(const Geometry &g, int64_t *near, int64_t *far) {
    const int64_t nl = int64_t(1) << g.depth;
    int64_t per_axis = g.direct ? nl * nl : nl + 2 * (nl - 1);
    int64_t n1 = per_axis, nn = 1;
    for (int d = 0; d < g.dim; ++d) nn *= n1;
    *near = nn;
    int64_t f = 0;
    if (g.far)
        for (int lev = 2; lev <= g.depth; ++lev) {
            int64_t nb = int64_t(1) << lev, a = 6 * nb - 8, b = 3 * nb - 2;
            int64_t pa = 1, pb = 1;
            for (int d = 0; d < g.dim; ++d) { pa *= a; pb *= b; }
            f += pa - pb;
        }
    *far = f;
}

// Workspace of hikf_cov_apply_noalloc: a fixed array in the library's
// device code object, so the call needs no allocation.  Each device holds its
// own copy; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device (the array's name is a
// host-side stand-in, not a device address).
constexpr size_t kNoAllocBytes = size_t(HIKF_NOALLOC_SCRATCH_BYTES);
static __device__ __align__(256) char scratch[kNoAllocBytes];

// Device address of `scratch` on device `dev`, looked up once per device
// (with that device current; the caller's current device is restored) and
// kept for the life of the process.  hikf_init performs the lookup for its
// device, so the entry point normally only reads the table.
hipError_t noalloc_scratch(int dev, char **out) {
    static std::mutex mu;
    static std::map<int, char *> addr;
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(dev);
    if (it == addr.end()) {
        int prev = 0;
        hipError_t e = hipGetDevice(&prev);
        if (e == hipSuccess && prev != dev) e = hipSetDevice(dev);
        if (e != hipSuccess) return e;
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (prev != dev) {
            hipError_t e2 = hipSetDevice(prev);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        if (!ptr || (reinterpret_cast<uintptr_t>(ptr) & 255)) return hipErrorInvalidSymbol;
        it = addr.emplace(dev, static_cast<char *>(ptr)).first;
    }
    *out = it->second;
    return hipSuccess;
}

// FNV-1a over the sizes, kernel and options that shape a filter's state
// (the device part covers H, R and x_0).
uint64_t host_hash(const hikf_problem *pr, const hikf_options *op) {
    uint64_t h = 1469598103934665603ull;
    auto eat = [&](const void *d, size_t n) {
        const unsigned char *b = static_cast<const unsigned char *>(d);
        for (size_t i = 0; i < n; ++i) {
            h ^= b[i];
            h *= 1099511628211ull;
        }
    };
    const int32_t ints[] = {pr->dim, pr->n, pr->kernel_family, pr->prior_kind, pr->p, op->n_c,
                            op->fmm_precision, op->direct, op->sparse, op->psd_guard};
    const double dbl[] = {pr->theta, pr->ell, pr->gamma, pr->alpha, op->m2l_eps};
    eat(ints, sizeof(ints));
    eat(dbl, sizeof(dbl));
    eat(&pr->nnz, sizeof(pr->nnz));
    return h;
}

hikf_status set_err(hikf_filter *f, hikf_status st, const char *what, hipError_t e) {
    if (f) snprintf(f->err, sizeof(f->err), "%s: %s", what, hipGetErrorString(e));
    return st;
}

}  // namespace

extern "C" {

hikf_status hikf_plan(const hikf_problem *prob, const hikf_options *opt, hikf_plan_info *out) {
    if (!out) return HIKF_E_INVALID;
    Geometry g;
    hikf_status st = build_geometry(prob, opt, &g);
    if (st != HIKF_OK) return st;
    hikf::Layout lay = hikf::make_layout(g);
    out->resident_bytes = lay.resident_bytes;
    out->scratch_bytes = lay.scratch_bytes;
    out->m = g.m;
    out->depth = g.depth;
    out->r = g.r;
    pair_counts(g, &out->near_pairs, &out->far_pairs);
    out->query_bytes = g.history ? query_plan(g).bytes : 0;
    out->rowpass_variant = resolve_rowpass_variant(g, opt);
    return HIKF_OK;
}

hikf_status hikf_init(const hikf_problem *prob, const hikf_options *opt, void *resident_dev,
                      size_t resident_bytes, void *scratch_dev, size_t scratch_bytes,
                      void *stream, hikf_filter **out) {
    if (!out) return HIKF_E_INVALID;
    *out = nullptr;
    Geometry g;
    hikf_status st = build_geometry(prob, opt, &g);
    if (st != HIKF_OK) return st;
    hikf::Layout lay = hikf::make_layout(g);
    if (!resident_dev || !scratch_dev || resident_bytes < lay.resident_bytes ||
        scratch_bytes < lay.scratch_bytes)
        return HIKF_E_NOMEM;
    if ((reinterpret_cast<uintptr_t>(resident_dev) & 255) ||
        (reinterpret_cast<uintptr_t>(scratch_dev) & 255))
        return HIKF_E_NOMEM;
    hikf_filter *f = new (std::nothrow) hikf_filter();
    if (!f) return HIKF_E_NOMEM;
    f->g = g;
    f->lay = lay;
    f->res = static_cast<char *>(resident_dev);
    hipStream_t s = static_cast<hipStream_t>(stream);
    f->last_stream = s;
    char *res = f->res, *scr = static_cast<char *>(scratch_dev);
    hipError_t e = hipGetDevice(&f->device);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&f->g.num_cu, hipDeviceAttributeMultiprocessorCount, f->device);
    if (e != hipSuccess) { hikf_status r = set_err(f, HIKF_E_DEVICE, "device query", e); delete f; return r; }
    if (f->g.num_cu < 1) f->g.num_cu = 1;
    {
        // the fixed workspace of hikf_cov_apply_noalloc: resolve its device
        // address now, with this device current.  A failure here only
        // affects that entry point (it retries and reports), so it is
        // cleared instead of failing the filter.
        char *unused = nullptr;
        if (noalloc_scratch(f->device, &unused) != hipSuccess) (void)hipGetLastError();
    }
#define HIKF_TRY(call, what)                                              \
    do {                                                                  \
        hipError_t e_ = (call);                                           \
        if (e_ != hipSuccess) {                                           \
            hikf_status r_ = set_err(f, HIKF_E_DEVICE, what, e_);         \
            (void)r_;                                                     \
            f->timing.destroy();                                          \
            delete f;                                                     \
            return HIKF_E_DEVICE;                                         \
        }                                                                 \
    } while (0)
    if (opt->timing) HIKF_TRY(f->timing.create(), "event create");
    HIKF_TRY(hipMemsetAsync(res + lay.status, 0, hikf::kNumStatus * 4, s), "status clear");
    HIKF_TRY(hipMemsetAsync(res + lay.steps, 0, 8, s), "steps clear");
    HIKF_TRY(hipMemsetAsync(res + lay.negvar, 0, 8, s), "counter clear");
    HIKF_TRY(hipMemsetAsync(res + lay.drift, 0, 3 * 8, s), "drift clear");
    HIKF_TRY(hipMemcpyAsync(res + lay.rowptr, prob->h_rowptr_dev, size_t(g.p + 1) * 8,
                            hipMemcpyDeviceToDevice, s), "copy rowptr");
    if (g.nnz > 0) {
        HIKF_TRY(hipMemcpyAsync(res + lay.col, prob->h_col_dev, size_t(g.nnz) * 4,
                                hipMemcpyDeviceToDevice, s), "copy col");
        HIKF_TRY(hipMemcpyAsync(res + lay.val, prob->h_val_dev, size_t(g.nnz) * 8,
                                hipMemcpyDeviceToDevice, s), "copy val");
    }
    HIKF_TRY(hipMemcpyAsync(res + lay.rdiag, prob->r_diag_dev, size_t(g.p) * 8,
                            hipMemcpyDeviceToDevice, s), "copy R");
    HIKF_TRY(hikf::launch_validate(g, lay, res, prob->x0_dev, s), "validate");
    HIKF_TRY(hikf::launch_hash(g, lay, res, prob->x0_dev, s), "hash");
    f->host_hash = host_hash(prob, opt);
    HIKF_TRY(hikf::launch_fmm(g, lay, res, scr, s, &f->timing, f->lr_ranks), "fmm");
    HIKF_TRY(hikf::launch_init_state(g, lay, res, prob->x0_dev, s), "init state");
    f->riccati = opt->riccati > 0 ? opt->riccati : 0;
    f->g.rp_variant = resolve_rowpass_variant(g, opt);
    // H C_Q: the fixed part of every step's G (and of the p-space recursion)
    HIKF_TRY(hikf::launch_gq(f->g, lay, res, s), "H C_Q");
    if (g.psd_guard) {
        // G_Q <- its PSD part; the first prior G = H C_0 + G_Q (2 G_Q for
        // P_0 = Q, whose H C_0 is G_Q itself) and h = H x_0, then carried
        double *GQ = reinterpret_cast<double *>(res + lay.GQ);
        HIKF_TRY(hikf::launch_psd_project(f->g, GQ, reinterpret_cast<double *>(scr + lay.psw), s),
                 "PSD guard");
        HIKF_TRY(hikf::launch_gather_g(f->g, lay, res, s), "guard start");
        if (g.prior == HIKF_PRIOR_KERNEL)
            HIKF_TRY(hikf::launch_pp_scal(f->g, 2.0, GQ, reinterpret_cast<double *>(res + lay.G), s),
                     "guard start");
        HIKF_TRY(hikf::launch_set_status(lay, res, hikf::kStCarried, 1, s), "guard start");
    }
    if (opt->graph && !opt->timing) {
        // capture on a private stream (the caller's may be the null stream,
        // which cannot be captured); the graph reads y from the resident copy
        hipStream_t cs = nullptr;
        HIKF_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "capture stream");
        // the gathering step (the only one without the recursion; with it,
        // the periodic check) and the carrying step (recursion or guard)
        const bool want_gather = !g.psd_guard || f->riccati > 0;
        const bool want_carry = f->riccati > 0 || g.psd_guard;
        hipError_t ce = hipSuccess;
        if (want_gather) {
            ce = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (ce == hipSuccess) {
                hipError_t le = hikf::launch_step(f->g, lay, res,
                                                  reinterpret_cast<const double *>(res + lay.ybuf),
                                                  cs, nullptr, true, f->riccati > 0);
                ce = hipStreamEndCapture(cs, &f->graph);
                if (ce == hipSuccess) ce = le;
            }
            if (ce == hipSuccess) ce = hipGraphInstantiate(&f->gexec, f->graph, nullptr, nullptr, 0);
        }
        if (ce == hipSuccess && want_carry) {
            ce = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (ce == hipSuccess) {
                hipError_t le = hikf::launch_step(f->g, lay, res,
                                                  reinterpret_cast<const double *>(res + lay.ybuf),
                                                  cs, nullptr, false, true);
                ce = hipStreamEndCapture(cs, &f->graph_ng);
                if (ce == hipSuccess) ce = le;
            }
            if (ce == hipSuccess)
                ce = hipGraphInstantiate(&f->gexec_ng, f->graph_ng, nullptr, nullptr, 0);
        }
        (void)hipStreamDestroy(cs);
        if (ce != hipSuccess) {
            if (f->gexec) (void)hipGraphExecDestroy(f->gexec);
            if (f->gexec_ng) (void)hipGraphExecDestroy(f->gexec_ng);
            if (f->graph) (void)hipGraphDestroy(f->graph);
            if (f->graph_ng) (void)hipGraphDestroy(f->graph_ng);
            f->gexec = f->gexec_ng = nullptr;
            f->graph = f->graph_ng = nullptr;
        }
        f->graphed = true;
        HIKF_TRY(ce, "step graph");
    }
#undef HIKF_TRY
    *out = f;
    return HIKF_OK;
}

hikf_status hikf_step(hikf_filter *f, const double *y_dev, double *x_out_dev, double *var_out_dev,
                      void *stream) {
    if (!f || !y_dev) return HIKF_E_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    f->last_stream = s;
    hipError_t e;
    // gather: without the guard, every step (no recursion), every riccati-th
    // step and the first after init or an import (recursion); with the
    // guard only every riccati-th step, as a check of the carried values
    bool gather;
    if (f->g.psd_guard)
        gather = f->riccati > 0 && f->issued > 0 && f->issued % f->riccati == 0;
    else
        gather = !f->riccati || f->force_gather || f->issued % f->riccati == 0;
    f->force_gather = false;
    ++f->issued;
    if (f->graphed) {
        e = hipMemcpyAsync(f->res + f->lay.ybuf, y_dev, size_t(f->g.p) * 8,
                           hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipGraphLaunch(gather ? f->gexec : f->gexec_ng, s);
    } else {
        e = hikf::launch_step(f->g, f->lay, f->res, y_dev, s, &f->timing, gather,
                              f->riccati > 0 || f->g.psd_guard);
    }
    if (e != hipSuccess) return set_err(f, HIKF_E_DEVICE, "step", e);
    const size_t mb = size_t(f->g.m) * 8;
    if (x_out_dev || var_out_dev) hikf::tbegin(&f->timing, HIKF_PHASE_OUTPUT, s);
    if (x_out_dev) {
        e = hipMemcpyAsync(x_out_dev, f->res + f->lay.xhat, mb, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return set_err(f, HIKF_E_DEVICE, "copy x", e);
    }
    if (var_out_dev) {
        e = hipMemcpyAsync(var_out_dev, f->res + f->lay.var, mb, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return set_err(f, HIKF_E_DEVICE, "copy var", e);
    }
    if (x_out_dev || var_out_dev) hikf::tend(&f->timing, HIKF_PHASE_OUTPUT, s);
    return HIKF_OK;
}

hikf_status hikf_cov_apply(hikf_filter *f, const double *v_dev, double *out_dev, void *scratch,
                           size_t scratch_bytes, void *stream) {
    if (!f || !v_dev || !out_dev || !scratch) return HIKF_E_INVALID;
    if (f->g.history == 0) return HIKF_E_UNSUPPORTED;
    const QueryPlan q = query_plan(f->g);
    if (scratch_bytes < q.bytes || (reinterpret_cast<uintptr_t>(scratch) & 255)) return HIKF_E_NOMEM;
    return cov_apply_run(f, q, v_dev, out_dev, static_cast<char *>(scratch), stream);
}

hikf_status hikf_cov_apply_noalloc(hikf_filter *f, const double *v_dev, double *out_dev,
                                   void *stream) {
    if (!f || !v_dev || !out_dev) return HIKF_E_INVALID;
    if (f->g.history == 0) return HIKF_E_UNSUPPORTED;
    const QueryPlan q = query_plan(f->g);
    if (q.bytes > kNoAllocBytes) {
        snprintf(f->err, sizeof(f->err),
                 "cov_apply_noalloc: the query needs %zu bytes of workspace, above the %zu-byte "
                 "fixed workspace (use hikf_cov_apply with a caller workspace)",
                 q.bytes, kNoAllocBytes);
        return HIKF_E_NOMEM;
    }
    char *scr = nullptr;
    hipError_t e = noalloc_scratch(f->device, &scr);
    if (e != hipSuccess) return set_err(f, HIKF_E_DEVICE, "noalloc workspace", e);
    return cov_apply_run(f, q, v_dev, out_dev, scr, stream);
}

hikf_status hikf_step_batch(hikf_filter *const *filters, const double *const *y_dev,
                            double *const *x_out_dev, double *const *var_out_dev, int32_t count,
                            void *stream) {
    if (count < 0 || (count > 0 && (!filters || !y_dev))) return HIKF_E_INVALID;
    for (int32_t i = 0; i < count; ++i) {
        if (!filters[i] || !y_dev[i]) return HIKF_E_INVALID;
        // one filter twice would be stepped concurrently on two streams
        for (int32_t j = 0; j < i; ++j)
            if (filters[j] == filters[i]) return HIKF_E_INVALID;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    StreamPool *pool = count > 1 ? stream_pool() : nullptr;
    if (!pool) {
        for (int32_t i = 0; i < count; ++i) {
            hikf_status st = hikf_step(filters[i], y_dev[i], x_out_dev ? x_out_dev[i] : nullptr,
                                       var_out_dev ? var_out_dev[i] : nullptr, stream);
            if (st != HIKF_OK) return st;
        }
        return HIKF_OK;
    }
    // Fork onto the device's internal streams (filter i on stream i mod
    // kPool), join back into the caller's stream; each filter's kernels stay
    // in order on one stream, so its result is that of a solo step.
    std::lock_guard<std::mutex> lock(pool->mu);
    const int used = count < kPool ? count : kPool;
    hipError_t e = hipEventRecord(pool->fork, s);
    for (int k = 0; e == hipSuccess && k < used; ++k) e = hipStreamWaitEvent(pool->s[k], pool->fork, 0);
    if (e != hipSuccess) return set_err(filters[0], HIKF_E_DEVICE, "batch fork", e);
    hikf_status st = HIKF_OK;
    int32_t done = 0;
    for (; done < count && st == HIKF_OK; ++done)
        st = hikf_step(filters[done], y_dev[done], x_out_dev ? x_out_dev[done] : nullptr,
                       var_out_dev ? var_out_dev[done] : nullptr, pool->s[done % kPool]);
    for (int k = 0; e == hipSuccess && k < used; ++k) {
        e = hipEventRecord(pool->join[k], pool->s[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, pool->join[k], 0);
    }
    for (int32_t i = 0; i < done; ++i) filters[i]->last_stream = s;
    if (e != hipSuccess) return set_err(filters[0], HIKF_E_DEVICE, "batch join", e);
    return st;
}

hikf_status hikf_query(hikf_filter *f, hikf_stats *out) {
    if (!f || !out) return HIKF_E_INVALID;
    hipError_t e = hipStreamSynchronize(f->last_stream);
    if (e != hipSuccess) return set_err(f, HIKF_E_DEVICE, "sync", e);
    int st[hikf::kNumStatus];
    double mp = 0.0;
    long long steps = 0;
    e = hipMemcpy(st, f->res + f->lay.status, sizeof(st), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&mp, f->res + f->lay.minpiv, 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&steps, f->res + f->lay.steps, 8, hipMemcpyDeviceToHost);
    unsigned long long neg = 0;
    if (e == hipSuccess) e = hipMemcpy(&neg, f->res + f->lay.negvar, 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return set_err(f, HIKF_E_DEVICE, "read status", e);
    out->steps_applied = steps;
    out->negative_variances = int64_t(neg);
    out->last_status = st[hikf::kStStep];
    out->init_status = st[hikf::kStInit];
    out->min_pivot = mp;
    out->rowpass_variant = f->g.rp_variant;
    double drift[3] = {0.0, 0.0, 0.0};
    e = hipMemcpy(drift, f->res + f->lay.drift, sizeof(drift), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return set_err(f, HIKF_E_DEVICE, "read drift", e);
    out->riccati_drift_g = drift[0];
    out->riccati_drift_h = drift[1];
    out->riccati_checks = int64_t(drift[2]);
    for (int lev = 0; lev < 20; ++lev) out->m2l_ranks[lev] = f->lr_ranks[lev];
    if (f->timing.on) {
        e = f->timing.collect();
        if (e != hipSuccess) return set_err(f, HIKF_E_DEVICE, "timing", e);
    }
    for (int ph = 0; ph < HIKF_NUM_PHASES; ++ph) {
        out->time_ms[ph] = f->timing.total_ms[ph];
        out->time_count[ph] = f->timing.count[ph];
    }
    return HIKF_OK;
}

hikf_status hikf_export_state(hikf_filter *f, double *x_dev, double *var_dev, double *c_dev,
                              void *stream) {
    if (!f) return HIKF_E_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    f->last_stream = s;
    const size_t mb = size_t(f->g.m) * 8;
    hipError_t e = hipSuccess;
    if (x_dev) e = hipMemcpyAsync(x_dev, f->res + f->lay.xhat, mb, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && var_dev)
        e = hipMemcpyAsync(var_dev, f->res + f->lay.var, mb, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && c_dev)
        e = hipMemcpyAsync(c_dev, f->res + f->lay.C, mb * f->g.p, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return set_err(f, HIKF_E_DEVICE, "export", e);
    return HIKF_OK;
}

hikf_status hikf_import_state(hikf_filter *f, const double *x_dev, const double *var_dev,
                              const double *c_dev, void *stream) {
    if (!f) return HIKF_E_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    f->last_stream = s;
    const size_t mb = size_t(f->g.m) * 8;
    hipError_t e = hipSuccess;
    if (x_dev) e = hipMemcpyAsync(f->res + f->lay.xhat, x_dev, mb, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && var_dev)
        e = hipMemcpyAsync(f->res + f->lay.var, var_dev, mb, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && c_dev)
        e = hipMemcpyAsync(f->res + f->lay.C, c_dev, mb * f->g.p, hipMemcpyDeviceToDevice, s);
    // the carried G, h no longer match: the next step gathers, and there is
    // nothing carried to check against
    if (e == hipSuccess)
        e = hipMemsetAsync(f->res + f->lay.status + 4 * hikf::kStCarried, 0, 4, s);
    if (e != hipSuccess) return set_err(f, HIKF_E_DEVICE, "import", e);
    f->force_gather = true;
    return HIKF_OK;
}

namespace {
// the filter's full problem hash (host part + the device digest of H, R, x_0)
hikf_status problem_hash(hikf_filter *f, uint64_t *out) {
    unsigned long long dev = 0;
    hipError_t e = hipStreamSynchronize(f->last_stream);
    if (e == hipSuccess) e = hipMemcpy(&dev, f->res + f->lay.hash, 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return set_err(f, HIKF_E_DEVICE, "read hash", e);
    *out = f->host_hash ^ (uint64_t(dev) * 0x9E3779B97F4A7C15ull);
    return HIKF_OK;
}
}  // namespace

hikf_status hikf_export_checkpoint(hikf_filter *f, double *x_dev, double *var_dev, double *c_dev,
                                   double *pspace_dev, hikf_checkpoint_info *info, void *stream) {
    if (!f || !info) return HIKF_E_INVALID;
    hikf_status st = hikf_export_state(f, x_dev, var_dev, c_dev, stream);
    if (st != HIKF_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t pp2 = size_t(f->g.p) * f->g.p;
    hipError_t e = hipSuccess;
    if (pspace_dev) {
        e = hipMemcpyAsync(pspace_dev, f->res + f->lay.G, pp2 * 8, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(pspace_dev + pp2, f->res + f->lay.hvec, size_t(f->g.p) * 8,
                               hipMemcpyDeviceToDevice, s);
    }
    if (e != hipSuccess) return set_err(f, HIKF_E_DEVICE, "export checkpoint", e);
    uint64_t h = 0;
    st = problem_hash(f, &h);             // synchronises the stream
    if (st != HIKF_OK) return st;
    long long steps = 0;
    int status[hikf::kNumStatus];
    e = hipMemcpy(&steps, f->res + f->lay.steps, 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(status, f->res + f->lay.status, sizeof(status), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return set_err(f, HIKF_E_DEVICE, "export checkpoint", e);
    info->problem_hash = h;
    info->steps_applied = steps;
    info->steps_issued = f->issued;
    info->p = f->g.p;
    info->carried = status[hikf::kStCarried] == 1 ? 1 : 0;
    return HIKF_OK;
}

hikf_status hikf_import_checkpoint(hikf_filter *f, const double *x_dev, const double *var_dev,
                                   const double *c_dev, const double *pspace_dev,
                                   const hikf_checkpoint_info *info, void *stream) {
    if (!f || !info) return HIKF_E_INVALID;
    if (info->p != f->g.p || (f->g.psd_guard && !(pspace_dev && info->carried)))
        return HIKF_E_INVALID;
    uint64_t h = 0;
    hikf_status st = problem_hash(f, &h);
    if (st != HIKF_OK) return st;
    if (h != info->problem_hash) {
        snprintf(f->err, sizeof(f->err), "checkpoint of another problem (hash %016llx, this "
                 "filter %016llx)", (unsigned long long)info->problem_hash, (unsigned long long)h);
        return HIKF_E_INVALID;
    }
    st = hikf_import_state(f, x_dev, var_dev, c_dev, stream);   // clears the carried flag
    if (st != HIKF_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t pp2 = size_t(f->g.p) * f->g.p;
    long long steps = info->steps_applied;
    hipError_t e = hipMemcpyAsync(f->res + f->lay.steps, &steps, 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);      // `steps` is a host local
    if (e == hipSuccess && pspace_dev && info->carried) {
        e = hipMemcpyAsync(f->res + f->lay.G, pspace_dev, pp2 * 8, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(f->res + f->lay.hvec, pspace_dev + pp2, size_t(f->g.p) * 8,
                               hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hikf::launch_set_status(f->lay, f->res, hikf::kStCarried, 1, s);
        if (e == hipSuccess) f->force_gather = false;
    }
    if (e != hipSuccess) return set_err(f, HIKF_E_DEVICE, "import checkpoint", e);
    f->issued = info->steps_issued;
    return HIKF_OK;
}

hikf_status hikf_export_cq(hikf_filter *f, double *cq_dev, void *stream) {
    if (!f || !cq_dev) return HIKF_E_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    f->last_stream = s;
    hipError_t e = hikf::launch_widen_cq(f->g, f->lay, f->res, cq_dev, s);
    if (e != hipSuccess) return set_err(f, HIKF_E_DEVICE, "export cq", e);
    return HIKF_OK;
}

void hikf_destroy(hikf_filter *f) {
    if (!f) return;
    if (f->gexec) (void)hipGraphExecDestroy(f->gexec);
    if (f->graph) (void)hipGraphDestroy(f->graph);
    if (f->gexec_ng) (void)hipGraphExecDestroy(f->gexec_ng);
    if (f->graph_ng) (void)hipGraphDestroy(f->graph_ng);
    f->timing.destroy();
    delete f;
}

const char *hikf_status_string(hikf_status s) {
    switch (s) {
        case HIKF_OK: return "ok";
        case HIKF_E_INVALID: return "invalid argument or input data";
        case HIKF_E_UNSUPPORTED: return "unsupported problem shape";
        case HIKF_E_NOMEM: return "workspace too small or misaligned";
        case HIKF_E_NOT_SPD: return "innovation covariance not positive definite";
        case HIKF_E_DEVICE: return "HIP runtime error";
    }
    return "unknown status";
}

const char *hikf_last_error(const hikf_filter *f) { return f ? f->err : ""; }

}  // extern "C"

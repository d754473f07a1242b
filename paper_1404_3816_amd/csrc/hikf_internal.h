// Internal declarations shared by the HiKF HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "hikf.h"

namespace hikf {

constexpr int kLeafPts = 64;      // points per leaf: 8x8 (2-D) or 4x4x4 (3-D)
constexpr int kMaxP = 512;        // measurements (rays) per step
constexpr int kMaxR = 64;         // Chebyshev nodes per box
constexpr int kNumStatus = 8;     // ints in the device status block
constexpr int kPsdIterations = 64; // Newton-Schulz sign iterations of the PSD guard

// device status block layout (int32 slots)
enum : int {
    kStStep = 0,                  // hikf_status of the last step
    kStInit = 1,                  // hikf_status of the device-side init checks
    kStCarried = 2,               // 1 while G, h hold values carried by the p-space recursion
};

struct KernelParams {
    int family;                   // HIKF_KERNEL_*
    double theta, ell, gamma;
};

// Covariance kernel evaluated from the squared distance r2.
template <typename T>
__device__ __forceinline__ T kernel_from_r2(T r2, const KernelParams &kp);

template <>
__device__ __forceinline__ double kernel_from_r2<double>(double r2, const KernelParams &kp) {
    if (kp.family == HIKF_KERNEL_TEST_R2) return kp.theta * r2;
    if (kp.gamma == 2.0) return kp.theta * exp(-r2 / (kp.ell * kp.ell));
    double r = sqrt(r2);
    if (kp.gamma == 1.0) return kp.theta * exp(-r / kp.ell);
    return kp.theta * exp(-pow(r / kp.ell, kp.gamma));
}

template <>
__device__ __forceinline__ float kernel_from_r2<float>(float r2, const KernelParams &kp) {
    const float theta = (float)kp.theta;
    if (kp.family == HIKF_KERNEL_TEST_R2) return theta * r2;
    const float ell = (float)kp.ell;
    if (kp.gamma == 2.0) return theta * expf(-r2 / (ell * ell));
    float r = sqrtf(r2);
    if (kp.gamma == 1.0) return theta * expf(-r / ell);
    return theta * expf(-powf(r / ell, (float)kp.gamma));
}

// Uniform-tree geometry of one filter.
struct Geometry {
    int dim = 2;
    int n = 0;                    // cells per axis
    int npad = 0;                 // cells per axis of the tree: ls * 2^depth >= n
    int ls = 8;                   // cells per leaf per axis
    int depth = 0;                // leaves per axis = 2^depth
    int nc = 4;                   // Chebyshev nodes per axis
    int r = 16;                   // nc^dim
    int p = 0;
    int pp = 32;                  // p rounded up to 32 (p-space layout)
    int cpr = 1;                  // gather chunks per ray
    int num_cu = 256;             // compute units of the device (persistent grids)
    int rp_variant = 0;           // row-pass variant (rowpass.h): bit 0 persistent, bit 1 narrow
    bool psd_guard = false;       // carry G, h with the PSD part of H C_Q (hikf_options.psd_guard)
    double m2l_eps = 0.0;         // low-rank M2L threshold (hikf_options.m2l_eps), 0 = dense
    int64_t m = 0;                // n^dim cells (state size)
    int64_t mpad = 0;             // npad^dim cells of the tree
    int64_t nnz = 0;
    bool direct = false;
    bool far = false;             // far field present (depth >= 2 and not direct)
    bool sparse = false;          // P2M / near field from the leaf-bucketed nonzeros of H
    int fmm_prec = HIKF_FMM_F32;
    int prior = HIKF_PRIOR_KERNEL;
    int history = 0;              // steps kept for covariance queries
    double alpha = 0.0;
    KernelParams kp{};
    int64_t boxes(int level) const {
        int64_t nb = int64_t(1) << level;
        return dim == 2 ? nb * nb : nb * nb * nb;
    }
    int noff() const { return dim == 2 ? 49 : 343; }   // 7^dim offset slots
    int kr32() const { return (r + 31) / 32 * 32; }    // nodes padded for BF16 MFMA
};

// Byte offsets of every array inside the two caller-owned regions.
struct Layout {
    // resident
    size_t C, CQ, xhat, var, sinv, xbuf, G, hvec, nu, partial;
    size_t rowptr, col, val, rdiag, status, minpiv, steps, negvar, ybuf;
    size_t GQ, Gn, hpart;                     // H C_Q, the next G, shares of the next h
    size_t histC, histS;                      // per-step C_prior and S^{-1} (history)
    size_t psA, pivs;                         // p-space ping-pong buffer (with xbuf), pivots
    size_t Gg, hg, drift;                     // gathered G, h (drift check), drift record
    size_t hash;                              // device part of the problem hash (uint64)
    size_t resident_bytes;
    // scratch
    size_t W, knear, sleaf, schild, m2l, lev_off;   // lev_off: start of M/L storage
    size_t ML_level[24];                      // per-level offset of M (L follows after all M)
    size_t L_base;
    size_t Wsplit, Tsplit, MS_level[24];      // BF16 hi/lo operands (BF16 modes only)
    size_t bcur, boff, btmp, bkey, bval;      // nonzeros of H by leaf (sparse mode only)
    size_t psw;                               // PSD guard: three p x p work matrices
    size_t lrA, lrU, lrW, lrC, lrUt, lrUe, lrM, lrL;   // low-rank M2L (m2l_eps > 0)
    size_t scratch_bytes;
};

Layout make_layout(const Geometry &g);

// HIP-event timing of the phases listed in hikf.h (HIKF_PHASE_*).  Each
// phase owns a ring of event pairs so that steps can be queued without a
// host synchronisation; a slot is drained before it is reused.
struct Timing {
    static constexpr int kRing = 64;
    bool on = false;
    hipEvent_t ev[HIKF_NUM_PHASES][kRing][2] = {};
    bool pending[HIKF_NUM_PHASES][kRing] = {};
    int next[HIKF_NUM_PHASES] = {};
    int cur[HIKF_NUM_PHASES] = {};
    double total_ms[HIKF_NUM_PHASES] = {};
    int64_t count[HIKF_NUM_PHASES] = {};
    hipError_t create();
    void destroy();
    hipError_t drain(int ph, int slot);
    void begin(int ph, hipStream_t s);
    void end(int ph, hipStream_t s);
    hipError_t collect();
};

// begin/end helpers that accept a null timer
inline void tbegin(Timing *t, int ph, hipStream_t s) { if (t && t->on) t->begin(ph, s); }
inline void tend(Timing *t, int ph, hipStream_t s) { if (t && t->on) t->end(ph, s); }

// ---- launch wrappers (defined in fmm.hip / step.hip) ----
// lr_ranks (levels 0..depth, optional): ranks of the low-rank M2L
hipError_t launch_fmm(const Geometry &g, const Layout &lay, char *res, char *scr,
                      hipStream_t s, Timing *t, int *lr_ranks = nullptr);
hipError_t launch_validate(const Geometry &g, const Layout &lay, char *res,
                           const double *x0, hipStream_t s);
hipError_t launch_init_state(const Geometry &g, const Layout &lay, char *res,
                             const double *x0, hipStream_t s);
// gather: form G, h from the rows of C (else use the carried ones);
// advance: afterwards carry G, h to the next step by the p-space recursion
// (with the PSD guard, gather only checks the carried G, h against the
// gathered ones and keeps the carried ones)
hipError_t launch_step(const Geometry &g, const Layout &lay, char *res,
                       const double *y, hipStream_t s, Timing *t, bool gather = true,
                       bool advance = false);
// fused row pass for p = 16 NT (rowpass.h, instantiated in rowpass_*.hip)
template <typename TQ, int NT>
hipError_t rowpass_launch(const Geometry &g, const Layout &lay, char *res, hipStream_t s);
hipError_t launch_pspace(const Geometry &g, const Layout &lay, char *res,
                         const double *y, hipStream_t s);
hipError_t launch_advance(const Geometry &g, const Layout &lay, char *res, hipStream_t s);
// PSD guard (pspace.hip): GQ <- PSD part of sym(GQ) in place; y = a x (p x p)
hipError_t launch_psd_project(const Geometry &g, double *GQ, double *work, hipStream_t s);
hipError_t launch_pp_scal(const Geometry &g, double a, const double *x, double *y, hipStream_t s);
// the device part of the problem hash: H, R and x_0 into res + lay.hash
hipError_t launch_hash(const Geometry &g, const Layout &lay, char *res, const double *x0,
                       hipStream_t s);
// set the status slot `slot` to `value` (a kernel, so graphs and streams order it)
hipError_t launch_set_status(const Layout &lay, char *res, int slot, int value, hipStream_t s);
hipError_t launch_gq(const Geometry &g, const Layout &lay, char *res, hipStream_t s);
hipError_t launch_gather_g(const Geometry &g, const Layout &lay, char *res, hipStream_t s);
hipError_t launch_widen_cq(const Geometry &g, const Layout &lay, char *res,
                           double *out, hipStream_t s);
// Q v into column 0 of out (m x g.p in the FMM precision) with the tree of g
hipError_t launch_fmm_apply(const Geometry &g, const Layout &lay, char *scr, const double *v,
                            void *out, hipStream_t s);
// out = P_0 v + t Q v - sum_{s<t} C_s S_s^{-1} C_s^T v from the history
hipError_t launch_cov_tail(const Geometry &g, const Layout &lay, char *res, int t,
                           const double *v, const void *qv, int qv_ld, double *part,
                           int nchunk, double *w, double *out, hipStream_t s);

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace hikf

struct hikf_filter {
    hikf::Geometry g;
    hikf::Layout lay;
    char *res = nullptr;          // resident region (caller-owned)
    hipStream_t last_stream = nullptr;
    int device = 0;
    hikf::Timing timing;
    hipGraph_t graph = nullptr;      // step captured at init (hikf_options.graph)
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph_ng = nullptr;   // the same without the gather (recursion or guard)
    hipGraphExec_t gexec_ng = nullptr;
    bool graphed = false;            // steps replay gexec / gexec_ng
    int riccati = 0;                 // gather period of the p-space recursion, 0 = off
    uint64_t host_hash = 0;          // host part of the problem hash (sizes, kernel, options)
    int lr_ranks[24] = {};           // ranks of the low-rank M2L per level (0: dense / none)
    int64_t issued = 0;              // steps issued since init or the last import
    bool force_gather = true;
    char err[256] = {0};
};

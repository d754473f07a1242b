// Per-step HiKF update on the GPU (Algorithm Algorithm_HiKF, Sec. 3.1).
//
// One assimilation step is:
//   1. k_gather   : partial sums of G = H (C + C_Q) and h = H x_hat over
//                   chunks of each ray's nonzeros (the prediction
//                   C_{t+1|t} = C_{t|t} + C_Q is formed on the fly).
//   2. k_reduce_g : chunk partials -> G (p x p), h (p), in a fixed order.
//   3. p-space    : S = (G + G^T)/2 + R, S^{-1} by a blocked symmetric
//                   sweep (Gauss-Jordan; its pivots are those of the
//                   Cholesky factorisation) on FP64 MFMA, and the innovation
//                   nu = y - h (pspace.hip); writes the step status.
//   4. k_rowpass  : K = C_prior S^{-1} on FP64 MFMA, fused with the state,
//                   variance and cross-covariance updates:
//                   x_hat += K nu, var += K(0) - sum_j K_ij C_prior,ij,
//                   C <- K R (= C_prior - K G).  Skipped when the status
//                   is not OK, so a failed step leaves the state untouched.
#include "hikf_internal.h"

namespace hikf {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

unsigned grid_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return unsigned(b);
}

// ---------------------------------------------------------------- init
__global__ void k_validate(int p, int64_t nnz, int64_t m, const int64_t *rowptr,
                           const int32_t *col, const double *val, const double *rdiag,
                           const double *x0, int *status) {
    int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int64_t stride = int64_t(gridDim.x) * blockDim.x;
    int bad = 0;
    for (int64_t i = tid; i <= p; i += stride) {
        if (i == 0 && rowptr[0] != 0) bad = 1;
        if (i == p && rowptr[p] != nnz) bad = 1;
        if (i < p && rowptr[i] > rowptr[i + 1]) bad = 1;
        if (i < p && !(rdiag[i] > 0.0 && isfinite(rdiag[i]))) bad = 1;
    }
    for (int64_t e = tid; e < nnz; e += stride) {
        int64_t c = col[e];
        if (c < 0 || c >= m || !isfinite(val[e])) bad = 1;
        int lo = 0, hi = p - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (rowptr[mid] <= e) lo = mid; else hi = mid - 1;
        }
        int64_t end = rowptr[lo + 1];
        if (e + 1 < nnz && e + 1 < end && col[e + 1] <= c) bad = 1;   // strictly increasing
    }
    if (x0)
        for (int64_t i = tid; i < m; i += stride)
            if (!isfinite(x0[i])) bad = 1;
    if (bad) status[kStInit] = HIKF_E_INVALID;
}

template <typename TQ>
__global__ void k_init_state(int64_t m, int p, int prior, double alpha, double kdiag,
                             const TQ *CQ, const double *x0, double *C, double *xhat,
                             double *var) {
    int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int64_t stride = int64_t(gridDim.x) * blockDim.x;
    int64_t mp = m * p;
    for (int64_t i = tid; i < mp; i += stride)
        C[i] = prior == HIKF_PRIOR_KERNEL ? (double)CQ[i] : 0.0;
    double v0 = prior == HIKF_PRIOR_KERNEL ? kdiag : (prior == HIKF_PRIOR_SCALED_I ? alpha : 0.0);
    for (int64_t i = tid; i < m; i += stride) {
        xhat[i] = x0 ? x0[i] : 0.0;
        var[i] = v0;
    }
}

// C_0 = alpha H^T for P_0 = alpha I
__global__ void k_scatter_c(int64_t nnz, int p, int64_t m, double alpha, const int64_t *rowptr,
                            const int32_t *col, const double *val, double *C) {
    int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    int lo = 0, hi = p - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (rowptr[mid] <= e) lo = mid; else hi = mid - 1;
    }
    if (rowptr[lo] > e || rowptr[lo + 1] <= e) return;
    int64_t c = col[e];
    if (c < 0 || c >= m) return;
    C[c * p + lo] = alpha * val[e];
}

template <typename TQ>
__global__ void k_widen(int64_t n, const TQ *src, double *dst) {
    int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = tid; i < n; i += stride) dst[i] = (double)src[i];
}

// ---------------------------------------------------------------- 1. gather
// One workgroup per (ray a, chunk ch of its nonzeros), taken 64 nonzeros at
// a time: their column indices and values go to LDS first (one load per
// thread, all in flight together), then thread t < p/2 sums columns 2t and
// 2t + 1 of sum_e H_ae X[col_e][.] with 16-byte loads, sixteen rows in
// flight per thread, where X is C (WITH_C; the step adds the fixed H C_Q
// afterwards, since H C_prior = H C + H C_Q) or C_Q (H C_Q, once at init),
// and the 64 threads after them split sum_e H_ae x_hat[col_e] (nonzero j
// mod 64 each, then summed in a fixed order).  A column index out of range
// contributes nothing.
template <typename TQ, bool WITH_C>
__global__ void __launch_bounds__(512)
k_gather(int p, int cpr, int64_t m, int64_t nnz, const int64_t *rowptr, const int32_t *col,
         const double *val, const double *C, const TQ *CQ, const double *xhat,
         double *partial, const int *status) {
    typedef double dv2 __attribute__((ext_vector_type(2)));
    typedef TQ qv2 __attribute__((ext_vector_type(2)));
    constexpr int U = 16;
    constexpr int kSub = 64;                           // nonzeros staged at a time
    __shared__ int64_t sc[kSub];
    __shared__ double sw[kSub];
    __shared__ double hsum[64];
    if (status[kStInit] != 0) return;
    const int a = blockIdx.x, ch = blockIdx.y;
    int64_t r0 = rowptr[a], r1 = rowptr[a + 1];
    r0 = r0 < 0 ? 0 : (r0 > nnz ? nnz : r0);
    r1 = r1 < r0 ? r0 : (r1 > nnz ? nnz : r1);
    const int64_t len = r1 - r0;
    const int64_t e0 = r0 + len * ch / cpr, e1 = r0 + len * (ch + 1) / cpr;
    double *out = partial + (int64_t(a) * cpr + ch) * (p + 1);
    const int half = p / 2;
    const int t = threadIdx.x;
    dv2 acc = dv2{0.0, 0.0};
    double hacc = 0.0;
    for (int64_t b = e0; b < e1; b += kSub) {
        const int n = int(e1 - b < kSub ? e1 - b : kSub);
        if (b > e0) __syncthreads();                   // previous entries consumed
        if (t < kSub) {
            int64_t c = 0;
            double w = 0.0;
            if (t < n) {
                c = col[b + t];
                w = val[b + t];
                if (c < 0 || c >= m) {
                    c = 0;
                    w = 0.0;
                }
            }
            sc[t] = c;
            sw[t] = w;
        }
        __syncthreads();
        if (t >= half && t < half + 64) {
            const int j = t - half;
            if (j < n) hacc += sw[j] * xhat[sc[j]];
        }
        if (t < half) {
            for (int e = 0; e < n; e += U) {
                dv2 x[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t o = (e + u < n ? sc[e + u] : 0) * p + 2 * t;
                    if constexpr (WITH_C) {
                        x[u] = *reinterpret_cast<const dv2 *>(C + o);
                    } else {
                        const qv2 qv = *reinterpret_cast<const qv2 *>(CQ + o);
                        x[u] = dv2{(double)qv[0], (double)qv[1]};
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (e + u < n) acc += sw[e + u] * x[u];
            }
        }
    }
    if (t >= half && t < half + 64) hsum[t - half] = hacc;
    if (t < half) {
        out[2 * t] = acc[0];
        out[2 * t + 1] = acc[1];
    }
    __syncthreads();
    if (t == half) {
        double s2 = 0.0;
        for (int j = 0; j < 64; ++j) s2 += hsum[j];
        out[p] = s2;
    }
}

// ---------------------------------------------------------------- 2. reduce
// G = the chunk sums (+ GQ = H C_Q when given), h = the chunk sums
__global__ void __launch_bounds__(256)
k_reduce_g(int p, int cpr, const double *partial, const double *GQ, double *G, double *hvec,
           const int *status) {
    if (status[kStInit] != 0) return;
    const int a = blockIdx.x;
    for (int b = threadIdx.x; b <= p; b += blockDim.x) {
        double s = 0.0;
        for (int c = 0; c < cpr; ++c) s += partial[(int64_t(a) * cpr + c) * (p + 1) + b];
        if (b < p) G[int64_t(a) * p + b] = GQ ? s + GQ[int64_t(a) * p + b] : s;
        else hvec[a] = s;
    }
}

// ---------------------------------------------------------------- drift check
// With the p-space recursion, every periodic gather is also a check: the G
// and h carried since the previous gather are compared with the gathered
// ones (max-norm difference relative to the max-norm of the gathered value),
// the largest drift seen so far is kept in drift[0] (G) and drift[1] (h) and
// the number of checks in drift[2]; then the gathered values replace the
// carried ones.  Skipped when nothing was carried (the first step, after an
// import, or if every step since the last gather failed).
__global__ void __launch_bounds__(256)
k_drift(int p, const double *Gg, const double *hg, double *G, double *h, double *drift,
        int *status, int keep_carried) {
    __shared__ double red[4][256];
    if (status[kStInit] != 0) return;
    const int t = threadIdx.x;
    const bool carried = status[kStCarried] == 1;
    double dg = 0.0, mg = 0.0, dh = 0.0, mh = 0.0;
    const int64_t n = int64_t(p) * p;
    for (int64_t i = t; i < n; i += 256) {
        const double a = Gg[i];
        dg = fmax(dg, fabs(G[i] - a));
        mg = fmax(mg, fabs(a));
    }
    for (int i = t; i < p; i += 256) {
        const double a = hg[i];
        dh = fmax(dh, fabs(h[i] - a));
        mh = fmax(mh, fabs(a));
    }
    red[0][t] = dg;
    red[1][t] = mg;
    red[2][t] = dh;
    red[3][t] = mh;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s)
            for (int k = 0; k < 4; ++k) red[k][t] = fmax(red[k][t], red[k][t + s]);
        __syncthreads();
    }
    if (t == 0 && carried) {
        const double rg = red[1][0] > 0.0 ? red[0][0] / red[1][0] : red[0][0];
        const double rh = red[3][0] > 0.0 ? red[2][0] / red[3][0] : red[2][0];
        drift[0] = fmax(drift[0], rg);
        drift[1] = fmax(drift[1], rh);
        drift[2] += 1.0;
    }
    if (keep_carried) return;                // the PSD guard keeps its own G, h
    __syncthreads();
    for (int64_t i = t; i < n; i += 256) G[i] = Gg[i];
    for (int i = t; i < p; i += 256) h[i] = hg[i];
    if (t == 0) status[kStCarried] = 0;
}

// ---------------------------------------------------------------- problem hash
// An order-independent 64-bit digest of H (row pointers, columns, values), R
// and x_0: every element's bits are mixed with its position and array
// (SplitMix64 finaliser) and the results are summed modulo 2^64.
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_hash(int p, int64_t nnz, int64_t m, const int64_t *rowptr, const int32_t *col,
                       const double *val, const double *rdiag, const double *x0,
                       unsigned long long *out) {
    unsigned long long acc = 0;
    const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = tid; i <= p; i += stride)
        acc += mix64((1ull << 60) ^ (unsigned long long)(i * 0x100000001B3ull) ^
                     mix64((unsigned long long)rowptr[i]));
    for (int64_t i = tid; i < nnz; i += stride) {
        acc += mix64((2ull << 60) ^ (unsigned long long)i ^ mix64((unsigned long long)(uint32_t)col[i]));
        acc += mix64((3ull << 60) ^ (unsigned long long)i ^
                     mix64(__builtin_bit_cast(unsigned long long, val[i])));
    }
    for (int64_t i = tid; i < p; i += stride)
        acc += mix64((4ull << 60) ^ (unsigned long long)i ^
                     mix64(__builtin_bit_cast(unsigned long long, rdiag[i])));
    if (x0)
        for (int64_t i = tid; i < m; i += stride)
            acc += mix64((5ull << 60) ^ (unsigned long long)i ^
                         mix64(__builtin_bit_cast(unsigned long long, x0[i])));
    if (acc) atomicAdd(out, acc);
}

__global__ void k_set_int(int *dst, int value) { *dst = value; }

// ---------------------------------------------------------------- history
// Covariance queries need every applied step's prior cross-covariance C_s
// and S_s^{-1}.  The slot of a step is the number of steps applied before
// it (read on the device, so a rejected step is overwritten by the next).
template <typename TQ>
__global__ void k_hist_c(int64_t mp, int history, const long long *steps, const double *C,
                         const TQ *CQ, double *histC) {
    const long long s = steps[0];
    if (s >= history) return;
    double *dst = histC + s * mp;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < mp;
         i += int64_t(gridDim.x) * blockDim.x)
        dst[i] = C[i] + (double)CQ[i];
}

__global__ void k_hist_s(int64_t pp, int history, const long long *steps, const int *status,
                         const double *Sinv, double *histS) {
    if (status[kStStep] != HIKF_OK) return;
    const long long s = steps[0] - 1;
    if (s < 0 || s >= history) return;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < pp;
         i += int64_t(gridDim.x) * blockDim.x)
        histS[s * pp + i] = Sinv[i];
}

// ---------------------------------------------------------------- queries
// part[s][ch][c] = sum over the rows of chunk ch of C_s[i][c] v[i]
__global__ void __launch_bounds__(256)
k_cov_u(int p, int64_t m, int nchunk, const double *histC, const double *v, double *part) {
    const int s = blockIdx.x, ch = blockIdx.y;
    const int64_t r0 = m * ch / nchunk, r1 = m * (ch + 1) / nchunk;
    const double *Cs = histC + int64_t(s) * m * p;
    for (int c = threadIdx.x; c < p; c += blockDim.x) {
        double acc = 0.0;
        for (int64_t i = r0; i < r1; ++i) acc += Cs[i * p + c] * v[i];
        part[(int64_t(s) * nchunk + ch) * p + c] = acc;
    }
}

// w_s = S_s^{-1} u_s with u_s the chunk sums in a fixed order
__global__ void __launch_bounds__(256)
k_cov_w(int p, int nchunk, const double *part, const double *histS, double *w) {
    __shared__ double su[kMaxP];
    const int s = blockIdx.x;
    for (int c = threadIdx.x; c < p; c += blockDim.x) {
        double u = 0.0;
        for (int ch = 0; ch < nchunk; ++ch) u += part[(int64_t(s) * nchunk + ch) * p + c];
        su[c] = u;
    }
    __syncthreads();
    const double *Ss = histS + int64_t(s) * p * p;
    for (int c = threadIdx.x; c < p; c += blockDim.x) {
        double acc = 0.0;
        for (int k = 0; k < p; ++k) acc += Ss[int64_t(c) * p + k] * su[k];
        w[int64_t(s) * p + c] = acc;
    }
}

// out_i = a v_i + b (Q v)_i - sum_s C_s[i][.] w_s; one wave per row
template <typename TQ>
__global__ void __launch_bounds__(256)
k_cov_out(int64_t m, int p, int t, double a, double b, const double *v, const TQ *qv, int qv_ld,
          const double *histC, const double *w, double *out) {
    const int64_t i = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= m) return;
    double d = 0.0;
    for (int s = 0; s < t; ++s) {
        const double *row = histC + (int64_t(s) * m + i) * p;
        for (int c = lane; c < p; c += 64) d += row[c] * w[int64_t(s) * p + c];
    }
    for (int off = 32; off > 0; off >>= 1) d += __shfl_xor(d, off, 64);
    if (lane == 0) out[i] = a * v[i] + b * (double)qv[i * qv_ld] - d;
}

// ---------------------------------------------------------------- 3. p-space
// (pspace.hip)

// ---------------------------------------------------------------- 4. row pass
// (rowpass.h; instantiated for every p / 16 in the rowpass_*.hip units)
template <typename TQ>
hipError_t launch_rowpass(const Geometry &g, const Layout &lay, char *res, hipStream_t s) {
    switch (g.p / 16) {
#define HIKF_NT(N) case N: return rowpass_launch<TQ, N>(g, lay, res, s);
        HIKF_NT(1) HIKF_NT(2) HIKF_NT(3) HIKF_NT(4) HIKF_NT(5) HIKF_NT(6) HIKF_NT(7) HIKF_NT(8)
        HIKF_NT(9) HIKF_NT(10) HIKF_NT(11) HIKF_NT(12) HIKF_NT(13) HIKF_NT(14) HIKF_NT(15)
        HIKF_NT(16) HIKF_NT(17) HIKF_NT(18) HIKF_NT(19) HIKF_NT(20) HIKF_NT(21) HIKF_NT(22)
        HIKF_NT(23) HIKF_NT(24) HIKF_NT(25) HIKF_NT(26) HIKF_NT(27) HIKF_NT(28) HIKF_NT(29)
        HIKF_NT(30) HIKF_NT(31) HIKF_NT(32)
#undef HIKF_NT
        default: return hipErrorInvalidValue;
    }
}

template <typename TQ>
void run_gather(const Geometry &g, const Layout &lay, char *res, bool with_c, double *G,
                double *h, hipStream_t s, Timing *tm) {
    const int p = g.p;
    tbegin(tm, HIKF_PHASE_GATHER, s);
    const unsigned gthreads = unsigned(((p / 2 + 64) + 63) / 64 * 64);
    const auto gk = with_c ? k_gather<TQ, true> : k_gather<TQ, false>;
    hipLaunchKernelGGL(gk, dim3(p, g.cpr), dim3(gthreads), 0, s, p, g.cpr, g.m, g.nnz,
                       reinterpret_cast<const int64_t *>(res + lay.rowptr),
                       reinterpret_cast<const int32_t *>(res + lay.col),
                       reinterpret_cast<const double *>(res + lay.val),
                       reinterpret_cast<const double *>(res + lay.C),
                       reinterpret_cast<const TQ *>(res + lay.CQ),
                       reinterpret_cast<const double *>(res + lay.xhat),
                       reinterpret_cast<double *>(res + lay.partial),
                       reinterpret_cast<const int *>(res + lay.status));
    tend(tm, HIKF_PHASE_GATHER, s);
    tbegin(tm, HIKF_PHASE_REDUCE, s);
    // the step's G adds the H C_Q formed at init
    hipLaunchKernelGGL(k_reduce_g, dim3(p), dim3(256), 0, s, p, g.cpr,
                       reinterpret_cast<const double *>(res + lay.partial),
                       with_c ? reinterpret_cast<const double *>(res + lay.GQ) : nullptr, G, h,
                       reinterpret_cast<const int *>(res + lay.status));
    tend(tm, HIKF_PHASE_REDUCE, s);
}

template <typename TQ>
hipError_t run_step(const Geometry &g, const Layout &lay, char *res, const double *y,
                    hipStream_t s, Timing *tm, bool gather, bool advance) {
    if (gather && !advance && !g.psd_guard) {
        run_gather<TQ>(g, lay, res, true, reinterpret_cast<double *>(res + lay.G),
                       reinterpret_cast<double *>(res + lay.hvec), s, tm);
    } else if (gather) {
        // recursion mode: gather aside, compare with the carried G, h, keep
        // the gathered ones (the PSD guard keeps the carried ones)
        run_gather<TQ>(g, lay, res, true, reinterpret_cast<double *>(res + lay.Gg),
                       reinterpret_cast<double *>(res + lay.hg), s, tm);
        hipLaunchKernelGGL(k_drift, dim3(1), dim3(256), 0, s, g.p,
                           reinterpret_cast<const double *>(res + lay.Gg),
                           reinterpret_cast<const double *>(res + lay.hg),
                           reinterpret_cast<double *>(res + lay.G),
                           reinterpret_cast<double *>(res + lay.hvec),
                           reinterpret_cast<double *>(res + lay.drift),
                           reinterpret_cast<int *>(res + lay.status), g.psd_guard ? 1 : 0);
    }
    if (g.psd_guard) advance = true;
    const long long *steps = reinterpret_cast<const long long *>(res + lay.steps);
    if (g.history)
        hipLaunchKernelGGL(k_hist_c<TQ>, dim3(grid_for(g.m * g.p)), dim3(256), 0, s, g.m * g.p,
                           g.history, steps, reinterpret_cast<const double *>(res + lay.C),
                           reinterpret_cast<const TQ *>(res + lay.CQ),
                           reinterpret_cast<double *>(res + lay.histC));
    tbegin(tm, HIKF_PHASE_PSPACE, s);
    {
        hipError_t e = launch_pspace(g, lay, res, y, s);
        if (e == hipSuccess && advance) e = launch_advance(g, lay, res, s);
        if (e != hipSuccess) return e;
    }
    tend(tm, HIKF_PHASE_PSPACE, s);
    if (g.history)
        hipLaunchKernelGGL(k_hist_s, dim3(grid_for(int64_t(g.p) * g.p)), dim3(256), 0, s,
                           int64_t(g.p) * g.p, g.history, steps,
                           reinterpret_cast<const int *>(res + lay.status),
                           reinterpret_cast<const double *>(res + lay.sinv),
                           reinterpret_cast<double *>(res + lay.histS));
    tbegin(tm, HIKF_PHASE_ROWPASS, s);
    {
        hipError_t e = launch_rowpass<TQ>(g, lay, res, s);
        if (e != hipSuccess) return e;
    }
    tend(tm, HIKF_PHASE_ROWPASS, s);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_cov_tail(const Geometry &g, const Layout &lay, char *res, int t,
                           const double *v, const void *qv, int qv_ld, double *part,
                           int nchunk, double *w, double *out, hipStream_t s) {
    const double *histC = reinterpret_cast<const double *>(res + lay.histC);
    if (t > 0) {
        hipLaunchKernelGGL(k_cov_u, dim3(t, nchunk), dim3(256), 0, s, g.p, g.m, nchunk, histC, v,
                           part);
        hipLaunchKernelGGL(k_cov_w, dim3(t), dim3(256), 0, s, g.p, nchunk, part,
                           reinterpret_cast<const double *>(res + lay.histS), w);
    }
    // P_0 v: Q v, alpha v or 0
    double a = 0.0, b = double(t);
    if (g.prior == HIKF_PRIOR_KERNEL) b += 1.0;
    else if (g.prior == HIKF_PRIOR_SCALED_I) a = g.alpha;
    const unsigned blocks = unsigned((g.m + 3) / 4);
    if (g.fmm_prec == HIKF_FMM_F64)
        hipLaunchKernelGGL(k_cov_out<double>, dim3(blocks), dim3(256), 0, s, g.m, g.p, t, a, b, v,
                           static_cast<const double *>(qv), qv_ld, histC, w, out);
    else
        hipLaunchKernelGGL(k_cov_out<float>, dim3(blocks), dim3(256), 0, s, g.m, g.p, t, a, b, v,
                           static_cast<const float *>(qv), qv_ld, histC, w, out);
    return hipGetLastError();
}

hipError_t launch_hash(const Geometry &g, const Layout &lay, char *res, const double *x0,
                       hipStream_t s) {
    unsigned long long *out = reinterpret_cast<unsigned long long *>(res + lay.hash);
    hipError_t e = hipMemsetAsync(out, 0, 8, s);
    if (e != hipSuccess) return e;
    int64_t n = g.nnz > g.m ? g.nnz : g.m;
    if (n < g.p + 1) n = g.p + 1;
    hipLaunchKernelGGL(k_hash, dim3(grid_for(n)), dim3(256), 0, s, g.p, g.nnz, g.m,
                       reinterpret_cast<const int64_t *>(res + lay.rowptr),
                       reinterpret_cast<const int32_t *>(res + lay.col),
                       reinterpret_cast<const double *>(res + lay.val),
                       reinterpret_cast<const double *>(res + lay.rdiag), x0, out);
    return hipGetLastError();
}

hipError_t launch_set_status(const Layout &lay, char *res, int slot, int value, hipStream_t s) {
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s,
                       reinterpret_cast<int *>(res + lay.status) + slot, value);
    return hipGetLastError();
}

hipError_t launch_validate(const Geometry &g, const Layout &lay, char *res, const double *x0,
                           hipStream_t s) {
    int64_t n = g.nnz > g.m ? g.nnz : g.m;
    if (n < g.p + 1) n = g.p + 1;
    hipLaunchKernelGGL(k_validate, dim3(grid_for(n)), dim3(256), 0, s, g.p, g.nnz, g.m,
                       reinterpret_cast<const int64_t *>(res + lay.rowptr),
                       reinterpret_cast<const int32_t *>(res + lay.col),
                       reinterpret_cast<const double *>(res + lay.val),
                       reinterpret_cast<const double *>(res + lay.rdiag), x0,
                       reinterpret_cast<int *>(res + lay.status));
    return hipGetLastError();
}

hipError_t launch_init_state(const Geometry &g, const Layout &lay, char *res, const double *x0,
                             hipStream_t s) {
    const double kdiag = g.kp.family == HIKF_KERNEL_TEST_R2 ? 0.0 : g.kp.theta;
    const unsigned grid = grid_for(g.m * g.p);
    if (g.fmm_prec == HIKF_FMM_F64)
        hipLaunchKernelGGL(k_init_state<double>, dim3(grid), dim3(256), 0, s, g.m, g.p, g.prior,
                           g.alpha, kdiag, reinterpret_cast<const double *>(res + lay.CQ), x0,
                           reinterpret_cast<double *>(res + lay.C),
                           reinterpret_cast<double *>(res + lay.xhat),
                           reinterpret_cast<double *>(res + lay.var));
    else
        hipLaunchKernelGGL(k_init_state<float>, dim3(grid), dim3(256), 0, s, g.m, g.p, g.prior,
                           g.alpha, kdiag, reinterpret_cast<const float *>(res + lay.CQ), x0,
                           reinterpret_cast<double *>(res + lay.C),
                           reinterpret_cast<double *>(res + lay.xhat),
                           reinterpret_cast<double *>(res + lay.var));
    if (g.prior == HIKF_PRIOR_SCALED_I && g.nnz > 0)
        hipLaunchKernelGGL(k_scatter_c, dim3(unsigned((g.nnz + 255) / 256)), dim3(256), 0, s,
                           g.nnz, g.p, g.m, g.alpha,
                           reinterpret_cast<const int64_t *>(res + lay.rowptr),
                           reinterpret_cast<const int32_t *>(res + lay.col),
                           reinterpret_cast<const double *>(res + lay.val),
                           reinterpret_cast<double *>(res + lay.C));
    return hipGetLastError();
}

hipError_t launch_step(const Geometry &g, const Layout &lay, char *res, const double *y,
                       hipStream_t s, Timing *t, bool gather, bool advance) {
    if (g.fmm_prec == HIKF_FMM_F64) return run_step<double>(g, lay, res, y, s, t, gather, advance);
    return run_step<float>(g, lay, res, y, s, t, gather, advance);
}

// G = H C + G_Q and h = H x_hat from the current state (the PSD guard's start)
hipError_t launch_gather_g(const Geometry &g, const Layout &lay, char *res, hipStream_t s) {
    double *G = reinterpret_cast<double *>(res + lay.G);
    double *h = reinterpret_cast<double *>(res + lay.hvec);
    if (g.fmm_prec == HIKF_FMM_F64) run_gather<double>(g, lay, res, true, G, h, s, nullptr);
    else run_gather<float>(g, lay, res, true, G, h, s, nullptr);
    return hipGetLastError();
}

// G_Q = H C_Q (p x p) for the p-space recursion; nu serves as a throw-away h
hipError_t launch_gq(const Geometry &g, const Layout &lay, char *res, hipStream_t s) {
    double *GQ = reinterpret_cast<double *>(res + lay.GQ);
    double *dummy = reinterpret_cast<double *>(res + lay.nu);
    if (g.fmm_prec == HIKF_FMM_F64) run_gather<double>(g, lay, res, false, GQ, dummy, s, nullptr);
    else run_gather<float>(g, lay, res, false, GQ, dummy, s, nullptr);
    return hipGetLastError();
}

hipError_t launch_widen_cq(const Geometry &g, const Layout &lay, char *res, double *out,
                           hipStream_t s) {
    const int64_t n = g.m * g.p;
    if (g.fmm_prec == HIKF_FMM_F64)
        hipLaunchKernelGGL(k_widen<double>, dim3(grid_for(n)), dim3(256), 0, s, n,
                           reinterpret_cast<const double *>(res + lay.CQ), out);
    else
        hipLaunchKernelGGL(k_widen<float>, dim3(grid_for(n)), dim3(256), 0, s, n,
                           reinterpret_cast<const float *>(res + lay.CQ), out);
    return hipGetLastError();
}

}  // namespace hikf

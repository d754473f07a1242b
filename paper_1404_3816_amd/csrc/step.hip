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
// One workgroup per (ray a, chunk ch of its nonzeros); thread t < p/2 sums
// columns 2t and 2t + 1 of sum_e H_ae X[col_e][.] with 16-byte loads, where
// X is C (WITH_C; the step adds the fixed H C_Q afterwards, since
// H C_prior = H C + H C_Q) or C_Q (H C_Q, once at init),
// and the 64 threads after them split sum_e H_ae x_hat[col_e] (nonzero j
// mod 64 each, then summed in a fixed order).  Eight nonzeros are loaded
// before any is accumulated, so the row loads of a chunk are in flight
// together.
template <typename TQ, bool WITH_C>
__global__ void __launch_bounds__(512)
k_gather(int p, int cpr, int64_t m, int64_t nnz, const int64_t *rowptr, const int32_t *col,
         const double *val, const double *C, const TQ *CQ, const double *xhat,
         double *partial, const int *status) {
    typedef double dv2 __attribute__((ext_vector_type(2)));
    typedef TQ qv2 __attribute__((ext_vector_type(2)));
    constexpr int U = 8;
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
    __shared__ double hsum[64];
    if (t >= half && t < half + 64) {
        double acc = 0.0;
        for (int64_t e = e0 + (t - half); e < e1; e += 64) {
            const int64_t c = col[e];
            if (c >= 0 && c < m) acc += val[e] * xhat[c];
        }
        hsum[t - half] = acc;
    }
    __syncthreads();
    if (t == half) {
        double acc = 0.0;
        for (int j = 0; j < 64; ++j) acc += hsum[j];
        out[p] = acc;
    }
    if (t < half) {
        dv2 acc = dv2{0.0, 0.0};
        int64_t e = e0;
        for (; e + U <= e1; e += U) {
            dv2 x[U];
            double w[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t c = col[e + u];
                const bool ok = c >= 0 && c < m;
                const int64_t o = (ok ? c : 0) * p + 2 * t;
                if constexpr (WITH_C) {
                    x[u] = *reinterpret_cast<const dv2 *>(C + o);
                } else {
                    const qv2 qv = *reinterpret_cast<const qv2 *>(CQ + o);
                    x[u] = dv2{(double)qv[0], (double)qv[1]};
                }
                w[u] = ok ? val[e + u] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) acc += w[u] * x[u];
        }
        for (; e < e1; ++e) {
            const int64_t c = col[e];
            if (c < 0 || c >= m) continue;
            const int64_t o = c * p + 2 * t;
            if constexpr (WITH_C) {
                acc += val[e] * *reinterpret_cast<const dv2 *>(C + o);
            } else {
                const qv2 qv = *reinterpret_cast<const qv2 *>(CQ + o);
                acc += val[e] * dv2{(double)qv[0], (double)qv[1]};
            }
        }
        out[2 * t] = acc[0];
        out[2 * t + 1] = acc[1];
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
// 512 threads = 8 waves per tile of 16 RG rows.  Wave w takes row group
// g = w % RG (rows [16 (RG b + g), +16); lane l owns row l % 16 of them) and
// column part c = w / RG (column tiles [T0, T1) of the P = 16 NT columns, the
// CS = 8 / RG parts splitting them as evenly as possible).  P <= 256 runs 4
// row groups x 2 column halves, P <= 512 runs 2 row groups x 4 quarters, so
// every wave holds at most 8 column tiles.
//
// v_mfma_f64_16x16x4 computes D += A B with lane l supplying A[l%16][l/16] and
// B[l/16][l%16] and holding D[l/16 + 4 r][l%16] (the FP64 variant interleaves
// the rows).  The kernel computes tiles of K^T = S^{-1} C_prior^T: A is a
// 16 x 4 piece of a slab of S^{-1} (symmetric) read from LDS and B is 4
// values of the lane's own row of C_prior, so the result stays in the lane
// that owns the row.  Columns are assigned so that every lane handles pairs
// of adjacent columns: with q = l/16, lane l holds, for tile t and r = 0..3,
//     K[row][16 t + col(q, r)],   col(q, r) = 8 (r/2) + 2 q + r % 2,
// (output row i = q + 4 r of the MFMA tile is column col(i%4, i/4)), and the
// MFMA step s of k block kb pairs lane group q with k = 16 kb + col(q, s).
// The C_prior values a lane loads in its own column part are then exactly
// the columns of K it ends up holding (no second read of C or C_Q), and every
// global access of C, C_Q and the stores of C are 16-byte (two-column)
// vector accesses.  S^{-1} is streamed through a double-buffered LDS slab of
// 16 rows (row pitch P + 8 doubles: lane groups q and q + 1 read rows two
// apart, which then fall on disjoint banks), prefetched into registers one
// block ahead as 16-byte loads; LDS operands are read two MFMAs ahead.
template <int NT, int CS, int RG_>
struct RowSplit {
    static constexpr int RG = RG_;
    static constexpr int NTH = 64 * CS * RG_;  // threads of the workgroup
    static constexpr int P = NT * 16;
    static constexpr int LDB = P + 8;           // row pitch of the LDS slab (doubles)
    static constexpr int SLAB = 16 * LDB;
    static constexpr int PER2 = (8 * P + NTH - 1) / NTH;  // slab column pairs per thread
    static constexpr int t0(int c) { return (c * NT + CS - 1) / CS; }
};

// column offset inside a 16-column tile of MFMA output row i (see above)
__device__ __forceinline__ constexpr int rp_col(int q, int r) { return 8 * (r >> 1) + 2 * q + (r & 1); }

template <typename TQ> struct Pair;
template <> struct Pair<float> { typedef float v2 __attribute__((ext_vector_type(2))); };
template <> struct Pair<double> { typedef double v2 __attribute__((ext_vector_type(2))); };
typedef double dv2 __attribute__((ext_vector_type(2)));

template <typename TQ, int NT, int CS, int RG_, int PART>
__device__ __forceinline__ void rowpass_part(double *sB, double *red, int64_t m, double *C,
                                             const TQ *CQ, const double *Sinv, const double *nu,
                                             const double *rdiag) {
    using RS = RowSplit<NT, CS, RG_>;
    typedef typename Pair<TQ>::v2 qv2;
    constexpr int RG = RS::RG, P = RS::P, LDB = RS::LDB, SLAB = RS::SLAB, PER2 = RS::PER2;
    constexpr int NTH = RS::NTH;
    constexpr int T0 = RS::t0(PART);
    constexpr int T1 = RS::t0(PART + 1);
    constexpr int NH = T1 - T0;
    constexpr int NQ = 4 * NH;                  // (s, t) pairs per k block
    constexpr int PH = PER2 > 4 && NQ >= 4 ? (PER2 + 1) / 2 : PER2;  // slab pairs in flight
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, q = lane >> 4, grp = wave % RG;
    const int64_t row = int64_t(blockIdx.x) * (16 * RG) + grp * 16 + lr;
    const bool ok = row < m;
    const int64_t rbase = (ok ? row : 0) * P + 2 * q;
    // A operand column of this lane inside a tile, and its slab row for step s
    const int acol = rp_col(lr & 3, lr >> 2);

    double keep[NH > 0 ? NH : 1][4];            // C_prior[row][16 t + col(q, s)], t in [T0, T1)
    double cur[4];
    dv2 nc[2];                                  // next block's C and C_Q, kept apart so the
    qv2 nq[2];                                  // loads are waited for only where they are used
    dv2 bpre[PH];
    d4 acc[NH > 0 ? NH : 1];
#pragma unroll
    for (int t = 0; t < NH; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};

#pragma unroll
    for (int u = 0; u < PER2; ++u) {
        const int idx = tid + NTH * u, rr = idx / (P / 2), c = 2 * (idx % (P / 2));
        if (idx < 8 * P)
            *reinterpret_cast<dv2 *>(sB + rr * LDB + c) =
                *reinterpret_cast<const dv2 *>(Sinv + int64_t(rr) * P + c);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const dv2 cv = *reinterpret_cast<const dv2 *>(C + rbase + 8 * h);
        const qv2 qv = *reinterpret_cast<const qv2 *>(CQ + rbase + 8 * h);
        cur[2 * h] = ok ? cv[0] + (double)qv[0] : 0.0;
        cur[2 * h + 1] = ok ? cv[1] + (double)qv[1] : 0.0;
    }
    __syncthreads();

#pragma unroll
    for (int kb = 0; kb < NT; ++kb) {
        if (kb > 0) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                cur[2 * h] = ok ? nc[h][0] + (double)nq[h][0] : 0.0;
                cur[2 * h + 1] = ok ? nc[h][1] + (double)nq[h][1] : 0.0;
            }
        }
        if (kb + 1 < NT) {
            // slab first: it is needed first (end of this block), C_prior next
#pragma unroll
            for (int u = 0; u < PH; ++u) {
                const int idx = tid + NTH * u, rr = idx / (P / 2), c = 2 * (idx % (P / 2));
                if (idx < 8 * P)
                    bpre[u] = *reinterpret_cast<const dv2 *>(Sinv + int64_t(16 * (kb + 1) + rr) * P + c);
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                nc[h] = *reinterpret_cast<const dv2 *>(C + rbase + 16 * (kb + 1) + 8 * h);
                nq[h] = *reinterpret_cast<const qv2 *>(CQ + rbase + 16 * (kb + 1) + 8 * h);
            }
        }
        if (kb >= T0 && kb < T1) {
#pragma unroll
            for (int s = 0; s < 4; ++s) keep[kb - T0][s] = cur[s];
        }
        if (NH > 0) {
            const double *B = sB + (kb & 1) * SLAB + 2 * q * LDB + acol + 16 * T0;
            // step s reads slab row col(q, s) = 8 (s/2) + 2 q + s % 2
            auto aop = [&](int i) {
                constexpr int NHp = NH > 0 ? NH : 1;
                const int si = i / NHp, ti = i % NHp;
                return B[(8 * (si >> 1) + (si & 1)) * LDB + 16 * ti];
            };
            double ring[3];
            ring[0] = aop(0);
            if (NQ > 1) ring[1] = aop(1);
#pragma unroll
            for (int i = 0; i < NQ; ++i) {
                if (i + 2 < NQ) ring[(i + 2) % 3] = aop(i + 2);
                const int si = i / NH, ti = i % NH;
                acc[ti] = __builtin_amdgcn_mfma_f64_16x16x4f64(ring[i % 3], cur[si], acc[ti], 0, 0, 0);
                if (PH < PER2 && i == NQ / 2 - 1 && kb + 1 < NT) {
                    // wide slabs go in two halves to bound the registers they hold;
                    // the target buffer was last read before the previous barrier
#pragma unroll
                    for (int u = 0; u < PH; ++u) {
                        const int idx = tid + NTH * u, rr = idx / (P / 2), c = 2 * (idx % (P / 2));
                        if (idx < 8 * P)
                            *reinterpret_cast<dv2 *>(sB + ((kb + 1) & 1) * SLAB + rr * LDB + c) = bpre[u];
                    }
#pragma unroll
                    for (int u = PH; u < PER2; ++u) {
                        const int idx = tid + NTH * u, rr = idx / (P / 2), c = 2 * (idx % (P / 2));
                        if (idx < 8 * P)
                            bpre[u - PH] = *reinterpret_cast<const dv2 *>(Sinv + int64_t(16 * (kb + 1) + rr) * P + c);
                    }
                }
            }
        }
        if (kb + 1 < NT) {
            constexpr int U0 = PH < PER2 ? PH : 0;
#pragma unroll
            for (int u = U0; u < PER2; ++u) {
                const int idx = tid + NTH * u, rr = idx / (P / 2), c = 2 * (idx % (P / 2));
                if (idx < 8 * P)
                    *reinterpret_cast<dv2 *>(sB + ((kb + 1) & 1) * SLAB + rr * LDB + c) = bpre[u - U0];
            }
        }
        __syncthreads();
    }

    // epilogue: lane holds K[row][16 t + col(q, r)] = acc[t - T0][r] and
    // C_prior[row][16 t + col(q, r)] = keep[t - T0][r]
    double dv = 0.0, dx = 0.0;
#pragma unroll
    for (int t = 0; t < NH; ++t)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = 16 * (T0 + t) + 8 * h + 2 * q;
            const dv2 nv = *reinterpret_cast<const dv2 *>(nu + c);
            const double k0 = acc[t][2 * h], k1 = acc[t][2 * h + 1];
            dv += k0 * keep[t][2 * h] + k1 * keep[t][2 * h + 1];
            dx += k0 * nv[0] + k1 * nv[1];
        }
    // C <- K R.  A row's 16 columns of tile t sit in its 4 lanes as two
    // 64-byte halves (h = 0: columns 0..7, h = 1: 8..15).  Lanes of rows 2j
    // and 2j + 1 (adjacent lanes) swap one half each (DPP quad permutation
    // [1,0,3,2]), so that every store instruction writes whole 128-byte rows:
    // first rows 2j (the even lane's h = 0 and, from the odd lane, the even
    // row's h = 1), then rows 2j + 1.
    {
        const bool odd = lr & 1;
        const int64_t r0 = row - odd;
        auto swap_pair = [](double x) {
            int2 v = __builtin_bit_cast(int2, x);
            v.x = __builtin_amdgcn_mov_dpp(v.x, 0xB1, 0xF, 0xF, false);
            v.y = __builtin_amdgcn_mov_dpp(v.y, 0xB1, 0xF, 0xF, false);
            return __builtin_bit_cast(double, v);
        };
#pragma unroll
        for (int t = 0; t < NH; ++t) {
            const int c0 = 16 * (T0 + t) + 2 * q;
            const dv2 ra = *reinterpret_cast<const dv2 *>(rdiag + c0);
            const dv2 rb = *reinterpret_cast<const dv2 *>(rdiag + c0 + 8);
            const dv2 a = dv2{acc[t][0] * ra[0], acc[t][1] * ra[1]};   // h = 0 of own row
            const dv2 b = dv2{acc[t][2] * rb[0], acc[t][3] * rb[1]};   // h = 1 of own row
            const dv2 g = dv2{swap_pair(odd ? a[0] : b[0]), swap_pair(odd ? a[1] : b[1])};
            const int cc = c0 + (odd ? 8 : 0);
            // streaming stores: C is not read again within this pass
            if (r0 < m) __builtin_nontemporal_store(odd ? g : a, reinterpret_cast<dv2 *>(C + r0 * P + cc));
            if (r0 + 1 < m)
                __builtin_nontemporal_store(odd ? b : g, reinterpret_cast<dv2 *>(C + (r0 + 1) * P + cc));
        }
    }
    dv += __shfl_xor(dv, 16, 64);
    dx += __shfl_xor(dx, 16, 64);
    dv += __shfl_xor(dv, 32, 64);
    dx += __shfl_xor(dx, 32, 64);
    if (q == 0) {
        red[((PART * RG + grp) * 16 + lr) * 2 + 0] = dv;
        red[((PART * RG + grp) * 16 + lr) * 2 + 1] = dx;
    }
}

template <typename TQ, int NT, int CS, int RG>
__global__ void __launch_bounds__(64 * CS * RG)
k_rowpass(int64_t m, double *C, const TQ *CQ, const double *Sinv, const double *nu,
          const double *rdiag, double *xhat, double *var, double kdiag, const int *status,
          unsigned long long *negvar) {
    using RS = RowSplit<NT, CS, RG>;
    __shared__ __align__(16) double sB[2 * RS::SLAB];
    __shared__ double red[CS * RG * 16 * 2];
    if (status[kStStep] != HIKF_OK) return;
    const int part = (threadIdx.x >> 6) / RG;
    if (part == 0)
        rowpass_part<TQ, NT, CS, RG, 0>(sB, red, m, C, CQ, Sinv, nu, rdiag);
    else if (part == 1)
        rowpass_part<TQ, NT, CS, RG, 1>(sB, red, m, C, CQ, Sinv, nu, rdiag);
    else if (CS > 2 && part == 2)
        rowpass_part<TQ, NT, CS, RG, (CS > 2 ? 2 : 0)>(sB, red, m, C, CQ, Sinv, nu, rdiag);
    else if (CS > 3)
        rowpass_part<TQ, NT, CS, RG, (CS > 3 ? 3 : 0)>(sB, red, m, C, CQ, Sinv, nu, rdiag);
    __syncthreads();
    const int tid = threadIdx.x;
    if (tid < 16 * RG) {
        const int64_t row = int64_t(blockIdx.x) * (16 * RG) + tid;
        if (row < m) {
            double dv = 0.0, dx = 0.0;
#pragma unroll
            for (int c = 0; c < CS; ++c) {
                dv += red[(c * 16 * RG + tid) * 2];
                dx += red[(c * 16 * RG + tid) * 2 + 1];
            }
            const double v = var[row] + kdiag - dv;
            var[row] = v;
            xhat[row] += dx;
            if (v < 0.0) atomicAdd(negvar, 1ull);
        }
    }
}

template <typename TQ, int NT>
void launch_rowpass_nt(const Geometry &g, const Layout &lay, char *res, hipStream_t s) {
    constexpr int CS = NT <= 16 ? 2 : 4;
    constexpr int RG = NT <= 16 ? 4 : 2;     // 8 waves; 4-wave workgroups of 32 rows measured slower
    constexpr int rows = 16 * RG;
    const unsigned blocks = unsigned((g.m + rows - 1) / rows);
    hipLaunchKernelGGL((k_rowpass<TQ, NT, CS, RG>), dim3(blocks), dim3(64 * CS * RG), 0, s, g.m,
                       reinterpret_cast<double *>(res + lay.C),
                       reinterpret_cast<const TQ *>(res + lay.CQ),
                       reinterpret_cast<const double *>(res + lay.sinv),
                       reinterpret_cast<const double *>(res + lay.nu),
                       reinterpret_cast<const double *>(res + lay.rdiag),
                       reinterpret_cast<double *>(res + lay.xhat),
                       reinterpret_cast<double *>(res + lay.var), g.kp.family == HIKF_KERNEL_TEST_R2 ? 0.0 : g.kp.theta,
                       reinterpret_cast<const int *>(res + lay.status),
                       reinterpret_cast<unsigned long long *>(res + lay.negvar));
}

template <typename TQ>
void launch_rowpass(const Geometry &g, const Layout &lay, char *res, hipStream_t s) {
    switch (g.p / 16) {
#define HIKF_NT(N) case N: launch_rowpass_nt<TQ, N>(g, lay, res, s); break;
        HIKF_NT(1) HIKF_NT(2) HIKF_NT(3) HIKF_NT(4) HIKF_NT(5) HIKF_NT(6) HIKF_NT(7) HIKF_NT(8)
        HIKF_NT(9) HIKF_NT(10) HIKF_NT(11) HIKF_NT(12) HIKF_NT(13) HIKF_NT(14) HIKF_NT(15)
        HIKF_NT(16) HIKF_NT(17) HIKF_NT(18) HIKF_NT(19) HIKF_NT(20) HIKF_NT(21) HIKF_NT(22)
        HIKF_NT(23) HIKF_NT(24) HIKF_NT(25) HIKF_NT(26) HIKF_NT(27) HIKF_NT(28) HIKF_NT(29)
        HIKF_NT(30) HIKF_NT(31) HIKF_NT(32)
#undef HIKF_NT
        default: break;
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
    if (gather)
        run_gather<TQ>(g, lay, res, true, reinterpret_cast<double *>(res + lay.G),
                       reinterpret_cast<double *>(res + lay.hvec), s, tm);
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
    launch_rowpass<TQ>(g, lay, res, s);
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

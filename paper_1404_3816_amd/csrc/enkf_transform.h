// Ensemble transform of the EnKF analysis (Sec. 2.3), included by the
// enkf_transform_*.hip units (each instantiates a few tile widths, so that
// the kernels compile in parallel): X <- (X + E) W for all
// m member rows, with the analysis sample mean (eq. equation_samplemean) and
// the diagonal of the sample covariance (eq. equation_samplecov1) of every
// row.  W = I + (I - 1 1^T / N) T / sqrt(N - 1) is the N x N matrix formed in
// enkf.hip; the product is the O(m N^2) part of a step, on FP64 MFMA.
//
// Tiling (the same lane layout as the HiKF row pass): a workgroup of 8
// waves takes a tile of 16 RG rows; wave w takes row group w % RG (lane l
// owns row l % 16 of it) and column part w / RG.  v_mfma_f64_16x16x4 computes
// tiles of Y^T = W^T X_f^T: the A operand is a 16 x 4 piece of a 16-row slab
// of W (rows k of W: W[k][c] is A[c][k]) read from LDS, the B operand is 4
// values of the lane's own row of X_f = X + E, so the output stays in the
// lane that owns the row.  With q = l / 16 the lane holds, for tile t and
// r = 0..3, Y[row][16 t + 8 (r/2) + 2 q + r % 2], and those are exactly the
// columns of X_f it loads as 16-byte pairs; every access of X and E is a
// 16-byte vector access.  The slabs of W stream through two LDS buffers
// (pitch ld + 8 doubles), prefetched into registers one block ahead.  Every
// row is read and written once; the row is written in place (a workgroup
// has loaded all of its rows before its first store).
#pragma once

#include "enkf_internal.h"
#include "hikf_internal.h"

namespace hikf {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double dv2 __attribute__((ext_vector_type(2)));

template <int NT, int CS, int RG>
struct EnSplit {
    static constexpr int NTH = 64 * CS * RG;
    static constexpr int P = NT * 16;
    static constexpr int LDB = P + 8;
    static constexpr int SLAB = 16 * LDB;
    static constexpr int PER2 = (8 * P + NTH - 1) / NTH;   // slab column pairs per thread
    static constexpr int t0(int c) { return (c * NT + CS - 1) / CS; }
};

__device__ __forceinline__ constexpr int en_col(int q, int r) { return 8 * (r >> 1) + 2 * q + (r & 1); }

template <int NT, int CS, int RG, int PART, bool HAS_E>
__device__ __forceinline__ void en_part(double *sB, double *red, double *red2, int64_t m,
                                        int n_ens, double *X, const double *E, const double *W,
                                        double *xmean, double *xvar) {
    using ES = EnSplit<NT, CS, RG>;
    constexpr int P = ES::P, LDB = ES::LDB, SLAB = ES::SLAB, PER2 = ES::PER2, NTH = ES::NTH;
    constexpr int T0 = ES::t0(PART);
    constexpr int T1 = ES::t0(PART + 1);
    constexpr int NH = T1 - T0;
    constexpr int NQ = 4 * NH;
    constexpr int PH = PER2 > 4 && NQ >= 4 ? (PER2 + 1) / 2 : PER2;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, q = lane >> 4, grp = wave % RG;
    const int acol = en_col(lr & 3, lr >> 2);
    const int64_t row = int64_t(blockIdx.x) * (16 * RG) + grp * 16 + lr;
    const bool ok = row < m;
    const int64_t rbase = (ok ? row : 0) * P + 2 * q;

    double cur[4];
    dv2 nx[2], ne[2];
    dv2 bpre[PH];
    d4 acc[NH > 0 ? NH : 1];

#pragma unroll
    for (int u = 0; u < PER2; ++u) {
        const int idx = tid + NTH * u, rr = idx / (P / 2), c = 2 * (idx % (P / 2));
        if (idx < 8 * P)
            *reinterpret_cast<dv2 *>(sB + rr * LDB + c) =
                *reinterpret_cast<const dv2 *>(W + int64_t(rr) * P + c);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        nx[h] = *reinterpret_cast<const dv2 *>(X + rbase + 8 * h);
        if (HAS_E) ne[h] = *reinterpret_cast<const dv2 *>(E + rbase + 8 * h);
    }
#pragma unroll
    for (int t = 0; t < NH; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
    __syncthreads();

#pragma unroll
    for (int kb = 0; kb < NT; ++kb) {
        // member columns 16 kb + 8 h + 2 q + i; columns at or beyond N hold
        // no member (E may hold anything there)
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int c = 16 * kb + 8 * h + 2 * q + i;
                const double v = HAS_E ? nx[h][i] + ne[h][i] : nx[h][i];
                cur[2 * h + i] = ok && c < n_ens ? v : 0.0;
            }
        const bool pf = kb + 1 < NT;
        const int nslab = 16 * (kb + 1);
        double *nbuf = sB + ((kb + 1) & 1) * SLAB;
        if (pf) {
#pragma unroll
            for (int u = 0; u < PH; ++u) {
                const int idx = tid + NTH * u, rr = idx / (P / 2), c = 2 * (idx % (P / 2));
                if (idx < 8 * P)
                    bpre[u] = *reinterpret_cast<const dv2 *>(W + int64_t(nslab + rr) * P + c);
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                nx[h] = *reinterpret_cast<const dv2 *>(X + rbase + 16 * (kb + 1) + 8 * h);
                if (HAS_E) ne[h] = *reinterpret_cast<const dv2 *>(E + rbase + 16 * (kb + 1) + 8 * h);
            }
        }
        if (NH > 0) {
            const double *B = sB + (kb & 1) * SLAB + 2 * q * LDB + acol + 16 * T0;
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
                if (PH < PER2 && i == NQ / 2 - 1 && pf) {
#pragma unroll
                    for (int u = 0; u < PH; ++u) {
                        const int idx = tid + NTH * u, rr = idx / (P / 2), c = 2 * (idx % (P / 2));
                        if (idx < 8 * P) *reinterpret_cast<dv2 *>(nbuf + rr * LDB + c) = bpre[u];
                    }
#pragma unroll
                    for (int u = PH; u < PER2; ++u) {
                        const int idx = tid + NTH * u, rr = idx / (P / 2), c = 2 * (idx % (P / 2));
                        if (idx < 8 * P)
                            bpre[u - PH] = *reinterpret_cast<const dv2 *>(W + int64_t(nslab + rr) * P + c);
                    }
                }
            }
        }
        if (pf) {
            constexpr int U0 = PH < PER2 ? PH : 0;
#pragma unroll
            for (int u = U0; u < PER2; ++u) {
                const int idx = tid + NTH * u, rr = idx / (P / 2), c = 2 * (idx % (P / 2));
                if (idx < 8 * P) *reinterpret_cast<dv2 *>(nbuf + rr * LDB + c) = bpre[u - U0];
            }
        }
        __syncthreads();
    }

    // epilogue: the lane holds Y[row][16 t + en_col(q, r)] = acc[t - T0][r]
    const double inv_n = 1.0 / n_ens, inv_n1 = 1.0 / (n_ens - 1);
    double s1 = 0.0;
#pragma unroll
    for (int t = 0; t < NH; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (16 * (T0 + t) + en_col(q, r) < n_ens) s1 += acc[t][r];
    s1 += __shfl_xor(s1, 16, 64);
    s1 += __shfl_xor(s1, 32, 64);
    if (q == 0) red[(PART * RG + grp) * 16 + lr] = s1;
    // store the row (in place): lanes of rows 2j and 2j + 1 swap one 64-byte
    // half per tile (DPP quad permutation [1,0,3,2]) so that every store
    // instruction writes whole 128-byte row pieces
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
            const dv2 a = dv2{acc[t][0], acc[t][1]};        // h = 0 of the own row
            const dv2 b = dv2{acc[t][2], acc[t][3]};        // h = 1 of the own row
            const dv2 g = dv2{swap_pair(odd ? a[0] : b[0]), swap_pair(odd ? a[1] : b[1])};
            const int cc = c0 + (odd ? 8 : 0);
            if (r0 < m) __builtin_nontemporal_store(odd ? g : a, reinterpret_cast<dv2 *>(X + r0 * P + cc));
            if (r0 + 1 < m)
                __builtin_nontemporal_store(odd ? b : g, reinterpret_cast<dv2 *>(X + (r0 + 1) * P + cc));
        }
    }
    __syncthreads();
    double mean = 0.0;
#pragma unroll
    for (int c = 0; c < CS; ++c) mean += red[(c * RG + grp) * 16 + lr];
    mean *= inv_n;
    double s2 = 0.0;
#pragma unroll
    for (int t = 0; t < NH; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (16 * (T0 + t) + en_col(q, r) < n_ens) {
                const double d = acc[t][r] - mean;
                s2 += d * d;
            }
    s2 += __shfl_xor(s2, 16, 64);
    s2 += __shfl_xor(s2, 32, 64);
    if (q == 0) red2[(PART * RG + grp) * 16 + lr] = s2;
    __syncthreads();
    if (PART == 0 && q == 0 && ok) {
        double v = 0.0;
#pragma unroll
        for (int c = 0; c < CS; ++c) v += red2[(c * RG + grp) * 16 + lr];
        xmean[row] = mean;
        xvar[row] = v * inv_n1;
    }
}

template <int NT, int CS, int RG, bool HAS_E>
__global__ void __launch_bounds__(64 * CS * RG)
k_en_transform(int64_t m, int n_ens, double *X, const double *E, const double *W, double *xmean,
               double *xvar, const int *status, long long *applied) {
    using ES = EnSplit<NT, CS, RG>;
    __shared__ __align__(16) double sB[2 * ES::SLAB];
    __shared__ double red[CS * RG * 16], red2[CS * RG * 16];
    if (status[kStStep] != HIKF_OK) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) applied[0] += 1;
    const int part = (threadIdx.x >> 6) / RG;
#define HIKF_EN_PART(K) en_part<NT, CS, RG, (K), HAS_E>(sB, red, red2, m, n_ens, X, E, W, xmean, xvar)
    // (with one column part only part 0 exists: no other part is compiled)
    if (CS == 1 || part == 0)
        HIKF_EN_PART(0);
    else if (part == 1)
        HIKF_EN_PART(CS > 1 ? 1 : 0);
    else if (CS > 2 && part == 2)
        HIKF_EN_PART(CS > 2 ? 2 : 0);
    else if (CS > 3)
        HIKF_EN_PART(CS > 3 ? 3 : 0);
#undef HIKF_EN_PART
}

template <int NT, int RG>
hipError_t en_go_rg(int64_t m, int n_ens, double *X, const double *E, const double *W,
                    double *xmean, double *xvar, const int *status, long long *applied,
                    hipStream_t s) {
    constexpr int CS = 8 / RG;
    const unsigned blocks = unsigned((m + 16 * RG - 1) / (16 * RG));
    if (E)
        hipLaunchKernelGGL((k_en_transform<NT, CS, RG, true>), dim3(blocks), dim3(64 * CS * RG), 0,
                           s, m, n_ens, X, E, W, xmean, xvar, status, applied);
    else
        hipLaunchKernelGGL((k_en_transform<NT, CS, RG, false>), dim3(blocks), dim3(64 * CS * RG), 0,
                           s, m, n_ens, X, E, W, xmean, xvar, status, applied);
    return hipGetLastError();
}

// tile_rows 64: 4 row groups x 2 column halves; 32: 2 row groups x 4
// column quarters (fewer accumulators per wave, twice the LDS reads of W
// per row); 128 (ld <= 256): 8 row groups, every wave on all columns (twice
// the MFMAs per k block and per slab of W); 0: 128 up to ld = 256, else 64.
// Measured on 1024^2 rows (ms, fraction of the FP64 peak):
//   N = 128: 128 rows 0.69 (0.64), 64 rows 0.82 (0.53)
//   N = 256: 128 rows 2.41 (0.73), 64 rows 2.67 (0.66), 32 rows 3.44
//   N = 400: 64 rows 6.27 (0.68), 32 rows 8.04;  N = 512: 64 rows 9.26
//   (0.76), 32 rows 11.73 (at ld >= 448 a wave spills a few registers).
template <int NT>
hipError_t en_go(int tile_rows, int64_t m, int n_ens, double *X, const double *E, const double *W,
                 double *xmean, double *xvar, const int *status, long long *applied,
                 hipStream_t s) {
    if constexpr (NT <= 16) {
        if (tile_rows == 128 || tile_rows == 0)
            return en_go_rg<NT, 8>(m, n_ens, X, E, W, xmean, xvar, status, applied, s);
    }
    if (tile_rows != 32) return en_go_rg<NT, 4>(m, n_ens, X, E, W, xmean, xvar, status, applied, s);
    return en_go_rg<NT, 2>(m, n_ens, X, E, W, xmean, xvar, status, applied, s);
}

}  // namespace

// one tile width: the unit that instantiates it compiles its kernels
template <int NT>
hipError_t enkf_transform_nt(int tile_rows, int64_t m, int n_ens, double *X, const double *E,
                             const double *W, double *xmean, double *xvar, const int *status,
                             long long *applied, hipStream_t s) {
    return en_go<NT>(tile_rows, m, n_ens, X, E, W, xmean, xvar, status, applied, s);
}

}  // namespace hikf

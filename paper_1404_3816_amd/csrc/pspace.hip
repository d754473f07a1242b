// p x p part of one assimilation step (Algorithm Algorithm_HiKF, gain row):
// S = (G + G^T)/2 + R with G = H C_prior, its Cholesky factor S = L L^T,
// X = L^{-1} and S^{-1} = X^T X, plus the innovation nu = y - h.
//
// Blocked with 32 x 32 FP64 blocks (the matrix is padded to PP = 32 NBk with
// an identity block), every block product on v_mfma_f64_16x16x4 with one
// 256-thread workgroup per block (each wave owns one 16 x 16 tile):
//   k_ps_factor   (1 WG)     : checks y, forms nu, factors block (0,0):
//                              L00 and D0 = L00^{-1}.
//   k_ps_update(kb)          : one WG per block (i, j), kb < j <= i: panel
//                              blocks L_ik = A_ik D_kb^T, L_jk = A_jk D_kb^T,
//                              A_ij -= L_ik L_jk^T; the WG of block
//                              (kb+1, kb+1) then factors it (L, D for kb+1).
//   k_ps_trtri    (NBk WGs)  : column j of X: X_jj = D_j,
//                              X_ij = -D_i sum_{k=j}^{i-1} L_ik X_kj.
//   k_ps_lauum    (one WG per lower block): S^{-1}_ij = sum_{k>=i} X_ki^T X_kj.
// A failed pivot (not > 0 or not finite) sets HIKF_E_NOT_SPD; every later
// kernel, and the row pass, then does nothing, so the state is untouched.
#include "hikf_internal.h"

namespace hikf {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int BS = 32;            // block size
constexpr int BP = 36;            // LDS pitch of a block (doubles)
constexpr int NT = 256;           // threads per workgroup
constexpr int kMaxNbk = kMaxP / BS;

// element (r, c) of block (bi, bj) of S = (G + G^T)/2 + R, identity beyond p
__device__ __forceinline__ double s_elem(const double *G, const double *rdiag, int p, int i, int j) {
    if (i < p && j < p)
        return 0.5 * (G[int64_t(i) * p + j] + G[int64_t(j) * p + i]) + (i == j ? rdiag[i] : 0.0);
    return i == j ? 1.0 : 0.0;
}

// Load block (bi, bj) of the working matrix into LDS: from G (first use,
// symmetrised, plus R) or from the PP x PP buffer A.
__device__ void blk_load(double *s, const double *A, int PP, const double *G, const double *rdiag,
                         int p, bool from_g, int bi, int bj) {
    for (int idx = threadIdx.x; idx < BS * BS; idx += NT) {
        const int r = idx / BS, c = idx % BS, i = bi * BS + r, j = bj * BS + c;
        s[r * BP + c] = from_g ? s_elem(G, rdiag, p, i, j) : A[int64_t(i) * PP + j];
    }
}

__device__ void blk_load_plain(double *s, const double *A, int PP, int bi, int bj) {
    for (int idx = threadIdx.x; idx < BS * BS; idx += NT) {
        const int r = idx / BS, c = idx % BS;
        s[r * BP + c] = A[int64_t(bi * BS + r) * PP + bj * BS + c];
    }
}

__device__ void blk_store(const double *s, double *A, int PP, int bi, int bj) {
    for (int idx = threadIdx.x; idx < BS * BS; idx += NT) {
        const int r = idx / BS, c = idx % BS;
        A[int64_t(bi * BS + r) * PP + bj * BS + c] = s[r * BP + c];
    }
}

// One wave's 16 x 16 tile (wi, wj) of op(A) op(B) over k = 0..31, added to acc.
// TA: use A^T; TB: use B^T.  Lane l supplies A[l%16][l/16], B[l/16][l%16];
// acc[r] holds C[16 wi + l/16 + 4 r][16 wj + l%16].
template <bool TA, bool TB>
__device__ __forceinline__ d4 tile_mma(d4 acc, const double *sA, const double *sB, double sign) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wi = wave >> 1, wj = wave & 1, lr = lane & 15, q = lane >> 4;
#pragma unroll
    for (int k0 = 0; k0 < BS; k0 += 4) {
        const int k = k0 + q;
        const double a = TA ? sA[k * BP + 16 * wi + lr] : sA[(16 * wi + lr) * BP + k];
        const double b = TB ? sB[(16 * wj + lr) * BP + k] : sB[k * BP + 16 * wj + lr];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sign * a, b, acc, 0, 0, 0);
    }
    return acc;
}

__device__ __forceinline__ d4 tile_read(const double *s) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wi = wave >> 1, wj = wave & 1, lr = lane & 15, q = lane >> 4;
    d4 v;
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = s[(16 * wi + q + 4 * r) * BP + 16 * wj + lr];
    return v;
}

__device__ __forceinline__ void tile_write(double *s, d4 v) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wi = wave >> 1, wj = wave & 1, lr = lane & 15, q = lane >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r) s[(16 * wi + q + 4 * r) * BP + 16 * wj + lr] = v[r];
}

// Factor the 32 x 32 SPD block in sA (in place) into L (lower, zero above)
// and write D = L^{-1} into sD.  Returns false on a failed pivot; *piv gets
// the smallest diagonal of L (or the failing pivot).  Uniform across the WG.
__device__ bool blk_factor(double *sA, double *sD, double *piv) {
    const int t = threadIdx.x, c = t % BS, r0 = t / BS;      // 4 rows per thread: r0 + 8 u
    double mp = 1.0e300;
    for (int j = 0; j < BS; ++j) {
        const double d2 = sA[j * BP + j];
        if (!(d2 > 0.0) || !isfinite(d2)) { *piv = d2; return false; }
        mp = fmin(mp, d2);
        const double inv = 1.0 / d2;
        const double acj = sA[c * BP + j];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = r0 + 8 * u;
            if (c > j && c <= i) sA[i * BP + c] -= sA[i * BP + j] * acj * inv;
        }
        __syncthreads();
    }
    // scale the columns: L_ij = A_ij / sqrt(A_jj); zero the upper part
    double vals[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int i = r0 + 8 * u;
        vals[u] = i >= c ? sA[i * BP + c] / sqrt(sA[c * BP + c]) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int i = r0 + 8 * u;
        sA[i * BP + c] = vals[u];
        sD[i * BP + c] = i == c ? 1.0 : 0.0;
    }
    *piv = sqrt(mp);
    __syncthreads();
    // D = L^{-1}: row k of D is final once divided by L_kk; then rows i > k
    // subtract L_ik D_k.
    for (int k = 0; k < BS; ++k) {
        if (k % 8 == r0) sD[k * BP + c] /= sA[k * BP + k];
        __syncthreads();
        const double dk = sD[k * BP + c];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = r0 + 8 * u;
            if (i > k) sD[i * BP + c] -= sA[i * BP + k] * dk;
        }
        __syncthreads();
    }
    return true;
}

struct PsArgs {
    int p, PP, nbk;
    const double *G, *rdiag, *y, *hvec;
    double *A, *L, *D, *X, *Sinv, *nu, *pivs, *minpiv;
    int *status;
    long long *steps;
};

__global__ void __launch_bounds__(NT) k_ps_factor(PsArgs a) {
    __shared__ double sA[BS * BP];
    __shared__ double sD[BS * BP];
    const int t = threadIdx.x;
    int bad = a.status[kStInit] != 0;
    for (int i = t; i < a.p; i += NT)
        if (!isfinite(a.y[i])) bad = 1;
    bad = __syncthreads_or(bad);
    if (bad) {
        if (t == 0) a.status[kStStep] = HIKF_E_INVALID;
        return;
    }
    for (int i = t; i < a.p; i += NT) a.nu[i] = a.y[i] - a.hvec[i];
    blk_load(sA, a.A, a.PP, a.G, a.rdiag, a.p, true, 0, 0);
    __syncthreads();
    double piv;
    const bool ok = blk_factor(sA, sD, &piv);
    if (t == 0) {
        a.status[kStStep] = ok ? HIKF_OK : HIKF_E_NOT_SPD;
        a.pivs[0] = piv;
        if (!ok) a.minpiv[0] = piv;
    }
    if (!ok) return;
    blk_store(sA, a.L, a.PP, 0, 0);
    blk_store(sD, a.D, BS, 0, 0);
}

// block (i, j) with kb < j <= i < nbk, enumerated row by row
__device__ __forceinline__ void pair_of(int w, int kb, int *bi, int *bj) {
    int i = kb + 1, base = 0;
    while (base + (i - kb) <= w) { base += i - kb; ++i; }
    *bi = i;
    *bj = kb + 1 + (w - base);
}

__global__ void __launch_bounds__(NT) k_ps_update(PsArgs a, int kb) {
    __shared__ double sD[BS * BP];
    __shared__ double sPi[BS * BP];
    __shared__ double sPj[BS * BP];
    __shared__ double sT[BS * BP];
    if (a.status[kStStep] != HIKF_OK) return;
    int bi, bj;
    pair_of(blockIdx.x, kb, &bi, &bj);
    const bool first = kb == 0;
    blk_load_plain(sD, a.D + int64_t(kb) * BS * BS, BS, 0, 0);
    blk_load(sPi, a.A, a.PP, a.G, a.rdiag, a.p, first, bi, kb);
    blk_load(sPj, a.A, a.PP, a.G, a.rdiag, a.p, first, bj, kb);
    blk_load(sT, a.A, a.PP, a.G, a.rdiag, a.p, first, bi, bj);
    __syncthreads();
    // panel blocks: L_ik = A_ik D^T, L_jk = A_jk D^T
    d4 pi = tile_mma<false, true>(d4{0, 0, 0, 0}, sPi, sD, 1.0);
    d4 pj = tile_mma<false, true>(d4{0, 0, 0, 0}, sPj, sD, 1.0);
    d4 acc = tile_read(sT);
    __syncthreads();
    tile_write(sPi, pi);
    tile_write(sPj, pj);
    __syncthreads();
    if (bj == kb + 1) blk_store(sPi, a.L, a.PP, bi, kb);
    // A_ij -= L_ik L_jk^T
    acc = tile_mma<false, true>(acc, sPi, sPj, -1.0);
    if (bi == bj && bi == kb + 1) {
        // the next diagonal block is final: factor it here
        tile_write(sT, acc);
        __syncthreads();
        double piv;
        const bool ok = blk_factor(sT, sD, &piv);
        if (threadIdx.x == 0) {
            a.pivs[bi] = piv;
            if (!ok) {
                a.status[kStStep] = HIKF_E_NOT_SPD;
                a.minpiv[0] = piv;
            }
        }
        if (!ok) return;
        blk_store(sT, a.L, a.PP, bi, bi);
        blk_store(sD, a.D + int64_t(bi) * BS * BS, BS, 0, 0);
    } else {
        __syncthreads();
        tile_write(sT, acc);
        __syncthreads();
        blk_store(sT, a.A, a.PP, bi, bj);
    }
}

__global__ void __launch_bounds__(NT) k_ps_trtri(PsArgs a) {
    // The blocks X_kj of column j are written to X as soon as they are final
    // and read back from there (they are needed by every later block of the
    // column; at PP = 512 they would not fit in LDS together).  The barrier
    // that follows each store makes them visible to the whole workgroup.
    __shared__ double sL[BS * BP];                // staged L_ik block
    __shared__ double sX[BS * BP];                // staged X_kj block
    __shared__ double sD[BS * BP];
    if (a.status[kStStep] != HIKF_OK) return;
    const int j = blockIdx.x;
    blk_load_plain(sD, a.D + int64_t(j) * BS * BS, BS, 0, 0);
    __syncthreads();
    blk_store(sD, a.X, a.PP, j, j);
    for (int i = j + 1; i < a.nbk; ++i) {
        d4 acc = d4{0, 0, 0, 0};
        for (int k = j; k < i; ++k) {
            __syncthreads();
            blk_load_plain(sL, a.L, a.PP, i, k);
            blk_load_plain(sX, a.X, a.PP, k, j);
            __syncthreads();
            acc = tile_mma<false, false>(acc, sL, sX, 1.0);
        }
        __syncthreads();
        tile_write(sL, acc);                       // T = sum_k L_ik X_kj
        blk_load_plain(sD, a.D + int64_t(i) * BS * BS, BS, 0, 0);
        __syncthreads();
        d4 x = tile_mma<false, false>(d4{0, 0, 0, 0}, sD, sL, -1.0);
        tile_write(sX, x);
        __syncthreads();
        blk_store(sX, a.X, a.PP, i, j);
    }
}

__global__ void __launch_bounds__(NT) k_ps_lauum(PsArgs a) {
    __shared__ double sXi[BS * BP];
    __shared__ double sXj[BS * BP];
    __shared__ double sT[BS * BP];
    if (a.status[kStStep] != HIKF_OK) return;
    int bi = 0, base = 0;
    while (base + bi + 1 <= (int)blockIdx.x) { base += bi + 1; ++bi; }
    const int bj = blockIdx.x - base;              // 0 <= bj <= bi
    d4 acc = d4{0, 0, 0, 0};
    for (int k = bi; k < a.nbk; ++k) {
        __syncthreads();
        blk_load_plain(sXi, a.X, a.PP, k, bi);
        blk_load_plain(sXj, a.X, a.PP, k, bj);
        __syncthreads();
        acc = tile_mma<true, false>(acc, sXi, sXj, 1.0);   // X_ki^T X_kj
    }
    __syncthreads();
    tile_write(sT, acc);
    __syncthreads();
    for (int idx = threadIdx.x; idx < BS * BS; idx += NT) {
        const int r = idx / BS, c = idx % BS, i = bi * BS + r, jj = bj * BS + c;
        // a diagonal block is written from its lower half only, so that both
        // triangles of S^{-1} receive the same value
        if (i < a.p && jj < a.p && (bi != bj || r >= c)) {
            a.Sinv[int64_t(i) * a.p + jj] = sT[r * BP + c];
            a.Sinv[int64_t(jj) * a.p + i] = sT[r * BP + c];
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double mp = a.pivs[0];
        for (int k = 1; k < a.nbk; ++k) mp = fmin(mp, a.pivs[k]);
        a.minpiv[0] = mp;
        a.steps[0] += 1;
    }
}

}  // namespace

hipError_t launch_pspace(const Geometry &g, const Layout &lay, char *res, const double *y,
                         hipStream_t s) {
    PsArgs a;
    a.p = g.p;
    a.PP = g.pp;
    a.nbk = g.pp / BS;
    a.G = reinterpret_cast<const double *>(res + lay.G);
    a.rdiag = reinterpret_cast<const double *>(res + lay.rdiag);
    a.y = y;
    a.hvec = reinterpret_cast<const double *>(res + lay.hvec);
    a.A = reinterpret_cast<double *>(res + lay.psA);
    a.L = reinterpret_cast<double *>(res + lay.psL);
    a.D = reinterpret_cast<double *>(res + lay.psD);
    a.X = reinterpret_cast<double *>(res + lay.xbuf);
    a.Sinv = reinterpret_cast<double *>(res + lay.sinv);
    a.nu = reinterpret_cast<double *>(res + lay.nu);
    a.pivs = reinterpret_cast<double *>(res + lay.pivs);
    a.minpiv = reinterpret_cast<double *>(res + lay.minpiv);
    a.status = reinterpret_cast<int *>(res + lay.status);
    a.steps = reinterpret_cast<long long *>(res + lay.steps);
    hipLaunchKernelGGL(k_ps_factor, dim3(1), dim3(NT), 0, s, a);
    for (int kb = 0; kb + 1 < a.nbk; ++kb) {
        const int n = a.nbk - 1 - kb;
        hipLaunchKernelGGL(k_ps_update, dim3(n * (n + 1) / 2), dim3(NT), 0, s, a, kb);
    }
    if (a.nbk > kMaxNbk) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_ps_trtri, dim3(a.nbk), dim3(NT), 0, s, a);
    hipLaunchKernelGGL(k_ps_lauum, dim3(a.nbk * (a.nbk + 1) / 2), dim3(NT), 0, s, a);
    return hipGetLastError();
}

}  // namespace hikf

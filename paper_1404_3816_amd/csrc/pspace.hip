// p x p part of one assimilation step (Algorithm Algorithm_HiKF, gain row):
// S = (G + G^T)/2 + R with G = H C_prior, S^{-1}, and the innovation
// nu = y - h.
//
// S^{-1} comes from the symmetric sweep operator (block Gauss-Jordan
// elimination without pivoting, valid for SPD matrices) over 32 x 32 FP64
// blocks; the matrix is padded to PP = 32 NBk with an identity block.
// Sweeping pivot block k maps
//     A_kk -> -A_kk^{-1},        A_ik -> A_ik A_kk^{-1},   A_kj -> A_kk^{-1} A_kj,
//     A_ij -> A_ij - A_ik A_kk^{-1} A_kj                       (i, j != k),
// and after all blocks the matrix is -S^{-1}.  The pivots are those of the
// Cholesky factorisation (LDL^T), so S is SPD exactly when every pivot is
// positive, and sqrt(pivot) is the Cholesky diagonal.
//   k_ps_sweep(k), one launch per pivot block, one 256-thread workgroup per
//   block (i, j) of the matrix (ping-pong between two PP x PP buffers):
//   wave 0 sweeps the 32 scalar pivots of block (k, k) in registers (no
//   barriers: column and row j pass through wave-private LDS), then the four
//   waves form the block's new value on v_mfma_f64_16x16x4 (each wave owns
//   one 16 x 16 tile).  Launch 0 also checks y and forms nu; the last launch
//   writes S^{-1}.
// A non-positive or non-finite pivot sets HIKF_E_NOT_SPD; every later
// launch, and the row pass, then does nothing, so the state is untouched.
#include "hikf_internal.h"
#include "sweep.h"

namespace hikf {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int BS = 32;            // block size
constexpr int BP = 36;            // LDS pitch of a block (doubles)
constexpr int NT = 256;           // threads per workgroup

// element (r, c) of block (bi, bj) of S = (G + G^T)/2 + R, identity beyond p
__device__ __forceinline__ double s_elem(const double *G, const double *rdiag, int p, int i, int j) {
    if (i < p && j < p)
        return 0.5 * (G[int64_t(i) * p + j] + G[int64_t(j) * p + i]) + (i == j ? rdiag[i] : 0.0);
    return i == j ? 1.0 : 0.0;
}

// Load block (bi, bj) of the working matrix into LDS: from G (first use,
// symmetrised, plus R) or from the PP x PP buffer A.
// (threads t0, t0 + nthr, ... of the workgroup take part)
__device__ void blk_load(double *s, const double *A, int PP, const double *G, const double *rdiag,
                         int p, bool from_g, int bi, int bj, int t0 = threadIdx.x, int nthr = NT) {
    for (int idx = t0; idx < BS * BS; idx += nthr) {
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

// Sweep the 32 x 32 block in sP (pitch BP) over its 32 pivots, in place:
// on return it holds -A^{-1}.  Run by one wave: lane l keeps column l % 32,
// rows 16 (l / 32) .. +15, in registers; cbuf / rbuf (32 doubles each,
// private to the wave) carry pivot column and row j to every lane.  Returns
// false on a non-positive or non-finite pivot; *pmin gets the smallest pivot.
__device__ bool blk_sweep_wave(double *sP, double *cbuf, double *rbuf, double *pmin) {
    const int lane = threadIdx.x & 63, c = lane & 31, h = lane >> 5;
    double a[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) a[e] = sP[(16 * h + e) * BP + c];
    double mp = 1.0e300;
    bool ok = true;
#pragma unroll
    for (int j = 0; j < BS; ++j) {
        if (c == j) {
#pragma unroll
            for (int e = 0; e < 16; ++e) cbuf[16 * h + e] = a[e];
        }
        if (h == (j >> 4)) rbuf[c] = a[j & 15];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const double piv = cbuf[j];
        ok = ok && piv > 0.0 && isfinite(piv);
        mp = fmin(mp, piv);
        const double inv = 1.0 / piv;
        const double rj = rbuf[c] * inv;                 // A_jc / A_jj
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int i = 16 * h + e;
            const double aij = cbuf[i];
            if (i == j) a[e] = c == j ? -inv : rj;
            else a[e] = c == j ? aij * inv : a[e] - aij * rj;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) sP[(16 * h + e) * BP + c] = a[e];
    *pmin = mp;
    return ok;
}

struct PsArgs {
    int p, PP, nbk;
    const double *G, *rdiag, *y, *hvec;
    double *A, *X, *Sinv, *nu, *pivs, *minpiv;
    int *status;
    long long *steps;
};

__global__ void __launch_bounds__(NT) k_ps_sweep(PsArgs a, int k) {
    __shared__ double sP[BS * BP];                // -A_kk^{-1} after the sweep
    __shared__ double sI[BS * BP];                // A_ik (or A_kk)
    __shared__ double sJ[BS * BP];                // A_kj
    __shared__ double sT[BS * BP];
    __shared__ double bufs[2 * BS];
    __shared__ int okflag;
    const int t = threadIdx.x;
    if (k == 0) {
        // a new step: clear the status (the previous step's may be a failure)
        if (a.status[kStInit] != 0) {
            if (blockIdx.x == 0 && t == 0) a.status[kStStep] = HIKF_E_INVALID;
            return;
        }
        if (blockIdx.x == 0) {
            int bad = 0;
            for (int i = t; i < a.p; i += NT) {
                if (!isfinite(a.y[i])) bad = 1;
                a.nu[i] = a.y[i] - a.hvec[i];
            }
            bad = __syncthreads_or(bad);
            if (t == 0) a.status[kStStep] = bad ? HIKF_E_INVALID : HIKF_OK;
            if (bad) return;
        }
    } else if (a.status[kStStep] != HIKF_OK) {
        return;
    }
    const int bi = blockIdx.x / a.nbk, bj = blockIdx.x % a.nbk;
    const double *src = (k & 1) ? a.X : a.A;
    double *dst = (k & 1) ? a.A : a.X;
    const bool first = k == 0;
    // the pivot block first; wave 0 then sweeps it while waves 1-3 load the
    // workgroup's other blocks
    blk_load(sP, src, a.PP, a.G, a.rdiag, a.p, first, k, k);
    __syncthreads();
    if (t < 64) {
        double pmin;
        const bool ok = blk_sweep_wave(sP, bufs, bufs + BS, &pmin);
        if (t == 0) {
            okflag = ok;
            if (bi == k && bj == k) {
                a.pivs[k] = ok ? sqrt(pmin) : pmin;
                if (!ok) {
                    a.status[kStStep] = HIKF_E_NOT_SPD;
                    a.minpiv[0] = pmin;
                }
            }
        }
    } else {
        const int t0 = t - 64, nthr = NT - 64;
        if (bi != k) blk_load(sI, src, a.PP, a.G, a.rdiag, a.p, first, bi, k, t0, nthr);
        if (bj != k) blk_load(sJ, src, a.PP, a.G, a.rdiag, a.p, first, k, bj, t0, nthr);
        if (bi != k && bj != k) blk_load(sT, src, a.PP, a.G, a.rdiag, a.p, first, bi, bj, t0, nthr);
    }
    __syncthreads();
    if (!okflag) return;
    d4 acc;
    if (bi == k && bj == k) {
        acc = tile_read(sP);                                    // -A_kk^{-1}
    } else if (bi == k) {
        acc = tile_mma<false, false>(d4{0, 0, 0, 0}, sP, sJ, -1.0);   // A_kk^{-1} A_kj
    } else if (bj == k) {
        acc = tile_mma<false, false>(d4{0, 0, 0, 0}, sI, sP, -1.0);   // A_ik A_kk^{-1}
    } else {
        // A_ij + A_ik (-A_kk^{-1}) A_kj
        d4 tik = tile_mma<false, false>(d4{0, 0, 0, 0}, sI, sP, 1.0);
        acc = tile_read(sT);
        __syncthreads();
        tile_write(sI, tik);
        __syncthreads();
        acc = tile_mma<false, false>(acc, sI, sJ, 1.0);
    }
    if (k + 1 < a.nbk) {
        __syncthreads();
        tile_write(sT, acc);
        __syncthreads();
        blk_store(sT, dst, a.PP, bi, bj);
        return;
    }
    // last pivot: the matrix is now -S^{-1}
    __syncthreads();
    tile_write(sT, acc);
    __syncthreads();
    for (int idx = t; idx < BS * BS; idx += NT) {
        const int r = idx / BS, c = idx % BS, i = bi * BS + r, j = bj * BS + c;
        if (i < a.p && j < a.p) a.Sinv[int64_t(i) * a.p + j] = -sT[r * BP + c];
    }
    if (bi == k && bj == k && t == 0) {
        double mp = a.pivs[0];
        for (int q = 1; q < a.nbk; ++q) mp = fmin(mp, a.pivs[q]);
        a.minpiv[0] = mp;
        a.steps[0] += 1;
    }
}

// ---------------------------------------------------------------- recursion
// Carry G = H C_prior and h = H x_hat to the next step without touching C:
// C_post = K R = C_prior S^{-1} R gives H C_post = G S^{-1} R, so the next
// prior G is G S^{-1} R + H C_Q, and H x_hat_post = h + G S^{-1} nu.
// k_ps_advance: one workgroup per 32 x 32 block (i, j) of G S^{-1}; it writes
// that block of Gn = G S^{-1} R + G_Q and the block's share of (G S^{-1} nu)_i
// to hpart[j][i].  k_ps_finish then copies Gn to G and adds the shares to h
// in a fixed order (no atomics: the result is deterministic).
__device__ void blk_load_p(double *s, const double *A, int p, int bi, int bj) {
    for (int idx = threadIdx.x; idx < BS * BS; idx += NT) {
        const int r = idx / BS, c = idx % BS, i = bi * BS + r, j = bj * BS + c;
        s[r * BP + c] = (i < p && j < p) ? A[int64_t(i) * p + j] : 0.0;
    }
}

__global__ void __launch_bounds__(NT)
k_ps_advance(int p, int nbk, const double *G, const double *Sinv, const double *rdiag,
             const double *GQ, const double *nu, double *Gn, double *hpart, const int *status) {
    __shared__ double sG[BS * BP];
    __shared__ double sS[BS * BP];
    if (status[kStStep] != HIKF_OK) return;          // failed step: keep G, h
    const int bi = blockIdx.x / nbk, bj = blockIdx.x % nbk, t = threadIdx.x;
    d4 acc = d4{0, 0, 0, 0};
    for (int kb = 0; kb < nbk; ++kb) {
        __syncthreads();
        blk_load_p(sG, G, p, bi, kb);
        blk_load_p(sS, Sinv, p, kb, bj);
        __syncthreads();
        acc = tile_mma<false, false>(acc, sG, sS, 1.0);
    }
    __syncthreads();
    tile_write(sG, acc);                              // (G S^{-1}) block
    __syncthreads();
    for (int idx = t; idx < BS * BS; idx += NT) {
        const int r = idx / BS, c = idx % BS, i = bi * BS + r, j = bj * BS + c;
        if (i < p && j < p)
            Gn[int64_t(i) * p + j] = sG[r * BP + c] * rdiag[j] + GQ[int64_t(i) * p + j];
    }
    if (t < BS && bi * BS + t < p) {
        double d = 0.0;
        for (int c = 0; c < BS && bj * BS + c < p; ++c) d += sG[t * BP + c] * nu[bj * BS + c];
        hpart[int64_t(bj) * p + bi * BS + t] = d;
    }
}

__global__ void k_ps_finish(int p, int nbk, const double *Gn, const double *hpart, double *G,
                            double *h, int *status) {
    if (status[kStStep] != HIKF_OK) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) status[kStCarried] = 1;
    const int64_t n = int64_t(p) * p;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        G[i] = Gn[i];
        if (i < p) {
            double d = 0.0;
            for (int j = 0; j < nbk; ++j) d += hpart[int64_t(j) * p + i];
            h[i] += d;
        }
    }
}

}  // namespace

hipError_t launch_sweep_inverse(const SweepArgs &w, hipStream_t s) {
    PsArgs a;
    a.p = w.p;
    a.PP = w.pp;
    a.nbk = w.pp / BS;
    a.G = w.G;
    a.rdiag = w.rdiag;
    a.y = w.y;
    a.hvec = w.hvec;
    a.A = w.A;
    a.X = w.X;
    a.Sinv = w.Sinv;
    a.nu = w.nu;
    a.pivs = w.pivs;
    a.minpiv = w.minpiv;
    a.status = w.status;
    a.steps = w.steps;
    for (int k = 0; k < a.nbk; ++k)
        hipLaunchKernelGGL(k_ps_sweep, dim3(a.nbk * a.nbk), dim3(NT), 0, s, a, k);
    return hipGetLastError();
}

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
    a.X = reinterpret_cast<double *>(res + lay.xbuf);
    a.Sinv = reinterpret_cast<double *>(res + lay.sinv);
    a.nu = reinterpret_cast<double *>(res + lay.nu);
    a.pivs = reinterpret_cast<double *>(res + lay.pivs);
    a.minpiv = reinterpret_cast<double *>(res + lay.minpiv);
    a.status = reinterpret_cast<int *>(res + lay.status);
    a.steps = reinterpret_cast<long long *>(res + lay.steps);
    for (int k = 0; k < a.nbk; ++k)
        hipLaunchKernelGGL(k_ps_sweep, dim3(a.nbk * a.nbk), dim3(NT), 0, s, a, k);
    return hipGetLastError();
}

}  // namespace hikf

namespace hikf {

hipError_t launch_advance(const Geometry &g, const Layout &lay, char *res, hipStream_t s) {
    const int nbk = g.pp / BS;
    const int *status = reinterpret_cast<const int *>(res + lay.status);
    double *Gn = reinterpret_cast<double *>(res + lay.Gn);
    double *hpart = reinterpret_cast<double *>(res + lay.hpart);
    hipLaunchKernelGGL(k_ps_advance, dim3(nbk * nbk), dim3(NT), 0, s, g.p, nbk,
                       reinterpret_cast<const double *>(res + lay.G),
                       reinterpret_cast<const double *>(res + lay.sinv),
                       reinterpret_cast<const double *>(res + lay.rdiag),
                       reinterpret_cast<const double *>(res + lay.GQ),
                       reinterpret_cast<const double *>(res + lay.nu), Gn, hpart, status);
    const int64_t n = int64_t(g.p) * g.p;
    hipLaunchKernelGGL(k_ps_finish, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, g.p, nbk,
                       Gn, hpart, reinterpret_cast<double *>(res + lay.G),
                       reinterpret_cast<double *>(res + lay.hvec), const_cast<int *>(status));
    return hipGetLastError();
}

}  // namespace hikf

namespace hikf {

// ---------------------------------------------------------------- PSD guard
// The H^2 approximation of a smooth kernel makes G_Q = H C_Q indefinite by
// about its approximation error; the random walk adds G_Q every step, so
// S = (G + G^T)/2 + R loses definiteness after a number of steps that the
// most negative eigenvalue sets.  The guard replaces G_Q by its positive
// semidefinite part (G_Q + |G_Q|) / 2, the projection onto the PSD cone,
// which is never farther from the exact H Q H^T than G_Q is.  |G_Q| =
// G_Q sign(G_Q) comes from the inverse-free Newton-Schulz iteration for the
// matrix sign,  X <- X (3 I - X^2) / 2  from X = G_Q / ||G_Q||_F, on FP64
// MFMA: an eigenvalue of relative size e grows by 1.5x per iteration, so a
// fixed count of iterations settles every eigenvalue above 1.5^-count of
// the largest; smaller ones (far below R) keep a partly converged sign and
// change by less than themselves.
namespace {

// Cout = alpha A B + beta D for p x p row-major matrices (D may be null);
// one 256-thread workgroup per 32 x 32 block, FP64 MFMA
__global__ void __launch_bounds__(NT)
k_pp_gemm(int p, int nbk, const double *A, const double *B, const double *D, double alpha,
          double beta, double *Cout) {
    __shared__ double sA[BS * BP];
    __shared__ double sBb[BS * BP];
    const int bi = blockIdx.x / nbk, bj = blockIdx.x % nbk, t = threadIdx.x;
    d4 acc = d4{0, 0, 0, 0};
    for (int kb = 0; kb < nbk; ++kb) {
        __syncthreads();
        blk_load_p(sA, A, p, bi, kb);
        blk_load_p(sBb, B, p, kb, bj);
        __syncthreads();
        acc = tile_mma<false, false>(acc, sA, sBb, 1.0);
    }
    __syncthreads();
    tile_write(sA, acc);
    __syncthreads();
    for (int idx = t; idx < BS * BS; idx += NT) {
        const int r = idx / BS, c = idx % BS, i = bi * BS + r, j = bj * BS + c;
        if (i < p && j < p) {
            const int64_t o = int64_t(i) * p + j;
            Cout[o] = alpha * sA[r * BP + c] + (D ? beta * D[o] : 0.0);
        }
    }
}

// X = sym(G) / ||sym(G)||_F (X = 0 for G = 0), one workgroup
__global__ void __launch_bounds__(NT) k_pp_scale(int p, const double *G, double *X) {
    __shared__ double red[NT];
    const int t = threadIdx.x;
    const int64_t n = int64_t(p) * p;
    double s = 0.0;
    for (int64_t i = t; i < n; i += NT) {
        const int64_t r = i / p, c = i % p;
        const double v = 0.5 * (G[i] + G[c * p + r]);
        s += v * v;
    }
    red[t] = s;
    __syncthreads();
    for (int k = NT / 2; k > 0; k >>= 1) {
        if (t < k) red[t] += red[t + k];
        __syncthreads();
    }
    const double inv = red[0] > 0.0 ? 1.0 / sqrt(red[0]) : 0.0;
    for (int64_t i = t; i < n; i += NT) {
        const int64_t r = i / p, c = i % p;
        X[i] = inv * 0.5 * (G[i] + G[c * p + r]);
    }
}

// G = (P + P^T) / 2 (the product of the last iteration, symmetrised)
__global__ void k_pp_sym(int p, const double *P, double *G) {
    const int64_t n = int64_t(p) * p;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int64_t r = i / p, c = i % p;
        G[i] = 0.5 * (P[i] + P[c * p + r]);
    }
}

// y = a x (p x p)
__global__ void k_pp_scal(int p, double a, const double *x, double *y) {
    const int64_t n = int64_t(p) * p;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        y[i] = a * x[i];
}

}  // namespace

// In place: GQ <- the PSD part of sym(GQ).  work: three p x p buffers.
hipError_t launch_psd_project(const Geometry &g, double *GQ, double *work, hipStream_t s) {
    const int p = g.p, nbk = g.pp / BS;
    const int64_t pp2 = int64_t(p) * p;
    double *X = work, *Y = work + pp2, *Z = work + 2 * pp2;
    const unsigned eb = unsigned((pp2 + 255) / 256);
    hipLaunchKernelGGL(k_pp_scale, dim3(1), dim3(NT), 0, s, p, GQ, X);
    for (int it = 0; it < kPsdIterations; ++it) {
        // Y = X X;  Z = 1.5 X - 0.5 X Y;  X <- Z
        hipLaunchKernelGGL(k_pp_gemm, dim3(nbk * nbk), dim3(NT), 0, s, p, nbk, X, X,
                           static_cast<const double *>(nullptr), 1.0, 0.0, Y);
        hipLaunchKernelGGL(k_pp_gemm, dim3(nbk * nbk), dim3(NT), 0, s, p, nbk, X, Y, X, -0.5, 1.5, Z);
        double *tmp = X;
        X = Z;
        Z = tmp;
    }
    // GQ <- sym((GQ + GQ X) / 2)
    hipLaunchKernelGGL(k_pp_gemm, dim3(nbk * nbk), dim3(NT), 0, s, p, nbk, GQ, X, GQ, 0.5, 0.5, Y);
    hipLaunchKernelGGL(k_pp_sym, dim3(eb), dim3(256), 0, s, p, Y, GQ);
    return hipGetLastError();
}

// y = a x for p x p matrices (the guard's start G = 2 G_Q+ for P_0 = Q)
hipError_t launch_pp_scal(const Geometry &g, double a, const double *x, double *y, hipStream_t s) {
    const int64_t pp2 = int64_t(g.p) * g.p;
    hipLaunchKernelGGL(k_pp_scal, dim3(unsigned((pp2 + 255) / 256)), dim3(256), 0, s, g.p, a, x, y);
    return hipGetLastError();
}

}  // namespace hikf

// Perturbed-observation ensemble Kalman filter (Sec. 2.3, eqs.
// equation_samplemean, equation_samplecov1, equation_samplegain_enkf) on the
// random-walk model of Sec. 2.1: host side of include/hikf_enkf.h and the
// small kernels of a step.
//
// A step, with X the stored ensemble (m x ld, members in columns 0..N-1),
// E the model-error draws, V the observation perturbations:
//   k_en_gather / k_en_reduce  HX = H (X + E): a workgroup per chunk of a
//                              ray's nonzeros reads those rows of X and E
//                              (16-byte loads over the members); the chunks
//                              of a ray are then summed in a fixed order
//   k_en_innov                 H A = (HX - mean) / sqrt(N - 1) and the
//                              innovations D = y 1^T + V - HX (p x ld)
//   k_en_gemm                  S0 = (H A)(H A)^T
//   launch_sweep_inverse       S = S0 + R, S^{-1} (blocked FP64-MFMA sweep;
//                              its pivots are the Cholesky pivots)
//   k_en_gemm (twice)          Z = S^{-1} D, T = (H A)^T Z   (N x N)
//   k_en_wmat                  W = I + (I - 1 1^T / N) T / sqrt(N - 1)
//   launch_enkf_transform      X <- (X + E) W, mean and variance rows
//                              (enkf_transform.h)
// so that every member gets x^j + K~ (d^j - H x^j) with K~ = A (H A)^T S^{-1}:
// (X + E) W = X_f + A T.  A failed step (S not positive definite, a NaN or
// Inf in y, V or the innovations) skips the transform: the ensemble is
// unchanged.
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "enkf_internal.h"
#include "hikf_enkf.h"
#include "hikf_internal.h"
#include "sweep.h"

namespace hikf {
namespace {

constexpr int kChunk = 256;        // nonzeros of one ray per gather workgroup
constexpr int kGemmTile = 32;

struct EnLayout {
    size_t X, xmean, xvar, rowptr, col, val, rdiag, ch_beg, ray_ch, part, HX, HA, D, S0,
        psA, xbuf, sinv, nu, hzero, pivs, minpiv, status, steps, applied, Z, T, W, bytes;
};

int64_t max_chunks(int64_t nnz, int p) { return nnz / kChunk + p; }

EnLayout en_layout(int64_t m, int p, int ld, int64_t nnz) {
    EnLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    const size_t pp = size_t((p + 31) / 32 * 32), P = size_t(p), LD = size_t(ld);
    const size_t nch = size_t(max_chunks(nnz, p));
    L.X = take(size_t(m) * LD * 8);
    L.xmean = take(size_t(m) * 8);
    L.xvar = take(size_t(m) * 8);
    L.rowptr = take((P + 1) * 8);
    L.col = take(size_t(nnz) * 4);
    L.val = take(size_t(nnz) * 8);
    L.rdiag = take(P * 8);
    L.ch_beg = take((nch + 1) * 8);
    L.ray_ch = take((P + 1) * 4);
    L.part = take(nch * LD * 8);
    L.HX = take(P * LD * 8);
    L.HA = take(P * LD * 8);
    L.D = take(P * LD * 8);
    L.S0 = take(P * P * 8);
    L.psA = take(pp * pp * 8);
    L.xbuf = take(pp * pp * 8);
    L.sinv = take(P * P * 8);
    L.nu = take(P * 8);
    L.hzero = take(P * 8);
    L.pivs = take(pp / 32 * 8);
    L.minpiv = take(8);
    L.status = take(kNumStatus * 4);
    L.steps = take(8);       // successful factorisations (the sweep's counter)
    L.applied = take(8);     // analyses applied (the transform's counter)
    L.Z = take(P * LD * 8);
    L.T = take(LD * LD * 8);
    L.W = take(LD * LD * 8);
    L.bytes = off;
    return L;
}

typedef double dv2 __attribute__((ext_vector_type(2)));

// H, R checks at init: a bad column, a non-finite value or R <= 0 sets
// status[kStInit]
__global__ void k_en_validate(int64_t m, int64_t nnz, int p, const int *col, const double *val,
                              const double *rdiag, int *status) {
    int bad = 0;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nnz;
         i += int64_t(gridDim.x) * blockDim.x)
        if (col[i] < 0 || col[i] >= m || !isfinite(val[i])) bad = 1;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < p;
         i += int64_t(gridDim.x) * blockDim.x)
        if (!(rdiag[i] > 0.0) || !isfinite(rdiag[i])) bad = 1;
    if (bad) status[kStInit] = HIKF_E_INVALID;
}

// dst (rows x dld) <- src (rows x sld) over the first `cols` columns; the
// columns cols..dld-1 of dst are zeroed
__global__ void k_en_copy(int64_t rows, int cols, const double *src, int64_t sld, double *dst,
                          int64_t dld) {
    const int64_t n = rows * dld;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int64_t r = i / dld, c = i % dld;
        dst[i] = c < cols ? src[r * sld + c] : 0.0;
    }
}

// one workgroup per chunk: part[chunk][c] = sum over the chunk's nonzeros
// (ray i, cell j, value h) of h (X[j][c] + E[j][c]) for c < N, 0 beyond.
// Nothing is read through H's columns once init found a bad one.
template <bool HAS_E>
__global__ void __launch_bounds__(256)
k_en_gather(int ld, int n_ens, const int64_t *ch_beg, const int *col, const double *val,
            const double *X, const double *E, double *part, const int *status) {
    if (status[kStInit] != HIKF_OK) return;
    const int64_t b = ch_beg[blockIdx.x], e = ch_beg[blockIdx.x + 1];
    const int c = 2 * threadIdx.x;
    if (c >= ld) return;
    const bool v0 = c < n_ens, v1 = c + 1 < n_ens;
    dv2 acc = dv2{0.0, 0.0};
    int64_t k = b;
    for (; k + 4 <= e; k += 4) {
        dv2 xs[4];
        double hv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t j = col[k + u];
            hv[u] = val[k + u];
            xs[u] = *reinterpret_cast<const dv2 *>(X + j * ld + c);
            if (HAS_E) {
                const dv2 ev = *reinterpret_cast<const dv2 *>(E + j * ld + c);
                xs[u] = dv2{xs[u][0] + (v0 ? ev[0] : 0.0), xs[u][1] + (v1 ? ev[1] : 0.0)};
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            acc[0] += hv[u] * xs[u][0];
            acc[1] += hv[u] * xs[u][1];
        }
    }
    for (; k < e; ++k) {
        const int64_t j = col[k];
        dv2 x = *reinterpret_cast<const dv2 *>(X + j * ld + c);
        if (HAS_E) {
            const dv2 ev = *reinterpret_cast<const dv2 *>(E + j * ld + c);
            x = dv2{x[0] + (v0 ? ev[0] : 0.0), x[1] + (v1 ? ev[1] : 0.0)};
        }
        acc[0] += val[k] * x[0];
        acc[1] += val[k] * x[1];
    }
    acc = dv2{v0 ? acc[0] : 0.0, v1 ? acc[1] : 0.0};
    *reinterpret_cast<dv2 *>(part + int64_t(blockIdx.x) * ld + c) = acc;
}

// HX[i] = sum of ray i's chunk rows, in chunk order
__global__ void k_en_reduce(int ld, const int *ray_ch, const double *part, double *HX,
                            const int *status) {
    if (status[kStInit] != HIKF_OK) return;
    const int i = blockIdx.x;
    const int c0 = ray_ch[i], c1 = ray_ch[i + 1];
    for (int c = threadIdx.x; c < ld; c += blockDim.x) {
        double s = 0.0;
        for (int k = c0; k < c1; ++k) s += part[int64_t(k) * ld + c];
        HX[int64_t(i) * ld + c] = s;
    }
}

// per ray i: HA[i][j] = (HX[i][j] - mean_j HX[i][j]) / sqrt(N - 1) and
// D[i][j] = y[i] + V[i][j] - HX[i][j] for j < N; 0 for N <= j < ld
__global__ void __launch_bounds__(256)
k_en_innov(int ld, int n_ens, const double *HX, const double *y, const double *V, double *HA,
           double *D) {
    __shared__ double red[256];
    const int i = blockIdx.x, t = threadIdx.x;
    const double *hx = HX + int64_t(i) * ld;
    double s = 0.0;
    for (int j = t; j < n_ens; j += 256) s += hx[j];
    red[t] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    const double mean = red[0] / n_ens, sc = 1.0 / sqrt(double(n_ens - 1));
    for (int j = t; j < ld; j += 256) {
        const bool in = j < n_ens;
        HA[int64_t(i) * ld + j] = in ? (hx[j] - mean) * sc : 0.0;
        D[int64_t(i) * ld + j] = in ? y[i] + V[int64_t(i) * n_ens + j] - hx[j] : 0.0;
    }
}

// C (M x N, ldc) = sum_k op(A)(i, k) op(B)(k, j), FP64; op(A)(i, k) =
// A[i lda + k] (TA false) or A[k lda + i] (TA true), likewise for B.  One
// 256-thread workgroup per 32 x 32 tile of C, k in steps of 32 through LDS.
template <bool TA, bool TB>
__global__ void __launch_bounds__(256)
k_en_gemm(int M, int N, int K, const double *A, int lda, const double *B, int ldb, double *C,
          int ldc, const int *status) {
    __shared__ double sA[kGemmTile][kGemmTile + 1];
    __shared__ double sB[kGemmTile][kGemmTile + 1];
    if (status[kStInit] != HIKF_OK) return;
    const int tilesN = (N + kGemmTile - 1) / kGemmTile;
    const int i0 = (blockIdx.x / tilesN) * kGemmTile, j0 = (blockIdx.x % tilesN) * kGemmTile;
    const int t = threadIdx.x, ti = t / 16, tj = t % 16;   // outputs (ti + 16 a, tj + 16 b)
    double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    for (int k0 = 0; k0 < K; k0 += kGemmTile) {
        for (int idx = t; idx < kGemmTile * kGemmTile; idx += 256) {
            const int r = idx / kGemmTile, c = idx % kGemmTile;
            // sA[r][c] = op(A)(i0 + r, k0 + c), sB[r][c] = op(B)(k0 + r, j0 + c)
            const int ia = i0 + r, ka = k0 + c, kb = k0 + r, jb = j0 + c;
            double a = 0.0, b = 0.0;
            if (ia < M && ka < K) a = TA ? A[int64_t(ka) * lda + ia] : A[int64_t(ia) * lda + ka];
            if (kb < K && jb < N) b = TB ? B[int64_t(jb) * ldb + kb] : B[int64_t(kb) * ldb + jb];
            sA[r][c] = a;
            sB[r][c] = b;
        }
        __syncthreads();
#pragma unroll 8
        for (int k = 0; k < kGemmTile; ++k) {
            const double a0 = sA[ti][k], a1 = sA[ti + 16][k];
            const double b0 = sB[k][tj], b1 = sB[k][tj + 16];
            acc[0][0] += a0 * b0;
            acc[0][1] += a0 * b1;
            acc[1][0] += a1 * b0;
            acc[1][1] += a1 * b1;
        }
        __syncthreads();
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            const int i = i0 + ti + 16 * a, j = j0 + tj + 16 * b;
            if (i < M && j < N) C[int64_t(i) * ldc + j] = acc[a][b];
        }
}

// W = I + (T - 1 colmean(T)) / sqrt(N - 1) on the N x N block, 0 elsewhere:
// one workgroup per column j (the column mean summed in a fixed order); a
// non-finite T entry fails the step
__global__ void __launch_bounds__(256) k_en_wmat(int ld, int n_ens, const double *T, double *W,
                                                 int *status) {
    __shared__ double red[256];
    __shared__ int bad;
    const int j = blockIdx.x, t = threadIdx.x;
    if (status[kStStep] != HIKF_OK) return;
    if (t == 0) bad = 0;
    const bool in = j < n_ens;
    double s = 0.0;
    int b = 0;
    if (in)
        for (int i = t; i < n_ens; i += 256) {
            const double v = T[int64_t(i) * ld + j];
            if (!isfinite(v)) b = 1;
            s += v;
        }
    red[t] = s;
    __syncthreads();
    if (b) bad = 1;
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    const double cm = red[0] / n_ens, sc = 1.0 / sqrt(double(n_ens - 1));
    for (int i = t; i < ld; i += 256) {
        double w = 0.0;
        if (in && i < n_ens) w = (i == j ? 1.0 : 0.0) + (T[int64_t(i) * ld + j] - cm) * sc;
        W[int64_t(i) * ld + j] = w;
    }
    if (t == 0 && bad) status[kStStep] = HIKF_E_INVALID;
}

template <typename T>
T *at(char *base, size_t off) { return reinterpret_cast<T *>(base + off); }

}  // namespace

hipError_t launch_enkf_transform(int tile_rows, int64_t m, int n_ens, int ld, double *X,
                                 const double *E, const double *W, double *xmean, double *xvar,
                                 const int *status, long long *applied, hipStream_t s) {
    switch (ld / 16) {
#define HIKF_EN_CASE(N) \
    case N: return enkf_transform_nt<N>(tile_rows, m, n_ens, X, E, W, xmean, xvar, status, applied, s);
        HIKF_EN_CASE(1) HIKF_EN_CASE(2) HIKF_EN_CASE(3) HIKF_EN_CASE(4) HIKF_EN_CASE(5)
        HIKF_EN_CASE(6) HIKF_EN_CASE(8) HIKF_EN_CASE(10) HIKF_EN_CASE(12) HIKF_EN_CASE(16)
        HIKF_EN_CASE(20) HIKF_EN_CASE(24) HIKF_EN_CASE(25) HIKF_EN_CASE(28) HIKF_EN_CASE(32)
#undef HIKF_EN_CASE
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hikf

using namespace hikf;

struct hikf_enkf {
    int64_t m = 0, nnz = 0;
    int p = 0, n = 0, ld = 0, pp = 0, nchunks = 0, device = 0, tile_rows = 0;
    bool timing = false;
    char *res = nullptr;
    EnLayout L{};
    hipStream_t last = nullptr;
    struct Pending { int phase; hipEvent_t a, b; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    double tsum[HIKF_ENKF_NUM_PHASES] = {};
    int64_t tcnt[HIKF_ENKF_NUM_PHASES] = {};
    std::string err;
};

namespace {

hikf_status en_fail(hikf_enkf *f, hikf_status s, const std::string &msg) {
    if (f) f->err = msg;
    return s;
}

hikf_status en_check(const hikf_enkf_problem *pr) {
    if (!pr || pr->m < 1 || pr->p < 1 || pr->n_ens < 2 || pr->nnz < 0) return HIKF_E_INVALID;
    if (!pr->h_rowptr_dev || !pr->r_diag_dev) return HIKF_E_INVALID;
    if (pr->nnz > 0 && (!pr->h_col_dev || !pr->h_val_dev)) return HIKF_E_INVALID;
    if (pr->tile_rows != 0 && pr->tile_rows != 32 && pr->tile_rows != 64 && pr->tile_rows != 128)
        return HIKF_E_INVALID;
    if (pr->tile_rows == 128 && pr->n_ens > 256) return HIKF_E_UNSUPPORTED;
    if (pr->p > kMaxP || pr->n_ens > kEnMaxMembers) return HIKF_E_UNSUPPORTED;
    return HIKF_OK;
}

hipEvent_t en_event(hikf_enkf *f) {
    if (!f->pool.empty()) {
        hipEvent_t e = f->pool.back();
        f->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// harvest finished phase timings (the caller has synchronised)
void en_harvest(hikf_enkf *f) {
    for (auto &pe : f->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, pe.a, pe.b) == hipSuccess) {
            f->tsum[pe.phase] += ms;
            f->tcnt[pe.phase] += 1;
        }
        f->pool.push_back(pe.a);
        f->pool.push_back(pe.b);
    }
    f->pending.clear();
}

}  // namespace

extern "C" {

hikf_status hikf_enkf_plan(const hikf_enkf_problem *pr, hikf_enkf_plan_info *out) {
    if (!out) return HIKF_E_INVALID;
    const hikf_status s = en_check(pr);
    if (s != HIKF_OK) return s;
    const int ld = enkf_ld(pr->n_ens);
    out->ld = ld;
    out->resident_bytes = en_layout(pr->m, pr->p, ld, pr->nnz).bytes;
    out->gather_chunks = 0;
    return HIKF_OK;
}

hikf_status hikf_enkf_init(const hikf_enkf_problem *pr, const double *x0_dev,
                           void *resident_dev, size_t resident_bytes, void *stream,
                           hikf_enkf **out) {
    if (!out) return HIKF_E_INVALID;
    *out = nullptr;
    hikf_status s = en_check(pr);
    if (s != HIKF_OK) return s;
    if (!x0_dev || !resident_dev) return HIKF_E_INVALID;
    const int ld = enkf_ld(pr->n_ens);
    const EnLayout L = en_layout(pr->m, pr->p, ld, pr->nnz);
    if (resident_bytes < L.bytes || (reinterpret_cast<uintptr_t>(resident_dev) & 255))
        return HIKF_E_NOMEM;
    hikf_enkf *f = new (std::nothrow) hikf_enkf;
    if (!f) return HIKF_E_NOMEM;
    f->m = pr->m;
    f->nnz = pr->nnz;
    f->p = pr->p;
    f->n = pr->n_ens;
    f->ld = ld;
    f->pp = (pr->p + 31) / 32 * 32;
    f->timing = pr->timing != 0;
    f->tile_rows = pr->tile_rows;
    f->res = static_cast<char *>(resident_dev);
    f->L = L;
    hipStream_t st = static_cast<hipStream_t>(stream);
    f->last = st;
    auto bail = [&](hikf_status code) {
        delete f;
        return code;
    };
    if (hipGetDevice(&f->device) != hipSuccess) return bail(HIKF_E_DEVICE);

    // the row pointer on the host: check it and cut every ray into chunks of
    // kChunk nonzeros; chunk c covers [beg[c], beg[c + 1]) (a ray's last chunk
    // ends where the next nonempty ray's first chunk begins, at its row end)
    std::vector<int64_t> rp(size_t(f->p) + 1);
    if (hipMemcpyAsync(rp.data(), pr->h_rowptr_dev, rp.size() * 8, hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return bail(HIKF_E_DEVICE);
    if (rp[0] != 0 || rp[size_t(f->p)] != f->nnz) return bail(HIKF_E_INVALID);
    std::vector<int> ray_ch(size_t(f->p) + 1);
    std::vector<int64_t> ch_beg;
    for (int i = 0; i < f->p; ++i) {
        if (rp[i + 1] < rp[i]) return bail(HIKF_E_INVALID);
        ray_ch[i] = int(ch_beg.size());
        for (int64_t b = rp[i]; b < rp[i + 1]; b += kChunk) ch_beg.push_back(b);
    }
    ray_ch[size_t(f->p)] = int(ch_beg.size());
    f->nchunks = int(ch_beg.size());
    ch_beg.push_back(f->nnz);
    if (f->nchunks > max_chunks(f->nnz, f->p)) return bail(HIKF_E_INVALID);

    char *r = f->res;
    hipError_t e = hipSuccess;
    auto cp = [&](size_t off, const void *src, size_t bytes, hipMemcpyKind kind) {
        if (e == hipSuccess && bytes) e = hipMemcpyAsync(r + off, src, bytes, kind, st);
    };
    cp(L.rowptr, pr->h_rowptr_dev, (size_t(f->p) + 1) * 8, hipMemcpyDeviceToDevice);
    cp(L.col, pr->h_col_dev, size_t(f->nnz) * 4, hipMemcpyDeviceToDevice);
    cp(L.val, pr->h_val_dev, size_t(f->nnz) * 8, hipMemcpyDeviceToDevice);
    cp(L.rdiag, pr->r_diag_dev, size_t(f->p) * 8, hipMemcpyDeviceToDevice);
    cp(L.ray_ch, ray_ch.data(), ray_ch.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemsetAsync(r + L.status, 0, kNumStatus * 4, st);
    if (e == hipSuccess) e = hipMemsetAsync(r + L.steps, 0, 8, st);
    if (e == hipSuccess) e = hipMemsetAsync(r + L.applied, 0, 8, st);
    if (e == hipSuccess) e = hipMemsetAsync(r + L.hzero, 0, size_t(f->p) * 8, st);
    if (e == hipSuccess) e = hipMemsetAsync(r + L.minpiv, 0, 8, st);
    cp(L.ch_beg, ch_beg.data(), ch_beg.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        hipLaunchKernelGGL(k_en_validate, dim3(256), dim3(256), 0, st, f->m, f->nnz, f->p,
                           at<const int>(r, L.col), at<const double>(r, L.val),
                           at<const double>(r, L.rdiag), at<int>(r, L.status));
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_en_copy, dim3(2048), dim3(256), 0, st, f->m, f->n, x0_dev,
                           int64_t(f->n), at<double>(r, L.X), int64_t(f->ld));
        e = hipGetLastError();
    }
    // the host vectors above are read by the queued copies: wait for them
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return bail(HIKF_E_DEVICE);
    *out = f;
    return HIKF_OK;
}

hikf_status hikf_enkf_step(hikf_enkf *f, const double *e_dev, const double *y_dev,
                           const double *v_dev, double *mean_out_dev, double *var_out_dev,
                           void *stream) {
    if (!f || !y_dev || !v_dev) return HIKF_E_INVALID;
    hipStream_t st = static_cast<hipStream_t>(stream);
    f->last = st;
    char *r = f->res;
    const EnLayout &L = f->L;
    const int p = f->p, ld = f->ld, n = f->n;
    int *status = at<int>(r, L.status);
    hipEvent_t ev[2 * HIKF_ENKF_NUM_PHASES] = {};
    auto mark = [&](int phase, int which) {
        if (!f->timing) return;
        hipEvent_t &x = ev[2 * phase + which];
        x = en_event(f);
        if (x) hipEventRecord(x, st);
    };

    mark(HIKF_ENKF_PHASE_GATHER, 0);
    if (f->nchunks > 0) {
        if (e_dev)
            hipLaunchKernelGGL(k_en_gather<true>, dim3(f->nchunks), dim3(256), 0, st, ld, n,
                               at<const int64_t>(r, L.ch_beg), at<const int>(r, L.col),
                               at<const double>(r, L.val), at<const double>(r, L.X), e_dev,
                               at<double>(r, L.part), status);
        else
            hipLaunchKernelGGL(k_en_gather<false>, dim3(f->nchunks), dim3(256), 0, st, ld, n,
                               at<const int64_t>(r, L.ch_beg), at<const int>(r, L.col),
                               at<const double>(r, L.val), at<const double>(r, L.X), e_dev,
                               at<double>(r, L.part), status);
    }
    hipLaunchKernelGGL(k_en_reduce, dim3(p), dim3(256), 0, st, ld, at<const int>(r, L.ray_ch),
                       at<const double>(r, L.part), at<double>(r, L.HX), status);
    mark(HIKF_ENKF_PHASE_GATHER, 1);

    mark(HIKF_ENKF_PHASE_NSPACE, 0);
    hipLaunchKernelGGL(k_en_innov, dim3(p), dim3(256), 0, st, ld, n, at<const double>(r, L.HX),
                       y_dev, v_dev, at<double>(r, L.HA), at<double>(r, L.D));
    auto tiles = [](int M, int N) {
        return unsigned(((M + kGemmTile - 1) / kGemmTile) * ((N + kGemmTile - 1) / kGemmTile));
    };
    // S0 = HA HA^T
    hipLaunchKernelGGL((k_en_gemm<false, true>), dim3(tiles(p, p)), dim3(256), 0, st, p, p, ld,
                       at<const double>(r, L.HA), ld, at<const double>(r, L.HA), ld,
                       at<double>(r, L.S0), p, status);
    SweepArgs sw;
    sw.p = p;
    sw.pp = f->pp;
    sw.G = at<const double>(r, L.S0);
    sw.rdiag = at<const double>(r, L.rdiag);
    sw.y = y_dev;
    sw.hvec = at<const double>(r, L.hzero);
    sw.A = at<double>(r, L.psA);
    sw.X = at<double>(r, L.xbuf);
    sw.Sinv = at<double>(r, L.sinv);
    sw.nu = at<double>(r, L.nu);
    sw.pivs = at<double>(r, L.pivs);
    sw.minpiv = at<double>(r, L.minpiv);
    sw.status = status;
    sw.steps = at<long long>(r, L.steps);
    hipError_t e = launch_sweep_inverse(sw, st);
    // Z = S^{-1} D, T = HA^T Z
    hipLaunchKernelGGL((k_en_gemm<false, false>), dim3(tiles(p, ld)), dim3(256), 0, st, p, ld, p,
                       at<const double>(r, L.sinv), p, at<const double>(r, L.D), ld,
                       at<double>(r, L.Z), ld, status);
    hipLaunchKernelGGL((k_en_gemm<true, false>), dim3(tiles(ld, ld)), dim3(256), 0, st, ld, ld, p,
                       at<const double>(r, L.HA), ld, at<const double>(r, L.Z), ld,
                       at<double>(r, L.T), ld, status);
    hipLaunchKernelGGL(k_en_wmat, dim3(ld), dim3(256), 0, st, ld, n,
                       at<const double>(r, L.T), at<double>(r, L.W), status);
    mark(HIKF_ENKF_PHASE_NSPACE, 1);

    mark(HIKF_ENKF_PHASE_TRANSFORM, 0);
    if (e == hipSuccess)
        e = launch_enkf_transform(f->tile_rows, f->m, n, ld, at<double>(r, L.X), e_dev,
                                  at<const double>(r, L.W),
                                  at<double>(r, L.xmean), at<double>(r, L.xvar), status,
                                  at<long long>(r, L.applied), st);
    mark(HIKF_ENKF_PHASE_TRANSFORM, 1);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess && mean_out_dev)
        e = hipMemcpyAsync(mean_out_dev, r + L.xmean, size_t(f->m) * 8, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && var_out_dev)
        e = hipMemcpyAsync(var_out_dev, r + L.xvar, size_t(f->m) * 8, hipMemcpyDeviceToDevice, st);
    if (f->timing)
        for (int ph = 0; ph < HIKF_ENKF_NUM_PHASES; ++ph)
            if (ev[2 * ph] && ev[2 * ph + 1])
                f->pending.push_back({ph, ev[2 * ph], ev[2 * ph + 1]});
    if (e != hipSuccess) return en_fail(f, HIKF_E_DEVICE, hipGetErrorString(e));
    return HIKF_OK;
}

hikf_status hikf_enkf_query(hikf_enkf *f, hikf_enkf_stats *out) {
    if (!f || !out) return HIKF_E_INVALID;
    hipError_t e = hipStreamSynchronize(f->last);
    int st[kNumStatus] = {};
    long long steps = 0;
    double minpiv = 0.0;
    if (e == hipSuccess) e = hipMemcpy(st, f->res + f->L.status, sizeof(st), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&steps, f->res + f->L.applied, 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&minpiv, f->res + f->L.minpiv, 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return en_fail(f, HIKF_E_DEVICE, hipGetErrorString(e));
    en_harvest(f);
    std::memset(out, 0, sizeof(*out));
    out->steps_applied = steps;
    out->last_status = st[kStStep];
    out->init_status = st[kStInit];
    out->min_pivot = minpiv;
    for (int ph = 0; ph < HIKF_ENKF_NUM_PHASES; ++ph) {
        out->time_ms[ph] = f->tsum[ph];
        out->time_count[ph] = f->tcnt[ph];
    }
    return HIKF_OK;
}

hikf_status hikf_enkf_export(hikf_enkf *f, double *x_dev, void *stream) {
    if (!f || !x_dev) return HIKF_E_INVALID;
    hipStream_t st = static_cast<hipStream_t>(stream);
    f->last = st;
    hipLaunchKernelGGL(k_en_copy, dim3(2048), dim3(256), 0, st, f->m, f->n,
                       at<const double>(f->res, f->L.X), int64_t(f->ld), x_dev, int64_t(f->n));
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? HIKF_OK : en_fail(f, HIKF_E_DEVICE, hipGetErrorString(e));
}

hikf_status hikf_enkf_import(hikf_enkf *f, const double *x_dev, void *stream) {
    if (!f || !x_dev) return HIKF_E_INVALID;
    hipStream_t st = static_cast<hipStream_t>(stream);
    f->last = st;
    hipLaunchKernelGGL(k_en_copy, dim3(2048), dim3(256), 0, st, f->m, f->n, x_dev, int64_t(f->n),
                       at<double>(f->res, f->L.X), int64_t(f->ld));
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? HIKF_OK : en_fail(f, HIKF_E_DEVICE, hipGetErrorString(e));
}

void hikf_enkf_destroy(hikf_enkf *f) {
    if (!f) return;
    hipStreamSynchronize(f->last);
    for (auto &pe : f->pending) {
        hipEventDestroy(pe.a);
        hipEventDestroy(pe.b);
    }
    for (hipEvent_t ev : f->pool) hipEventDestroy(ev);
    delete f;
}

const char *hikf_enkf_last_error(const hikf_enkf *f) { return f ? f->err.c_str() : ""; }

}  // extern "C"

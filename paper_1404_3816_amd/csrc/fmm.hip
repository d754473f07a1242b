// H^2 / black-box FMM product C_Q = Q H^T on a uniform grid (Sec. 3.2).
//
// Sec. 3.2 writes Q H^T = [Q h^(1) ... Q h^(p)], each column a kernel sum
// (Q h)_i = sum_j K(x_i, x_j) h_j, and evaluates it with the fast multipole
// method whose far field is represented by Chebyshev interpolation (the
// black-box FMM of Fong & Darve 2009 that the paper cites).  All p right-hand
// sides travel together through every pass.
//
// Tree: the N^dim cell-centred grid is split into leaves of 8x8 (2-D) or
// 4x4x4 (3-D) cells (64 points); level l has 2^l boxes per axis.  Box arrays
// are [box][node k][column] with the p columns contiguous; node index
// k = kx + nc*ky (+ nc^2*kz), box index b = bx + nb*by (+ nb^2*bz).
//
// Passes: P2M (leaf anterpolation), M2M (upward, levels D-1..2), M2L
// (interaction lists, levels 2..D), L2L (downward), and the fused L2P + P2P
// (leaf interpolation plus the near-field sum with kernel entries generated
// on the fly).  Operators are built on the device in FP64 and stored in the
// pass precision T (float or double).
#include <algorithm>
#include <cmath>
#include <vector>

#include "hikf_internal.h"

namespace hikf {
namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ double cheb_node(int nc, int k) {
    return cos((2 * k + 1) * M_PI / (2.0 * nc));
}

// S_nc(xi, x) = 1/nc + (2/nc) sum_{l=1}^{nc-1} T_l(xi) T_l(x)
__device__ double cheb_S(int nc, double xi, double x) {
    double s = 0.0;
    double a0 = 1.0, a1 = xi, b0 = 1.0, b1 = x;
    for (int l = 1; l < nc; ++l) {
        s += a1 * b1;
        double a2 = 2.0 * xi * a1 - a0;
        double b2 = 2.0 * x * b1 - b0;
        a0 = a1; a1 = a2; b0 = b1; b1 = b2;
    }
    return (1.0 + 2.0 * s) / nc;
}

__device__ __forceinline__ void node_idx(int k, int nc, int *kk) {
    kk[0] = k % nc;
    kk[1] = (k / nc) % nc;
    kk[2] = k / (nc * nc);
}

__device__ __forceinline__ void leaf_local(int j, int dim, int *l) {
    if (dim == 2) { l[0] = j & 7; l[1] = j >> 3; l[2] = 0; }
    else          { l[0] = j & 3; l[1] = (j >> 2) & 3; l[2] = j >> 4; }
}

__device__ __forceinline__ void box_coords(int64_t b, int nb, int dim, int *c) {
    c[0] = int(b % nb);
    c[1] = int((b / nb) % nb);
    c[2] = dim == 3 ? int(b / (int64_t(nb) * nb)) : 0;
}

__device__ __forceinline__ int64_t box_index(const int *c, int nb, int dim) {
    int64_t b = c[0] + int64_t(nb) * c[1];
    if (dim == 3) b += int64_t(nb) * nb * c[2];
    return b;
}

// grid-order index of local point j of leaf with coordinates bc
__device__ __forceinline__ int64_t leaf_point(const int *bc, int j, int dim, int n, int ls) {
    int l[3];
    leaf_local(j, dim, l);
    int64_t g = int64_t(bc[0]) * ls + l[0];
    g += int64_t(n) * (int64_t(bc[1]) * ls + l[1]);
    if (dim == 3) g += int64_t(n) * n * (int64_t(bc[2]) * ls + l[2]);
    return g;
}

// grid-order index of local point j of leaf bc among the N^dim real cells,
// or -1 for a padding cell of the tree (grids that are not leaf * 2^D)
__device__ __forceinline__ int64_t leaf_point_real(const int *bc, int j, int dim, int n, int ls) {
    int l[3];
    leaf_local(j, dim, l);
    const int x = bc[0] * ls + l[0], y = bc[1] * ls + l[1], z = dim == 3 ? bc[2] * ls + l[2] : 0;
    if (x >= n || y >= n || z >= n) return -1;
    return x + int64_t(n) * (y + int64_t(n) * z);
}

// ---------------------------------------------------------------- operators
template <typename T>
__global__ void k_ops_sleaf(int dim, int nc, int ls, int r, T *out) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= r * kLeafPts) return;
    int k = idx / kLeafPts, j = idx % kLeafPts;
    int kk[3], l[3];
    node_idx(k, nc, kk);
    leaf_local(j, dim, l);
    double half = 0.5 * ls, v = 1.0;
    for (int ax = 0; ax < dim; ++ax)
        v *= cheb_S(nc, cheb_node(nc, kk[ax]), (l[ax] + 0.5 - half) / half);
    out[idx] = (T)v;
}

template <typename T>
__global__ void k_ops_schild(int dim, int nc, int r, T *out) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    int nch = 1 << dim;
    if (idx >= nch * r * r) return;
    int ch = idx / (r * r), rem = idx % (r * r);
    int k = rem / r, kq = rem % r;
    int kk[3], kq3[3];
    node_idx(k, nc, kk);
    node_idx(kq, nc, kq3);
    double v = 1.0;
    for (int ax = 0; ax < dim; ++ax) {
        double shift = ((ch >> ax) & 1) ? 0.5 : -0.5;
        v *= cheb_S(nc, cheb_node(nc, kk[ax]), shift + 0.5 * cheb_node(nc, kq3[ax]));
    }
    out[idx] = (T)v;
}

// T_{l,o}[k][k'] = K(s_l * |o + (xi_k' - xi_k)/2|), o in [-3,3]^dim, slot
// oi = (ox+3) + 7 (oy+3) (+ 49 (oz+3)); slots with max|o| < 2 are zero.
template <typename T>
__global__ void k_ops_m2l(int dim, int nc, int r, int lev0, int nlev, double root, KernelParams kp,
                          T *out) {
    int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int noff = dim == 2 ? 49 : 343;
    int64_t per_lev = int64_t(noff) * r * r;
    if (idx >= per_lev * nlev) return;
    int lev = lev0 + int(idx / per_lev);
    int64_t rem = idx % per_lev;
    int oi = int(rem / (r * r));
    int rr = int(rem % (r * r));
    int k = rr / r, kq = rr % r;
    int o[3] = {oi % 7 - 3, (oi / 7) % 7 - 3, oi / 49 - 3};
    int omax = 0;
    for (int ax = 0; ax < dim; ++ax) omax = max(omax, abs(o[ax]));
    if (omax < 2) { out[idx] = (T)0; return; }
    int kk[3], kq3[3];
    node_idx(k, nc, kk);
    node_idx(kq, nc, kq3);
    double s = root / double(int64_t(1) << lev), r2 = 0.0;      // box side
    for (int ax = 0; ax < dim; ++ax) {
        double d = s * (o[ax] + 0.5 * (cheb_node(nc, kq3[ax]) - cheb_node(nc, kk[ax])));
        r2 += d * d;
    }
    out[idx] = (T)kernel_from_r2<double>(r2, kp);
}

// Near-field kernel blocks: on a uniform grid the 64 x 64 block between a
// target leaf b and a source leaf b + o depends on o only.  For the 3^dim
// offsets o in [-1, 1]^dim (slot (ox+1) + 3 (oy+1) (+ 9 (oz+1))):
// out[slot][i][j] = K(h |o ls + l_j - l_i|).
template <typename T>
__global__ void k_ops_near(int dim, int ls, KernelParams kp, double h, T *out) {
    const int nslot = dim == 2 ? 9 : 27;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nslot * kLeafPts * kLeafPts) return;
    const int sl = idx / (kLeafPts * kLeafPts), i = (idx / kLeafPts) % kLeafPts, j = idx % kLeafPts;
    const int o[3] = {sl % 3 - 1, (sl / 3) % 3 - 1, sl / 9 - 1};
    int li[3], lj[3];
    leaf_local(i, dim, li);
    leaf_local(j, dim, lj);
    int dsq = 0;
    for (int q = 0; q < dim; ++q) {
        const int d = o[q] * ls + lj[q] - li[q];
        dsq += d * d;
    }
    out[idx] = kernel_from_r2<T>((T)dsq * (T)(h * h), kp);
}

// ---------------------------------------------------------------- W = H^T
template <typename T>
__global__ void k_scatter_w(int64_t nnz, int p, int64_t m, int dim, int n, int npad,
                            const int64_t *rowptr, const int32_t *col, const double *val, T *W) {
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
    // W is laid out over the tree's Npad^dim cells
    const int64_t x = c % n, y = (c / n) % n, z = dim == 3 ? c / (int64_t(n) * n) : 0;
    W[(x + int64_t(npad) * (y + int64_t(npad) * z)) * p + lo] = (T)val[e];
}

// ---------------------------------------------------------------- sparse W
// W = H^T has nnz(H) nonzeros: a ray crosses O(N) of the m cells.  In the
// sparse mode the nonzeros are bucketed by the leaf of their cell (a counting
// sort), and each bucket is then put in nonzero order, so that every sum
// over a bucket runs in the same order whatever order the atomic placement
// took.  A bucket entry is (ray * 64 + point of the leaf, value); nonzero
// order is ray-major, so the entries of one ray within a leaf are adjacent.

// ray of nonzero e, or -1 if e lies in no row of the CSR arrays or its cell
// is out of range; *leaf and *pt receive the cell's leaf and point index
__device__ __forceinline__ int sparse_entry(int64_t e, int p, int64_t m, int dim, int n, int ls,
                                            int depth, const int64_t *rowptr, const int32_t *col,
                                            int64_t *leaf, int *pt) {
    int lo = 0, hi = p - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (rowptr[mid] <= e) lo = mid; else hi = mid - 1;
    }
    if (rowptr[lo] > e || rowptr[lo + 1] <= e) return -1;
    const int64_t c = col[e];
    if (c < 0 || c >= m) return -1;
    const int64_t x = c % n, y = (c / n) % n, z = dim == 3 ? c / (int64_t(n) * n) : 0;
    const int64_t nb = int64_t(1) << depth;
    *leaf = x / ls + nb * (y / ls + nb * (z / ls));
    *pt = int(x % ls + ls * (y % ls) + ls * ls * (z % ls));
    return lo;
}

__global__ void k_sp_count(int64_t nnz, int p, int64_t m, int dim, int n, int ls, int depth,
                           const int64_t *rowptr, const int32_t *col, int *cnt) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    int64_t leaf;
    int pt;
    if (sparse_entry(e, p, m, dim, n, ls, depth, rowptr, col, &leaf, &pt) >= 0)
        atomicAdd(cnt + leaf, 1);
}

// exclusive prefix sum of the bucket sizes (one workgroup of 1024 threads):
// off[0..nl] = offsets, cnt[0..nl) = the same offsets as placement cursors
__global__ void __launch_bounds__(1024) k_sp_scan(int64_t nl, int *cnt, int *off) {
    __shared__ int sv[1024];
    __shared__ int carry;
    const int t = threadIdx.x;
    if (t == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nl; base += 1024) {
        const int v = base + t < nl ? cnt[base + t] : 0;
        sv[t] = v;
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {
            const int u = t >= d ? sv[t - d] : 0;
            __syncthreads();
            sv[t] += u;
            __syncthreads();
        }
        const int excl = carry + sv[t] - v;
        if (base + t < nl) { off[base + t] = excl; cnt[base + t] = excl; }
        __syncthreads();
        if (t == 1023) carry += sv[1023];
        __syncthreads();
    }
    if (t == 0) off[nl] = carry;
}

__global__ void k_sp_fill(int64_t nnz, int p, int64_t m, int dim, int n, int ls, int depth,
                          const int64_t *rowptr, const int32_t *col, int *cur, int *tmp) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    int64_t leaf;
    int pt;
    if (sparse_entry(e, p, m, dim, n, ls, depth, rowptr, col, &leaf, &pt) >= 0)
        tmp[atomicAdd(cur + leaf, 1)] = int(e);
}

// one workgroup per leaf: entry of rank k (by nonzero index) to slot k
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_sp_order(int p, int64_t m, int dim, int n, int ls, int depth, const int64_t *rowptr,
           const int32_t *col, const double *val, const int *off, const int *tmp, int *key, T *bv) {
    const int64_t L = blockIdx.x;
    const int o0 = off[L], cnt = off[L + 1] - o0;
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
        const int e = tmp[o0 + i];
        int rank = 0;
        for (int j = 0; j < cnt; ++j) rank += tmp[o0 + j] < e;
        int64_t leaf;
        int pt;
        const int ray = sparse_entry(e, p, m, dim, n, ls, depth, rowptr, col, &leaf, &pt);
        key[o0 + rank] = ray * kLeafPts + pt;
        bv[o0 + rank] = (T)val[e];
    }
}

// P2M from the buckets: one workgroup per leaf; M_B[k][a] sums the entries
// of ray a (one run of the bucket) times S_leaf[k][point].  Buckets of up to
// kCap entries are staged in LDS first.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_p2m_sparse(int r, int p, const int *off, const int *key, const T *bv, const T *Sleaf, T *Mleaf) {
    constexpr int kCap = 1024;
    __shared__ T sS[kMaxR * kLeafPts];
    __shared__ int rs[kMaxP], re[kMaxP];
    __shared__ int sk[kCap];
    __shared__ T sv[kCap];
    const int64_t B = blockIdx.x;
    const int o0 = off[B], cnt = off[B + 1] - o0;
    const bool staged = cnt <= kCap;
    for (int a = threadIdx.x; a < p; a += blockDim.x) { rs[a] = 0; re[a] = 0; }
    for (int idx = threadIdx.x; idx < r * kLeafPts; idx += blockDim.x) sS[idx] = Sleaf[idx];
    if (staged)
        for (int i = threadIdx.x; i < cnt; i += blockDim.x) { sk[i] = key[o0 + i]; sv[i] = bv[o0 + i]; }
    __syncthreads();
    // the entries from LDS (staged) or from memory; two instances, so that
    // each keeps its pointers' address space (a pointer chosen between LDS
    // and global memory at run time would make every access a flat access)
    auto sum_runs = [&](const int *ek, const T *ev) __attribute__((always_inline)) {
        for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
            const int a = ek[i] / kLeafPts;
            if (i == 0 || ek[i - 1] / kLeafPts != a) rs[a] = i;
            if (i == cnt - 1 || ek[i + 1] / kLeafPts != a) re[a] = i + 1;
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < r * p; idx += blockDim.x) {
            const int k = idx / p, a = idx % p;
            T acc = (T)0;
            for (int i = rs[a]; i < re[a]; ++i) acc += sS[k * kLeafPts + ek[i] % kLeafPts] * ev[i];
            Mleaf[(B * r + k) * p + a] = acc;
        }
    };
    if (staged)
        sum_runs(sk, sv);
    else
        sum_runs(key + o0, bv + o0);
}

// ---------------------------------------------------------------- P2M
// The W panel and the interpolation operator, which every output of the
// workgroup reads, are staged in LDS (W with 16-byte loads: rows of PT
// values are contiguous and 16-byte aligned, p and PT being multiples of 16).
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_p2m(int dim, int n, int ls, int depth, int r, int p, int PT, const T *W,
      const T *Sleaf, T *Mleaf) {
    constexpr int VW = 16 / sizeof(T);
    typedef T tv __attribute__((ext_vector_type(VW)));
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sW = reinterpret_cast<T *>(smem_raw);           // [64][PT]
    T *sS = sW + kLeafPts * PT;                        // [r][64]
    const int64_t B = blockIdx.x;
    const int c0 = blockIdx.y * PT;
    const int ncols = min(PT, p - c0);
    const int nb = 1 << depth;
    int bc[3];
    box_coords(B, nb, dim, bc);
    const int chunks = PT / VW;
    for (int idx = threadIdx.x; idx < kLeafPts * chunks; idx += blockDim.x) {
        const int j = idx / chunks, ch = idx % chunks;
        tv v;
        if (VW * ch < ncols) {
            v = *reinterpret_cast<const tv *>(W + leaf_point(bc, j, dim, n, ls) * p + c0 + VW * ch);
        } else {
#pragma unroll
            for (int e = 0; e < VW; ++e) v[e] = (T)0;
        }
        *reinterpret_cast<tv *>(sW + j * PT + VW * ch) = v;
    }
    for (int idx = threadIdx.x; idx < r * kLeafPts; idx += blockDim.x) sS[idx] = Sleaf[idx];
    __syncthreads();
    for (int idx = threadIdx.x; idx < r * PT; idx += blockDim.x) {
        const int k = idx / PT, c = idx % PT;
        if (c >= ncols) continue;
        T acc = (T)0;
        const T *srow = sS + k * kLeafPts;
#pragma unroll 16
        for (int j = 0; j < kLeafPts; ++j) acc += srow[j] * sW[j * PT + c];
        Mleaf[(B * r + k) * p + c0 + c] = acc;
    }
}

// ---------------------------------------------------------------- M2L
// Interaction list of B at level l: boxes A = B + o with max|o| >= 2 whose
// parent is adjacent to (or equal to) B's parent.
__device__ __forceinline__ bool il_member(const int *b, const int *o, int nb, int dim) {
    int omax = 0;
    for (int ax = 0; ax < dim; ++ax) {
        int a = b[ax] + o[ax];
        if (a < 0 || a >= nb) return false;
        int lo = (b[ax] & 1) ? -3 : -2, hi = (b[ax] & 1) ? 2 : 3;
        if (o[ax] < lo || o[ax] > hi) return false;
        omax = max(omax, abs(o[ax]));
    }
    return omax >= 2;
}

// ---------------------------------------------------------------- MFMA forms
// v_mfma_{f32,f64}_16x16x4: D += A B with lane l supplying A[l%16][l/16] and
// B[l/16][l%16]; lane l holds D[row(l/16, r)][l%16] for r = 0..3, where the
// FP32 variant returns rows 4 (l/16) + r and the FP64 variant rows l/16 + 4 r.
template <typename T> struct Mma;
template <> struct Mma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int q, int r) { return 4 * q + r; }
    static constexpr int pad = 16;          // LDS pitch padding of a B operand tile
};
template <> struct Mma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int q, int r) { return q + 4 * r; }
    static constexpr int pad = 8;
};

// ---------------------------------------------------------------- L2P + P2P (MFMA)
// One workgroup per (target leaf B, PT-column tile); wave w owns target rows
// [16 w, 16 w + 16) of the leaf and all PT columns.  For every source leaf A
// within `rad` boxes the 64 x 64 kernel block K(x_i - x_j) is generated in
// LDS from the integer cell offsets, W_A (64 x PT) is staged next to it, and
// the product accumulates on MFMA; the far field then adds
// S_leaf^T (64 x r) L_B (r x PT) the same way.
template <typename T, int PT>
__global__ void __launch_bounds__(kBlock)
k_l2p_p2p_mma(int dim, int n, int npad, int ls, int depth, int r, int rpad, int p, int rad, int far,
              KernelParams kp, T h2, const T *W, const T *Sleaf, const T *Lleaf, const T *Knear,
              T *CQ) {
    typedef typename Mma<T>::v4 v4;
    constexpr int NTI = PT / 16;
    constexpr int WP = PT + Mma<T>::pad;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int KP = max(kLeafPts, rpad) + 4;
    T *sK = reinterpret_cast<T *>(smem_raw);           // [64][KP]
    T *sW = sK + kLeafPts * KP;                        // [max(64, rpad)][WP]
    const int64_t B = blockIdx.x;
    const int c0 = blockIdx.y * PT;
    const int ncols = min(PT, p - c0);
    const int nb = 1 << depth;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, q = lane >> 4;
    int b[3];
    box_coords(B, nb, dim, b);
    v4 acc[NTI];
#pragma unroll
    for (int t = 0; t < NTI; ++t) acc[t] = v4{0, 0, 0, 0};
    constexpr int VW = 16 / sizeof(T), CH = PT / VW, KC = kLeafPts / VW;
    typedef T tv __attribute__((ext_vector_type(VW)));
    if (Knear) {
        // Neighbour leaves only (3^dim offsets, kernel blocks from the table),
        // software-pipelined: the next source's W rows and kernel block are
        // loaded into registers while the MFMAs of the current one run.
        constexpr int WPT = (kLeafPts * CH + kBlock - 1) / kBlock;
        constexpr int KPT = (kLeafPts * KC + kBlock - 1) / kBlock;
        const int nsl = dim == 2 ? 9 : 27;
        auto next_src = [&](int sl) {
            for (++sl; sl < nsl; ++sl) {
                const int a0 = b[0] + sl % 3 - 1, a1 = b[1] + (sl / 3) % 3 - 1, a2 = b[2] + sl / 9 - 1;
                if (a0 >= 0 && a0 < nb && a1 >= 0 && a1 < nb && (dim == 2 || (a2 >= 0 && a2 < nb))) break;
            }
            return sl;
        };
        tv wreg[WPT], kreg[KPT];
#define HIKF_P2P_FETCH(SL)                                                                        \
        do {                                                                                      \
            const int fs = (SL);                                                                  \
            const int fa[3] = {b[0] + fs % 3 - 1, b[1] + (fs / 3) % 3 - 1,                        \
                               dim == 3 ? b[2] + fs / 9 - 1 : 0};                                 \
            _Pragma("unroll") for (int u = 0; u < WPT; ++u) {                                     \
                const int idx = tid + kBlock * u, j = idx / CH, ch = idx % CH;                    \
                if (VW * ch < ncols) {                                                            \
                    wreg[u] = *reinterpret_cast<const tv *>(W + leaf_point(fa, j, dim, npad, ls) * p \
                                                             + c0 + VW * ch);                     \
                } else {                                                                          \
                    _Pragma("unroll") for (int e = 0; e < VW; ++e) wreg[u][e] = (T)0;             \
                }                                                                                 \
            }                                                                                     \
            const T *kt = Knear + int64_t(fs) * kLeafPts * kLeafPts;                              \
            _Pragma("unroll") for (int u = 0; u < KPT; ++u) {                                     \
                const int idx = tid + kBlock * u, i = idx / KC, ch = idx % KC;                    \
                kreg[u] = *reinterpret_cast<const tv *>(kt + i * kLeafPts + VW * ch);             \
            }                                                                                     \
        } while (0)
        int sl = next_src(-1);
        HIKF_P2P_FETCH(sl);                              // the leaf itself always exists
        while (sl < nsl) {
            __syncthreads();                             // LDS free (previous MFMAs done)
#pragma unroll
            for (int u = 0; u < WPT; ++u) {
                const int idx = tid + kBlock * u, j = idx / CH, ch = idx % CH;
                *reinterpret_cast<tv *>(sW + j * WP + VW * ch) = wreg[u];
            }
#pragma unroll
            for (int u = 0; u < KPT; ++u) {
                const int idx = tid + kBlock * u, i = idx / KC, ch = idx % KC;
                *reinterpret_cast<tv *>(sK + i * KP + VW * ch) = kreg[u];
            }
            __syncthreads();
            const int sn = next_src(sl);
            if (sn < nsl) HIKF_P2P_FETCH(sn);            // in flight during the MFMAs
            const T *arow = sK + (16 * wave + lr) * KP + q;
            const T *bcol = sW + q * WP + lr;
#pragma unroll 4
            for (int k0 = 0; k0 < kLeafPts; k0 += 4) {
                const T av = arow[k0];
#pragma unroll
                for (int t = 0; t < NTI; ++t) acc[t] = Mma<T>::op(av, bcol[k0 * WP + 16 * t], acc[t]);
            }
            sl = sn;
        }
#undef HIKF_P2P_FETCH
    }
    const int zlo = dim == 3 ? max(0, b[2] - rad) : 0;
    const int zhi = dim == 3 ? min(nb - 1, b[2] + rad) : 0;
    if (!Knear)
    for (int az = zlo; az <= zhi; ++az)
    for (int ay = max(0, b[1] - rad); ay <= min(nb - 1, b[1] + rad); ++ay)
    for (int ax = max(0, b[0] - rad); ax <= min(nb - 1, b[0] + rad); ++ax) {
        int a[3] = {ax, ay, az};
        __syncthreads();
        // W_A: 64 rows of PT values as 16-byte pieces
        for (int idx = tid; idx < kLeafPts * CH; idx += kBlock) {
            const int j = idx / CH, ch = idx % CH;
            tv v;
            if (VW * ch < ncols) {
                v = *reinterpret_cast<const tv *>(W + leaf_point(a, j, dim, npad, ls) * p + c0 + VW * ch);
            } else {
#pragma unroll
                for (int e = 0; e < VW; ++e) v[e] = (T)0;
            }
            *reinterpret_cast<tv *>(sW + j * WP + VW * ch) = v;
        }
        {
            for (int idx = tid; idx < kLeafPts * kLeafPts; idx += kBlock) {
                const int i = idx / kLeafPts, j = idx % kLeafPts;
                int li[3], lj[3];
                leaf_local(i, dim, li);
                leaf_local(j, dim, lj);
                int dsq = 0;
                for (int qq = 0; qq < dim; ++qq) {
                    const int d = (a[qq] - b[qq]) * ls + lj[qq] - li[qq];
                    dsq += d * d;
                }
                sK[i * KP + j] = kernel_from_r2<T>((T)dsq * h2, kp);
            }
        }
        __syncthreads();
        const T *arow = sK + (16 * wave + lr) * KP + q;
        const T *bcol = sW + q * WP + lr;
#pragma unroll 4
        for (int k0 = 0; k0 < kLeafPts; k0 += 4) {
            const T av = arow[k0];
#pragma unroll
            for (int t = 0; t < NTI; ++t) acc[t] = Mma<T>::op(av, bcol[k0 * WP + 16 * t], acc[t]);
        }
    }
    if (far) {
        __syncthreads();
        for (int idx = tid; idx < kLeafPts * rpad; idx += kBlock) {
            const int i = idx / rpad, k = idx % rpad;
            sK[i * KP + k] = k < r ? Sleaf[k * kLeafPts + i] : (T)0;
        }
        for (int idx = tid; idx < rpad * PT; idx += kBlock) {
            const int k = idx / PT, c = idx % PT;
            sW[k * WP + c] = (k < r && c < ncols) ? Lleaf[(B * r + k) * p + c0 + c] : (T)0;
        }
        __syncthreads();
        const T *arow = sK + (16 * wave + lr) * KP + q;
        const T *bcol = sW + q * WP + lr;
        for (int k0 = 0; k0 < rpad; k0 += 4) {
            const T av = arow[k0];
#pragma unroll
            for (int t = 0; t < NTI; ++t) acc[t] = Mma<T>::op(av, bcol[k0 * WP + 16 * t], acc[t]);
        }
    }
#pragma unroll
    for (int t = 0; t < NTI; ++t) {
        const int c = 16 * t + lr;
        if (c >= ncols) continue;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int i = 16 * wave + Mma<T>::row(q, rr);
            const int64_t g = leaf_point_real(b, i, dim, n, ls);
            if (g >= 0) CQ[g * p + c0 + c] = acc[t][rr];
        }
    }
}

// value of lane src (uniform) of x, through the scalar unit
__device__ __forceinline__ float lane_value(float x, int src) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), src));
}
__device__ __forceinline__ double lane_value(double x, int src) {
    int2 v = __builtin_bit_cast(int2, x);
    v.x = __builtin_amdgcn_readlane(v.x, src);
    v.y = __builtin_amdgcn_readlane(v.y, src);
    return __builtin_bit_cast(double, v);
}

// ---------------------------------------------------------------- L2P + P2P (sparse W)
// One workgroup per (target leaf B, PT-column tile).  Near field: for every
// bucket entry (ray a, point j, value v) of the NSL = 3^dim neighbour leaves
// with a in the tile, all 64 targets add K(x_i - x_j) v to their column a of
// an LDS tile; wave w takes the columns a = w (mod 4), so every tile element
// is updated by one lane, in bucket order.  The far-field operands and the
// first 64 entries of every neighbour bucket (one per lane) are all loaded up
// front, so a workgroup waits for memory about twice; a wave then keeps its
// own entries by a ballot and walks them with the kernel value generated from
// the integer cell offset.  A bucket is ray-major, so a ray's entries (its
// cells in the leaf) come in a run: the run is summed in a register and
// added to the LDS tile once, when the column changes.  The far field adds
// S_leaf^T L_B on MFMA as in the dense kernel, and the two meet in the
// epilogue.
template <typename T, int PT, int NSL>
__global__ void __launch_bounds__(kBlock)
k_l2p_p2p_sparse(int n, int ls, int depth, int r, int rpad, int p, int far, KernelParams kp,
                 T h2, const int *off, const int *key, const T *bv, const T *Sleaf,
                 const T *Lleaf, T *CQ) {
    typedef typename Mma<T>::v4 v4;
    constexpr int dim = NSL == 9 ? 2 : 3;
    constexpr int NTI = PT / 16;
    constexpr int NFP = kLeafPts;                      // pitch of the near-field tile
    constexpr int KT = kLeafPts + 16;                  // pitch of S_leaf^T ([k][point])
    constexpr int WP = PT + Mma<T>::pad;
    constexpr int FU = (kLeafPts * kMaxR + kBlock - 1) / kBlock;   // far operand loads per thread
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *nf = reinterpret_cast<T *>(smem_raw);           // [PT][NFP], swizzled (nfi)
    T *sK = nf + PT * NFP;                             // [rpad][KT] S_leaf^T
    T *sW = sK + rpad * KT;                            // [rpad][WP] L_B tile
    // element (column c, target i) of the near-field tile: i XOR a function
    // of the low four bits of c, so that both the per-column writes (64
    // targets) and the epilogue reads (16 columns x 4 target rows in the
    // MFMA output layout) fall on distinct LDS banks
    auto nfi = [](int c, int i) {
        const int l = c & 15;
        return c * NFP + (i ^ ((l & 3) | ((l & 4) << 2) | ((l & 8) ? 0x28 : 0)));
    };
    const int64_t B = blockIdx.x;
    const int c0 = blockIdx.y * PT;
    const int ncols = min(PT, p - c0);
    const int nb = 1 << depth;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    int b[3];
    box_coords(B, nb, dim, b);
    // lane t < NSL: bucket range of the neighbour leaf in slot t (empty if
    // that leaf lies outside the tree)
    int my_lo = 0, my_hi = 0;
    if (lane < NSL) {
        const int a[3] = {b[0] + lane % 3 - 1, b[1] + (lane / 3) % 3 - 1,
                          dim == 3 ? b[2] + lane / 9 - 1 : 0};
        if (a[0] >= 0 && a[0] < nb && a[1] >= 0 && a[1] < nb && (dim == 2 || (a[2] >= 0 && a[2] < nb))) {
            const int64_t A = box_index(a, nb, dim);
            my_lo = off[A];
            my_hi = off[A + 1];
        }
    }
    // far operands into registers (in flight while the buckets are read)
    T kreg[FU], lreg[FU];
    if (far) {
#pragma unroll
        for (int u = 0; u < FU; ++u) {
            const int idx = tid + kBlock * u;
            kreg[u] = (T)0;
            lreg[u] = (T)0;
            if (idx < kLeafPts * rpad) {
                const int i = idx / rpad, k = idx % rpad;
                if (k < r) kreg[u] = Sleaf[k * kLeafPts + i];
            }
            if (idx < rpad * PT) {
                const int k = idx / PT, c = idx % PT;
                if (k < r && c < ncols) lreg[u] = Lleaf[(B * r + k) * p + c0 + c];
            }
        }
    }
    for (int idx = tid; idx < PT * NFP; idx += kBlock) nf[idx] = (T)0;
    // the first 64 entries of every neighbour bucket, one per lane
    int kk[NSL];
    T vv[NSL];
#pragma unroll
    for (int sl = 0; sl < NSL; ++sl) {
        const int e = __builtin_amdgcn_readlane(my_lo, sl) + lane;
        const bool in = e < __builtin_amdgcn_readlane(my_hi, sl);
        kk[sl] = in ? key[e] : -1;
        vv[sl] = in ? bv[e] : (T)0;
    }
    if (far) {
#pragma unroll
        for (int u = 0; u < FU; ++u) {
            const int idx = tid + kBlock * u;
            if (idx < kLeafPts * rpad) sK[(idx % rpad) * KT + idx / rpad] = kreg[u];
            if (idx < rpad * PT) sW[(idx / PT) * WP + idx % PT] = lreg[u];
        }
    }
    int li[3];
    leaf_local(lane, dim, li);                         // this lane's target point
    __syncthreads();                                   // tile cleared, far operands staged
    // the current run: its tile column (uniform; -1 before the first) and
    // this lane's sum over it
    int run_c = -1;
    T run = (T)0;
    auto flush = [&]() {
        if (run_c >= 0) nf[nfi(run_c, lane)] += run;
    };
    auto add_entries = [&](int kkl, T vl, int sl) {
        const int c = kkl / kLeafPts - c0;
        uint64_t mask = __ballot(kkl >= 0 && c >= 0 && c < ncols && (c & 3) == wave);
        const int o[3] = {sl % 3 - 1, (sl / 3) % 3 - 1, sl / 9 - 1};
        while (mask) {
            const int src = __builtin_ctzll(mask);
            mask &= mask - 1;
            const int ks = __builtin_amdgcn_readlane(kkl, src);
            const T vs = lane_value(vl, src);
            int lj[3];
            leaf_local(ks % kLeafPts, dim, lj);
            int dsq = 0;
#pragma unroll
            for (int ax = 0; ax < dim; ++ax) {
                const int d = o[ax] * ls + lj[ax] - li[ax];
                dsq += d * d;
            }
            const int cs = ks / kLeafPts - c0;
            if (cs != run_c) {                         // uniform
                flush();
                run_c = cs;
                run = (T)0;
            }
            run += kernel_from_r2<T>((T)dsq * h2, kp) * vs;
        }
    };
#pragma unroll
    for (int sl = 0; sl < NSL; ++sl) {
        add_entries(kk[sl], vv[sl], sl);
        // buckets of more than 64 entries: the rest, 64 at a time
        const int lo = __builtin_amdgcn_readlane(my_lo, sl), hi = __builtin_amdgcn_readlane(my_hi, sl);
        for (int base = lo + 64; base < hi; base += 64) {
            const int e = base + lane;
            add_entries(e < hi ? key[e] : -1, e < hi ? bv[e] : (T)0, sl);
        }
    }
    flush();
    v4 acc[NTI];
#pragma unroll
    for (int t = 0; t < NTI; ++t) acc[t] = v4{0, 0, 0, 0};
    const int lr = lane & 15, q = lane >> 4;
    __syncthreads();                                   // near-field tile complete
    if (far) {
        const T *arow = sK + q * KT + 16 * wave + lr;
        const T *bcol = sW + q * WP + lr;
        for (int k0 = 0; k0 < rpad; k0 += 4) {
            const T av = arow[k0 * KT];
#pragma unroll
            for (int t = 0; t < NTI; ++t) acc[t] = Mma<T>::op(av, bcol[k0 * WP + 16 * t], acc[t]);
        }
    }
#pragma unroll
    for (int t = 0; t < NTI; ++t) {
        const int c = 16 * t + lr;
        if (c >= ncols) continue;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int i = 16 * wave + Mma<T>::row(q, rr);
            const int64_t g = leaf_point_real(b, i, dim, n, ls);
            if (g >= 0) CQ[g * p + c0 + c] = acc[t][rr] + nf[nfi(c, i)];
        }
    }
}

// ---------------------------------------------------------------- M2L, M2M, L2L (MFMA)
// One workgroup per (output box B, PT-column tile).  The output r x PT tile is
// cut into 16 x 16 MFMA tiles (target-node rows padded to RT = ceil(r/16)
// tiles), dealt round-robin to the 4 waves; for every source box A the r x r
// translation and M_A (r x PT) are staged in LDS (k padded to a multiple of 4
// with zeros) and multiplied on MFMA.  The three translations differ only in
// their sources and operators:
//   M2L: B at level lev, A over its interaction list, T_{lev, offset};
//        L_B = the sum (levels are written before any L2L adds to them)
//   M2M: B a parent at level lev, A its 2^dim children, S_child; M_B = the sum
//   L2L: B a child at level lev + 1, A its parent, S_child^T; L_B += the product
enum { kM2L = 0, kM2M = 1, kL2L = 2 };
template <typename T, int PT, int RMAX, int MODE>
__global__ void __launch_bounds__(kBlock)
k_trans_mma(int dim, int r, int p, int lev, const T *M, const T *Tlev, T *L) {
    typedef typename Mma<T>::v4 v4;
    constexpr int NCT = PT / 16;
    constexpr int MAXT = 8;                            // tiles per wave (r <= 64)
    constexpr int WP = PT + Mma<T>::pad;
    constexpr int VW = 16 / sizeof(T);                 // values per 16-byte load
    typedef T tv __attribute__((ext_vector_type(VW)));
    constexpr int MPT = (RMAX * PT / VW + kBlock - 1) / kBlock;    // M loads per thread (r <= RMAX)
    constexpr int TPT = (RMAX * RMAX + kBlock - 1) / kBlock;       // T values per thread
    extern __shared__ __align__(16) unsigned char smem_raw[];
    // TP = 68 (4 mod 64 words) spreads the 16 rows x 4 k of an A-operand
    // read over distinct LDS banks
    const int RT = (r + 15) / 16, KR = (r + 3) / 4 * 4, TP = 68;
    T *sM = reinterpret_cast<T *>(smem_raw);           // [KR][WP]
    T *sT = sM + KR * WP;                              // [16 RT][TP]
    const int64_t B = blockIdx.x;
    const int c0 = blockIdx.y * PT;
    const int ncols = min(PT, p - c0);
    const int nb = 1 << lev;                           // boxes per axis at level lev
    const int nbB = MODE == kL2L ? 2 * nb : nb;        // ... at the output box's level
    // sources: the interaction list (M2L, over the 7^dim offset slots), the
    // 2^dim children (M2M) or the parent (L2L)
    const int noff = MODE == kM2L ? (dim == 2 ? 49 : 343) : MODE == kM2M ? (1 << dim) : 1;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, q = lane >> 4;
    const int ntiles = RT * NCT;
    const int nm = KR * (PT / VW), nt = 16 * RT * KR;
    int b[3];
    box_coords(B, nbB, dim, b);
    const int bch = (b[0] & 1) | ((b[1] & 1) << 1) | ((b[2] & 1) << 2);   // L2L: child slot of B
    // The next source is loaded into registers while the
    // MFMAs of the current one run, then moved to LDS between two barriers.
    tv mreg[MPT];
    T treg[TPT];
#define HIKF_M2L_FETCH(OI)                                                                    \
    do {                                                                                      \
        const int fo = (OI);                                                                  \
        int64_t A;                                                                            \
        if (MODE == kM2L) {                                                                   \
            const int fa[3] = {b[0] + fo % 7 - 3, b[1] + (fo / 7) % 7 - 3,                    \
                               dim == 3 ? b[2] + fo / 49 - 3 : 0};                            \
            A = box_index(fa, nb, dim);                                                       \
        } else if (MODE == kM2M) {                                                            \
            const int fa[3] = {2 * b[0] + (fo & 1), 2 * b[1] + ((fo >> 1) & 1),               \
                               2 * b[2] + ((fo >> 2) & 1)};                                   \
            A = box_index(fa, 2 * nb, dim);                                                   \
        } else {                                                                              \
            const int fa[3] = {b[0] >> 1, b[1] >> 1, b[2] >> 1};                              \
            A = box_index(fa, nb, dim);                                                       \
        }                                                                                     \
        const T *Toff = Tlev + int64_t(MODE == kL2L ? bch : fo) * r * r;                      \
        _Pragma("unroll") for (int u = 0; u < MPT; ++u) {                                     \
            const int idx = tid + kBlock * u, k = idx / (PT / VW), ch = idx % (PT / VW);      \
            tv v;                                                                             \
            if (idx < nm && k < r && VW * ch < ncols) {                                       \
                v = *reinterpret_cast<const tv *>(M + (A * r + k) * p + c0 + VW * ch);        \
            } else {                                                                          \
                _Pragma("unroll") for (int e = 0; e < VW; ++e) v[e] = (T)0;                   \
            }                                                                                 \
            mreg[u] = v;                                                                      \
        }                                                                                     \
        _Pragma("unroll") for (int u = 0; u < TPT; ++u) {                                     \
            const int idx = tid + kBlock * u, i = idx / KR, k = idx % KR;                     \
            treg[u] = (idx < nt && i < r && k < r) ? Toff[MODE == kL2L ? k * r + i : i * r + k] \
                                                   : (T)0;                                    \
        }                                                                                     \
    } while (0)
    auto next_il = [&](int oi) {
        if (MODE != kM2L) return oi + 1;
        for (++oi; oi < noff; ++oi) {
            int o[3] = {oi % 7 - 3, (oi / 7) % 7 - 3, oi / 49 - 3};
            if (il_member(b, o, nb, dim)) break;
        }
        return oi;
    };
    v4 acc[MAXT];
#pragma unroll
    for (int u = 0; u < MAXT; ++u) acc[u] = v4{0, 0, 0, 0};
    int oi = next_il(-1);
    if (oi < noff) HIKF_M2L_FETCH(oi);
    while (oi < noff) {
        __syncthreads();                               // LDS free (previous MFMAs done)
#pragma unroll
        for (int u = 0; u < MPT; ++u) {
            const int idx = tid + kBlock * u, k = idx / (PT / VW), ch = idx % (PT / VW);
            if (idx < nm) *reinterpret_cast<tv *>(sM + k * WP + VW * ch) = mreg[u];
        }
#pragma unroll
        for (int u = 0; u < TPT; ++u) {
            const int idx = tid + kBlock * u, i = idx / KR, k = idx % KR;
            if (idx < nt) sT[i * TP + k] = treg[u];
        }
        __syncthreads();
        const int on = next_il(oi);
        if (on < noff) HIKF_M2L_FETCH(on);             // in flight during the MFMAs
#pragma unroll
        for (int u = 0; u < MAXT; ++u) {
            const int tile = wave + 4 * u;
            if (tile >= ntiles) break;                 // uniform per wave
            const int rt = tile / NCT, ct = tile % NCT;
            const T *arow = sT + (16 * rt + lr) * TP + q;
            const T *bcol = sM + q * WP + 16 * ct + lr;
            for (int k0 = 0; k0 < KR; k0 += 4)
                acc[u] = Mma<T>::op(arow[k0], bcol[k0 * WP], acc[u]);
        }
        oi = on;
    }
#undef HIKF_M2L_FETCH
#pragma unroll
    for (int u = 0; u < MAXT; ++u) {
        const int tile = wave + 4 * u;
        if (tile >= ntiles) break;
        const int rt = tile / NCT, ct = tile % NCT;
        const int c = 16 * ct + lr;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int k = 16 * rt + Mma<T>::row(q, rr);
            if (k < r && c < ncols) {
                T *dst = L + (B * r + k) * p + c0 + c;
                *dst = MODE == kL2L ? *dst + acc[u][rr] : acc[u][rr];
            }
        }
    }
}

// M2L in FP32 on the 32 x 32 x 2 MFMA (16 < r <= 64; RMAX = 32 or 64 rows):
// as k_trans_mma, with 32 x 32 output tiles.  Per 2-deep k step a lane
// supplies one A value (translation row l % 32, k = l / 32) and one B value
// (M row k, column l % 32) for 32 x 32 x 2 products, half the LDS operand
// reads per flop of the 16 x 16 x 4 shape, and the k padding drops from a
// multiple of 4 to a multiple of 2 (r = 25: 26 instead of 28).  A wave's
// tiles share their row tile when RMAX = 32, so one A read feeds all of
// them.  Lane l holds D[8 (v / 4) + 4 (l / 32) + v % 4][l % 32] in v.
template <int PT, int RMAX>
__global__ void __launch_bounds__(kBlock)
k_m2l_f32w(int dim, int r, int p, int lev, const float *M, const float *Tlev, float *L) {
    typedef float v16 __attribute__((ext_vector_type(16)));
    typedef float f4 __attribute__((ext_vector_type(4)));
    constexpr int NCT = PT / 32;                       // 32-column tiles
    constexpr int RT = RMAX / 32;                      // 32-row tiles
    constexpr int NTILE = RT * NCT;
    constexpr int TW = NTILE / 4;                      // tiles per wave
    static_assert(NTILE % 4 == 0 && TW >= 1, "tiles must split over the 4 waves");
    constexpr int WP = PT + 4;                         // B row pitch (floats)
    constexpr int TP = RMAX + 1;                       // A row pitch: odd, 32 rows on 32 banks
    constexpr int MPT = (RMAX * PT / 4 + kBlock - 1) / kBlock;   // M float4 loads per thread
    constexpr int TPT = (32 * RT * RMAX + kBlock - 1) / kBlock;  // T values per thread
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int KR2 = (r + 1) / 2 * 2;
    float *sM = reinterpret_cast<float *>(smem_raw);   // [KR2][WP]
    float *sT = sM + KR2 * WP;                         // [32 RT][TP]
    const int64_t B = blockIdx.x;
    const int c0 = blockIdx.y * PT;
    const int ncols = min(PT, p - c0);
    const int nb = 1 << lev;
    const int noff = dim == 2 ? 49 : 343;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int l32 = lane & 31, h = lane >> 5;
    const int nm = KR2 * (PT / 4), nt = 32 * RT * KR2;
    int b[3];
    box_coords(B, nb, dim, b);
    auto next_il = [&](int oi) {
        for (++oi; oi < noff; ++oi) {
            int o[3] = {oi % 7 - 3, (oi / 7) % 7 - 3, oi / 49 - 3};
            if (il_member(b, o, nb, dim)) break;
        }
        return oi;
    };
    f4 mreg[MPT];
    float treg[TPT];
    // the multipoles and translation tile of list entry fo into registers
    auto fetch = [&](int fo) __attribute__((always_inline)) {
        const int fa[3] = {b[0] + fo % 7 - 3, b[1] + (fo / 7) % 7 - 3, dim == 3 ? b[2] + fo / 49 - 3 : 0};
        const int64_t A = box_index(fa, nb, dim);
        const float *Toff = Tlev + int64_t(fo) * r * r;
#pragma unroll
        for (int u = 0; u < MPT; ++u) {
            const int idx = tid + kBlock * u, k = idx / (PT / 4), ch = idx % (PT / 4);
            f4 v = f4{0.f, 0.f, 0.f, 0.f};
            if (idx < nm && k < r && 4 * ch < ncols)
                v = *reinterpret_cast<const f4 *>(M + (A * r + k) * p + c0 + 4 * ch);
            mreg[u] = v;
        }
#pragma unroll
        for (int u = 0; u < TPT; ++u) {
            const int idx = tid + kBlock * u, i = idx / KR2, k = idx % KR2;
            treg[u] = (idx < nt && i < r && k < r) ? Toff[i * r + k] : 0.f;
        }
    };
    v16 acc[TW];
#pragma unroll
    for (int u = 0; u < TW; ++u)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[u][v] = 0.f;
    int oi = next_il(-1);
    if (oi < noff) fetch(oi);
    while (oi < noff) {
        __syncthreads();                               // LDS free (previous MFMAs done)
#pragma unroll
        for (int u = 0; u < MPT; ++u) {
            const int idx = tid + kBlock * u, k = idx / (PT / 4), ch = idx % (PT / 4);
            if (idx < nm) *reinterpret_cast<f4 *>(sM + k * WP + 4 * ch) = mreg[u];
        }
#pragma unroll
        for (int u = 0; u < TPT; ++u) {
            const int idx = tid + kBlock * u, i = idx / KR2, k = idx % KR2;
            if (idx < nt) sT[i * TP + k] = treg[u];
        }
        __syncthreads();
        const int on = next_il(oi);
        if (on < noff) fetch(on);                      // in flight during the MFMAs
        for (int k0 = 0; k0 < KR2; k0 += 2) {
            float a[RT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) a[rt] = sT[(32 * rt + l32) * TP + k0 + h];
#pragma unroll
            for (int u = 0; u < TW; ++u) {
                const int tile = wave + 4 * u, rt = tile / NCT, ct = tile % NCT;
                const float bv = sM[(k0 + h) * WP + 32 * ct + l32];
                acc[u] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[rt], bv, acc[u], 0, 0, 0);
            }
        }
        oi = on;
    }
#pragma unroll
    for (int u = 0; u < TW; ++u) {
        const int tile = wave + 4 * u, rt = tile / NCT, ct = tile % NCT;
        const int c = 32 * ct + l32;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int k = 32 * rt + 8 * (v >> 2) + 4 * h + (v & 3);
            if (k < r && c < ncols) L[(B * r + k) * p + c0 + c] = acc[u][v];
        }
    }
}

// ---------------------------------------------------------------- low-rank M2L
// The compressed M2L of the black-box FMM: a level's translations T_o share
// one basis U (r x k), the left singular vectors of [T_o1 T_o2 ...] (all
// offsets with max|o| >= 2) whose singular values are at least eps times the
// largest, and T_o ~ U (U^T T_o U) U^T.  The multipoles are compressed once
// (U^T M, k x p per box), translated by the k x k operators C_o = U^T T_o U
// and expanded once (U L~), so a list entry costs 2 k^2 p instead of 2 r^2 p.
// U comes from the eigenvectors of the r x r Gram matrix sum_o T_o T_o^T
// (FP64, evaluated from the kernel), found on the host by the cyclic Jacobi
// method.

// A[i][j] = sum_o sum_q T_o[i][q] T_o[j][q] for the level's box side s:
// one workgroup per (i, j >= i), its threads over the (slot, q) pairs, a
// fixed-order tree sum at the end
__global__ void __launch_bounds__(kBlock)
k_lr_gram(int dim, int nc, int r, double s, KernelParams kp, double *A) {
    __shared__ double red[kBlock];
    const int i = blockIdx.x / r, j = blockIdx.x % r;
    if (j < i) return;
    const int noff = dim == 2 ? 49 : 343;
    int ki[3], kj[3], kq[3];
    node_idx(i, nc, ki);
    node_idx(j, nc, kj);
    double acc = 0.0;
    for (int t = threadIdx.x; t < noff * r; t += kBlock) {
        const int oi = t / r, q = t % r;
        const int o[3] = {oi % 7 - 3, (oi / 7) % 7 - 3, oi / 49 - 3};
        int omax = 0;
        for (int ax = 0; ax < dim; ++ax) omax = max(omax, abs(o[ax]));
        if (omax < 2) continue;
        node_idx(q, nc, kq);
        double r2i = 0.0, r2j = 0.0;
        for (int ax = 0; ax < dim; ++ax) {
            const double xq = cheb_node(nc, kq[ax]);
            const double di = s * (o[ax] + 0.5 * (xq - cheb_node(nc, ki[ax])));
            const double dj = s * (o[ax] + 0.5 * (xq - cheb_node(nc, kj[ax])));
            r2i += di * di;
            r2j += dj * dj;
        }
        acc += kernel_from_r2<double>(r2i, kp) * kernel_from_r2<double>(r2j, kp);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int k = kBlock / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        A[i * r + j] = red[0];
        A[j * r + i] = red[0];
    }
}

// W[slot][i][b] = sum_q T_slot[i][q] U[q][b] (U: r x k, row stride k)
__global__ void k_lr_w(int dim, int nc, int r, int k, double s, KernelParams kp, const double *U,
                       double *W) {
    const int noff = dim == 2 ? 49 : 343;
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= int64_t(noff) * r * k) return;
    const int oi = int(idx / (int64_t(r) * k)), i = int((idx / k) % r), b = int(idx % k);
    const int o[3] = {oi % 7 - 3, (oi / 7) % 7 - 3, oi / 49 - 3};
    int omax = 0;
    for (int ax = 0; ax < dim; ++ax) omax = max(omax, abs(o[ax]));
    if (omax < 2) { W[idx] = 0.0; return; }
    int ki[3], kq[3];
    node_idx(i, nc, ki);
    double acc = 0.0;
    for (int q = 0; q < r; ++q) {
        node_idx(q, nc, kq);
        double r2 = 0.0;
        for (int ax = 0; ax < dim; ++ax) {
            const double d = s * (o[ax] + 0.5 * (cheb_node(nc, kq[ax]) - cheb_node(nc, ki[ax])));
            r2 += d * d;
        }
        acc += kernel_from_r2<double>(r2, kp) * U[q * k + b];
    }
    W[idx] = acc;
}

// C[slot][a][b] = sum_i U[i][a] W[slot][i][b] in the pass precision, and
// the compress / expand operators Ut = U^T (k x r), Ue = U (r x k)
template <typename T>
__global__ void k_lr_c(int noff, int r, int k, const double *U, const double *W, T *C, T *Ut,
                       T *Ue) {
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t nc_ = int64_t(noff) * k * k;
    if (idx < nc_) {
        const int sl = int(idx / (int64_t(k) * k)), a = int((idx / k) % k), b = int(idx % k);
        const double *Ws = W + int64_t(sl) * r * k;
        double acc = 0.0;
        for (int i = 0; i < r; ++i) acc += U[i * k + a] * Ws[i * k + b];
        C[idx] = (T)acc;
    }
    if (idx < int64_t(r) * k) {
        const int i = int(idx / k), a = int(idx % k);
        Ut[a * r + i] = (T)U[i * k + a];
        Ue[i * k + a] = (T)U[i * k + a];
    }
}

// out[box][a][c] = sum_b op[a][b] in[box][b][c] (op: na x nb <= 64 x 64),
// one workgroup per (box, 64 columns); the operator and the input panel are
// staged in LDS
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_box_op(int na, int nb, int p, const T *op, const T *in, T *out) {
    __shared__ T sop[64 * 64];
    __shared__ T sin_[64 * 64];
    const int64_t B = blockIdx.x;
    const int c0 = blockIdx.y * 64;
    const int ncol = min(64, p - c0);
    for (int idx = threadIdx.x; idx < na * nb; idx += kBlock)
        sop[(idx / nb) * 64 + idx % nb] = op[idx];
    for (int idx = threadIdx.x; idx < nb * 64; idx += kBlock) {
        const int b = idx / 64, c = idx % 64;
        sin_[b * 64 + c] = c < ncol ? in[(B * nb + b) * p + c0 + c] : (T)0;
    }
    __syncthreads();
    const int c = threadIdx.x & 63;
    for (int a = threadIdx.x >> 6; a < na; a += kBlock / 64) {
        T acc = 0;
        for (int b = 0; b < nb; ++b) acc += sop[a * 64 + b] * sin_[b * 64 + c];
        if (c < ncol) out[(B * na + a) * p + c0 + c] = acc;
    }
}

// ---------------------------------------------------------------- BF16 split (MFMA)
// v_mfma_f32_16x16x32_bf16: D += A B with lane l supplying the 8 values
// A[l%16][8 (l/16) + i] and B[8 (l/16) + i][l%16], i = 0..7, and holding
// D[4 (l/16) + r][l%16] (the FP32 16x16x4 layout).  Every FP32 operand a is
// split as hi = bf16(a), lo = bf16(a - hi); a product is accumulated in FP32
// as A_hi B_hi + A_hi B_lo + A_lo B_hi (SPLIT) or A_hi B_hi alone.  Operands
// are stored k-contiguous ([row][k] for A, [column][k] for B) so that a
// lane's 8 values are one 16-byte LDS read; LDS rows are padded by 8 values.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void split_bf16(float a, __bf16 *hi, __bf16 *lo) {
    const __bf16 h = (__bf16)a;
    *hi = h;
    *lo = (__bf16)(a - (float)h);
}

template <bool SPLIT>
__device__ __forceinline__ f4v mma_bf16(const bf8 &ah, const bf8 &al, const bf8 &bh, const bf8 &bl,
                                        f4v acc) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
    if (SPLIT) {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
    }
    return acc;
}

// W = H^T split per leaf as [leaf][column][point] (hi block, then lo block);
// the region is zeroed first.  Each nonzero of H is one entry.
__global__ void k_split_w(int64_t nnz, int p, int64_t m, int dim, int n, int npad, int ls,
                          const int64_t *rowptr, const int32_t *col, const double *val,
                          __bf16 *Wh, __bf16 *Wl) {
    int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    int lo = 0, hi = p - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (rowptr[mid] <= e) lo = mid; else hi = mid - 1;
    }
    if (rowptr[lo] > e || rowptr[lo + 1] <= e) return;
    const int64_t c = col[e];
    if (c < 0 || c >= m) return;
    int g[3] = {int(c % n), int((c / n) % n), dim == 3 ? int(c / (int64_t(n) * n)) : 0};
    int bc[3] = {g[0] / ls, g[1] / ls, g[2] / ls};
    const int j = dim == 2 ? (g[0] % ls) + 8 * (g[1] % ls)
                           : (g[0] % ls) + 4 * (g[1] % ls) + 16 * (g[2] % ls);
    const int64_t leaf = box_index(bc, npad / ls, dim);
    const int64_t o = (leaf * p + lo) * kLeafPts + j;
    split_bf16((float)val[e], Wh + o, Wl + o);
}

// Multipoles [box][node][p] (FP32) -> [box][column][kr] hi / lo, nodes >= r
// zero.  One workgroup per (box, 64 columns), transposed through LDS.
__global__ void __launch_bounds__(kBlock)
k_split_m(int r, int kr, int p, const float *M, __bf16 *Mh, __bf16 *Ml) {
    __shared__ float s[64 * 65];
    const int64_t B = blockIdx.x;
    const int c0 = blockIdx.y * 64;
    const int nc = min(64, p - c0);
    for (int k0 = 0; k0 < kr; k0 += 64) {
        __syncthreads();
        for (int idx = threadIdx.x; idx < 64 * 64; idx += kBlock) {
            const int kk = idx / 64, c = idx % 64, k = k0 + kk;
            s[kk * 65 + c] = (k < r && c < nc) ? M[(B * r + k) * p + c0 + c] : 0.f;
        }
        __syncthreads();
        const int kw = min(64, kr - k0);
        for (int idx = threadIdx.x; idx < 64 * kw; idx += kBlock) {
            const int c = idx / kw, kk = idx % kw;
            if (c >= nc) continue;
            const int64_t o = (B * p + c0 + c) * kr + k0 + kk;
            split_bf16(s[kk * 65 + c], Mh + o, Ml + o);
        }
    }
}

// M2L tables [level][slot][r][r] -> [level][slot][rt][kr] hi / lo (zero padded)
__global__ void k_split_t(int64_t nslots, int r, int rt, int kr, const float *T, __bf16 *Th,
                          __bf16 *Tl) {
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= nslots * rt * kr) return;
    const int64_t sl = idx / (int64_t(rt) * kr);
    const int i = int((idx / kr) % rt), k = int(idx % kr);
    const float v = (i < r && k < r) ? T[(sl * r + i) * r + k] : 0.f;
    split_bf16(v, Th + idx, Tl + idx);
}

// M2L on BF16 MFMA: as k_trans_mma, with the translation tile (A, [target
// node][source node]) and M_A (B, [column][source node]) staged as hi / lo.
// Software-pipelined two sources deep over the interaction list: the tiles
// of the next two sources sit in two register sets while the MFMAs of the
// current one run, and each set is moved to LDS between two barriers when
// its turn comes.  KR (nodes padded to 32) is a template parameter so that
// the per-thread staging counts are compile-time.
template <bool SPLIT, int PT, int KR>
__global__ void __launch_bounds__(kBlock)
k_m2l_bf16(int dim, int r, int p, int lev, const __bf16 *Mh, const __bf16 *Ml,
           const __bf16 *Th, const __bf16 *Tl, float *L) {
    constexpr int NCT = PT / 16;
    constexpr int MAXT = 8;                            // tiles per wave
    constexpr int CW = NCT / 4;                        // column tiles per wave
    static_assert(NCT % 4 == 0 && CW <= MAXT, "column tiles must split over the 4 waves");
    constexpr int KP = KR + 8;
    constexpr int KCH = KR / 8;                        // 16-byte chunks per row
    constexpr int TPT = (KR * KCH + kBlock - 1) / kBlock;   // T chunks per thread (rt16 <= KR)
    constexpr int MPT = (PT * KCH + kBlock - 1) / kBlock;   // M chunks per thread
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int RT = (r + 15) / 16, rt16 = 16 * RT;
    __bf16 *sTh = reinterpret_cast<__bf16 *>(smem_raw);
    __bf16 *sTl = sTh + rt16 * KP;
    __bf16 *sMh = sTl + rt16 * KP;
    __bf16 *sMl = sMh + PT * KP;
    const int64_t B = blockIdx.x;
    const int c0 = blockIdx.y * PT;
    const int ncols = min(PT, p - c0);
    const int nb = 1 << lev;
    const int noff = dim == 2 ? 49 : 343;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, q = lane >> 4;
    const int ntiles = RT * NCT;
    int b[3];
    box_coords(B, nb, dim, b);
    // next interaction-list offset after oi (noff when none); uniform
    auto next_il = [&](int oi) {
        for (++oi; oi < noff; ++oi) {
            int o[3] = {oi % 7 - 3, (oi / 7) % 7 - 3, oi / 49 - 3};
            if (il_member(b, o, nb, dim)) break;
        }
        return oi;
    };
    const bf8 zero8 = {};
    // the tiles of interaction-list offset FO into register set S
#define HIKF_M2L_FETCH(FO, S)                                                                     \
    do {                                                                                          \
        const int fo = (FO);                                                                      \
        const int fa[3] = {b[0] + fo % 7 - 3, b[1] + (fo / 7) % 7 - 3,                            \
                           dim == 3 ? b[2] + fo / 49 - 3 : 0};                                    \
        const int64_t A = box_index(fa, nb, dim);                                                 \
        const int64_t tbase = int64_t(fo) * rt16 * KR;                                            \
        _Pragma("unroll") for (int u = 0; u < TPT; ++u) {                                         \
            const int idx = tid + kBlock * u, i = idx / KCH, ch = idx % KCH;                      \
            if (i < rt16) {                                                                       \
                th##S[u] = *reinterpret_cast<const bf8 *>(Th + tbase + int64_t(i) * KR + 8 * ch); \
                tl##S[u] = *reinterpret_cast<const bf8 *>(Tl + tbase + int64_t(i) * KR + 8 * ch); \
            }                                                                                     \
        }                                                                                         \
        _Pragma("unroll") for (int u = 0; u < MPT; ++u) {                                         \
            const int idx = tid + kBlock * u, c = idx / KCH, ch = idx % KCH;                      \
            if (c < ncols) {                                                                      \
                const int64_t g = (A * p + c0 + c) * KR + 8 * ch;                                 \
                mh##S[u] = *reinterpret_cast<const bf8 *>(Mh + g);                                \
                ml##S[u] = *reinterpret_cast<const bf8 *>(Ml + g);                                \
            } else {                                                                              \
                mh##S[u] = ml##S[u] = zero8;                                                      \
            }                                                                                     \
        }                                                                                         \
    } while (0)
    // register set S -> LDS, between two barriers
#define HIKF_M2L_STAGE(S)                                                                         \
    do {                                                                                          \
        __syncthreads();                           /* LDS free (previous MFMAs done) */           \
        _Pragma("unroll") for (int u = 0; u < TPT; ++u) {                                         \
            const int idx = tid + kBlock * u, i = idx / KCH, ch = idx % KCH;                      \
            if (i < rt16) {                                                                       \
                *reinterpret_cast<bf8 *>(sTh + i * KP + 8 * ch) = th##S[u];                       \
                *reinterpret_cast<bf8 *>(sTl + i * KP + 8 * ch) = tl##S[u];                       \
            }                                                                                     \
        }                                                                                         \
        _Pragma("unroll") for (int u = 0; u < MPT; ++u) {                                         \
            const int idx = tid + kBlock * u, c = idx / KCH, ch = idx % KCH;                      \
            *reinterpret_cast<bf8 *>(sMh + c * KP + 8 * ch) = mh##S[u];                           \
            *reinterpret_cast<bf8 *>(sMl + c * KP + 8 * ch) = ml##S[u];                           \
        }                                                                                         \
        __syncthreads();                                                                          \
    } while (0)
    f4v acc[MAXT];
#pragma unroll
    for (int u = 0; u < MAXT; ++u) acc[u] = f4v{0, 0, 0, 0};
    // the wave's tiles are every row tile rt < RT times the column tiles
    // wave + 4 c (c < CW), u = rt CW + c: per k step the hi / lo A values
    // of a row tile and B values of a column tile feed independent MFMAs
    // (128^3, r = 64: 146 -> 129 ms over the levels; in the FP32 / FP64
    // kernel above the same order measured slower, 3.52 -> 3.78 ms at
    // 1024^2, r = 25, so that one keeps a tile's k loop innermost)
    auto compute = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int k0 = 0; k0 < KR; k0 += 32) {
            bf8 bh[CW], bl[CW];
#pragma unroll
            for (int c = 0; c < CW; ++c) {
                const int off = (16 * (wave + 4 * c) + lr) * KP + 8 * q + k0;
                bh[c] = *reinterpret_cast<const bf8 *>(sMh + off);
                bl[c] = *reinterpret_cast<const bf8 *>(sMl + off);
            }
#pragma unroll
            for (int rt = 0; rt < MAXT / CW; ++rt) {
                if (rt < RT) {                          // uniform
                    const int off = (16 * rt + lr) * KP + 8 * q + k0;
                    const bf8 ah = *reinterpret_cast<const bf8 *>(sTh + off);
                    const bf8 al = *reinterpret_cast<const bf8 *>(sTl + off);
#pragma unroll
                    for (int c = 0; c < CW; ++c)
                        acc[rt * CW + c] = mma_bf16<SPLIT>(ah, al, bh[c], bl[c], acc[rt * CW + c]);
                }
            }
        }
    };
    // Software pipeline two sources deep: while the MFMAs of list entry o0
    // run, the tiles of o1 are already in registers (set 1 or 0) and those
    // of o2 are being loaded into the set o0 came from.  The two register
    // sets alternate (phase 0 / phase 1) so that each has a fixed name.
    bf8 th0[TPT], tl0[TPT], mh0[MPT], ml0[MPT];
    bf8 th1[TPT], tl1[TPT], mh1[MPT], ml1[MPT];
    int o0 = next_il(-1);
    int o1 = o0 < noff ? next_il(o0) : noff;
    if (o0 < noff) HIKF_M2L_FETCH(o0, 0);
    if (o1 < noff) HIKF_M2L_FETCH(o1, 1);
    while (o0 < noff) {
        HIKF_M2L_STAGE(0);
        int o2 = o1 < noff ? next_il(o1) : noff;
        if (o2 < noff) HIKF_M2L_FETCH(o2, 0);
        compute();
        o0 = o1;
        o1 = o2;
        if (o0 >= noff) break;
        HIKF_M2L_STAGE(1);
        o2 = o1 < noff ? next_il(o1) : noff;
        if (o2 < noff) HIKF_M2L_FETCH(o2, 1);
        compute();
        o0 = o1;
        o1 = o2;
    }
#undef HIKF_M2L_FETCH
#undef HIKF_M2L_STAGE
#pragma unroll
    for (int u = 0; u < MAXT; ++u) {
        const int tile = wave + 4 * u;
        if (tile >= ntiles) break;
        const int rt = tile / NCT, ct = tile % NCT;
        const int c = 16 * ct + lr;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int k = 16 * rt + 4 * q + rr;
            if (k < r && c < ncols) L[(B * r + k) * p + c0 + c] = acc[u][rr];
        }
    }
}

// L2P + P2P with the near field on BF16 MFMA: the 64 x 64 kernel tile is
// generated in FP32 and split into LDS ([target][source] hi / lo), W_A comes
// pre-split ([column][source]); the far field S_leaf^T L_B stays on FP32 MFMA.
template <bool SPLIT, int PT>
__global__ void __launch_bounds__(kBlock)
k_l2p_p2p_bf16(int dim, int n, int npad, int ls, int depth, int r, int rpad, int p, int rad, int far,
               KernelParams kp, float h2, const __bf16 *Wh, const __bf16 *Wl,
               const float *Sleaf, const float *Lleaf, const float *Knear, float *CQ) {
    constexpr int NTI = PT / 16;
    constexpr int KPB = kLeafPts + 8;                  // bf16 row pitch
    constexpr int WP = PT + Mma<float>::pad;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __bf16 *sKh = reinterpret_cast<__bf16 *>(smem_raw);
    __bf16 *sKl = sKh + kLeafPts * KPB;
    __bf16 *sWh = sKl + kLeafPts * KPB;
    __bf16 *sWl = sWh + PT * KPB;
    const int64_t B = blockIdx.x;
    const int c0 = blockIdx.y * PT;
    const int ncols = min(PT, p - c0);
    const int nb = 1 << depth;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, q = lane >> 4;
    int b[3];
    box_coords(B, nb, dim, b);
    f4v acc[NTI];
#pragma unroll
    for (int t = 0; t < NTI; ++t) acc[t] = f4v{0, 0, 0, 0};
    if (Knear) {
        // neighbour leaves only, software-pipelined as in k_l2p_p2p_mma: the
        // next source's split W panel and FP32 kernel block are loaded into
        // registers during the current MFMAs; the block is split at staging
        constexpr int WPT = (PT * 8 + kBlock - 1) / kBlock;
        constexpr int KPT = (kLeafPts * kLeafPts / 4 + kBlock - 1) / kBlock;
        typedef float f4 __attribute__((ext_vector_type(4)));
        const int nsl = dim == 2 ? 9 : 27;
        auto next_src = [&](int sl) {
            for (++sl; sl < nsl; ++sl) {
                const int a0 = b[0] + sl % 3 - 1, a1 = b[1] + (sl / 3) % 3 - 1, a2 = b[2] + sl / 9 - 1;
                if (a0 >= 0 && a0 < nb && a1 >= 0 && a1 < nb && (dim == 2 || (a2 >= 0 && a2 < nb))) break;
            }
            return sl;
        };
        bf8 whr[WPT], wlr[WPT];
        f4 kr4[KPT];
        const bf8 zero8 = {};
#define HIKF_P2P16_FETCH(SL)                                                                      \
        do {                                                                                      \
            const int fs = (SL);                                                                  \
            const int fa[3] = {b[0] + fs % 3 - 1, b[1] + (fs / 3) % 3 - 1,                        \
                               dim == 3 ? b[2] + fs / 9 - 1 : 0};                                 \
            const int64_t A = box_index(fa, nb, dim);                                             \
            _Pragma("unroll") for (int u = 0; u < WPT; ++u) {                                     \
                const int idx = tid + kBlock * u, c = idx / 8, ch = idx % 8;                      \
                if (c < ncols) {                                                                  \
                    const int64_t g = (A * p + c0 + c) * kLeafPts + 8 * ch;                       \
                    whr[u] = *reinterpret_cast<const bf8 *>(Wh + g);                              \
                    wlr[u] = *reinterpret_cast<const bf8 *>(Wl + g);                              \
                } else {                                                                          \
                    whr[u] = wlr[u] = zero8;                                                      \
                }                                                                                 \
            }                                                                                     \
            const float *kt = Knear + int64_t(fs) * kLeafPts * kLeafPts;                          \
            _Pragma("unroll") for (int u = 0; u < KPT; ++u)                                       \
                kr4[u] = *reinterpret_cast<const f4 *>(kt + 4 * (tid + kBlock * u));              \
        } while (0)
        int sl = next_src(-1);
        HIKF_P2P16_FETCH(sl);
        while (sl < nsl) {
            __syncthreads();
#pragma unroll
            for (int u = 0; u < WPT; ++u) {
                const int idx = tid + kBlock * u, c = idx / 8, ch = idx % 8;
                *reinterpret_cast<bf8 *>(sWh + c * KPB + 8 * ch) = whr[u];
                *reinterpret_cast<bf8 *>(sWl + c * KPB + 8 * ch) = wlr[u];
            }
#pragma unroll
            for (int u = 0; u < KPT; ++u) {
                const int e0 = 4 * (tid + kBlock * u), i = e0 / kLeafPts, j = e0 % kLeafPts;
#pragma unroll
                for (int e = 0; e < 4; ++e) split_bf16(kr4[u][e], sKh + i * KPB + j + e, sKl + i * KPB + j + e);
            }
            __syncthreads();
            const int sn = next_src(sl);
            if (sn < nsl) HIKF_P2P16_FETCH(sn);
            const __bf16 *ah = sKh + (16 * wave + lr) * KPB + 8 * q;
            const __bf16 *al = sKl + (16 * wave + lr) * KPB + 8 * q;
#pragma unroll
            for (int k0 = 0; k0 < kLeafPts; k0 += 32) {
                const bf8 avh = *reinterpret_cast<const bf8 *>(ah + k0);
                const bf8 avl = *reinterpret_cast<const bf8 *>(al + k0);
#pragma unroll
                for (int t = 0; t < NTI; ++t) {
                    const __bf16 *bh = sWh + (16 * t + lr) * KPB + 8 * q + k0;
                    const __bf16 *bl = sWl + (16 * t + lr) * KPB + 8 * q + k0;
                    acc[t] = mma_bf16<SPLIT>(avh, avl, *reinterpret_cast<const bf8 *>(bh),
                                             *reinterpret_cast<const bf8 *>(bl), acc[t]);
                }
            }
            sl = sn;
        }
#undef HIKF_P2P16_FETCH
    }
    const int zlo = dim == 3 ? max(0, b[2] - rad) : 0;
    const int zhi = dim == 3 ? min(nb - 1, b[2] + rad) : 0;
    if (!Knear)
    for (int az = zlo; az <= zhi; ++az)
    for (int ay = max(0, b[1] - rad); ay <= min(nb - 1, b[1] + rad); ++ay)
    for (int ax = max(0, b[0] - rad); ax <= min(nb - 1, b[0] + rad); ++ax) {
        int a[3] = {ax, ay, az};
        const int64_t A = box_index(a, nb, dim);
        __syncthreads();
        for (int idx = tid; idx < PT * 8; idx += kBlock) {
            const int c = idx / 8, ch = idx % 8;
            bf8 vh, vl;
            if (c < ncols) {
                const int64_t g = (A * p + c0 + c) * kLeafPts + 8 * ch;
                vh = *reinterpret_cast<const bf8 *>(Wh + g);
                vl = *reinterpret_cast<const bf8 *>(Wl + g);
            } else {
                for (int e = 0; e < 8; ++e) vh[e] = vl[e] = (__bf16)0.f;
            }
            *reinterpret_cast<bf8 *>(sWh + c * KPB + 8 * ch) = vh;
            *reinterpret_cast<bf8 *>(sWl + c * KPB + 8 * ch) = vl;
        }
        const int sl = (a[0] - b[0] + 1) + 3 * (a[1] - b[1] + 1) + (dim == 3 ? 9 * (a[2] - b[2] + 1) : 0);
        for (int idx = tid; idx < kLeafPts * kLeafPts; idx += kBlock) {
            const int i = idx / kLeafPts, j = idx % kLeafPts;
            float kv;
            if (Knear) {
                kv = Knear[int64_t(sl) * kLeafPts * kLeafPts + idx];
            } else {
                int li[3], lj[3];
                leaf_local(i, dim, li);
                leaf_local(j, dim, lj);
                int dsq = 0;
                for (int qq = 0; qq < dim; ++qq) {
                    const int d = (a[qq] - b[qq]) * ls + lj[qq] - li[qq];
                    dsq += d * d;
                }
                kv = kernel_from_r2<float>((float)dsq * h2, kp);
            }
            split_bf16(kv, sKh + i * KPB + j, sKl + i * KPB + j);
        }
        __syncthreads();
        const __bf16 *ah = sKh + (16 * wave + lr) * KPB + 8 * q;
        const __bf16 *al = sKl + (16 * wave + lr) * KPB + 8 * q;
#pragma unroll
        for (int k0 = 0; k0 < kLeafPts; k0 += 32) {
            const bf8 avh = *reinterpret_cast<const bf8 *>(ah + k0);
            const bf8 avl = *reinterpret_cast<const bf8 *>(al + k0);
#pragma unroll
            for (int t = 0; t < NTI; ++t) {
                const __bf16 *bh = sWh + (16 * t + lr) * KPB + 8 * q + k0;
                const __bf16 *bl = sWl + (16 * t + lr) * KPB + 8 * q + k0;
                acc[t] = mma_bf16<SPLIT>(avh, avl, *reinterpret_cast<const bf8 *>(bh),
                                         *reinterpret_cast<const bf8 *>(bl), acc[t]);
            }
        }
    }
    if (far) {
        // S_leaf^T (64 x r) L_B (r x PT) on FP32 MFMA, staged in the same LDS
        const int KP = max(kLeafPts, rpad) + 4;
        float *sK = reinterpret_cast<float *>(smem_raw);
        float *sW = sK + kLeafPts * KP;
        __syncthreads();
        for (int idx = tid; idx < kLeafPts * rpad; idx += kBlock) {
            const int i = idx / rpad, k = idx % rpad;
            sK[i * KP + k] = k < r ? Sleaf[k * kLeafPts + i] : 0.f;
        }
        for (int idx = tid; idx < rpad * PT; idx += kBlock) {
            const int k = idx / PT, c = idx % PT;
            sW[k * WP + c] = (k < r && c < ncols) ? Lleaf[(B * r + k) * p + c0 + c] : 0.f;
        }
        __syncthreads();
        const float *arow = sK + (16 * wave + lr) * KP + q;
        const float *bcol = sW + q * WP + lr;
        for (int k0 = 0; k0 < rpad; k0 += 4) {
            const float av = arow[k0];
#pragma unroll
            for (int t = 0; t < NTI; ++t) acc[t] = Mma<float>::op(av, bcol[k0 * WP + 16 * t], acc[t]);
        }
    }
#pragma unroll
    for (int t = 0; t < NTI; ++t) {
        const int c = 16 * t + lr;
        if (c >= ncols) continue;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int i = 16 * wave + 4 * q + rr;
            const int64_t g = leaf_point_real(b, i, dim, n, ls);
            if (g >= 0) CQ[g * p + c0 + c] = acc[t][rr];
        }
    }
}

// Allow a kernel more than the default 64 KiB of dynamic LDS (gfx950 has
// 160 KiB per workgroup).
template <typename K>
hipError_t allow_lds(K kernel, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    if (bytes > 160 * 1024) return hipErrorInvalidValue;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
}

int floor_pow2(int x) {
    int v = 1;
    while (v * 2 <= x) v *= 2;
    return v;
}

// column 0 of W from a dense m-vector (the other columns stay zero)
template <typename T>
__global__ void k_dense_w(int64_t m, int dim, int n, int npad, int p, const double *v, T *W) {
    for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < m;
         c += int64_t(gridDim.x) * blockDim.x) {
        const int64_t x = c % n, y = (c / n) % n, z = dim == 3 ? c / (int64_t(n) * n) : 0;
        W[(x + int64_t(npad) * (y + int64_t(npad) * z)) * p] = (T)v[c];
    }
}

// Eigenvectors of the symmetric r x r matrix A (row-major) by the cyclic
// Jacobi method (rotations zeroing a[p][q] with tan 2t = 2 a_pq / (a_qq -
// a_pp)) until the off-diagonal mass is negligible; then the basis of the
// low-rank M2L: the eigenvectors whose sqrt(eigenvalue) is at least eps
// times the largest, sorted by decreasing eigenvalue, as U (r x k, row
// stride k).  Returns k (at least 1).
int lowrank_basis_host(int r, const double *A_in, double eps, double *U) {
    std::vector<double> av(A_in, A_in + size_t(r) * r), vv(size_t(r) * r, 0.0);
    double *a = av.data(), *v = vv.data();
    for (int i = 0; i < r; ++i) v[i * r + i] = 1.0;
    double scale = 0.0;
    for (int i = 0; i < r * r; ++i) scale += a[i] * a[i];
    // sweeps until the off-diagonal part is below 1e-13 of the whole (the
    // kept eigenvalues are at least eps^2 of the largest, eps >= 1e-7 in use)
    for (int sweep = 0; sweep < 50 && scale > 0.0; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < r; ++i)
            for (int j = i + 1; j < r; ++j) off += a[i * r + j] * a[i * r + j];
        if (off <= 1e-26 * scale) break;
        for (int pp = 0; pp < r; ++pp)
            for (int qq = pp + 1; qq < r; ++qq) {
                const double apq = a[pp * r + qq];
                const double app = a[pp * r + pp], aqq = a[qq * r + qq];
                if (std::fabs(apq) <= 1e-18 * std::sqrt(std::fabs(app * aqq)) || apq == 0.0) continue;
                const double th = 0.5 * (aqq - app) / apq;
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < r; ++k) {                    // columns pp, qq
                    double *row = a + k * r;
                    const double akp = row[pp], akq = row[qq];
                    row[pp] = c * akp - sn * akq;
                    row[qq] = sn * akp + c * akq;
                }
                double *rp = a + pp * r, *rq = a + qq * r;       // rows pp, qq
                for (int k = 0; k < r; ++k) {
                    const double apk = rp[k], aqk = rq[k];
                    rp[k] = c * apk - sn * aqk;
                    rq[k] = sn * apk + c * aqk;
                }
                for (int k = 0; k < r; ++k) {                    // eigenvector columns
                    double *row = v + k * r;
                    const double vkp = row[pp], vkq = row[qq];
                    row[pp] = c * vkp - sn * vkq;
                    row[qq] = sn * vkp + c * vkq;
                }
            }
    }
    std::vector<int> order(r);
    for (int i = 0; i < r; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return a[x * r + x] > a[y * r + y]; });
    const double top = std::max(a[order[0] * r + order[0]], 0.0);
    int k = 0;
    while (k < r && top > 0.0 &&
           std::sqrt(std::max(a[order[k] * r + order[k]], 0.0)) >= eps * std::sqrt(top))
        ++k;
    if (k < 1) k = 1;
    for (int i = 0; i < r; ++i)
        for (int b = 0; b < k; ++b) U[size_t(i) * k + b] = v[i * r + order[b]];
    return k;
}

// Low-rank M2L of every level (g.m2l_eps > 0): bases from the Gram matrices
// (one host synchronisation), compressed operators, then per level
// compress -> translate on MFMA (FP32 / FP64, or BF16 split) -> expand into L.
// lr_ranks (optional, levels 0..D) receives the rank used at each level.
template <typename T>
hipError_t run_lowrank_m2l(const Geometry &g, const Layout &lay, char *scr, hipStream_t s,
                           int *lr_ranks) {
    const int p = g.p, r = g.r, dim = g.dim, D = g.depth, nlev = D - 1;
    const int noff = g.noff();
    const double root = double(g.npad) / g.n;
    const bool bf16 = g.fmm_prec == HIKF_FMM_BF16X3 || g.fmm_prec == HIKF_FMM_BF16;
    double *Ag = reinterpret_cast<double *>(scr + lay.lrA);
    double *Ud = reinterpret_cast<double *>(scr + lay.lrU);
    double *Wd = reinterpret_cast<double *>(scr + lay.lrW);
    T *Ct = reinterpret_cast<T *>(scr + lay.lrC);
    T *Ut = reinterpret_cast<T *>(scr + lay.lrUt);
    T *Ue = reinterpret_cast<T *>(scr + lay.lrUe);
    T *MT = reinterpret_cast<T *>(scr + lay.lrM);
    T *LT = reinterpret_cast<T *>(scr + lay.lrL);
    const size_t rr = size_t(r) * r;
    for (int lev = 2; lev <= D; ++lev)
        hipLaunchKernelGGL(k_lr_gram, dim3(unsigned(rr)), dim3(kBlock), 0, s, dim, g.nc, r,
                           root / double(int64_t(1) << lev), g.kp, Ag + (lev - 2) * rr);
    std::vector<double> Ah(size_t(nlev) * rr), Uh(size_t(nlev) * rr, 0.0);
    hipError_t e = hipMemcpyAsync(Ah.data(), Ag, Ah.size() * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    std::vector<int> kl(nlev);
    for (int l = 0; l < nlev; ++l)
        kl[l] = lowrank_basis_host(r, Ah.data() + l * rr, g.m2l_eps, Uh.data() + l * rr);
    e = hipMemcpyAsync(Ud, Uh.data(), Uh.size() * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);     // Uh is a host local
    if (e != hipSuccess) return e;
    if (lr_ranks)
        for (int lev = 0; lev <= D; ++lev) lr_ranks[lev] = lev >= 2 ? kl[lev - 2] : 0;
    for (int lev = 2; lev <= D; ++lev) {
        const int k = kl[lev - 2];
        const double sl = root / double(int64_t(1) << lev);
        const int64_t nw = int64_t(noff) * r * k;
        hipLaunchKernelGGL(k_lr_w, dim3(unsigned((nw + 255) / 256)), dim3(256), 0, s, dim, g.nc, r, k,
                           sl, g.kp, Ud + (lev - 2) * rr, Wd);
        const int64_t nc_ = std::max<int64_t>(int64_t(noff) * k * k, int64_t(r) * k);
        hipLaunchKernelGGL(k_lr_c<T>, dim3(unsigned((nc_ + 255) / 256)), dim3(256), 0, s, noff, r, k,
                           Ud + (lev - 2) * rr, Wd, Ct + size_t(lev - 2) * noff * rr,
                           Ut + (lev - 2) * rr, Ue + (lev - 2) * rr);
    }
    auto Mlev = [&](int lev) { return reinterpret_cast<T *>(scr + lay.ML_level[lev]); };
    auto Llev = [&](int lev) {
        return reinterpret_cast<T *>(scr + lay.L_base + (lay.ML_level[lev] - lay.ML_level[2]));
    };
    for (int lev = 2; lev <= D; ++lev) {
        const int k = kl[lev - 2];
        const int64_t nbx = g.boxes(lev);
        const dim3 gop(unsigned(nbx), (p + 63) / 64);
        hipLaunchKernelGGL(k_box_op<T>, gop, dim3(kBlock), 0, s, k, r, p,
                           static_cast<const T *>(Ut + (lev - 2) * rr),
                           static_cast<const T *>(Mlev(lev)), MT);
        const T *Cl = Ct + size_t(lev - 2) * noff * rr;
        bool done = false;
        if constexpr (sizeof(T) == 4) {
            if (bf16) {
                const int kr = (k + 31) / 32 * 32, rt16 = (k + 15) / 16 * 16;
                __bf16 *Th = reinterpret_cast<__bf16 *>(scr + lay.Tsplit);
                __bf16 *Tl = Th + int64_t(noff) * rt16 * kr;
                hipLaunchKernelGGL(k_split_t, dim3(unsigned((int64_t(noff) * rt16 * kr + 255) / 256)),
                                   dim3(256), 0, s, int64_t(noff), k, rt16, kr, Cl, Th, Tl);
                __bf16 *Mh = reinterpret_cast<__bf16 *>(scr + lay.MS_level[lev]);
                __bf16 *Ml = Mh + nbx * p * kr;
                hipLaunchKernelGGL(k_split_m, dim3(unsigned(nbx), (p + 63) / 64), dim3(kBlock), 0, s, k,
                                   kr, p, MT, Mh, Ml);
                const size_t lds = size_t(rt16 + 128) * (kr + 8) * 2 * sizeof(__bf16);
                const dim3 grid(unsigned(nbx), (p + 127) / 128);
                const bool split = g.fmm_prec == HIKF_FMM_BF16X3;
#define HIKF_LR_BF16(SPL, KRV)                                                                   \
    do {                                                                                         \
        e = allow_lds(k_m2l_bf16<SPL, 128, KRV>, lds);                                           \
        if (e != hipSuccess) return e;                                                           \
        hipLaunchKernelGGL((k_m2l_bf16<SPL, 128, KRV>), grid, dim3(kBlock), lds, s, dim, k, p, lev, \
                           Mh, Ml, Th, Tl, LT);                                                  \
    } while (0)
                if (split) { if (kr == 32) HIKF_LR_BF16(true, 32); else HIKF_LR_BF16(true, 64); }
                else       { if (kr == 32) HIKF_LR_BF16(false, 32); else HIKF_LR_BF16(false, 64); }
#undef HIKF_LR_BF16
                done = true;
            }
        }
        if (!done) {
            // the column tile of the dense M2L below (twice as wide at k <= 32)
            constexpr int MPT = sizeof(T) == 4 ? 128 : 64, MPTW = 2 * MPT;
            const int RT = (k + 15) / 16, KR = (k + 3) / 4 * 4;
            const bool wide = k <= 32 && p > MPT;
            const int pt = wide ? MPTW : MPT;
            const size_t lds = (size_t(KR) * (pt + Mma<T>::pad) + size_t(16 * RT) * 68) * sizeof(T);
            const dim3 grid(unsigned(nbx), (p + pt - 1) / pt);
            if (wide) {
                e = allow_lds(k_trans_mma<T, MPTW, 32, kM2L>, lds);
                if (e != hipSuccess) return e;
                hipLaunchKernelGGL((k_trans_mma<T, MPTW, 32, kM2L>), grid, dim3(kBlock), lds, s, dim, k,
                                   p, lev, static_cast<const T *>(MT), Cl, LT);
            } else if (k <= 32) {
                e = allow_lds(k_trans_mma<T, MPT, 32, kM2L>, lds);
                if (e != hipSuccess) return e;
                hipLaunchKernelGGL((k_trans_mma<T, MPT, 32, kM2L>), grid, dim3(kBlock), lds, s, dim, k,
                                   p, lev, static_cast<const T *>(MT), Cl, LT);
            } else {
                e = allow_lds(k_trans_mma<T, MPT, 64, kM2L>, lds);
                if (e != hipSuccess) return e;
                hipLaunchKernelGGL((k_trans_mma<T, MPT, 64, kM2L>), grid, dim3(kBlock), lds, s, dim, k,
                                   p, lev, static_cast<const T *>(MT), Cl, LT);
            }
        }
        hipLaunchKernelGGL(k_box_op<T>, gop, dim3(kBlock), 0, s, r, k, p,
                           static_cast<const T *>(Ue + (lev - 2) * rr),
                           static_cast<const T *>(LT), Llev(lev));
    }
    return hipGetLastError();
}

// vdense == nullptr: W = H^T from the CSR arrays in RES, result into C_Q.
// Otherwise W's first column is vdense and the result goes to out (m x p).
template <typename T>
hipError_t run_fmm(const Geometry &g, const Layout &lay, char *res, char *scr, hipStream_t s,
                   Timing *tm, const double *vdense = nullptr, T *out = nullptr,
                   int *lr_ranks = nullptr) {
    const int p = g.p, r = g.r, dim = g.dim, D = g.depth;
    const int64_t m = g.m;
    const bool bf16 = g.fmm_prec == HIKF_FMM_BF16X3 || g.fmm_prec == HIKF_FMM_BF16;
    const bool split = g.fmm_prec == HIKF_FMM_BF16X3;
    (void)split;
    T *W = reinterpret_cast<T *>(scr + lay.W);
    T *CQ = vdense ? out : reinterpret_cast<T *>(res + lay.CQ);
    const int64_t *rowptr = res ? reinterpret_cast<const int64_t *>(res + lay.rowptr) : nullptr;
    const int32_t *col = res ? reinterpret_cast<const int32_t *>(res + lay.col) : nullptr;
    const double *val = res ? reinterpret_cast<const double *>(res + lay.val) : nullptr;
    const bool sparse = g.sparse && !vdense;
    const int64_t leaves = g.boxes(D);
    int *bcur = sparse ? reinterpret_cast<int *>(scr + lay.bcur) : nullptr;
    int *boff = sparse ? reinterpret_cast<int *>(scr + lay.boff) : nullptr;
    int *bkey = sparse ? reinterpret_cast<int *>(scr + lay.bkey) : nullptr;
    T *bval = sparse ? reinterpret_cast<T *>(scr + lay.bval) : nullptr;
    tbegin(tm, HIKF_PHASE_INIT, s);
    hipError_t e = hipSuccess;
    if (sparse) {
        // bucket the nonzeros of H by leaf (no dense W)
        int *btmp = reinterpret_cast<int *>(scr + lay.btmp);
        e = hipMemsetAsync(bcur, 0, size_t(leaves) * sizeof(int), s);
        if (e != hipSuccess) return e;
        const unsigned nblk = unsigned(std::max<int64_t>(1, (g.nnz + kBlock - 1) / kBlock));
        if (g.nnz > 0)
            hipLaunchKernelGGL(k_sp_count, dim3(nblk), dim3(kBlock), 0, s, g.nnz, p, m, dim, g.n,
                               g.ls, D, rowptr, col, bcur);
        hipLaunchKernelGGL(k_sp_scan, dim3(1), dim3(1024), 0, s, leaves, bcur, boff);
        if (g.nnz > 0) {
            hipLaunchKernelGGL(k_sp_fill, dim3(nblk), dim3(kBlock), 0, s, g.nnz, p, m, dim, g.n,
                               g.ls, D, rowptr, col, bcur, btmp);
            hipLaunchKernelGGL(k_sp_order<T>, dim3(unsigned(leaves)), dim3(kBlock), 0, s, p, m, dim,
                               g.n, g.ls, D, rowptr, col, val, boff, btmp, bkey, bval);
        }
    } else {
        e = hipMemsetAsync(W, 0, size_t(g.mpad) * p * sizeof(T), s);
        if (e != hipSuccess) return e;
        if (vdense) {
            hipLaunchKernelGGL(k_dense_w<T>, dim3(unsigned(std::min<int64_t>((m + 255) / 256, 65536))),
                               dim3(256), 0, s, m, dim, g.n, g.npad, p, vdense, W);
        } else if (g.nnz > 0) {
            int64_t blocks = (g.nnz + kBlock - 1) / kBlock;
            hipLaunchKernelGGL(k_scatter_w<T>, dim3(unsigned(blocks)), dim3(kBlock), 0, s,
                               g.nnz, p, m, dim, g.n, g.npad, rowptr, col, val, W);
        }
    }
    tend(tm, HIKF_PHASE_INIT, s);
    T *Sleaf = reinterpret_cast<T *>(scr + lay.sleaf);
    T *Schild = reinterpret_cast<T *>(scr + lay.schild);
    T *Tm2l = reinterpret_cast<T *>(scr + lay.m2l);
    auto Mlev = [&](int lev) { return reinterpret_cast<T *>(scr + lay.ML_level[lev]); };
    auto Llev = [&](int lev) {
        return reinterpret_cast<T *>(scr + lay.L_base + (lay.ML_level[lev] - lay.ML_level[2]));
    };
    if (g.far) {
        tbegin(tm, HIKF_PHASE_OPERATORS, s);
        int tot = r * kLeafPts;
        hipLaunchKernelGGL(k_ops_sleaf<T>, dim3((tot + 255) / 256), dim3(256), 0, s,
                           dim, g.nc, g.ls, r, Sleaf);
        tot = (1 << dim) * r * r;
        hipLaunchKernelGGL(k_ops_schild<T>, dim3((tot + 255) / 256), dim3(256), 0, s,
                           dim, g.nc, r, Schild);
        int64_t tot64 = int64_t(D - 1) * g.noff() * r * r;
        hipLaunchKernelGGL(k_ops_m2l<T>, dim3(unsigned((tot64 + 255) / 256)), dim3(256), 0, s,
                           dim, g.nc, r, 2, D - 1, double(g.npad) / g.n, g.kp, Tm2l);
        tend(tm, HIKF_PHASE_OPERATORS, s);
        // P2M
        tbegin(tm, HIKF_PHASE_P2M, s);
        int PT = min(64, p);
        if (sparse)
            hipLaunchKernelGGL(k_p2m_sparse<T>, dim3(unsigned(leaves)), dim3(kBlock), 0, s, r, p,
                               boff, bkey, bval, Sleaf, Mlev(D));
        else
            hipLaunchKernelGGL(k_p2m<T>, dim3(unsigned(g.boxes(D)), (p + PT - 1) / PT), dim3(kBlock),
                               (kLeafPts * PT + r * kLeafPts) * sizeof(T), s, dim, g.npad, g.ls, D, r,
                               p, PT, W, Sleaf, Mlev(D));
        tend(tm, HIKF_PHASE_P2M, s);
        // M2M (and L2L below) on MFMA: the tile kernel of M2L with the children
        // (or the parent) as sources
        constexpr int TPT = sizeof(T) == 4 ? 128 : 64;
        const int RTt = (r + 15) / 16, KRt = (r + 3) / 4 * 4;
        const size_t tlds = (size_t(KRt) * (TPT + Mma<T>::pad) + size_t(16 * RTt) * 68) * sizeof(T);
        tbegin(tm, HIKF_PHASE_M2M, s);
        e = r <= 32 ? allow_lds(k_trans_mma<T, TPT, 32, kM2M>, tlds) : allow_lds(k_trans_mma<T, TPT, 64, kM2M>, tlds);
        if (e == hipSuccess)
            e = r <= 32 ? allow_lds(k_trans_mma<T, TPT, 32, kL2L>, tlds) : allow_lds(k_trans_mma<T, TPT, 64, kL2L>, tlds);
        if (e != hipSuccess) return e;
        for (int lev = D - 1; lev >= 2; --lev) {
            const dim3 grid(unsigned(g.boxes(lev)), (p + TPT - 1) / TPT);
            if (r <= 32)
                hipLaunchKernelGGL((k_trans_mma<T, TPT, 32, kM2M>), grid, dim3(kBlock), tlds, s, dim, r, p,
                                   lev, Mlev(lev + 1), Schild, Mlev(lev));
            else
                hipLaunchKernelGGL((k_trans_mma<T, TPT, 64, kM2M>), grid, dim3(kBlock), tlds, s, dim, r, p,
                                   lev, Mlev(lev + 1), Schild, Mlev(lev));
        }
        tend(tm, HIKF_PHASE_M2M, s);
        // M2L
        tbegin(tm, HIKF_PHASE_M2L, s);
        const bool lowrank = g.m2l_eps > 0.0 && !vdense;
        if (lowrank) {
            e = run_lowrank_m2l<T>(g, lay, scr, s, lr_ranks);
            if (e != hipSuccess) return e;
        }
        if constexpr (sizeof(T) == 4) {
            if (bf16 && !lowrank) {
                const int kr = g.kr32(), rt16 = (r + 15) / 16 * 16;
                const int64_t nslots = int64_t(D - 1) * g.noff();
                __bf16 *Th = reinterpret_cast<__bf16 *>(scr + lay.Tsplit);
                __bf16 *Tl = Th + nslots * rt16 * kr;
                hipLaunchKernelGGL(k_split_t, dim3(unsigned((nslots * rt16 * kr + 255) / 256)),
                                   dim3(256), 0, s, nslots, r, rt16, kr, Tm2l, Th, Tl);
                const size_t lds = size_t(rt16 + 128) * (kr + 8) * 2 * sizeof(__bf16);
                e = kr == 32 ? allow_lds(k_m2l_bf16<true, 128, 32>, lds) : allow_lds(k_m2l_bf16<true, 128, 64>, lds);
                if (e == hipSuccess)
                    e = kr == 32 ? allow_lds(k_m2l_bf16<false, 128, 32>, lds) : allow_lds(k_m2l_bf16<false, 128, 64>, lds);
                if (e != hipSuccess) return e;
                for (int lev = 2; lev <= D; ++lev) {
                    const int64_t nbx = g.boxes(lev);
                    __bf16 *Mh = reinterpret_cast<__bf16 *>(scr + lay.MS_level[lev]);
                    __bf16 *Ml = Mh + nbx * p * kr;
                    hipLaunchKernelGGL(k_split_m, dim3(unsigned(nbx), (p + 63) / 64), dim3(kBlock), 0,
                                       s, r, kr, p, Mlev(lev), Mh, Ml);
                    const __bf16 *Thl = Th + int64_t(lev - 2) * g.noff() * rt16 * kr;
                    const __bf16 *Tll = Tl + int64_t(lev - 2) * g.noff() * rt16 * kr;
                    const dim3 grid(unsigned(nbx), (p + 127) / 128);
#define HIKF_M2L_BF16(SPL, KRV)                                                            \
    hipLaunchKernelGGL((k_m2l_bf16<SPL, 128, KRV>), grid, dim3(kBlock), lds, s, dim, r, p, lev, \
                       Mh, Ml, Thl, Tll, Llev(lev))
                    if (split) { if (kr == 32) HIKF_M2L_BF16(true, 32); else HIKF_M2L_BF16(true, 64); }
                    else       { if (kr == 32) HIKF_M2L_BF16(false, 32); else HIKF_M2L_BF16(false, 64); }
#undef HIKF_M2L_BF16
                }
            }
        }
        bool wdone = false;
        if constexpr (sizeof(T) == 4) {
            if (!bf16 && !lowrank && r > 16) {
                // FP32 with r > 16 on the 32 x 32 x 2 MFMA; 256-column tiles
                // when p fills them and r <= 32 (at r > 32 they would hold
                // the registers of a single wave per SIMD)
                const int rmax = r <= 32 ? 32 : 64;
                const int pt = p > 128 && rmax == 32 ? 256 : 128, KR2 = (r + 1) / 2 * 2;
                const size_t lds = (size_t(KR2) * (pt + 4) + size_t(rmax) * (rmax + 1)) * sizeof(float);
#define HIKF_M2L_F32W(PTV, RMV)                                                                   \
    do {                                                                                          \
        e = allow_lds(k_m2l_f32w<PTV, RMV>, lds);                                                 \
        if (e != hipSuccess) return e;                                                            \
        for (int lev = 2; lev <= D; ++lev) {                                                      \
            const dim3 grid(unsigned(g.boxes(lev)), (p + PTV - 1) / PTV);                         \
            hipLaunchKernelGGL((k_m2l_f32w<PTV, RMV>), grid, dim3(kBlock), lds, s, dim, r, p, lev, \
                               Mlev(lev), Tm2l + int64_t(lev - 2) * g.noff() * r * r, Llev(lev)); \
        }                                                                                         \
    } while (0)
                if (pt == 256) HIKF_M2L_F32W(256, 32);
                else if (rmax == 32) HIKF_M2L_F32W(128, 32);
                else HIKF_M2L_F32W(128, 64);
#undef HIKF_M2L_F32W
                wdone = true;
            }
        }
        if (!bf16 && !lowrank && !wdone) {
            // column tile: with r <= 32 the output is 2 node tiles high, so a
            // tile twice as wide (256 FP32 / 128 FP64 columns) still fits 8
            // MFMA tiles per wave and doubles the products per staged source
            // (FP32 at 1024^2, p = 256, r = 25, before the 32 x 32 kernel above took
            // that case: 3.85 -> 3.52 ms); used when p fills it
            constexpr int MPT = sizeof(T) == 4 ? 128 : 64, MPTW = 2 * MPT;
            const int RT = (r + 15) / 16, KR = (r + 3) / 4 * 4;
            const bool wide = r <= 32 && p > MPT;
            const int pt = wide ? MPTW : MPT;
            const size_t lds = (size_t(KR) * (pt + Mma<T>::pad) + size_t(16 * RT) * 68) * sizeof(T);
            e = wide ? allow_lds(k_trans_mma<T, MPTW, 32, kM2L>, lds)
                     : r <= 32 ? allow_lds(k_trans_mma<T, MPT, 32, kM2L>, lds)
                               : allow_lds(k_trans_mma<T, MPT, 64, kM2L>, lds);
            if (e != hipSuccess) return e;
            for (int lev = 2; lev <= D; ++lev) {
                const dim3 grid(unsigned(g.boxes(lev)), (p + pt - 1) / pt);
                const T *Tl = Tm2l + int64_t(lev - 2) * g.noff() * r * r;
                if (wide)
                    hipLaunchKernelGGL((k_trans_mma<T, MPTW, 32, kM2L>), grid, dim3(kBlock), lds, s, dim, r, p,
                                       lev, Mlev(lev), Tl, Llev(lev));
                else if (r <= 32)
                    hipLaunchKernelGGL((k_trans_mma<T, MPT, 32, kM2L>), grid, dim3(kBlock), lds, s, dim, r, p,
                                       lev, Mlev(lev), Tl, Llev(lev));
                else
                    hipLaunchKernelGGL((k_trans_mma<T, MPT, 64, kM2L>), grid, dim3(kBlock), lds, s, dim, r, p,
                                       lev, Mlev(lev), Tl, Llev(lev));
            }
        }
        tend(tm, HIKF_PHASE_M2L, s);
        // L2L
        tbegin(tm, HIKF_PHASE_L2L, s);
        for (int lev = 2; lev < D; ++lev) {
            const dim3 grid(unsigned(g.boxes(lev + 1)), (p + TPT - 1) / TPT);
            if (r <= 32)
                hipLaunchKernelGGL((k_trans_mma<T, TPT, 32, kL2L>), grid, dim3(kBlock), tlds, s, dim, r, p,
                                   lev, Llev(lev), Schild, Llev(lev + 1));
            else
                hipLaunchKernelGGL((k_trans_mma<T, TPT, 64, kL2L>), grid, dim3(kBlock), tlds, s, dim, r, p,
                                   lev, Llev(lev), Schild, Llev(lev + 1));
        }
        tend(tm, HIKF_PHASE_L2L, s);
    }
    // near-field kernel blocks by leaf offset (all neighbours are within one
    // leaf unless the exact all-pairs sum is requested)
    T *Knear = nullptr;
    if (!g.direct && !sparse) {
        Knear = reinterpret_cast<T *>(scr + lay.knear);
        const int tot = (dim == 2 ? 9 : 27) * kLeafPts * kLeafPts;
        hipLaunchKernelGGL(k_ops_near<T>, dim3((tot + 255) / 256), dim3(256), 0, s, dim, g.ls, g.kp,
                           1.0 / g.n, Knear);
    }
    if (sparse) {
        constexpr int PPT = sizeof(T) == 4 ? 64 : 32;
        const int rpad = (r + 3) / 4 * 4;
        const size_t lds = (size_t(PPT) * kLeafPts + size_t(rpad) * (kLeafPts + 16) +
                            size_t(rpad) * (PPT + Mma<T>::pad)) * sizeof(T);
        e = dim == 2 ? allow_lds(k_l2p_p2p_sparse<T, PPT, 9>, lds) : allow_lds(k_l2p_p2p_sparse<T, PPT, 27>, lds);
        if (e != hipSuccess) return e;
        tbegin(tm, HIKF_PHASE_P2P, s);
        const double h = 1.0 / g.n;
        const dim3 grid(unsigned(leaves), (p + PPT - 1) / PPT);
#define HIKF_P2P_SPARSE(NSLV)                                                                   \
        hipLaunchKernelGGL((k_l2p_p2p_sparse<T, PPT, NSLV>), grid, dim3(kBlock), lds, s, g.n, g.ls, D, \
                           r, rpad, p, g.far ? 1 : 0, g.kp, (T)(h * h), boff, bkey, bval, Sleaf,  \
                           g.far ? Llev(D) : nullptr, CQ)
        if (dim == 2) HIKF_P2P_SPARSE(9); else HIKF_P2P_SPARSE(27);
#undef HIKF_P2P_SPARSE
        tend(tm, HIKF_PHASE_P2P, s);
        return hipGetLastError();
    }
    if constexpr (sizeof(T) == 4) {
        if (bf16) {
            const int rpad = (r + 3) / 4 * 4;
            const int rad = g.direct ? (1 << D) : 1;
            const double h = 1.0 / g.n;
            __bf16 *Wh = reinterpret_cast<__bf16 *>(scr + lay.Wsplit);
            __bf16 *Wl = Wh + leaves * p * kLeafPts;
            tbegin(tm, HIKF_PHASE_P2P, s);
            e = hipMemsetAsync(Wh, 0, size_t(2 * leaves * p * kLeafPts) * sizeof(__bf16), s);
            if (e != hipSuccess) return e;
            if (g.nnz > 0)
                hipLaunchKernelGGL(k_split_w, dim3(unsigned((g.nnz + kBlock - 1) / kBlock)),
                                   dim3(kBlock), 0, s, g.nnz, p, m, dim, g.n, g.npad, g.ls, rowptr, col, val,
                                   Wh, Wl);
            const size_t near_lds = size_t(kLeafPts + 128) * (kLeafPts + 8) * 2 * sizeof(__bf16);
            const size_t far_lds = (size_t(kLeafPts) * (max(kLeafPts, rpad) + 4) +
                                    size_t(max(kLeafPts, rpad)) * (128 + Mma<float>::pad)) * sizeof(float);
            const size_t lds = max(near_lds, far_lds);
            e = allow_lds(k_l2p_p2p_bf16<true, 128>, lds);
            if (e == hipSuccess) e = allow_lds(k_l2p_p2p_bf16<false, 128>, lds);
            if (e != hipSuccess) return e;
            if (split)
                hipLaunchKernelGGL((k_l2p_p2p_bf16<true, 128>), dim3(unsigned(leaves), (p + 127) / 128),
                                   dim3(kBlock), lds, s, dim, g.n, g.npad, g.ls, D, r, rpad, p, rad,
                                   g.far ? 1 : 0, g.kp, (float)(h * h), Wh, Wl, Sleaf,
                                   g.far ? Llev(D) : W, Knear, CQ);
            else
                hipLaunchKernelGGL((k_l2p_p2p_bf16<false, 128>), dim3(unsigned(leaves), (p + 127) / 128),
                                   dim3(kBlock), lds, s, dim, g.n, g.npad, g.ls, D, r, rpad, p, rad,
                                   g.far ? 1 : 0, g.kp, (float)(h * h), Wh, Wl, Sleaf,
                                   g.far ? Llev(D) : W, Knear, CQ);
            tend(tm, HIKF_PHASE_P2P, s);
            return hipGetLastError();
        }
    }
    {
        constexpr int PPT = sizeof(T) == 4 ? 128 : 64;
        const int rpad = (r + 3) / 4 * 4;
        const int rows = max(kLeafPts, rpad);
        const int rad = g.direct ? (1 << D) : 1;
        const double h = 1.0 / g.n;
        const size_t lds = (size_t(kLeafPts) * (rows + 4) + size_t(rows) * (PPT + Mma<T>::pad)) * sizeof(T);
        e = allow_lds(k_l2p_p2p_mma<T, PPT>, lds);
        if (e != hipSuccess) return e;
        tbegin(tm, HIKF_PHASE_P2P, s);
        hipLaunchKernelGGL((k_l2p_p2p_mma<T, PPT>), dim3(unsigned(g.boxes(D)), (p + PPT - 1) / PPT),
                           dim3(kBlock), lds, s, dim, g.n, g.npad, g.ls, D, r, rpad, p, rad, g.far ? 1 : 0,
                           g.kp, (T)(h * h), W, Sleaf, g.far ? Llev(D) : W, Knear, CQ);
        tend(tm, HIKF_PHASE_P2P, s);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fmm(const Geometry &g, const Layout &lay, char *res, char *scr, hipStream_t s,
                      Timing *t, int *lr_ranks) {
    if (g.fmm_prec == HIKF_FMM_F64)
        return run_fmm<double>(g, lay, res, scr, s, t, nullptr, nullptr, lr_ranks);
    return run_fmm<float>(g, lay, res, scr, s, t, nullptr, nullptr, lr_ranks);
}

hipError_t launch_fmm_apply(const Geometry &g, const Layout &lay, char *scr, const double *v,
                            void *out, hipStream_t s) {
    if (g.fmm_prec == HIKF_FMM_F64)
        return run_fmm<double>(g, lay, nullptr, scr, s, nullptr, v, static_cast<double *>(out));
    return run_fmm<float>(g, lay, nullptr, scr, s, nullptr, v, static_cast<float *>(out));
}

}  // namespace hikf

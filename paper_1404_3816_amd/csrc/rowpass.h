// Fused row pass of one assimilation step (Algorithm Algorithm_HiKF: gain,
// state, variance and cross-covariance rows), included by the rowpass_*.hip
// units, each of which instantiates rowpass_launch for a quarter of the
// supported p / 16 values and one C_Q type (the 64 variants compile in
// parallel).  Selected by HIKF_RP_TQ (float or double) and HIKF_RP_SEL
// (p / 16 mod 4).
#pragma once

#include "hikf_internal.h"

namespace hikf {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

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

// The row pass of one or (PERSIST) several row tiles.  A persistent
// workgroup takes tiles blockIdx.x, blockIdx.x + gridDim.x, ...; during the
// last k block of a tile it already loads the first S^{-1} slab and the first
// C_prior values of its next tile, so that tile's MFMAs start as soon as the
// epilogue of the current one has issued its stores (the stores then drain
// while the next tile computes).
template <typename TQ, int NT, int CS, int RG_, int PART, bool PERSIST>
__device__ __forceinline__ void rowpass_part(double *sB, double *red, double *sNR, double *sVX,
                                             int64_t m, int64_t ntiles,
                                             double *C, const TQ *CQ, const double *Sinv,
                                             const double *nu, const double *rdiag, double *xhat,
                                             double *var, double kdiag,
                                             unsigned long long *negvar) {
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
    // A operand column of this lane inside a tile, and its slab row for step s
    const int acol = rp_col(lr & 3, lr >> 2);
    int64_t tile = blockIdx.x;
    auto row_of = [&](int64_t tl) { return tl * (16 * RG) + grp * 16 + lr; };

    double keep[NH > 0 ? NH : 1][4];            // C_prior[row][16 t + col(q, s)], t in [T0, T1)
    double cur[4];
    dv2 nc[2];                                  // next block's C and C_Q, kept apart so the
    qv2 nq[2];                                  // loads are waited for only where they are used
    dv2 bpre[PH];
    d4 acc[NH > 0 ? NH : 1];

    // prologue: slab 0 into buffer 0, the first tile's first C_prior block
#pragma unroll
    for (int u = 0; u < PER2; ++u) {
        const int idx = tid + NTH * u, rr = idx / (P / 2), c = 2 * (idx % (P / 2));
        if (idx < 8 * P)
            *reinterpret_cast<dv2 *>(sB + rr * LDB + c) =
                *reinterpret_cast<const dv2 *>(Sinv + int64_t(rr) * P + c);
    }
    {
        const int64_t r = row_of(tile);
        const int64_t rb = (r < m ? r : 0) * P + 2 * q;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            nc[h] = *reinterpret_cast<const dv2 *>(C + rb + 8 * h);
            nq[h] = *reinterpret_cast<const qv2 *>(CQ + rb + 8 * h);
        }
    }
    // nu and R for the epilogue, once per workgroup (the epilogue then
    // reads LDS instead of waiting on L2 at the end of every tile)
    for (int i = tid; i < P; i += NTH) {
        sNR[i] = nu[i];
        sNR[P + i] = rdiag[i];
    }
    __syncthreads();
    // LDS buffer of k block kb: kb % 2 (a tile has an even number of k
    // blocks in the persistent form, so every tile starts in buffer 0)
    static_assert(!PERSIST || NT % 2 == 0, "persistent row pass needs an even block count");

    for (;;) {
        const int64_t row = row_of(tile);
        const bool ok = row < m;
        const int64_t rbase = (ok ? row : 0) * P + 2 * q;
        const int64_t next = tile + gridDim.x;
        const bool more = PERSIST && next < ntiles;
        int64_t nrbase = 0;
        if (more) {
            const int64_t nr = row_of(next);
            nrbase = (nr < m ? nr : 0) * P + 2 * q;
        }
#pragma unroll
        for (int t = 0; t < NH; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
        // this tile's variance and state entries, read now and parked in LDS
        // at the end of the first k block, so that the epilogue does not
        // wait for them
        double vpre = 0.0, xpre = 0.0;
        const int64_t vrow = tile * (16 * RG) + tid;
        if (tid < 16 * RG && vrow < m) {
            vpre = var[vrow];
            xpre = xhat[vrow];
        }
        // the S^{-1} slabs are the same for every tile: the empty asm keeps
        // their loads inside this tile's k loop instead of hoisted out of
        // the tile loop.  It hides an offset, not the pointer: a pointer
        // passed through asm loses its global address space, the loads
        // become flat loads, and every wait for them becomes a full wait.
        int soff = 0;
        if (PERSIST) asm volatile("" : "+s"(soff));
        const double *Sv = Sinv + soff;

#pragma unroll
        for (int kb = 0; kb < NT; ++kb) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                cur[2 * h] = ok ? nc[h][0] + (double)nq[h][0] : 0.0;
                cur[2 * h + 1] = ok ? nc[h][1] + (double)nq[h][1] : 0.0;
            }
            // what the next k block needs: slab kb + 1 and this tile's
            // C_prior block kb + 1, or after the last block slab 0 and the
            // next tile's first block
            const bool pf = kb + 1 < NT || more;
            const int nslab = kb + 1 < NT ? 16 * (kb + 1) : 0;
            const int64_t pbase = kb + 1 < NT ? rbase + 16 * (kb + 1) : nrbase;
            double *nbuf = sB + ((kb + 1) & 1) * SLAB;
            if (pf) {
                // slab first: it is needed first (end of this block), C_prior next
#pragma unroll
                for (int u = 0; u < PH; ++u) {
                    const int idx = tid + NTH * u, rr = idx / (P / 2), c = 2 * (idx % (P / 2));
                    if (idx < 8 * P)
                        bpre[u] = *reinterpret_cast<const dv2 *>(Sv + int64_t(nslab + rr) * P + c);
                }
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    nc[h] = *reinterpret_cast<const dv2 *>(C + pbase + 8 * h);
                    nq[h] = *reinterpret_cast<const qv2 *>(CQ + pbase + 8 * h);
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
                    if (PH < PER2 && i == NQ / 2 - 1 && pf) {
                        // wide slabs go in two halves to bound the registers they
                        // hold; the target buffer was last read before the
                        // previous barrier
#pragma unroll
                        for (int u = 0; u < PH; ++u) {
                            const int idx = tid + NTH * u, rr = idx / (P / 2), c = 2 * (idx % (P / 2));
                            if (idx < 8 * P)
                                *reinterpret_cast<dv2 *>(nbuf + rr * LDB + c) = bpre[u];
                        }
#pragma unroll
                        for (int u = PH; u < PER2; ++u) {
                            const int idx = tid + NTH * u, rr = idx / (P / 2), c = 2 * (idx % (P / 2));
                            if (idx < 8 * P)
                                bpre[u - PH] = *reinterpret_cast<const dv2 *>(Sv + int64_t(nslab + rr) * P + c);
                        }
                    }
                }
            }
            if (pf) {
                constexpr int U0 = PH < PER2 ? PH : 0;
#pragma unroll
                for (int u = U0; u < PER2; ++u) {
                    const int idx = tid + NTH * u, rr = idx / (P / 2), c = 2 * (idx % (P / 2));
                    if (idx < 8 * P)
                        *reinterpret_cast<dv2 *>(nbuf + rr * LDB + c) = bpre[u - U0];
                }
            }
            if (kb == 0 && tid < 16 * RG) {
                sVX[2 * tid] = vpre;
                sVX[2 * tid + 1] = xpre;
            }
            __syncthreads();
        }

        // epilogue: lane holds K[row][16 t + col(q, r)] = acc[t - T0][r] and
        // C_prior[row][16 t + col(q, r)] = keep[t - T0][r].  nu and R come
        // from LDS; their offset passes through an empty asm statement so
        // that the reads stay here and are not hoisted out of the tile loop
        // (which would hold them in registers for the whole kernel).
        int zoff = 0;
        if (PERSIST) asm volatile("" : "+s"(zoff));
        const double *nu_t = sNR + zoff, *rdiag_t = sNR + P + zoff;
        double dv = 0.0, dx = 0.0;
#pragma unroll
        for (int t = 0; t < NH; ++t)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int c = 16 * (T0 + t) + 8 * h + 2 * q;
                const dv2 nv = *reinterpret_cast<const dv2 *>(nu_t + c);
                const double k0 = acc[t][2 * h], k1 = acc[t][2 * h + 1];
                dv += k0 * keep[t][2 * h] + k1 * keep[t][2 * h + 1];
                dx += k0 * nv[0] + k1 * nv[1];
            }
        // C <- K R.  A row's 16 columns of tile t sit in its 4 lanes as two
        // 64-byte halves (h = 0: columns 0..7, h = 1: 8..15).  Lanes of rows
        // 2j and 2j + 1 (adjacent lanes) swap one half each (DPP quad
        // permutation [1,0,3,2]), so that every store instruction writes whole
        // 128-byte rows: first rows 2j (the even lane's h = 0 and, from the
        // odd lane, the even row's h = 1), then rows 2j + 1.
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
                const dv2 ra = *reinterpret_cast<const dv2 *>(rdiag_t + c0);
                const dv2 rb = *reinterpret_cast<const dv2 *>(rdiag_t + c0 + 8);
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
        __syncthreads();
        // the parts' sums, in a fixed order: x_hat += K nu, var += K(0) - K . C_prior
        if (tid < 16 * RG) {
            const int64_t r = tile * (16 * RG) + tid;
            if (r < m) {
                double sv = 0.0, sx = 0.0;
#pragma unroll
                for (int c = 0; c < CS; ++c) {
                    sv += red[(c * 16 * RG + tid) * 2];
                    sx += red[(c * 16 * RG + tid) * 2 + 1];
                }
                const double v = sVX[2 * tid] + kdiag - sv;
                var[r] = v;
                xhat[r] = sVX[2 * tid + 1] + sx;
                if (v < 0.0) atomicAdd(negvar, 1ull);
            }
        }
        // `red` and `sVX` are written again only after the next tile's
        // first k block, whose barrier orders it after these reads
        if (!more) break;
        tile = next;
    }
}

template <typename TQ, int NT, int CS, int RG, bool PERSIST>
__global__ void __launch_bounds__(64 * CS * RG)
k_rowpass(int64_t m, int64_t ntiles, double *C, const TQ *CQ, const double *Sinv,
          const double *nu, const double *rdiag, double *xhat, double *var, double kdiag,
          const int *status, unsigned long long *negvar) {
    using RS = RowSplit<NT, CS, RG>;
    __shared__ __align__(16) double sB[2 * RS::SLAB];
    __shared__ double red[CS * RG * 16 * 2];
    __shared__ __align__(16) double sNR[2 * RS::P];
    __shared__ double sVX[2 * 16 * RG];
    if (status[kStStep] != HIKF_OK) return;
    if (int64_t(blockIdx.x) >= ntiles) return;
    const int part = (threadIdx.x >> 6) / RG;
#define HIKF_RP_PART(K)                                                                        \
    rowpass_part<TQ, NT, CS, RG, (K), PERSIST>(sB, red, sNR, sVX, m, ntiles, C, CQ, Sinv, nu, rdiag, xhat, \
                                             var, kdiag, negvar)
    if (part == 0)
        HIKF_RP_PART(0);
    else if (part == 1)
        HIKF_RP_PART(1);
    else if (CS > 2 && part == 2)
        HIKF_RP_PART(CS > 2 ? 2 : 0);
    else if (CS > 3)
        HIKF_RP_PART(CS > 3 ? 3 : 0);
#undef HIKF_RP_PART
}

template <typename TQ, int NT, int CS, int RG, bool PERSIST>
hipError_t rowpass_go(const Geometry &g, const Layout &lay, char *res, hipStream_t s) {
    constexpr int rows = 16 * RG;
    const int64_t ntiles = (g.m + rows - 1) / rows;
    int64_t blocks = ntiles;
    if (PERSIST) {
        // one resident workgroup per compute unit (the LDS slabs and the
        // registers of an 8-wave group leave room for one)
        blocks = g.num_cu > 0 ? g.num_cu : 256;
        if (blocks > ntiles) blocks = ntiles;
    }
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL((k_rowpass<TQ, NT, CS, RG, PERSIST>), dim3(unsigned(blocks)),
                       dim3(64 * CS * RG), 0, s, g.m, ntiles,
                       reinterpret_cast<double *>(res + lay.C),
                       reinterpret_cast<const TQ *>(res + lay.CQ),
                       reinterpret_cast<const double *>(res + lay.sinv),
                       reinterpret_cast<const double *>(res + lay.nu),
                       reinterpret_cast<const double *>(res + lay.rdiag),
                       reinterpret_cast<double *>(res + lay.xhat),
                       reinterpret_cast<double *>(res + lay.var),
                       g.kp.family == HIKF_KERNEL_TEST_R2 ? 0.0 : g.kp.theta,
                       reinterpret_cast<const int *>(res + lay.status),
                       reinterpret_cast<unsigned long long *>(res + lay.negvar));
    return hipGetLastError();
}

// ---------------------------------------------------------------- dual form
// One wave per SIMD: 256 threads = 4 waves per tile of 64 rows, P <= 256.
// Wave w takes the row pair rp = w % 2 (row groups 2 rp and 2 rp + 1, 16
// rows each) and the column half c = w / 2.  Every S^{-1} value read from LDS
// feeds two MFMAs (one per row group), which halves the LDS traffic per
// MFMA, and the register file a single wave per SIMD may use (accumulators
// in AGPRs) leaves room to load C_prior two k blocks ahead, so the loads are
// in flight for two blocks of MFMAs instead of one.  The column mapping, the
// slab layout and the epilogue are those of the form above, per row group.
template <typename TQ, int NT, bool PERSIST>
__device__ __forceinline__ void rowpass_dual_part(double *sB, double *red, int64_t m,
                                                  int64_t ntiles, double *C, const TQ *CQ,
                                                  const double *Sinv, const double *nu,
                                                  const double *rdiag, double *xhat,
                                                  double *var, double kdiag,
                                                  unsigned long long *negvar, const int part) {
    typedef typename Pair<TQ>::v2 qv2;
    constexpr int P = NT * 16, LDB = P + 8, SLAB = 16 * LDB, NTH = 256;
    constexpr int PER2 = (8 * P + NTH - 1) / NTH;       // slab column pairs per thread
    constexpr int NH = (NT + 1) / 2;                    // tiles of column half 0
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, q = lane >> 4, rp = wave & 1;
    const int T0 = part ? NH : 0, NHp = part ? NT - NH : NH;
    const int acol = rp_col(lr & 3, lr >> 2);
    int64_t tile = blockIdx.x;

    double keep[2][NH][4];                      // C_prior of the own columns, per row group
    double cur[2][4];
    dv2 pc[2][2][2];                            // C blocks in flight: [stage][group][half]
    qv2 pq[2][2][2];
    dv2 bpre[PER2];
    d4 acc[2][NH];

    auto rbase_of = [&](int64_t tl, int gg) -> int64_t {
        const int64_t r = tl * 64 + (2 * rp + gg) * 16 + lr;
        return (r < m ? r : 0) * P + 2 * q;
    };
    auto load_block = [&](int st, int64_t tl, int kb) {
#pragma unroll
        for (int gg = 0; gg < 2; ++gg) {
            const int64_t b = rbase_of(tl, gg) + 16 * kb;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                pc[st][gg][h] = *reinterpret_cast<const dv2 *>(C + b + 8 * h);
                pq[st][gg][h] = *reinterpret_cast<const qv2 *>(CQ + b + 8 * h);
            }
        }
    };

    // prologue: slab 0 into buffer 0, C_prior blocks 0 and 1 of the first tile
#pragma unroll
    for (int u = 0; u < PER2; ++u) {
        const int idx = tid + NTH * u, rr = idx / (P / 2), c = 2 * (idx % (P / 2));
        if (idx < 8 * P)
            *reinterpret_cast<dv2 *>(sB + rr * LDB + c) =
                *reinterpret_cast<const dv2 *>(Sinv + int64_t(rr) * P + c);
    }
    load_block(0, tile, 0);
    if (NT > 1) load_block(1, tile, 1);
    __syncthreads();

    for (;;) {
        const int64_t next = tile + gridDim.x;
        const bool more = PERSIST && next < ntiles;
        bool okg[2];
#pragma unroll
        for (int gg = 0; gg < 2; ++gg) okg[gg] = tile * 64 + (2 * rp + gg) * 16 + lr < m;
#pragma unroll
        for (int gg = 0; gg < 2; ++gg)
#pragma unroll
            for (int t = 0; t < NH; ++t) acc[gg][t] = d4{0.0, 0.0, 0.0, 0.0};
        int soff = 0;                                  // as in rowpass_part
        if (PERSIST) asm volatile("" : "+s"(soff));
        const double *Sv = Sinv + soff;

#pragma unroll
        for (int kb = 0; kb < NT; ++kb) {
            const int st = kb & 1;
#pragma unroll
            for (int gg = 0; gg < 2; ++gg)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    cur[gg][2 * h] = okg[gg] ? pc[st][gg][h][0] + (double)pq[st][gg][h][0] : 0.0;
                    cur[gg][2 * h + 1] = okg[gg] ? pc[st][gg][h][1] + (double)pq[st][gg][h][1] : 0.0;
                }
            // the block two ahead goes into the stage just consumed: this
            // tile's block kb + 2, or the next tile's block kb + 2 - NT
            if (kb + 2 < NT) load_block(st, tile, kb + 2);
            else if (more && kb + 2 - NT < NT) load_block(st, next, kb + 2 - NT);
            const bool pfs = kb + 1 < NT || more;
            const int nslab = kb + 1 < NT ? 16 * (kb + 1) : 0;
            if (pfs) {
#pragma unroll
                for (int u = 0; u < PER2; ++u) {
                    const int idx = tid + NTH * u, rr = idx / (P / 2), c = 2 * (idx % (P / 2));
                    if (idx < 8 * P)
                        bpre[u] = *reinterpret_cast<const dv2 *>(Sv + int64_t(nslab + rr) * P + c);
                }
            }
            if (kb >= T0 && kb < T0 + NHp) {
#pragma unroll
                for (int gg = 0; gg < 2; ++gg)
#pragma unroll
                    for (int s4 = 0; s4 < 4; ++s4) keep[gg][kb - T0][s4] = cur[gg][s4];
            }
            {
                const double *B = sB + (kb & 1) * SLAB + 2 * q * LDB + acol + 16 * T0;
                constexpr int NQ = 4 * NH;
                auto aop = [&](int i) {
                    const int si = i / NH, ti = i % NH;
                    return B[(8 * (si >> 1) + (si & 1)) * LDB + 16 * ti];
                };
                double ring[4];
                ring[0] = aop(0);
                if (NQ > 1) ring[1] = aop(1);
                if (NQ > 2) ring[2] = aop(2);
#pragma unroll
                for (int i = 0; i < NQ; ++i) {
                    if (i + 3 < NQ) ring[(i + 3) % 4] = aop(i + 3);
                    const int si = i / NH, ti = i % NH;
                    if (ti < NHp) {
                        acc[0][ti] = __builtin_amdgcn_mfma_f64_16x16x4f64(ring[i % 4], cur[0][si], acc[0][ti], 0, 0, 0);
                        acc[1][ti] = __builtin_amdgcn_mfma_f64_16x16x4f64(ring[i % 4], cur[1][si], acc[1][ti], 0, 0, 0);
                    }
                }
            }
            if (pfs) {
#pragma unroll
                for (int u = 0; u < PER2; ++u) {
                    const int idx = tid + NTH * u, rr = idx / (P / 2), c = 2 * (idx % (P / 2));
                    if (idx < 8 * P)
                        *reinterpret_cast<dv2 *>(sB + ((kb + 1) & 1) * SLAB + rr * LDB + c) = bpre[u];
                }
            }
            __syncthreads();
        }
        // with NT = 1 only one block was prefetched per tile; load the next
        // tile's now
        if (NT == 1 && more) load_block(0, next, 0);

        int eoff = 0;                                  // an offset, as for the slabs
        if (PERSIST) asm volatile("" : "+s"(eoff));
        const double *nu_t = nu + eoff, *rdiag_t = rdiag + eoff;
        const bool odd = lr & 1;
        auto swap_pair = [](double x) {
            int2 v = __builtin_bit_cast(int2, x);
            v.x = __builtin_amdgcn_mov_dpp(v.x, 0xB1, 0xF, 0xF, false);
            v.y = __builtin_amdgcn_mov_dpp(v.y, 0xB1, 0xF, 0xF, false);
            return __builtin_bit_cast(double, v);
        };
#pragma unroll
        for (int gg = 0; gg < 2; ++gg) {
            double dv = 0.0, dx = 0.0;
#pragma unroll
            for (int t = 0; t < NH; ++t) {
                if (t >= NHp) continue;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int c = 16 * (T0 + t) + 8 * h + 2 * q;
                    const dv2 nv = *reinterpret_cast<const dv2 *>(nu_t + c);
                    const double k0 = acc[gg][t][2 * h], k1 = acc[gg][t][2 * h + 1];
                    dv += k0 * keep[gg][t][2 * h] + k1 * keep[gg][t][2 * h + 1];
                    dx += k0 * nv[0] + k1 * nv[1];
                }
            }
            // C <- K R with whole-row stores (see the form above)
            const int64_t row = tile * 64 + (2 * rp + gg) * 16 + lr;
            const int64_t r0 = row - odd;
#pragma unroll
            for (int t = 0; t < NH; ++t) {
                if (t >= NHp) continue;
                const int c0 = 16 * (T0 + t) + 2 * q;
                const dv2 ra = *reinterpret_cast<const dv2 *>(rdiag_t + c0);
                const dv2 rb = *reinterpret_cast<const dv2 *>(rdiag_t + c0 + 8);
                const dv2 a = dv2{acc[gg][t][0] * ra[0], acc[gg][t][1] * ra[1]};
                const dv2 b = dv2{acc[gg][t][2] * rb[0], acc[gg][t][3] * rb[1]};
                const dv2 g2 = dv2{swap_pair(odd ? a[0] : b[0]), swap_pair(odd ? a[1] : b[1])};
                const int cc = c0 + (odd ? 8 : 0);
                if (r0 < m) __builtin_nontemporal_store(odd ? g2 : a, reinterpret_cast<dv2 *>(C + r0 * P + cc));
                if (r0 + 1 < m)
                    __builtin_nontemporal_store(odd ? b : g2, reinterpret_cast<dv2 *>(C + (r0 + 1) * P + cc));
            }
            dv += __shfl_xor(dv, 16, 64);
            dx += __shfl_xor(dx, 16, 64);
            dv += __shfl_xor(dv, 32, 64);
            dx += __shfl_xor(dx, 32, 64);
            if (q == 0) {
                red[((part * 4 + 2 * rp + gg) * 16 + lr) * 2 + 0] = dv;
                red[((part * 4 + 2 * rp + gg) * 16 + lr) * 2 + 1] = dx;
            }
        }
        __syncthreads();
        if (tid < 64) {
            const int64_t r = tile * 64 + tid;
            if (r < m) {
                const double sv = red[tid * 2] + red[(64 + tid) * 2];
                const double sx = red[tid * 2 + 1] + red[(64 + tid) * 2 + 1];
                const double v = var[r] + kdiag - sv;
                var[r] = v;
                xhat[r] += sx;
                if (v < 0.0) atomicAdd(negvar, 1ull);
            }
        }
        if (!more) break;
        tile = next;
    }
}

template <typename TQ, int NT, bool PERSIST>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_rowpass_dual(int64_t m, int64_t ntiles, double *C, const TQ *CQ, const double *Sinv,
               const double *nu, const double *rdiag, double *xhat, double *var, double kdiag,
               const int *status, unsigned long long *negvar) {
    __shared__ __align__(16) double sB[2 * 16 * (NT * 16 + 8)];
    __shared__ double red[2 * 64 * 2];
    if (status[kStStep] != HIKF_OK) return;
    if (int64_t(blockIdx.x) >= ntiles) return;
    const int part = (threadIdx.x >> 6) >> 1;
    rowpass_dual_part<TQ, NT, PERSIST>(sB, red, m, ntiles, C, CQ, Sinv, nu, rdiag, xhat, var,
                                       kdiag, negvar, part);
}

template <typename TQ, int NT, bool PERSIST>
hipError_t rowpass_go_dual(const Geometry &g, const Layout &lay, char *res, hipStream_t s) {
    const int64_t ntiles = (g.m + 63) / 64;
    int64_t blocks = ntiles;
    if (PERSIST) {
        blocks = g.num_cu > 0 ? g.num_cu : 256;
        if (blocks > ntiles) blocks = ntiles;
    }
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL((k_rowpass_dual<TQ, NT, PERSIST>), dim3(unsigned(blocks)), dim3(256), 0, s,
                       g.m, ntiles, reinterpret_cast<double *>(res + lay.C),
                       reinterpret_cast<const TQ *>(res + lay.CQ),
                       reinterpret_cast<const double *>(res + lay.sinv),
                       reinterpret_cast<const double *>(res + lay.nu),
                       reinterpret_cast<const double *>(res + lay.rdiag),
                       reinterpret_cast<double *>(res + lay.xhat),
                       reinterpret_cast<double *>(res + lay.var),
                       g.kp.family == HIKF_KERNEL_TEST_R2 ? 0.0 : g.kp.theta,
                       reinterpret_cast<const int *>(res + lay.status),
                       reinterpret_cast<unsigned long long *>(res + lay.negvar));
    return hipGetLastError();
}

}  // namespace

// Row-pass variants (Geometry::rp_variant): bit 0 = persistent workgroups
// (for an even number of 16-column blocks in the 8-wave forms; otherwise
// ignored), bit 1 = the narrow split (32-row tiles, columns in four parts)
// instead of 64-row tiles in two column halves; p > 256 always uses the
// narrow split, which its register budget needs; bit 2 = the dual form
// (4 waves, one per SIMD, two row groups per wave; built for p = 64, 128
// and 256, ignored for other p).
template <typename TQ, int NT>
hipError_t rowpass_launch(const Geometry &g, const Layout &lay, char *res, hipStream_t s) {
    constexpr bool kCanPersist = NT % 2 == 0;
    const bool persist = kCanPersist && (g.rp_variant & 1);
    if constexpr (NT == 4 || NT == 8 || NT == 16) {
        if (g.rp_variant & 4)
            return (g.rp_variant & 1) ? rowpass_go_dual<TQ, NT, true>(g, lay, res, s)
                                      : rowpass_go_dual<TQ, NT, false>(g, lay, res, s);
    }
    const bool narrow = NT > 16 || (g.rp_variant & 2);
    if (narrow)
        return persist ? rowpass_go<TQ, NT, 4, 2, kCanPersist>(g, lay, res, s)
                       : rowpass_go<TQ, NT, 4, 2, false>(g, lay, res, s);
    return persist ? rowpass_go<TQ, NT, (NT > 16 ? 4 : 2), (NT > 16 ? 2 : 4), kCanPersist>(g, lay, res, s)
                   : rowpass_go<TQ, NT, (NT > 16 ? 4 : 2), (NT > 16 ? 2 : 4), false>(g, lay, res, s);
}

#define HIKF_RP(N) \
    template hipError_t rowpass_launch<HIKF_RP_TQ, N>(const Geometry &, const Layout &, char *, hipStream_t);
#if HIKF_RP_SEL == 1
HIKF_RP(1) HIKF_RP(5) HIKF_RP(9) HIKF_RP(13) HIKF_RP(17) HIKF_RP(21) HIKF_RP(25) HIKF_RP(29)
#elif HIKF_RP_SEL == 2
HIKF_RP(2) HIKF_RP(6) HIKF_RP(10) HIKF_RP(14) HIKF_RP(18) HIKF_RP(22) HIKF_RP(26) HIKF_RP(30)
#elif HIKF_RP_SEL == 3
HIKF_RP(3) HIKF_RP(7) HIKF_RP(11) HIKF_RP(15) HIKF_RP(19) HIKF_RP(23) HIKF_RP(27) HIKF_RP(31)
#else
HIKF_RP(4) HIKF_RP(8) HIKF_RP(12) HIKF_RP(16) HIKF_RP(20) HIKF_RP(24) HIKF_RP(28) HIKF_RP(32)
#endif
#undef HIKF_RP

}  // namespace hikf

// Device kernels of the EP sweep for gfx950 (CDNA4, wave64).
//
// Dense linear algebra works on 64 x 64 FP64 tiles of the multifrontal
// fronts.  Every tile product goes through one MFMA core
// (v_mfma_f64_16x16x4f64: four waves, each owning a 32 x 32 quarter of the
// output tile as 2 x 2 MFMA blocks), fed from LDS.  Tasks are either listed
// explicitly (GemmTask) or enumerated implicitly from a per-front batch so a
// right-looking Cholesky step over many fronts is one launch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>

#include "kernels.h"

namespace ep {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int LDP = TS + 1;   // padded LDS row (doubles)

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// star of launch slot i (block i / 4, wave i % 4), -1 if none
__device__ __forceinline__ int64_t star_of_slot(const StarsDev& s, int64_t i) {
    if (s.order) return i < s.norder ? (int64_t)s.order[i] : -1;
    return i < s.n ? i : -1;
}
static unsigned star_blocks(const StarsDev& s) {
    return (unsigned)(((s.order ? s.norder : s.n) + 3) / 4);
}

__device__ __forceinline__ int64_t batch_find(const BatchEnt* be, int nbe, int64_t t) {
    int lo = 0, hi = nbe - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (be[mid].base <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// t -> (i, j) with i >= j >= 0, row-major over the lower triangle
__device__ __forceinline__ void tri_decode(int64_t t, int& i, int& j) {
    int64_t r = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((r + 1) * (r + 2) / 2 <= t) r++;
    while (r * (r + 1) / 2 > t) r--;
    i = (int)r;
    j = (int)(t - r * (r + 1) / 2);
}

__device__ __forceinline__ double* buf_of(const Bufs& b, int id) {
    return id == BUF_FRONTS ? b.fronts : (id == BUF_X ? b.X : b.W);
}

// ---------------------------------------------------------------------------
// MFMA tile core: acc += sum_t op(A_t) op(B_t) over nk tiles.
// sA holds op(A) as [k][i], sB holds op(B) as [k][j] (row stride LDP).
// ---------------------------------------------------------------------------
// Register staging of one A tile and one B tile (16 + 16 doubles per thread),
// so the global loads of the next K tile overlap the MFMAs of the current one.
struct Stage {
    double a[16], b[16];
};

// Thread (lo = tid % 64, hi = tid / 64) reads element lo + (hi + 4r) ld of a
// column-major tile: row lo of column hi + 4r.  Whether that is A[i][k] or
// A[k][i] (transposed operand) is decided when it is written to LDS.
template <typename TA, typename TB>
__device__ __forceinline__ void stage_load(Stage& p, const TA* A, int lda, const TB* B, int ldb) {
    const int tid = threadIdx.x, lo = tid & 63, hi = tid >> 6;
#pragma unroll
    for (int r = 0; r < 16; r++) p.a[r] = (double)A[lo + (int64_t)(hi + 4 * r) * lda];
#pragma unroll
    for (int r = 0; r < 16; r++) p.b[r] = (double)B[lo + (int64_t)(hi + 4 * r) * ldb];
}

// sA holds op(A) as [k][i], sB holds op(B) as [k][j] (row stride LDP)
__device__ __forceinline__ void stage_store(const Stage& p, double* sA, double* sB, bool ta, bool tb, double sgn) {
    const int tid = threadIdx.x, lo = tid & 63, hi = tid >> 6;
    if (!ta) {
#pragma unroll
        for (int r = 0; r < 16; r++) sA[(hi + 4 * r) * LDP + lo] = sgn * p.a[r];
    } else {
#pragma unroll
        for (int r = 0; r < 16; r++) sA[lo * LDP + hi + 4 * r] = sgn * p.a[r];
    }
    if (!tb) {
#pragma unroll
        for (int r = 0; r < 16; r++) sB[lo * LDP + hi + 4 * r] = p.b[r];
    } else {
#pragma unroll
        for (int r = 0; r < 16; r++) sB[(hi + 4 * r) * LDP + lo] = p.b[r];
    }
}

__device__ __forceinline__ void tile_mma(d4 acc[2][2], const double* sA, const double* sB) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
#pragma unroll 4
    for (int kk = 0; kk < TS; kk += 4) {
        const double* ra = sA + (kk + lk) * LDP;
        const double* rb = sB + (kk + lk) * LDP;
        double a0 = ra[wr + li], a1 = ra[wr + 16 + li];
        double b0 = rb[wc + li], b1 = rb[wc + 16 + li];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
}

template <typename TA, typename TB>
__device__ __forceinline__ void seg_run(d4 acc[2][2], double* sA, double* sB, const TA* A, int64_t sa, int lda,
                                        bool ta, double sgn, const TB* B, int64_t sb, int ldb, bool tb, int nk) {
    if (nk <= 0) return;
    Stage p;
    stage_load(p, A, lda, B, ldb);
    for (int t = 0; t < nk; t++) {
        __syncthreads();
        stage_store(p, sA, sB, ta, tb, sgn);
        __syncthreads();
        if (t + 1 < nk) stage_load(p, A + (t + 1) * sa, lda, B + (t + 1) * sb, ldb);
        tile_mma(acc, sA, sB);
    }
}

// Write acc to C (mode: 0 accumulate, 1 overwrite, 2 atomic).  Uses sA as
// staging for a coalesced column-major store.
__device__ __forceinline__ void tile_store(d4 acc[2][2], double* sC, double* C, int ldc, int mode) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    __syncthreads();
#pragma unroll
    for (int bi = 0; bi < 2; bi++)
#pragma unroll
        for (int bj = 0; bj < 2; bj++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                // v_mfma_f64_16x16x4f64 output: lane l, item r -> row l/16 + 4r, column l%16
                int row = wr + 16 * bi + (lane >> 4) + 4 * r;
                int col = wc + 16 * bj + (lane & 15);
                sC[col * LDP + row] = acc[bi][bj][r];
            }
    __syncthreads();
    const int row = threadIdx.x & 63;
#pragma unroll
    for (int r = 0; r < 16; r++) {
        int col = (threadIdx.x >> 6) + 4 * r;
        double v = sC[col * LDP + row];
        double* p = C + row + (int64_t)col * ldc;
        if (mode == 1) *p = v;
        else if (mode == 0) *p += v;
        else atomicAdd(p, v);
    }
}

__device__ __forceinline__ void acc_zero(d4 acc[2][2]) {
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
}

// Blocks are dealt round-robin to the 8 XCDs; give each XCD a contiguous
// range of tasks instead, so neighbouring tasks (which share operand tiles)
// meet in the same L2.
__device__ __forceinline__ int64_t xcd_task(int64_t n) {
    const int64_t b = blockIdx.x, G = gridDim.x;
    const int64_t per = (G + 7) / 8;
    const int64_t x = b % 8, q = b / 8;
    const int64_t full = G % 8 == 0 ? 8 : G % 8;   // XCDs that own 'per' blocks
    const int64_t t = x < full ? x * per + q : full * per + (x - full) * (per - 1) + q;
    (void)n;
    return t;
}

// ---------------------------------------------------------------------------
// Task-list GEMM on 256 x 128 output blocks (trailing updates, diagonal-block
// inverses, selected inversion).  One block of eight waves per CU, two waves
// per SIMD; wave w owns the 64 x 64 quadrant (row quarter w >> 1, column
// half w & 1) as 4 x 4 v_mfma_f64_16x16x4f64 blocks.  K advances in slabs of
// 16 through a ring of three LDS buffers and one register stage.  Within
// slab h: MFMA groups 0 and 1 (k 0-7), then slab h + 1 goes from registers
// to LDS and slab h + 2's global loads (16-byte pairs) are issued, then the
// slab's one barrier, then groups 2 and 3.  Each group's operands are read
// from LDS while the previous group's MFMAs run, and group 0 of slab h + 1
// (visible after the barrier) while group 3 of slab h runs, so the matrix
// units do not wait on LDS at the barrier.  Three buffers make the middle
// barrier enough: a buffer is rewritten two slabs after it was last read,
// with a barrier in between.
// ---------------------------------------------------------------------------
constexpr int BM = 256;              // output rows per block (op(A) side)
constexpr int BN = 128;              // output columns per block (op(B) side)
constexpr int KH = 16;               // K slab depth
constexpr int LDA2 = BM + 4;         // LDS row strides (doubles)
constexpr int LDB2 = BN + 4;
constexpr int SLA = KH * LDA2, SLB = KH * LDB2;
constexpr int GT_THREADS = 512;

template <typename T> struct Pair;
template <> struct Pair<double> { typedef double2 type; };
template <> struct Pair<float> { typedef float2 type; };

// One R x 16 operand slab op(M)(i, k), i in [0, R), k in [0, 16), loaded as
// 16-byte pairs by all 512 threads (NP pairs each).  kc: k is the contiguous
// index in memory (element at M[k + i ld]): a thread loads (k, k+1) of one
// i.  Otherwise i is contiguous: a thread loads (i, i+1) of one k.  Every
// offset and leading dimension is even, so the pairs are aligned.  Row
// quarters a task does not have are loaded all the same: every buffer ends
// in a pad of 256 leading dimensions, so the reads stay in the allocation,
// and only waves whose quadrant is absent (and which skip their MFMAs) ever
// read those rows of LDS.
template <int R, typename T>
__device__ __forceinline__ void slab_load(double* r, const T* M, int ld, bool kc) {
    typedef typename Pair<T>::type P2;
    constexpr int NP = R * KH / 2 / GT_THREADS;
    const int t = threadIdx.x;
    if (!kc) {
        constexpr int PR = R / 2;   // pairs per column
        constexpr int KS = GT_THREADS / PR;
        const int p = t % PR, k0 = t / PR;
        const T* Mp = M + 2 * p + (int64_t)k0 * ld;
#pragma unroll
        for (int q = 0; q < NP; q++) {
            const P2 v = *(const P2*)(Mp + (int64_t)(KS * q) * ld);
            r[2 * q] = (double)v.x;
            r[2 * q + 1] = (double)v.y;
        }
    } else {
        const int kp = t & 7, i0 = t >> 3;   // 64 columns per round
        const T* Mp = M + 2 * kp + (int64_t)i0 * ld;
#pragma unroll
        for (int q = 0; q < NP; q++) {
            const P2 v = *(const P2*)(Mp + (int64_t)(64 * q) * ld);
            r[2 * q] = (double)v.x;
            r[2 * q + 1] = (double)v.y;
        }
    }
}

// Write a slab to LDS as s[k][i] (row stride LD).
template <int R, int LD>
__device__ __forceinline__ void slab_store(const double* r, double* s, bool kc) {
    constexpr int NP = R * KH / 2 / GT_THREADS;
    const int t = threadIdx.x;
    if (!kc) {
        constexpr int PR = R / 2;
        constexpr int KS = GT_THREADS / PR;
        const int p = t % PR, k0 = t / PR;
#pragma unroll
        for (int q = 0; q < NP; q++) *(double2*)&s[(k0 + KS * q) * LD + 2 * p] = double2{r[2 * q], r[2 * q + 1]};
    } else {
        const int kp = t & 7, i0 = t >> 3;
#pragma unroll
        for (int q = 0; q < NP; q++) {
            s[(2 * kp) * LD + i0 + 64 * q] = r[2 * q];
            s[(2 * kp + 1) * LD + i0 + 64 * q] = r[2 * q + 1];
        }
    }
}

// This wave's operands of group g (k = 4g .. 4g + 3) of a slab in LDS.
__device__ __forceinline__ void group_read(double a[4], double b[4], const double* sA, const double* sB, int g) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
    const int li = lane & 15, lk = lane >> 4;
    const double* ra = sA + (4 * g + lk) * LDA2 + wr + li;
    const double* rb = sB + (4 * g + lk) * LDB2 + wc + li;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        a[q] = ra[16 * q];
        b[q] = rb[16 * q];
    }
}

// acc (this wave's quadrant) += one group's rank-4 update
__device__ __forceinline__ void group_mma(d4 acc[4][4], const double a[4], const double b[4]) {
#pragma unroll
    for (int x = 0; x < 4; x++)
#pragma unroll
        for (int y = 0; y < 4; y++) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
}

__device__ __forceinline__ void acc_negate(d4 acc[4][4]) {
#pragma unroll
    for (int x = 0; x < 4; x++)
#pragma unroll
        for (int y = 0; y < 4; y++) acc[x][y] = -acc[x][y];
}

// One segment: acc += sum over its K of op(A) op(B) (acc -= with the negate
// flag: acc is negated before and after, which rounds exactly as adding the
// negated product).  ACT: this wave's quadrant is present; waves without one
// load, store and wait like the others but issue no MFMA and read no LDS.
// All 512 threads take every barrier; ends with a barrier after the last
// read of smem.
template <bool ACT, typename TA>
__device__ __forceinline__ void seg_run(d4 acc[4][4], double* smem, const TA* A, const double* B, const GemmSeg& S) {
    const int sflags = S.flags, lda = S.lda, ldb = S.ldb;
    // op(A)(i, k): transposed A has k contiguous; op(B)(k, j): plain B has k contiguous
    const bool kca = sflags & 1, kcb = !(sflags & 2);
    const bool neg = (sflags & 4) != 0;
    const int nh = (TS / KH) * S.nk;
    const int64_t ha = S.sa / (TS / KH), hb = S.sb / (TS / KH);
    if (nh <= 0) return;
    if (ACT && neg) acc_negate(acc);
    double ra[BM * KH / GT_THREADS], rb[BN * KH / GT_THREADS];
    slab_load<BM>(ra, A, lda, kca);
    slab_load<BN>(rb, B, ldb, kcb);
    slab_store<BM, LDA2>(ra, smem, kca);
    slab_store<BN, LDB2>(rb, smem + SLA, kcb);
    if (nh > 1) {
        slab_load<BM>(ra, A + ha, lda, kca);
        slab_load<BN>(rb, B + hb, ldb, kcb);
    }
    __syncthreads();
    // x: operands of groups 0 and 2, y: of groups 1 and 3
    double xa[4], xb[4], ya[4], yb[4];
    if (ACT) group_read(xa, xb, smem, smem + SLA, 0);
    double* cur = smem;
    double* nxt = smem + (SLA + SLB);
    double* spare = smem + 2 * (SLA + SLB);
    for (int h = 0; h < nh; h++) {
        if (ACT) {
            group_read(ya, yb, cur, cur + SLA, 1);
            group_mma(acc, xa, xb);
            group_read(xa, xb, cur, cur + SLA, 2);
            group_mma(acc, ya, yb);
        }
        if (h + 1 < nh) {
            slab_store<BM, LDA2>(ra, nxt, kca);
            slab_store<BN, LDB2>(rb, nxt + SLA, kcb);
            if (h + 2 < nh) {
                slab_load<BM>(ra, A + (h + 2) * ha, lda, kca);
                slab_load<BN>(rb, B + (h + 2) * hb, ldb, kcb);
            }
        }
        __syncthreads();
        if (ACT) {
            group_read(ya, yb, cur, cur + SLA, 3);
            group_mma(acc, xa, xb);
            if (h + 1 < nh) group_read(xa, xb, nxt, nxt + SLA, 0);
            group_mma(acc, ya, yb);
        }
        double* t = cur;
        cur = nxt;
        nxt = spare;
        spare = t;
    }
    // the last slab's buffer is the next segment's first
    __syncthreads();
    if (ACT && neg) acc_negate(acc);
}

// A32: the launch's tasks have one segment whose A operand is in the FP32
// copy of the factor (mixed precision), upcast on load; B is FP64.
template <bool A32>
__global__ __launch_bounds__(GT_THREADS) void k_gemm_tasks(const GemmTask* __restrict__ tasks, int64_t n, Bufs bufs) {
    __shared__ double smem[3 * (SLA + SLB)];
    const int64_t t = xcd_task(n);
    if (t >= n) return;
    const GemmTask& T = tasks[t];
    if (((T.flags >> 4) & 3) == 0) return;   // padding entry
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int qr = w >> 1, qc = w & 1;
    const int nqa = gt_rows(T.flags), nqb = (T.flags & GT_COLS2) ? 2 : 1;
    // this wave's quadrant is (qr, qc)
    const bool mine = qr < nqa && qc < nqb && (!(T.flags & GT_LOWER) || gt_diag(T.flags) + qr - qc >= 0);
    d4 acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; x++)
#pragma unroll
        for (int y = 0; y < 4; y++) acc[x][y] = d4{0.0, 0.0, 0.0, 0.0};
    if (A32) {
        const GemmSeg& S = T.s[0];
        const float* A = bufs.F32 + S.a;
        const double* B = buf_of(bufs, (S.flags >> 10) & 3) + S.b;
        if (mine) seg_run<true>(acc, smem, A, B, S);
        else seg_run<false>(acc, smem, A, B, S);
    } else {
        const int nseg = (T.flags >> 4) & 3;
        for (int q = 0; q < 2; q++) {
            if (q >= nseg) break;
            const GemmSeg& S = T.s[q];
            const double* A = buf_of(bufs, (S.flags >> 8) & 3) + S.a;
            const double* B = buf_of(bufs, (S.flags >> 10) & 3) + S.b;
            if (mine) seg_run<true>(acc, smem, A, B, S);
            else seg_run<false>(acc, smem, A, B, S);
        }
    }
    if (!mine) return;
    const bool over = T.flags & 1, atom = (T.flags & 2) != 0;
    const int64_t rs = (T.flags & GT_TSTORE) ? T.ldc : 1, cs = (T.flags & GT_TSTORE) ? 1 : T.ldc;
    double* C = buf_of(bufs, (T.flags >> 8) & 3) + T.c + (qr * 64 + (lane >> 4)) * rs + (qc * 64 + (lane & 15)) * cs;
    // v_mfma_f64_16x16x4f64 output: lane l, item r -> row l/16 + 4r, column l%16
#pragma unroll
    for (int x = 0; x < 4; x++)
#pragma unroll
        for (int y = 0; y < 4; y++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                double* p = C + (16 * x + 4 * r) * rs + (16 * y) * cs;
                if (atom) atomicAdd(p, acc[x][y][r]);
                else *p = over ? acc[x][y][r] : *p + acc[x][y][r];
            }
}

void launch_gemm_tasks(hipStream_t st, const GemmTask* t, int64_t n, Bufs b, bool a32) {
    if (n <= 0) return;
    if (a32)
        hipLaunchKernelGGL(k_gemm_tasks<true>, dim3((unsigned)n), dim3(GT_THREADS), 0, st, t, n, b);
    else
        hipLaunchKernelGGL(k_gemm_tasks<false>, dim3((unsigned)n), dim3(GT_THREADS), 0, st, t, n, b);
}

// ---------------------------------------------------------------------------
// Diagonal tile: Cholesky of tile (k,k) of each listed front, and the
// inverse of the factor (kept in X as the diagonal tile of L11^{-1}).
// ---------------------------------------------------------------------------
// One block of four waves per tile (potrf_tile below); the loops are fully
// unrolled, so every register index is static.
__device__ __forceinline__ double lane_bcast(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// FT: the element type of the fronts being factored (double, or float for
// the FP32 copy of a mixed-precision level); the arithmetic is FP64 either
// way and X is FP64.
template <typename FT> __device__ __forceinline__ FT* fronts_of(const Bufs& b);
template <> __device__ __forceinline__ double* fronts_of<double>(const Bufs& b) { return b.fronts; }
template <> __device__ __forceinline__ float* fronts_of<float>(const Bufs& b) { return b.F32; }

// LDS ordering within one wave: the lanes' LDS writes are seen by the
// lanes' later reads (one wave, so no barrier is needed beyond keeping the
// compiler and the counters in order).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// A block of four waves, all of whose threads call this: Cholesky of tile
// (k, k) of front f in place, and the inverse of the factor into X.  Lane i
// holds row i and wave w the columns c = 4 t + w (t = 0..15), so each pivot
// step updates about a quarter of the later columns per wave.  The pivot
// column goes through LDS (C; row i at (i mod 4) 16 + i / 4, so that the
// entries of a wave's columns are contiguous), one barrier per step.  The
// inverse is forward substitution by the first wave, lane j solving for
// column j of X.  T: TS x LDP doubles of LDS; C: TS x TS + TS doubles.
template <typename FT>
__device__ __forceinline__ void potrf_tile(int f, int k, const FrontsDev& F, const Bufs& bufs, int* err, double* T,
                                           double* C) {
    const int m = F.m[f];
    FT* A = fronts_of<FT>(bufs) + F.off[f] + (int64_t)TS * k + (int64_t)TS * k * m;
    const int i = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int pi = (i & 3) * 16 + (i >> 2);
    double a[16];
#pragma unroll
    for (int t = 0; t < 16; t++) a[t] = (double)A[i + (int64_t)(4 * t + w) * m];
    bool bad = false;
#pragma unroll
    for (int j = 0; j < TS; j++) {
        const int s = j >> 2;
        if (w == (j & 3)) {   // the wave holding column j
            double d = lane_bcast(a[s], j);
            if (!(d > 0.0) || !isfinite(d)) {
                bad = true;
                d = 1.0;
            }
            const double l = sqrt(d);
            a[s] = (i == j) ? l : a[s] / l;   // rows above j hold unused values
            C[j * TS + pi] = a[s];
        }
        __syncthreads();
        const double lij = C[j * TS + pi];
        const double* cj = C + j * TS + 16 * w;   // L(4 t + w, j) at cj[t]
        if (w > (j & 3)) a[s] -= lij * cj[s];     // column 4 s + w comes after j
#pragma unroll
        for (int t = s + 1; t < 16; t++) a[t] -= lij * cj[t];
    }
    // L (zeros above the diagonal) to the front and to LDS
#pragma unroll
    for (int t = 0; t < 16; t++) {
        const int c = 4 * t + w;
        const double v = (i >= c) ? a[t] : 0.0;
        A[i + (int64_t)c * m] = (FT)v;
        T[i * LDP + c] = v;
    }
    if (i == 0 && bad) atomicCAS(err, 0, f + 1);
    __syncthreads();
    if (w != 0) return;
    double* dinv = C + TS * TS;
    dinv[i] = 1.0 / T[i * LDP + i];
    wave_sync();
    // X = L^{-1}: lane j solves L x = e_j column by column, so the updates of
    // one step are independent (no chain of dependent FMAs through a sum)
    double x[TS];
#pragma unroll
    for (int r = 0; r < TS; r++) x[r] = (i == r) ? 1.0 : 0.0;
#pragma unroll
    for (int q = 0; q < TS; q++) {
        x[q] *= dinv[q];
#pragma unroll
        for (int r = q + 1; r < TS; r++) x[r] -= T[r * LDP + q] * x[q];
        __builtin_amdgcn_sched_barrier(0);   // keeps the LDS reads of later steps from piling up in registers
    }
    wave_sync();
#pragma unroll
    for (int r = 0; r < TS; r++) T[r * LDP + i] = x[r];
    wave_sync();
    double* Xk = bufs.X + F.xoff[f] + (int64_t)TS * k + (int64_t)TS * k * F.nvpad[f];
    const int ldx = F.nvpad[f];
#pragma unroll
    for (int c = 0; c < TS; c++) {
        Xk[i + (int64_t)c * ldx] = T[i * LDP + c];
        if (c % 16 == 15) __builtin_amdgcn_sched_barrier(0);
    }
}

template <typename FT>
__global__ __launch_bounds__(256) void k_potrf(const int32_t* __restrict__ flist, int k, FrontsDev F, Bufs bufs,
                                               int* err) {
    __shared__ double T[TS * LDP];
    __shared__ double C[TS * TS + TS];
    potrf_tile<FT>(flist[blockIdx.x], k, F, bufs, err, T, C);
}

void launch_potrf(hipStream_t st, const int32_t* flist, int nf, int k, FrontsDev F, Bufs b, int* err) {
    if (nf <= 0) return;
    hipLaunchKernelGGL(k_potrf<double>, dim3(nf), dim3(256), 0, st, flist, k, F, b, err);
}

// ---------------------------------------------------------------------------
// Right-looking step k, implicit tasks.
//   trsm: L_ik = A_ik X_kk^T for row tiles i > k
//   syrk: A_ij -= L_ik L_jk^T for i >= j > k
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_trsm_step(const BatchEnt* __restrict__ be, int nbe, int64_t ntasks, int k,
                                                   FrontsDev F, Bufs bufs) {
    __shared__ double sA[TS * LDP];
    __shared__ double sB[TS * LDP];
    const int64_t t = blockIdx.x;
    if (t >= ntasks) return;
    const int e = (int)batch_find(be, nbe, t);
    const int f = be[e].front;
    const int i = k + 1 + (int)(t - be[e].base);
    const int m = F.m[f];
    double* Aik = bufs.fronts + F.off[f] + (int64_t)TS * i + (int64_t)TS * k * m;
    const double* Xkk = bufs.X + F.xoff[f] + (int64_t)TS * k + (int64_t)TS * k * F.nvpad[f];
    d4 acc[2][2];
    acc_zero(acc);
    seg_run(acc, sA, sB, Aik, 0, m, false, 1.0, Xkk, 0, F.nvpad[f], true, 1);
    tile_store(acc, sA, Aik, m, 1);
}

// In-panel update at pivot step kk (left-looking): column j = kk + 1 of the
// panel, rows i >= j, takes the updates of the panel's pivot columns
// k0 .. kk (K = kk - k0 + 1 tiles), once, after the column solve of kk.
// FACTOR: the block of the diagonal tile (j, j), whose update is then
// complete, goes on to factor it (the next pivot step's diagonal tile)
// while the other blocks update the rest of the column.
template <bool FACTOR>
__global__ __launch_bounds__(256, 2) void k_syrk_inner(const BatchEnt* __restrict__ be, int nbe, int64_t ntasks,
                                                       int kk, FrontsDev F, Bufs bufs, int* err) {
    __shared__ double sA[TS * LDP];
    __shared__ double sB[TS * LDP];
    const int64_t t = blockIdx.x;
    if (t >= ntasks) return;
    const int e = (int)batch_find(be, nbe, t);
    const int f = be[e].front;
    const int m = F.m[f];
    const int j = kk + 1, i = j + (int)(t - be[e].base);
    const int k0 = PW * (kk / PW);
    double* base = bufs.fronts + F.off[f];
    d4 acc[2][2];
    acc_zero(acc);
    seg_run(acc, sA, sB, base + (int64_t)TS * i + (int64_t)TS * k0 * m, (int64_t)TS * m, m, false, -1.0,
            base + (int64_t)TS * j + (int64_t)TS * k0 * m, (int64_t)TS * m, m, true, kk - k0 + 1);
    tile_store(acc, sA, base + (int64_t)TS * i + (int64_t)TS * j * m, m, 0);
    if (FACTOR && i == j) {   // uniform over the block
        __syncthreads();      // the tile's stores are visible to the block
        potrf_tile<double>(f, j, F, bufs, err, sA, sB);
    }
}

void launch_trsm_step(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, int k, FrontsDev F, Bufs b) {
    if (ntasks <= 0) return;
    hipLaunchKernelGGL(k_trsm_step, dim3((unsigned)ntasks), dim3(256), 0, st, be, nbe, ntasks, k, F, b);
}
void launch_syrk_inner(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, int kk, FrontsDev F, Bufs b,
                       int* factor_err) {
    if (ntasks <= 0) return;
    if (factor_err)
        hipLaunchKernelGGL(k_syrk_inner<true>, dim3((unsigned)ntasks), dim3(256), 0, st, be, nbe, ntasks, kk, F, b,
                           factor_err);
    else
        hipLaunchKernelGGL(k_syrk_inner<false>, dim3((unsigned)ntasks), dim3(256), 0, st, be, nbe, ntasks, kk, F, b,
                           factor_err);
}

// ---------------------------------------------------------------------------
// Extend-add: the update block (R x R, lower) of each front is added into
// its parent at the relative rows.  Sigma gather is the reverse copy of the
// parent's selected inverse into the child's R x R block (both triangles of
// diagonal tiles, zeros on padding).
// ---------------------------------------------------------------------------
// ATOMIC: fronts of one launch may share a parent (FP64 atomic adds);
// otherwise the launch holds at most one child per parent, whose rows map
// injectively into the parent, so a plain read-add-write is race-free.
template <bool ATOMIC>
__global__ __launch_bounds__(256) void k_extend_add(const BatchEnt* __restrict__ be, int nbe, int64_t ntasks,
                                                    FrontsDev F, Bufs bufs) {
    __shared__ int32_t rel_i[TS], rel_j[TS];
    const int64_t t = blockIdx.x;
    if (t >= ntasks) return;
    const int e = (int)batch_find(be, nbe, t);
    const int f = be[e].front;
    int ti, tj;
    tri_decode(t - be[e].base, ti, tj);
    const int p = F.parent[f];
    const int nr = F.nr[f], nvp = F.nvpad[f], m = F.m[f], mp = F.m[p];
    const int32_t* rel = F.relmap + F.rptr[f];
    if (threadIdx.x < TS) {
        int a = TS * ti + threadIdx.x;
        rel_i[threadIdx.x] = a < nr ? rel[a] : -1;
    } else if (threadIdx.x < 2 * TS) {
        int b = TS * tj + threadIdx.x - TS;
        rel_j[threadIdx.x - TS] = b < nr ? rel[b] : -1;
    }
    __syncthreads();
    const double* src = bufs.fronts + F.off[f] + nvp + (int64_t)nvp * m;
    double* dst = bufs.fronts + F.off[p];
    const int r = threadIdx.x & 63;
    const int a = TS * ti + r;
    if (rel_i[r] < 0) return;
    for (int q = threadIdx.x >> 6; q < TS; q += 4) {
        const int b = TS * tj + q;
        if (rel_j[q] < 0 || b > a) continue;
        double* d = dst + rel_i[r] + (int64_t)rel_j[q] * mp;
        if (ATOMIC) atomicAdd(d, src[a + (int64_t)b * m]);
        else *d += src[a + (int64_t)b * m];
    }
}

__global__ __launch_bounds__(256) void k_sigma_gather(const BatchEnt* __restrict__ be, int nbe, int64_t ntasks,
                                                      FrontsDev F, Bufs bufs) {
    __shared__ int32_t rel_i[TS], rel_j[TS];
    const int64_t t = blockIdx.x;
    if (t >= ntasks) return;
    const int e = (int)batch_find(be, nbe, t);
    const int f = be[e].front;
    int ti, tj;
    tri_decode(t - be[e].base, ti, tj);
    const int p = F.parent[f];
    const int nr = F.nr[f], nvp = F.nvpad[f], m = F.m[f], mp = F.m[p];
    const int32_t* rel = F.relmap + F.rptr[f];
    if (threadIdx.x < TS) {
        int a = TS * ti + threadIdx.x;
        rel_i[threadIdx.x] = a < nr ? rel[a] : -1;
    } else if (threadIdx.x < 2 * TS) {
        int b = TS * tj + threadIdx.x - TS;
        rel_j[threadIdx.x - TS] = b < nr ? rel[b] : -1;
    }
    __syncthreads();
    double* dst = bufs.fronts + F.off[f] + nvp + (int64_t)nvp * m;
    const double* src = bufs.fronts + F.off[p];
    const int r = threadIdx.x & 63;
    const int a = TS * ti + r;
    for (int q = threadIdx.x >> 6; q < TS; q += 4) {
        const int b = TS * tj + q;
        double v = 0.0;
        if (rel_i[r] >= 0 && rel_j[q] >= 0) {
            int ra = rel_i[r], rb = rel_j[q];
            v = (ra >= rb) ? src[ra + (int64_t)rb * mp] : src[rb + (int64_t)ra * mp];
        }
        if (ti == tj) {
            if (b <= a) { dst[a + (int64_t)b * m] = v; dst[b + (int64_t)a * m] = v; }
        } else {
            dst[a + (int64_t)b * m] = v;
        }
    }
}

void launch_extend_add(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, FrontsDev F, Bufs b) {
    if (ntasks <= 0) return;
    hipLaunchKernelGGL(k_extend_add<true>, dim3((unsigned)ntasks), dim3(256), 0, st, be, nbe, ntasks, F, b);
}
void launch_extend_add_plain(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, FrontsDev F, Bufs b) {
    if (ntasks <= 0) return;
    hipLaunchKernelGGL(k_extend_add<false>, dim3((unsigned)ntasks), dim3(256), 0, st, be, nbe, ntasks, F, b);
}
// one block per lower tile (ti >= tj) of a front; 16-byte stores down the columns
__global__ __launch_bounds__(256) void k_zero_lower(const BatchEnt* __restrict__ be, int nbe, int64_t ntasks,
                                                    FrontsDev F, double* fronts) {
    const int64_t t = blockIdx.x;
    if (t >= ntasks) return;
    const int e = (int)batch_find(be, nbe, t);
    const int f = be[e].front;
    int ti, tj;
    tri_decode(t - be[e].base, ti, tj);
    const int64_t m = F.m[f];
    double* base = fronts + F.off[f] + (int64_t)TS * ti + (int64_t)TS * tj * m;
    const int r2 = (threadIdx.x & 31) * 2, c0 = threadIdx.x >> 5;
#pragma unroll
    for (int c = c0; c < TS; c += 8) *(double2*)(base + r2 + (int64_t)c * m) = make_double2(0.0, 0.0);
}
void launch_zero_lower(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, FrontsDev F, double* fronts) {
    if (ntasks <= 0) return;
    hipLaunchKernelGGL(k_zero_lower, dim3((unsigned)ntasks), dim3(256), 0, st, be, nbe, ntasks, F, fronts);
}

void launch_sigma_gather(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, FrontsDev F, Bufs b) {
    if (ntasks <= 0) return;
    hipLaunchKernelGGL(k_sigma_gather, dim3((unsigned)ntasks), dim3(256), 0, st, be, nbe, ntasks, F, b);
}

// ---------------------------------------------------------------------------
// Triangular solves with the fronts.  Vectors are in the new node order.
//   forward : z_V = X y_V ; y_R -= L21 z_V ; y_V = z_V
//   backward: t_V = y_V - L21^T x_R ; x_V = X^T t_V
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fwd_xv(const BatchEnt* __restrict__ be, int nbe, int64_t ntasks,
                                                FrontsDev F, Bufs bufs, const double* __restrict__ y,
                                                double* __restrict__ tout) {
    __shared__ double v[TS];
    __shared__ double part[4][TS];
    const int64_t t = blockIdx.x;
    if (t >= ntasks) return;
    const int e = (int)batch_find(be, nbe, t);
    const int f = be[e].front;
    const int i = (int)(t - be[e].base);
    const int nv = F.nv[f], ldx = F.nvpad[f];
    const int64_t first = F.first[f];
    const double* Xb = bufs.X + F.xoff[f];
    const int r = threadIdx.x & 63, cg = threadIdx.x >> 6;
    double acc = 0.0;
    for (int k = 0; k <= i; k++) {
        __syncthreads();
        if (threadIdx.x < TS) {
            int l = TS * k + threadIdx.x;
            v[threadIdx.x] = l < nv ? y[first + l] : 0.0;
        }
        __syncthreads();
        const double* T = Xb + (int64_t)TS * i + (int64_t)TS * k * ldx;
#pragma unroll
        for (int c = 0; c < 16; c++) acc += T[r + (int64_t)(cg * 16 + c) * ldx] * v[cg * 16 + c];
    }
    part[cg][r] = acc;
    __syncthreads();
    if (threadIdx.x < TS) {
        int l = TS * i + threadIdx.x;
        double s = part[0][threadIdx.x] + part[1][threadIdx.x] + part[2][threadIdx.x] + part[3][threadIdx.x];
        if (l < nv) tout[first + l] = s;
    }
}

// y[update rows] -= L21 z; with stage, the products go to stage[rptr + row]
// instead (no atomics) and k_gather_sub applies them in a fixed order
template <typename LT>
__global__ __launch_bounds__(256) void k_fwd_r(const BatchEnt* __restrict__ be, int nbe, int64_t ntasks,
                                               FrontsDev F, const LT* __restrict__ Lbuf, const double* __restrict__ z,
                                               double* __restrict__ y, double* __restrict__ stage) {
    __shared__ double v[TS];
    __shared__ double part[4][TS];
    const int64_t t = blockIdx.x;
    if (t >= ntasks) return;
    const int e = (int)batch_find(be, nbe, t);
    const int f = be[e].front;
    const int i = (int)(t - be[e].base);
    const int nv = F.nv[f], nvp = F.nvpad[f], m = F.m[f], nr = F.nr[f];
    const int64_t first = F.first[f];
    const LT* base = Lbuf + F.off[f];
    const int r = threadIdx.x & 63, cg = threadIdx.x >> 6;
    double acc = 0.0;
    const int P = nvp / TS;
    for (int k = 0; k < P; k++) {
        __syncthreads();
        if (threadIdx.x < TS) {
            int l = TS * k + threadIdx.x;
            v[threadIdx.x] = l < nv ? z[first + l] : 0.0;
        }
        __syncthreads();
        const LT* T = base + nvp + (int64_t)TS * i + (int64_t)TS * k * m;
#pragma unroll
        for (int c = 0; c < 16; c++) acc += (double)T[r + (int64_t)(cg * 16 + c) * m] * v[cg * 16 + c];
    }
    part[cg][r] = acc;
    __syncthreads();
    if (threadIdx.x < TS) {
        int a = TS * i + threadIdx.x;
        double s = part[0][threadIdx.x] + part[1][threadIdx.x] + part[2][threadIdx.x] + part[3][threadIdx.x];
        if (a < nr) {
            if (stage) stage[F.rptr[f] + a] = s;
            else atomicAdd(y + F.rrows[F.rptr[f] + a], -s);
        }
    }
}

// y[tgt[i]] -= sum over e in [tptr[i], tptr[i+1]) of stage[src[e]], in that order
__global__ void k_gather_sub(const int32_t* __restrict__ tgt, const int64_t* __restrict__ tptr,
                             const int64_t* __restrict__ src, int64_t n, const double* __restrict__ stage,
                             double* __restrict__ y) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double v = y[tgt[i]];
        for (int64_t e = tptr[i]; e < tptr[i + 1]; e++) v -= stage[src[e]];
        y[tgt[i]] = v;
    }
}

__global__ void k_copy_v(const int32_t* __restrict__ flist, FrontsDev F, const double* __restrict__ src,
                         double* __restrict__ dst) {
    const int f = flist[blockIdx.x];
    const int64_t first = F.first[f];
    for (int l = threadIdx.x; l < F.nv[f]; l += blockDim.x) dst[first + l] = src[first + l];
}

// transposed tile-vector product through LDS: out[c] += sum_r T[r][c] v[r]
template <typename LT>
__device__ __forceinline__ void tgemv_tile(double* sT, const LT* T, int64_t ld, const double* v, double& acc) {
    const int tid = threadIdx.x;
    __syncthreads();
    {
        const int r = tid & 63;
#pragma unroll
        for (int q = 0; q < 16; q++) {
            int c = (tid >> 6) + 4 * q;
            sT[c * LDP + r] = (double)T[r + (int64_t)c * ld];
        }
    }
    __syncthreads();
    const int c = tid & 63, rg = tid >> 6;
#pragma unroll
    for (int q = 0; q < 16; q++) acc += sT[c * LDP + rg * 16 + q] * v[rg * 16 + q];
}

template <typename LT>
__global__ __launch_bounds__(256) void k_bwd_t(const BatchEnt* __restrict__ be, int nbe, int64_t ntasks,
                                               FrontsDev F, const LT* __restrict__ Lbuf, const double* __restrict__ y,
                                               const double* __restrict__ x, double* __restrict__ tout) {
    __shared__ double sT[TS * LDP];
    __shared__ double v[TS];
    __shared__ double part[4][TS];
    const int64_t t = blockIdx.x;
    if (t >= ntasks) return;
    const int e = (int)batch_find(be, nbe, t);
    const int f = be[e].front;
    const int k = (int)(t - be[e].base);
    const int nv = F.nv[f], nvp = F.nvpad[f], m = F.m[f], nr = F.nr[f];
    const int64_t first = F.first[f];
    const LT* base = Lbuf + F.off[f];
    const int32_t* rows = F.rrows + F.rptr[f];
    const int MR = (nr + TS - 1) / TS;
    double acc = 0.0;
    for (int i = 0; i < MR; i++) {
        __syncthreads();
        if (threadIdx.x < TS) {
            int a = TS * i + threadIdx.x;
            v[threadIdx.x] = a < nr ? x[rows[a]] : 0.0;
        }
        tgemv_tile(sT, base + nvp + (int64_t)TS * i + (int64_t)TS * k * m, m, v, acc);
    }
    const int c = threadIdx.x & 63, rg = threadIdx.x >> 6;
    __syncthreads();
    part[rg][c] = acc;
    __syncthreads();
    if (threadIdx.x < TS) {
        int l = TS * k + threadIdx.x;
        double s = part[0][threadIdx.x] + part[1][threadIdx.x] + part[2][threadIdx.x] + part[3][threadIdx.x];
        if (l < nv) tout[first + l] = y[first + l] - s;
    }
}

__global__ __launch_bounds__(256) void k_bwd_x(const BatchEnt* __restrict__ be, int nbe, int64_t ntasks,
                                               FrontsDev F, Bufs bufs, const double* __restrict__ tin,
                                               double* __restrict__ x) {
    __shared__ double sT[TS * LDP];
    __shared__ double v[TS];
    __shared__ double part[4][TS];
    const int64_t t = blockIdx.x;
    if (t >= ntasks) return;
    const int e = (int)batch_find(be, nbe, t);
    const int f = be[e].front;
    const int k = (int)(t - be[e].base);
    const int nv = F.nv[f], nvp = F.nvpad[f];
    const int64_t first = F.first[f];
    const double* Xb = bufs.X + F.xoff[f];
    const int P = nvp / TS;
    double acc = 0.0;
    for (int i = k; i < P; i++) {
        __syncthreads();
        if (threadIdx.x < TS) {
            int l = TS * i + threadIdx.x;
            v[threadIdx.x] = l < nv ? tin[first + l] : 0.0;
        }
        tgemv_tile(sT, Xb + (int64_t)TS * i + (int64_t)TS * k * nvp, nvp, v, acc);
    }
    const int c = threadIdx.x & 63, rg = threadIdx.x >> 6;
    __syncthreads();
    part[rg][c] = acc;
    __syncthreads();
    if (threadIdx.x < TS) {
        int l = TS * k + threadIdx.x;
        double s = part[0][threadIdx.x] + part[1][threadIdx.x] + part[2][threadIdx.x] + part[3][threadIdx.x];
        if (l < nv) x[first + l] = s;
    }
}

void launch_fwd_xv(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, FrontsDev F, Bufs b,
                   const double* y, double* t) {
    if (ntasks <= 0) return;
    hipLaunchKernelGGL(k_fwd_xv, dim3((unsigned)ntasks), dim3(256), 0, st, be, nbe, ntasks, F, b, y, t);
}
void launch_fwd_r(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, FrontsDev F, Bufs b,
                  const double* t, double* y, double* stage) {
    if (ntasks <= 0) return;
    if (b.F32)
        hipLaunchKernelGGL(k_fwd_r<float>, dim3((unsigned)ntasks), dim3(256), 0, st, be, nbe, ntasks, F,
                           (const float*)b.F32, t, y, (double*)nullptr);
    else
        hipLaunchKernelGGL(k_fwd_r<double>, dim3((unsigned)ntasks), dim3(256), 0, st, be, nbe, ntasks, F,
                           (const double*)b.fronts, t, y, stage);
}

void launch_gather_sub(hipStream_t st, const int32_t* tgt, const int64_t* tptr, const int64_t* src, int64_t n,
                       const double* stage, double* y) {
    if (n <= 0) return;
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_gather_sub, dim3(blocks), dim3(256), 0, st, tgt, tptr, src, n, stage, y);
}
void launch_copy_v(hipStream_t st, const int32_t* flist, int nf, FrontsDev F, const double* t, double* y) {
    if (nf <= 0) return;
    hipLaunchKernelGGL(k_copy_v, dim3(nf), dim3(256), 0, st, flist, F, t, y);
}
void launch_bwd_t(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, FrontsDev F, Bufs b,
                  const double* y, const double* x, double* t) {
    if (ntasks <= 0) return;
    if (b.F32)
        hipLaunchKernelGGL(k_bwd_t<float>, dim3((unsigned)ntasks), dim3(256), 0, st, be, nbe, ntasks, F,
                           (const float*)b.F32, y, x, t);
    else
        hipLaunchKernelGGL(k_bwd_t<double>, dim3((unsigned)ntasks), dim3(256), 0, st, be, nbe, ntasks, F,
                           (const double*)b.fronts, y, x, t);
}
void launch_bwd_x(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, FrontsDev F, Bufs b,
                  const double* t, double* x) {
    if (ntasks <= 0) return;
    hipLaunchKernelGGL(k_bwd_x, dim3((unsigned)ntasks), dim3(256), 0, st, be, nbe, ntasks, F, b, t, x);
}

// ---------------------------------------------------------------------------
// Elementwise helpers
// ---------------------------------------------------------------------------
__global__ void k_fill(double* p, int64_t n, double v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_scatter_set(double* base, const int64_t* dest, const double* val, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        base[dest[i]] = val[i];
}
__global__ void k_scatter_const(double* base, const int64_t* dest, int64_t n, double v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        base[dest[i]] = v;
}
__global__ void k_gather_perm(const int32_t* perm, const double* src, double* dst, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[perm[i]];
}
__global__ void k_scatter_perm(const int32_t* perm, const double* src, double* dst, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[perm[i]] = src[i];
}
__global__ void k_diag(const int32_t* perm, const int32_t* snode, FrontsDev F, const double* fronts, double* var,
                       int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int f = snode[i];
        int64_t l = i - F.first[f];
        var[perm[i]] = fronts[F.off[f] + l + l * (int64_t)F.m[f]];
    }
}

static unsigned grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (unsigned)g;
}
void launch_fill(hipStream_t st, double* p, int64_t n, double v) {
    if (n > 0) hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(256), 0, st, p, n, v);
}
void launch_scatter_set(hipStream_t st, double* base, const int64_t* dest, const double* val, int64_t n) {
    if (n > 0) hipLaunchKernelGGL(k_scatter_set, dim3(grid_for(n)), dim3(256), 0, st, base, dest, val, n);
}
void launch_scatter_const(hipStream_t st, double* base, const int64_t* dest, int64_t n, double v) {
    if (n > 0) hipLaunchKernelGGL(k_scatter_const, dim3(grid_for(n)), dim3(256), 0, st, base, dest, n, v);
}
void launch_gather_perm(hipStream_t st, const int32_t* perm, const double* src, double* dst, int64_t n) {
    if (n > 0) hipLaunchKernelGGL(k_gather_perm, dim3(grid_for(n)), dim3(256), 0, st, perm, src, dst, n);
}
void launch_scatter_perm(hipStream_t st, const int32_t* perm, const double* src, double* dst, int64_t n) {
    if (n > 0) hipLaunchKernelGGL(k_scatter_perm, dim3(grid_for(n)), dim3(256), 0, st, perm, src, dst, n);
}
void launch_diag(hipStream_t st, const int32_t* perm, const int32_t* snode, FrontsDev F, const double* fronts,
                 double* var, int64_t n) {
    if (n > 0) hipLaunchKernelGGL(k_diag, dim3(grid_for(n)), dim3(256), 0, st, perm, snode, F, fronts, var, n);
}

// ---------------------------------------------------------------------------
// Line-of-sight linearisation, one wavefront per star.
//   A_n = sum_t w_t exp(F(s_t)), s_t = o + (t/T)(x_n - o), trapezoid weights
//   g_n = d ln A_n / d f over the support, c_n = ln A_n - g_n . f
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_los(GridDev g, StarsDev s, const double* __restrict__ f, int cap) {
    extern __shared__ char smem[];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int32_t* snodes = (int32_t*)(smem) + w * cap;
    double* sg = (double*)(smem + (size_t)4 * cap * sizeof(int32_t)) + w * cap;
    const int64_t star = (int64_t)blockIdx.x * 4 + w;
    const bool active = star < s.n;
    int64_t p0 = 0;
    int cnt = 0;
    if (active) {
        p0 = s.ptr[star];
        cnt = (int)(s.ptr[star + 1] - p0);
        for (int k = lane; k < cnt; k += 64) { snodes[k] = s.nodes[p0 + k]; sg[k] = 0.0; }
    }
    __syncthreads();
    double Asum = 0.0;
    if (active) {
        const double dx = s.xyz[3 * star] - g.ox, dy = s.xyz[3 * star + 1] - g.oy, dz = s.xyz[3 * star + 2] - g.oz;
        const int T = s.nsamp[star];
        const double d = sqrt(dx * dx + dy * dy + dz * dz);
        const double delta = d / (double)T;
        const int n = g.n;
        for (int t = lane; t <= T; t += 64) {
            const double fr = (double)t / (double)T;
            double p[3] = {g.ox + fr * dx, g.oy + fr * dy, g.oz + fr * dz};
            int cc[3];
            double wv[3];
#pragma unroll
            for (int a = 0; a < 3; a++) {
                double c = floor(p[a] / g.h);
                c = c < 0 ? 0 : (c > n - 2 ? n - 2 : c);
                cc[a] = (int)c;
                wv[a] = p[a] / g.h - c;
            }
            double phi[8];
            int nd[8];
            double F = 0.0;
#pragma unroll
            for (int c8 = 0; c8 < 8; c8++) {
                int bi = c8 & 1, bj = (c8 >> 1) & 1, bk = (c8 >> 2) & 1;
                phi[c8] = (bi ? wv[0] : 1.0 - wv[0]) * (bj ? wv[1] : 1.0 - wv[1]) * (bk ? wv[2] : 1.0 - wv[2]);
                nd[c8] = (cc[0] + bi) + n * ((cc[1] + bj) + n * (cc[2] + bk));
                F += phi[c8] * f[nd[c8]];
            }
            const double wt = (t == 0 || t == T) ? 0.5 * delta : delta;
            const double ev = wt * exp(F);
            Asum += ev;
#pragma unroll
            for (int c8 = 0; c8 < 8; c8++) {
                int lo = 0, hi = cnt - 1;
                while (lo < hi) {
                    int mid = (lo + hi) >> 1;
                    if (snodes[mid] < nd[c8]) lo = mid + 1; else hi = mid;
                }
                atomicAdd(&sg[lo], ev * phi[c8]);
            }
        }
    }
    const double A = wave_sum(Asum);
    __syncthreads();
    if (!active) return;
    const double iA = 1.0 / A;
    double gf = 0.0;
    for (int k = lane; k < cnt; k += 64) {
        double gv = sg[k] * iA;
        s.g[p0 + k] = gv;
        gf += gv * f[snodes[k]];
    }
    gf = wave_sum(gf);
    if (lane == 0) {
        s.lnA[star] = log(A);
        s.c[star] = log(A) - gf;
    }
}

void launch_los(hipStream_t st, GridDev g, StarsDev s, const double* f, int cap) {
    if (s.n <= 0) return;
    size_t sh = (size_t)4 * cap * (sizeof(int32_t) + sizeof(double));
    hipLaunchKernelGGL(k_los, dim3((unsigned)((s.n + 3) / 4)), dim3(256), sh, st, g, s, f, cap);
}

// ---------------------------------------------------------------------------
// Assembly of the sites into the fronts: tau_n g_n g_n^T lands in the front
// of the star's first-eliminated support node (its whole clique is there).
// ---------------------------------------------------------------------------
// Clique assembly by tile owner.  Every front tile that star cliques touch
// is assembled by one wave (or, when it has many incidences, by several
// waves whose partial tiles are then summed in order): the wave accumulates
// tau g_a g_b of each of its incidences in a 64 x 64 LDS tile, incidence after
// incidence in star order, and adds the tile to the front once.  No global
// atomics, and every summation order is fixed, so the result is
// reproducible bit for bit.
__global__ void k_sort_g(const int64_t* __restrict__ ptr, const int32_t* __restrict__ sord,
                         const double* __restrict__ g, double* __restrict__ gs, int64_t S) {
    // one wave per star: gs[p0 + k] = g[p0 + sord[p0 + k]]
    const int64_t star = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (star >= S) return;
    const int64_t p0 = ptr[star], p1 = ptr[star + 1];
    for (int64_t q = p0 + (threadIdx.x & 63); q < p1; q += 64) gs[q] = g[p0 + sord[q]];
}

__device__ __forceinline__ int64_t lane_bcast64(int64_t v, int lane) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), lane);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// One incidence's slot data held by the lanes: lane j < nr holds row slot j,
// lane j < nc column slot j.
struct IncData {
    double rg, cg;
    int32_t rl, cl;
};

constexpr int TA_DEPTH = 8;   // incidences whose slot data is in flight ahead of the ones applied

// Order of one wave's LDS accesses: the LDS executes a wave's instructions in
// order, so the compiler only has to keep them in program order (no wait).
__device__ __forceinline__ void wave_order() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_wave_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// One block of four waves per chunk; wave w owns rows 16 w .. 16 w + 15 of
// the tile and runs through all the chunk's incidences, applying only the
// pairs whose row is its own (the rows of an incidence are sorted, so they
// are a contiguous range; a wave with none skips the incidence).  The waves
// share nothing, so no barrier, and each entry's sum runs in incidence order.
__global__ __launch_bounds__(256) void k_assemble_tiles(const TileChunk* __restrict__ ch, const TileInc* __restrict__ inc,
                                                        const int64_t* __restrict__ ptr, const double* __restrict__ tau,
                                                        const double* __restrict__ gs, const int32_t* __restrict__ ls,
                                                        FrontsDev F, double* fronts, double* __restrict__ parts) {
    __shared__ double T[TS * LDP];
    __shared__ double sr_all[4][TS], sc_all[4][TS];
    __shared__ int32_t lr_all[4][TS], lc_all[4][TS];
    const TileChunk C = ch[blockIdx.x];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double* sr = sr_all[w];
    double* sc = sc_all[w];
    int32_t* lr = lr_all[w];
    int32_t* lc = lc_all[w];
    double* Tw = T + 16 * w * LDP;   // this wave's 16 rows
    for (int q = lane; q < 16 * LDP; q += 64) Tw[q] = 0.0;
    const int rb = TS * C.ti, cb = TS * C.tj;
    const bool diag = C.ti == C.tj;
    __shared__ int32_t list_all[4][64];
    int32_t* list = list_all[w];
    for (int64_t e0 = C.i0; e0 < C.i0 + C.n; e0 += 64) {
        const int nbatch = (int)std::min<int64_t>(64, C.i0 + C.n - e0);
        // lane j holds incidence e0 + j; the wave keeps those whose row run
        // reaches its stripe, in order (their positions compacted in LDS)
        const TileInc I0 = inc[e0 + (lane < nbatch ? lane : nbatch - 1)];
        const bool member = lane < nbatch && (I0.rlo >> 4) <= w && w <= (I0.rhi >> 4);
        const uint64_t mm = __ballot(member);
        const int nb = __popcll(mm);
        if (nb == 0) continue;
        wave_order();
        if (member) list[__builtin_amdgcn_mbcnt_hi((uint32_t)(mm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mm, 0))] = lane;
        wave_order();
        const int src = list[lane < nb ? lane : nb - 1];
        const TileInc I = inc[e0 + src];
        const int64_t p0 = ptr[I.star];
        const int64_t rp = p0 + I.r0, cp = p0 + I.c0;
        const int nrc = ((int)I.nr << 16) | (int)I.nc;
        const double t = tau[I.star];
        // loads without branches (indices clamped into the incidence and the
        // batch), so that their waits fall where the data is used
        auto fetch = [&](int j, IncData& D) {
            const int jj = j < nb ? j : nb - 1;
            const int64_t r0 = lane_bcast64(rp, jj), c0 = lane_bcast64(cp, jj);
            const int x = __builtin_amdgcn_readlane(nrc, jj);
            const int nr = x >> 16, nc = x & 0xffff;
            const int ia = lane < nr ? lane : nr - 1, ib = lane < nc ? lane : nc - 1;
            D.rl = ls[r0 + ia] - rb;
            D.rg = gs[r0 + ia];
            D.cl = ls[c0 + ib] - cb;
            D.cg = gs[c0 + ib];
        };
        IncData cur[TA_DEPTH], nxt[TA_DEPTH];
#pragma unroll
        for (int d = 0; d < TA_DEPTH; d++) fetch(d, cur[d]);
        for (int j0 = 0; j0 < nb; j0 += TA_DEPTH) {
#pragma unroll
            for (int d = 0; d < TA_DEPTH; d++) fetch(j0 + TA_DEPTH + d, nxt[d]);
#pragma unroll
            for (int d = 0; d < TA_DEPTH; d++) {
                const int j = j0 + d;
                if (j >= nb) break;
                const double tj = lane_bcast(t, j);
                const int x = __builtin_amdgcn_readlane(nrc, j);
                const int nr = x >> 16, nc = x & 0xffff;
                // this wave's rows of the incidence: a contiguous range
                const uint64_t mine = __ballot(lane < nr && (cur[d].rl >> 4) == w);
                if (tj == 0.0 || mine == 0) continue;
                const int a_lo = __ffsll((unsigned long long)mine) - 1, na = __popcll(mine);
                // stage the slots (the previous incidence's reads of the
                // staging arrays precede these writes in this wave's LDS order)
                wave_order();
                lr[lane] = cur[d].rl;
                sr[lane] = tj * cur[d].rg;
                lc[lane] = cur[d].cl;
                sc[lane] = cur[d].cg;
                wave_order();
                // the na x nc (row slot, column slot) pairs dealt to the lanes
                // row after row, 64 at a time (pair k: row k / nc, column
                // k mod nc; the quotient from a float product, exact since
                // k < 1024 keeps (k + 1/2) / nc at least 1/128 from an
                // integer); within one incidence every pair is a different tile
                // entry.  LDS adds without return: the wave does not wait for
                // them, and the LDS applies one wave's instructions in order
                const int npair = na * nc;
                const float inv_nc = 1.0f / (float)nc;
                for (int k = lane; k < npair; k += 64) {
                    const int ai = (int)(((float)k + 0.5f) * inv_nc);
                    const int a = a_lo + ai, b = k - ai * nc;
                    if (!diag || a >= b) atomicAdd(&T[lr[a] * LDP + lc[b]], sr[a] * sc[b]);
                }
            }
#pragma unroll
            for (int d = 0; d < TA_DEPTH; d++) cur[d] = nxt[d];
        }
    }
    wave_order();
    // this wave's 16 rows: lane = (column mod 4) x 16 + row
    const int r = 16 * w + (lane & 15);
    if (C.part < 0) {
        const int64_t m = F.m[C.f];
        double* dst = fronts + F.off[C.f] + rb + (int64_t)cb * m;
        // the 16 front entries loaded before the first store (the compiler
        // cannot tell the columns apart and would wait out each one in turn)
        double v[TS / 4];
#pragma unroll
        for (int i = 0; i < TS / 4; i++) v[i] = dst[r + (int64_t)((lane >> 4) + 4 * i) * m];
#pragma unroll
        for (int i = 0; i < TS / 4; i++) {
            const int c = (lane >> 4) + 4 * i;
            dst[r + (int64_t)c * m] = v[i] + T[r * LDP + c];
        }
    } else {
        double* dst = parts + (int64_t)C.part * TS * TS;
#pragma unroll 4
        for (int c = lane >> 4; c < TS; c += 4) dst[r + c * TS] = T[r * LDP + c];
    }
}

// Tiles assembled in several chunks: their partial tiles summed in chunk
// order and added to the front (one wave per tile, lane = tile row).
__global__ __launch_bounds__(64) void k_tiles_reduce(const TileRed* __restrict__ red, const double* __restrict__ parts,
                                                     FrontsDev F, double* fronts) {
    const TileRed R = red[blockIdx.x];
    const int lane = threadIdx.x;
    const int64_t m = F.m[R.f];
    double* dst = fronts + F.off[R.f] + TS * R.ti + (int64_t)TS * R.tj * m;
    // eight columns at a time, every load of them ahead of their stores
    for (int c0 = 0; c0 < TS; c0 += 8) {
        double d[8], v[8];
#pragma unroll
        for (int u = 0; u < 8; u++) {
            d[u] = dst[lane + (int64_t)(c0 + u) * m];
            v[u] = 0.0;
        }
        for (int q = 0; q < R.np; q++) {
            const double* pp = parts + (int64_t)(R.p0 + q) * TS * TS + lane + c0 * TS;
#pragma unroll
            for (int u = 0; u < 8; u++) v[u] += pp[u * TS];
        }
#pragma unroll
        for (int u = 0; u < 8; u++) dst[lane + (int64_t)(c0 + u) * m] = d[u] + v[u];
    }
}

void launch_sort_g(hipStream_t st, StarsDev s, double* gs, int64_t nslots) {
    (void)nslots;
    if (s.n <= 0) return;
    hipLaunchKernelGGL(k_sort_g, dim3((unsigned)((s.n + 3) / 4)), dim3(256), 0, st, s.ptr, s.sord, s.g, gs, s.n);
}
void launch_assemble_tiles(hipStream_t st, const TileChunk* ch, int64_t nch, const TileInc* inc, const int64_t* ptr,
                           const double* tau, const double* gs, const int32_t* ls, FrontsDev F, double* fronts,
                           double* parts) {
    if (nch <= 0) return;
    hipLaunchKernelGGL(k_assemble_tiles, dim3((unsigned)nch), dim3(256), 0, st, ch, inc, ptr, tau, gs, ls, F, fronts,
                       parts);
}
void launch_tiles_reduce(hipStream_t st, const TileRed* red, int64_t nred, const double* parts, FrontsDev F,
                         double* fronts) {
    if (nred <= 0) return;
    hipLaunchKernelGGL(k_tiles_reduce, dim3((unsigned)nred), dim3(64), 0, st, red, parts, F, fronts);
}

__global__ void k_assemble_b(StarsDev s, double* b) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t star = star_of_slot(s, (int64_t)blockIdx.x * 4 + w);
    if (star < 0) return;
    const double coef = s.nu[star] - s.tau[star] * s.c[star];
    if (coef == 0.0) return;
    const int64_t p0 = s.ptr[star];
    const int cnt = (int)(s.ptr[star + 1] - p0);
    for (int k = lane; k < cnt; k += 64) atomicAdd(b + s.nodes[p0 + k], coef * s.g[p0 + k]);
}

// Deterministic right-hand side: b[node] += sum over the node's slots (in
// star order) of (nu - tau c) g, one wave per node: lane l sums the slots
// l, l + 64, ... in order, then a fixed butterfly adds the lanes.  (The
// nodes next to the observer lie on every sightline.)
__global__ __launch_bounds__(256) void k_assemble_b_nodes(StarsDev s, const int64_t* __restrict__ nptr,
                                                          const int64_t* __restrict__ nslot,
                                                          const int32_t* __restrict__ nstar, double* b, int64_t N) {
    const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= N) return;
    const int lane = threadIdx.x & 63;
    double v = 0.0;
    for (int64_t e = nptr[p] + lane; e < nptr[p + 1]; e += 64) {
        const int32_t star = nstar[e];
        v += (s.nu[star] - s.tau[star] * s.c[star]) * s.g[nslot[e]];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) b[p] += v;
}

void launch_assemble_b_nodes(hipStream_t st, StarsDev s, const int64_t* nptr, const int64_t* nslot,
                             const int32_t* nstar, double* b, int64_t N) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_assemble_b_nodes, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, st, s, nptr, nslot, nstar, b,
                       N);
}

void launch_assemble_b(hipStream_t st, StarsDev s, double* b) {
    if (s.n <= 0) return;
    hipLaunchKernelGGL(k_assemble_b, dim3(star_blocks(s)), dim3(256), 0, st, s, b);
}

// ---------------------------------------------------------------------------
// Cavity: q-marginal of a_n = c_n + g_n . f: mean c_n + g_n . mu and variance
// g_n^T Sigma g_n, all pairs read from the star's front (lower triangle).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_cavity(StarsDev s, FrontsDev F, const double* __restrict__ fronts,
                                                const double* __restrict__ mu, int cap) {
    extern __shared__ char smem[];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int32_t* sl = (int32_t*)smem + w * cap;
    double* sg = (double*)(smem + (size_t)4 * cap * sizeof(int32_t)) + w * cap;
    const int64_t star = star_of_slot(s, (int64_t)blockIdx.x * 4 + w);
    const bool active = star >= 0;
    int64_t p0 = 0;
    int cnt = 0;
    double mean = 0.0;
    if (active) {
        p0 = s.ptr[star];
        cnt = (int)(s.ptr[star + 1] - p0);
        for (int k = lane; k < cnt; k += 64) {
            int slot = s.sord[p0 + k];
            sl[k] = s.loc[p0 + slot];
            double gv = s.g[p0 + slot];
            sg[k] = gv;
            mean += gv * mu[s.nodes[p0 + slot]];
        }
    }
    __syncthreads();
    if (!active) return;
    const int f = s.front[star];
    const double* base = fronts + F.off[f];
    const int64_t m = F.m[f];
    double acc = 0.0;
    for (int b = 0; b < cnt; b++) {
        const double* col = base + (int64_t)sl[b] * m;
        double part = 0.0;
        for (int a = b + lane; a < cnt; a += 64) part += (a == b ? 1.0 : 2.0) * sg[a] * col[sl[a]];
        acc += part * sg[b];
    }
    acc = wave_sum(acc);
    mean = wave_sum(mean);
    if (lane == 0) {
        s.cav_mu[star] = s.c[star] + mean;
        s.cav_var[star] = acc;
    }
}

void launch_cavity(hipStream_t st, StarsDev s, FrontsDev F, const double* fronts, const double* mu, int cap) {
    if (s.n <= 0) return;
    size_t sh = (size_t)4 * cap * (sizeof(int32_t) + sizeof(double));
    hipLaunchKernelGGL(k_cavity, dim3(star_blocks(s)), dim3(256), sh, st, s, F, fronts, mu, cap);
}

// ---------------------------------------------------------------------------
// Tilted moments of N(a; mu, v) N(A; e^a, s^2), one wavefront per star.
//
// The log-integrand l(a) has at most two local maxima: its inflection points
// solve 2y^2 - A y + s^2/v = 0 (y = e^a) and split the line into pieces
// where l' is monotone.  Each side of each maximum is cut where l falls
// 1, 2, 4, 8, 12, ..., 32, 40, 50, 60 below that maximum (one bisection per
// lane), and every piece gets a 16-point Gauss-Legendre rule; a piece between
// two maxima ends at the local minimum.
// ---------------------------------------------------------------------------
__constant__ double c_glx[16];
__constant__ double c_glw[16];
__constant__ double c_depth[13] = {1, 2, 4, 8, 12, 16, 20, 24, 28, 32, 40, 50, 60};

struct TiltP {
    double mu, v, A, s2;
};
__device__ __forceinline__ double t_ell(const TiltP& t, double a) {
    double y = exp(a), r = t.A - y;
    return -(a - t.mu) * (a - t.mu) / (2.0 * t.v) - r * r / (2.0 * t.s2);
}
__device__ __forceinline__ double t_d1(const TiltP& t, double a) {
    double y = exp(a);
    return -(a - t.mu) / t.v + (t.A - y) * y / t.s2;
}
__device__ __forceinline__ double t_d2(const TiltP& t, double a) {
    double y = exp(a);
    return -1.0 / t.v + (t.A * y - 2.0 * y * y) / t.s2;
}
// zero of l' on [lo, hi] (l' changes sign), bisection to full precision
__device__ __forceinline__ double t_root(const TiltP& t, double lo, double hi) {
    double flo = t_d1(t, lo);
    for (int it = 0; it < 200; it++) {
        double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        double fm = t_d1(t, mid);
        if (fm == 0.0) return mid;
        if ((fm > 0.0) == (flo > 0.0)) { lo = mid; flo = fm; } else hi = mid;
    }
    return 0.5 * (lo + hi);
}

// Computes (lnZ, mean, var) with all 64 lanes of the calling wave.
__device__ void tilted_wave(const TiltP& t, double* sb, double& lnZ, double& mean, double& var) {
    const int lane = threadIdx.x & 63;
    double maxima[2] = {t.mu, t.mu};
    int nmax = 0;
    double amin = 0.0;
    bool bimodal = false;
    const double disc = t.A * t.A - 8.0 * t.s2 / t.v;
    if (t.A > 0.0 && disc > 0.0) {
        double y1 = 0.25 * (t.A - sqrt(disc)), y2 = 0.25 * (t.A + sqrt(disc));
        double a1 = log(y1), a2 = log(y2);
        double d1a = t_d1(t, a1), d1b = t_d1(t, a2);
        if (d1a < 0.0) {
            double step = 1.0, lo = a1 - step;
            for (int it = 0; it < 200 && !(t_d1(t, lo) > 0.0); it++) { step *= 2.0; lo = a1 - step; }
            maxima[nmax++] = t_root(t, lo, a1);
        }
        if (d1b > 0.0) {
            double step = 1.0, hi = a2 + step;
            for (int it = 0; it < 200 && !(t_d1(t, hi) < 0.0); it++) { step *= 2.0; hi = a2 + step; }
            maxima[nmax++] = t_root(t, a2, hi);
        }
        if (d1a < 0.0 && d1b > 0.0) { amin = t_root(t, a1, a2); bimodal = true; }
    } else {
        double step = 1.0, lo = t.mu - step, hi = t.mu + step;
        for (int it = 0; it < 200 && !(t_d1(t, lo) > 0.0); it++) { step *= 2.0; lo = t.mu - step; }
        step = 1.0;
        for (int it = 0; it < 200 && !(t_d1(t, hi) < 0.0); it++) { step *= 2.0; hi = t.mu + step; }
        maxima[nmax++] = t_root(t, lo, hi);
    }
    if (nmax == 0) { maxima[0] = t.mu; nmax = 1; }
    const double l0 = t_ell(t, maxima[0]), l1 = t_ell(t, maxima[nmax - 1]);
    const double astar = (nmax == 2 && l1 > l0) ? maxima[1] : maxima[0];
    const double lmax = (nmax == 2 && l1 > l0) ? l1 : l0;
    // segment ends: outer tails where l drops 60 below the adjacent maximum
    double sL = 1.0 / sqrt(-t_d2(t, maxima[0]));
    double sR = 1.0 / sqrt(-t_d2(t, maxima[nmax - 1]));
    if (!isfinite(sL) || sL <= 0.0) sL = sqrt(t.v);
    if (!isfinite(sR) || sR <= 0.0) sR = sqrt(t.v);
    double Lend = maxima[0] - sL, Uend = maxima[nmax - 1] + sR;
    {
        double st = sL;
        for (int it = 0; it < 200 && t_ell(t, Lend) - l0 > -60.0; it++) { st *= 2.0; Lend = maxima[0] - st; }
        st = sR;
        for (int it = 0; it < 200 && t_ell(t, Uend) - l1 > -60.0; it++) { st *= 2.0; Uend = maxima[nmax - 1] + st; }
    }
    // four segments: (anchor, far end, anchor level); unused ones are empty
    // 0: left of the first maximum, 1: right of the last maximum,
    // 2: first maximum -> local minimum, 3: last maximum -> local minimum
    const int seg = lane / 13, di = lane % 13;
    if (lane < 52) {
        double anc, end, lv;
        bool live = true;
        if (seg == 0) { anc = maxima[0]; end = Lend; lv = l0; }
        else if (seg == 1) { anc = maxima[nmax - 1]; end = Uend; lv = l1; }
        else if (seg == 2) { anc = maxima[0]; end = amin; lv = l0; live = bimodal; }
        else { anc = maxima[nmax - 1]; end = amin; lv = l1; live = bimodal; }
        double bpt = anc;
        if (live) {
            const double target = lv - c_depth[di];
            if (di == 12 || !(t_ell(t, end) < target)) {
                bpt = end;   // the segment ends before this depth
            } else {
                double lo = anc, hi = end;   // l(lo) > target >= l(hi)
                for (int it = 0; it < 200; it++) {
                    double mid = 0.5 * (lo + hi);
                    if (mid == lo || mid == hi) break;
                    if (t_ell(t, mid) > target) lo = mid; else hi = mid;
                }
                bpt = 0.5 * (lo + hi);
            }
        }
        sb[lane] = bpt;
        if (di == 0) sb[64 + seg] = live ? anc : bpt;   // segment start
    }
    __syncthreads();
    // 52 panels x 16 nodes
    double I0 = 0.0, I1 = 0.0, I2 = 0.0;
    for (int idx = lane; idx < 52 * 16; idx += 64) {
        const int pnl = idx >> 4, q = idx & 15;
        const int sg = pnl / 13, dk = pnl % 13;
        const double a0 = (dk == 0) ? sb[64 + sg] : sb[sg * 13 + dk - 1];
        const double a1 = sb[sg * 13 + dk];
        const double hw = 0.5 * (a1 - a0);
        if (hw == 0.0) continue;
        const double a = 0.5 * (a0 + a1) + hw * c_glx[q];
        const double e = fabs(hw) * c_glw[q] * exp(t_ell(t, a) - lmax);
        const double u = a - astar;
        I0 += e;
        I1 += e * u;
        I2 += e * u * u;
    }
    I0 = wave_sum(I0);
    I1 = wave_sum(I1);
    I2 = wave_sum(I2);
    const double m1 = I1 / I0;
    mean = astar + m1;
    var = I2 / I0 - m1 * m1;
    const double twopi = 6.283185307179586476925286766559;
    lnZ = lmax + log(I0) - 0.5 * log(twopi * t.v) - 0.5 * log(twopi * t.s2);
}

__device__ __forceinline__ void tilted_gauss(const TiltP& t, double& lnZ, double& mean, double& var) {
    double vh = 1.0 / (1.0 / t.v + 1.0 / t.s2);
    var = vh;
    mean = vh * (t.mu / t.v + t.A / t.s2);
    double tv = t.v + t.s2, r = t.A - t.mu;
    lnZ = -0.5 * log(6.283185307179586476925286766559 * tv) - 0.5 * r * r / tv;
}

// Cavity from the q-marginal, tilted moments, damped site update.
__global__ __launch_bounds__(256) void k_tilted_update(StarsDev s, EpParams P, const int32_t* list, int64_t nlist) {
    __shared__ double sbw[4][72];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + w;
    const bool active = list ? i < nlist : i < s.n;
    const int64_t star = list ? (active ? (int64_t)list[i] : 0) : i;
    double tau = 0.0, nu = 0.0, tau_c = 1.0, nu_c = 0.0, mu_c = 0.0, v_c = 1.0;
    bool skip = !active;
    TiltP tp{0.0, 1.0, 1.0, 1.0};   // benign stand-in for idle waves
    if (active) {
        const double qm = s.cav_mu[star], qv = s.cav_var[star];
        tau = s.tau[star];
        nu = s.nu[star];
        tau_c = 1.0 / qv - tau;
        nu_c = qm / qv - nu;
        if (!(tau_c > 0.0)) {
            skip = true;
        } else {
            v_c = 1.0 / tau_c;
            if (v_c < P.vfloor) v_c = P.vfloor;
            mu_c = nu_c / tau_c;
            tau_c = 1.0 / v_c;
            nu_c = mu_c / v_c;
            const double sig = s.sigma[star];
            tp = TiltP{mu_c, v_c, s.A[star], sig * sig};
        }
    }
    double lnZ, mh, vh;
    if (P.mode == 1) tilted_gauss(tp, lnZ, mh, vh);
    else tilted_wave(tp, sbw[w], lnZ, mh, vh);   // every wave reaches the block barrier inside
    if (!active || lane != 0) return;
    if (skip) {
        s.status[star] = 1;
        s.dtau[star] = 0.0;
        return;
    }
    s.cav_mu[star] = mu_c;
    s.cav_var[star] = v_c;
    s.lnZ[star] = lnZ;
    s.tmean[star] = mh;
    s.tvar[star] = vh;
    const double tn = 1.0 / vh - tau_c;
    const double nn = mh / vh - nu_c;
    if (!(tn >= 0.0) || !isfinite(tn) || !isfinite(nn)) {
        s.status[star] = 2;
        s.dtau[star] = 0.0;
    } else {
        const double d = P.damping;
        const double t2 = (1.0 - d) * tau + d * tn;
        s.status[star] = 0;
        s.dtau[star] = fabs(t2 - tau);
        s.tau[star] = t2;
        s.nu[star] = (1.0 - d) * nu + d * nn;
    }
}

void launch_tilted_update(hipStream_t st, StarsDev s, EpParams p, const int32_t* list, int64_t nlist) {
    const int64_t n = list ? nlist : s.n;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_tilted_update, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, s, p, list, nlist);
}

__global__ __launch_bounds__(256) void k_tilted_batch(int mode, int64_t n, const double* mu, const double* v,
                                                      const double* A, const double* sig, double* lnZ,
                                                      double* mean, double* var) {
    __shared__ double sbw[4][72];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + w;
    const bool active = i < n;
    TiltP tp{0.0, 1.0, 1.0, 1.0};
    if (active) tp = TiltP{mu[i], v[i], A[i], sig[i] * sig[i]};
    double a, b, c;
    if (mode == 1) tilted_gauss(tp, a, b, c);
    else tilted_wave(tp, sbw[w], a, b, c);
    if (active && lane == 0) { lnZ[i] = a; mean[i] = b; var[i] = c; }
}

void launch_tilted_batch(hipStream_t st, int mode, int64_t n, const double* mu, const double* v, const double* A,
                         const double* sig, double* lnZ, double* mean, double* var) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_tilted_batch, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, mode, n, mu, v, A, sig,
                       lnZ, mean, var);
}

// Gauss-Legendre 16-point nodes and weights from Newton's iteration on the
// three-term Legendre recurrence, started from the asymptotic node estimate
// cos(pi (i + 3/4) / (n + 1/2)) (the standard construction, e.g. Press et
// al., Numerical Recipes, Sec. 4.5); computed on the host, copied to
// constant memory.
void gauss_legendre16(double* x, double* wgt) {
    const int n = 16;
    for (int i = 0; i < n; i++) {
        double z = cos(3.14159265358979323846 * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; k++) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-17) break;
        }
        {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; k++) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
        }
        x[i] = z;
        wgt[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

hipError_t set_gauss_legendre(hipStream_t st) {
    double x[16], wgt[16];
    gauss_legendre16(x, wgt);
    hipError_t e = hipMemcpyToSymbolAsync(HIP_SYMBOL(c_glx), x, sizeof(x), 0, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyToSymbolAsync(HIP_SYMBOL(c_glw), wgt, sizeof(wgt), 0, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
}

// ===========================================================================
// Mixed precision: the partial Cholesky of every front in FP32 storage with
// FP32 MFMA (v_mfma_f32_16x16x4f32) for the column solves and the updates;
// the diagonal tiles are factored (and inverted) in FP64 from their FP32
// values.  Extend-add goes back into the FP64 fronts, which each level
// converts to FP32 before it is factored.
// ===========================================================================
typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int LDF = TS + 4;   // padded LDS row (floats)

struct Stage32 {
    float a[16], b[16];
};

template <typename TA, typename TB>
__device__ __forceinline__ void stage32_load(Stage32& p, const TA* A, int lda, const TB* B, int ldb) {
    const int tid = threadIdx.x, lo = tid & 63, hi = tid >> 6;
#pragma unroll
    for (int r = 0; r < 16; r++) p.a[r] = (float)A[lo + (int64_t)(hi + 4 * r) * lda];
#pragma unroll
    for (int r = 0; r < 16; r++) p.b[r] = (float)B[lo + (int64_t)(hi + 4 * r) * ldb];
}

__device__ __forceinline__ void stage32_store(const Stage32& p, float* sA, float* sB, bool ta, bool tb, float sgn) {
    const int tid = threadIdx.x, lo = tid & 63, hi = tid >> 6;
    if (!ta) {
#pragma unroll
        for (int r = 0; r < 16; r++) sA[(hi + 4 * r) * LDF + lo] = sgn * p.a[r];
    } else {
#pragma unroll
        for (int r = 0; r < 16; r++) sA[lo * LDF + hi + 4 * r] = sgn * p.a[r];
    }
    if (!tb) {
#pragma unroll
        for (int r = 0; r < 16; r++) sB[lo * LDF + hi + 4 * r] = p.b[r];
    } else {
#pragma unroll
        for (int r = 0; r < 16; r++) sB[(hi + 4 * r) * LDF + lo] = p.b[r];
    }
}

__device__ __forceinline__ void tile_mma32(f4 acc[2][2], const float* sA, const float* sB) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
#pragma unroll 4
    for (int kk = 0; kk < TS; kk += 4) {
        const float* ra = sA + (kk + lk) * LDF;
        const float* rb = sB + (kk + lk) * LDF;
        float a0 = ra[wr + li], a1 = ra[wr + 16 + li];
        float b0 = rb[wc + li], b1 = rb[wc + 16 + li];
        acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
    }
}

template <typename TA, typename TB>
__device__ __forceinline__ void seg_run32(f4 acc[2][2], float* sA, float* sB, const TA* A, int64_t sa, int lda,
                                          bool ta, float sgn, const TB* B, int64_t sb, int ldb, bool tb, int nk) {
    if (nk <= 0) return;
    Stage32 p;
    stage32_load(p, A, lda, B, ldb);
    for (int t = 0; t < nk; t++) {
        __syncthreads();
        stage32_store(p, sA, sB, ta, tb, sgn);
        __syncthreads();
        if (t + 1 < nk) stage32_load(p, A + (t + 1) * sa, lda, B + (t + 1) * sb, ldb);
        tile_mma32(acc, sA, sB);
    }
}

// mode 0 accumulate, 1 overwrite
__device__ __forceinline__ void tile_store32(f4 acc[2][2], float* sC, float* C, int ldc, int mode) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    __syncthreads();
#pragma unroll
    for (int bi = 0; bi < 2; bi++)
#pragma unroll
        for (int bj = 0; bj < 2; bj++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                // v_mfma_f32_16x16x4f32 output: lane l, item r -> row 4(l/16) + r, column l%16
                int row = wr + 16 * bi + 4 * (lane >> 4) + r;
                int col = wc + 16 * bj + (lane & 15);
                sC[col * LDF + row] = acc[bi][bj][r];
            }
    __syncthreads();
    const int row = threadIdx.x & 63;
#pragma unroll
    for (int r = 0; r < 16; r++) {
        int col = (threadIdx.x >> 6) + 4 * r;
        float v = sC[col * LDF + row];
        float* p = C + row + (int64_t)col * ldc;
        if (mode == 1) *p = v;
        else *p += v;
    }
}

__device__ __forceinline__ void acc32_zero(f4 acc[2][2]) {
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
}

// FP64 -> FP32 copy of every front of a level; task = (front, 64-column tile)
__global__ __launch_bounds__(256) void k_to_f32(const BatchEnt* __restrict__ be, int nbe, int64_t ntasks, FrontsDev F,
                                                Bufs bufs) {
    const int64_t t = blockIdx.x;
    if (t >= ntasks) return;
    const int e = (int)batch_find(be, nbe, t);
    const int f = be[e].front;
    const int j0 = TS * (int)(t - be[e].base);
    const int64_t m = F.m[f];
    const double* src = bufs.fronts + F.off[f] + j0 * m;
    float* dst = bufs.F32 + F.off[f] + j0 * m;
    for (int64_t q = threadIdx.x; q < (int64_t)TS * m; q += 256) dst[q] = (float)src[q];
}

__global__ __launch_bounds__(256) void k_trsm32(const BatchEnt* __restrict__ be, int nbe, int64_t ntasks, int k,
                                                FrontsDev F, Bufs bufs) {
    __shared__ float sA[TS * LDF];
    __shared__ float sB[TS * LDF];
    const int64_t t = blockIdx.x;
    if (t >= ntasks) return;
    const int e = (int)batch_find(be, nbe, t);
    const int f = be[e].front;
    const int i = k + 1 + (int)(t - be[e].base);
    const int m = F.m[f];
    float* Aik = bufs.F32 + F.off[f] + (int64_t)TS * i + (int64_t)TS * k * m;
    const double* Xkk = bufs.X + F.xoff[f] + (int64_t)TS * k + (int64_t)TS * k * F.nvpad[f];
    f4 acc[2][2];
    acc32_zero(acc);
    seg_run32(acc, sA, sB, Aik, 0, m, false, 1.0f, Xkk, 0, F.nvpad[f], true, 1);
    tile_store32(acc, sA, Aik, m, 1);
}

__global__ __launch_bounds__(256) void k_syrk_inner32(const BatchEnt* __restrict__ be, int nbe, int64_t ntasks,
                                                      int kk, FrontsDev F, Bufs bufs) {
    __shared__ float sA[TS * LDF];
    __shared__ float sB[TS * LDF];
    const int64_t t = blockIdx.x;
    if (t >= ntasks) return;
    const int e = (int)batch_find(be, nbe, t);
    const int f = be[e].front;
    const int m = F.m[f];
    const int j = kk + 1, i = j + (int)(t - be[e].base);
    const int k0 = PW * (kk / PW);
    float* base = bufs.F32 + F.off[f];
    f4 acc[2][2];
    acc32_zero(acc);
    seg_run32(acc, sA, sB, base + (int64_t)TS * i + (int64_t)TS * k0 * m, (int64_t)TS * m, m, false, -1.0f,
              base + (int64_t)TS * j + (int64_t)TS * k0 * m, (int64_t)TS * m, m, true, kk - k0 + 1);
    tile_store32(acc, sA, base + (int64_t)TS * i + (int64_t)TS * j * m, m, 0);
}

// update block of the FP32 front added into the FP64 parent
__global__ __launch_bounds__(256) void k_extend_add32(const BatchEnt* __restrict__ be, int nbe, int64_t ntasks,
                                                      FrontsDev F, Bufs bufs) {
    __shared__ int32_t rel_i[TS], rel_j[TS];
    const int64_t t = blockIdx.x;
    if (t >= ntasks) return;
    const int e = (int)batch_find(be, nbe, t);
    const int f = be[e].front;
    int ti, tj;
    tri_decode(t - be[e].base, ti, tj);
    const int p = F.parent[f];
    const int nr = F.nr[f], nvp = F.nvpad[f], m = F.m[f], mp = F.m[p];
    const int32_t* rel = F.relmap + F.rptr[f];
    if (threadIdx.x < TS) {
        int a = TS * ti + threadIdx.x;
        rel_i[threadIdx.x] = a < nr ? rel[a] : -1;
    } else if (threadIdx.x < 2 * TS) {
        int b = TS * tj + threadIdx.x - TS;
        rel_j[threadIdx.x - TS] = b < nr ? rel[b] : -1;
    }
    __syncthreads();
    const float* src = bufs.F32 + F.off[f] + nvp + (int64_t)nvp * m;
    double* dst = bufs.fronts + F.off[p];
    const int r = threadIdx.x & 63;
    const int a = TS * ti + r;
    if (rel_i[r] < 0) return;
    for (int q = threadIdx.x >> 6; q < TS; q += 4) {
        const int b = TS * tj + q;
        if (rel_j[q] < 0 || b > a) continue;
        atomicAdd(dst + rel_i[r] + (int64_t)rel_j[q] * mp, (double)src[a + (int64_t)b * m]);
    }
}

void launch_to_f32(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, FrontsDev F, Bufs b) {
    if (ntasks <= 0) return;
    hipLaunchKernelGGL(k_to_f32, dim3((unsigned)ntasks), dim3(256), 0, st, be, nbe, ntasks, F, b);
}
void launch_potrf32(hipStream_t st, const int32_t* flist, int nf, int k, FrontsDev F, Bufs b, int* err) {
    if (nf <= 0) return;
    hipLaunchKernelGGL(k_potrf<float>, dim3(nf), dim3(256), 0, st, flist, k, F, b, err);
}
void launch_trsm32(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, int k, FrontsDev F, Bufs b) {
    if (ntasks <= 0) return;
    hipLaunchKernelGGL(k_trsm32, dim3((unsigned)ntasks), dim3(256), 0, st, be, nbe, ntasks, k, F, b);
}
void launch_syrk_inner32(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, int kk, FrontsDev F, Bufs b) {
    if (ntasks <= 0) return;
    hipLaunchKernelGGL(k_syrk_inner32, dim3((unsigned)ntasks), dim3(256), 0, st, be, nbe, ntasks, kk, F, b);
}
void launch_extend_add32(hipStream_t st, const BatchEnt* be, int nbe, int64_t ntasks, FrontsDev F, Bufs b) {
    if (ntasks <= 0) return;
    hipLaunchKernelGGL(k_extend_add32, dim3((unsigned)ntasks), dim3(256), 0, st, be, nbe, ntasks, F, b);
}

// ===========================================================================
// FP64 residual of the posterior system for iterative refinement:
//   r = b - Q x,  Q x = (I-B)^T D^{-1} (I-B) x + sum_n tau_n g_n (g_n . x)
// ===========================================================================
// u = D^{-1} (I - B) x  (rows of B)
__global__ void k_q0_rows(int64_t N, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                          const double* __restrict__ val, const double* __restrict__ d, const double* __restrict__ x,
                          double* __restrict__ u) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
        double s = x[p];
        for (int64_t e = rp[p]; e < rp[p + 1]; e++) s -= val[e] * x[col[e]];
        u[p] = s / d[p];
    }
}
// w = u - B^T u  (w initialised to u by the caller)
__global__ void k_q0_cols(int64_t N, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                          const double* __restrict__ val, const double* __restrict__ u, double* __restrict__ w) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
        const double up = u[p];
        if (up == 0.0) continue;
        for (int64_t e = rp[p]; e < rp[p + 1]; e++) atomicAdd(w + col[e], -val[e] * up);
    }
}
// w += sum_n tau_n g_n (g_n . x), one wavefront per star
__global__ __launch_bounds__(256) void k_gtg(StarsDev s, const double* __restrict__ x, double* __restrict__ w) {
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t star = (int64_t)blockIdx.x * 4 + wv;
    if (star >= s.n) return;
    const double tau = s.tau[star];
    if (tau == 0.0) return;
    const int64_t p0 = s.ptr[star];
    const int cnt = (int)(s.ptr[star + 1] - p0);
    double dot = 0.0;
    for (int k = lane; k < cnt; k += 64) dot += s.g[p0 + k] * x[s.nodes[p0 + k]];
    dot = wave_sum(dot);
    const double c = tau * dot;
    for (int k = lane; k < cnt; k += 64) atomicAdd(w + s.nodes[p0 + k], c * s.g[p0 + k]);
}
// r = b - w
__global__ void k_sub(int64_t n, const double* __restrict__ b, const double* __restrict__ w, double* __restrict__ r) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        r[i] = b[i] - w[i];
}
// x += dx
__global__ void k_add(int64_t n, double* __restrict__ x, const double* __restrict__ dx) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] += dx[i];
}

void launch_residual(hipStream_t st, int64_t N, const int64_t* rp, const int32_t* col, const double* val,
                     const double* d, StarsDev s, const double* b, const double* x, double* u, double* w, double* r) {
    unsigned g = grid_for(N);
    hipLaunchKernelGGL(k_q0_rows, dim3(g), dim3(256), 0, st, N, rp, col, val, d, x, u);
    (void)hipMemcpyAsync(w, u, sizeof(double) * N, hipMemcpyDeviceToDevice, st);
    hipLaunchKernelGGL(k_q0_cols, dim3(g), dim3(256), 0, st, N, rp, col, val, u, w);
    if (s.n > 0) hipLaunchKernelGGL(k_gtg, dim3((unsigned)((s.n + 3) / 4)), dim3(256), 0, st, s, x, w);
    hipLaunchKernelGGL(k_sub, dim3(g), dim3(256), 0, st, N, b, w, r);
}
void launch_add(hipStream_t st, int64_t n, double* x, const double* dx) {
    if (n > 0) hipLaunchKernelGGL(k_add, dim3(grid_for(n)), dim3(256), 0, st, n, x, dx);
}

}  // namespace ep

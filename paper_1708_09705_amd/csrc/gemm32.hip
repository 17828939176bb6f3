// FP32 task-list GEMM for the trailing updates of the mixed-precision
// factorization, on the FP32 copy of the fronts.  The layout is that of the
// FP64 task kernel: 256 x 128 output blocks, eight waves, wave w owning the
// 64 x 64 quadrant (row quarter w >> 1, column half w & 1) as 4 x 4
// v_mfma_f32_16x16x4f32 blocks; K advances in slabs of 16 through two LDS
// buffers and two register stages (a slab's global loads are issued two MFMA
// phases before they are stored to LDS; one barrier per slab).  Operand and
// output offsets of the tasks address the FP32 buffer; the buffer ids in the
// flags are not used.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace ep {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int BM = 256, BN = 128, KH = 16;
// LDS row strides (floats): 16 mod 64, so that the 16 columns x 4 k rows
// of an MFMA operand read fall in distinct banks
constexpr int LDA = BM + 16, LDB = BN + 16;
constexpr int SLA = KH * LDA, SLB = KH * LDB;
constexpr int NT = 512;

__device__ __forceinline__ int64_t xcd_task32(int64_t n) {
    const int64_t b = blockIdx.x, G = gridDim.x;
    const int64_t per = (G + 7) / 8;
    const int64_t x = b % 8, q = b / 8;
    const int64_t full = G % 8 == 0 ? 8 : G % 8;
    (void)n;
    return x < full ? x * per + q : full * per + (x - full) * (per - 1) + q;
}

template <typename T> struct Pair2;
template <> struct Pair2<float> { typedef float2 type; };
template <> struct Pair2<double> { typedef double2 type; };

// One R x 16 slab op(M)(i, k) into registers as pairs (NP per thread),
// read in the element type of the memory (T: float, or double for the FP64
// buffers, rounded to FP32 in the registers).  kc: k contiguous in memory
// (M[k + i ld]); else i contiguous.
template <int R, typename T>
__device__ __forceinline__ void load_slab(float* r, const T* M, int ld, bool kc) {
    typedef typename Pair2<T>::type P2;
    constexpr int NP = R * KH / 2 / NT;
    const int t = threadIdx.x;
    if (!kc) {
        constexpr int PR = R / 2, KS = NT / PR;
        const int p = t % PR, k0 = t / PR;
        const T* Mp = M + 2 * p + (int64_t)k0 * ld;
#pragma unroll
        for (int q = 0; q < NP; q++) {
            const P2 v = *(const P2*)(Mp + (int64_t)(KS * q) * ld);
            r[2 * q] = (float)v.x;
            r[2 * q + 1] = (float)v.y;
        }
    } else {
        const int kp = t & 7, i0 = t >> 3;   // 64 i per round
        const T* Mp = M + 2 * kp + (int64_t)i0 * ld;
#pragma unroll
        for (int q = 0; q < NP; q++) {
            const P2 v = *(const P2*)(Mp + (int64_t)(64 * q) * ld);
            r[2 * q] = (float)v.x;
            r[2 * q + 1] = (float)v.y;
        }
    }
}

// The slab to LDS as s[k][i] (row stride LD), scaled by sgn
template <int R, int LD>
__device__ __forceinline__ void store_slab(const float* r, float* s, bool kc, float sgn) {
    constexpr int NP = R * KH / 2 / NT;
    const int t = threadIdx.x;
    if (!kc) {
        constexpr int PR = R / 2, KS = NT / PR;
        const int p = t % PR, k0 = t / PR;
#pragma unroll
        for (int q = 0; q < NP; q++) {
            s[(k0 + KS * q) * LD + 2 * p] = sgn * r[2 * q];
            s[(k0 + KS * q) * LD + 2 * p + 1] = sgn * r[2 * q + 1];
        }
    } else {
        const int kp = t & 7, i0 = t >> 3;
#pragma unroll
        for (int q = 0; q < NP; q++) {
            s[(2 * kp) * LD + i0 + 64 * q] = sgn * r[2 * q];
            s[(2 * kp + 1) * LD + i0 + 64 * q] = sgn * r[2 * q + 1];
        }
    }
}

// acc (this wave's quadrant) += sum over the slab's k of sA[k][i] sB[k][j]
__device__ __forceinline__ void mma_slab(f4v acc[4][4], const float* sA, const float* sB) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
    const int li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int kk = 0; kk < KH; kk += 4) {
        const float* ra = sA + (kk + lk) * LDA + wr + li;
        const float* rb = sB + (kk + lk) * LDB + wc + li;
        float a[4], b[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            a[q] = ra[16 * q];
            b[q] = rb[16 * q];
        }
#pragma unroll
        for (int x = 0; x < 4; x++)
#pragma unroll
            for (int y = 0; y < 4; y++) acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[x], b[y], acc[x][y], 0, 0, 0);
    }
}

// One segment: acc += sum over its K of op(A) op(B).  Ends with a barrier
// after the last read of smem.
// Adds the FP32 sums into the FP64 accumulators and clears them.
__device__ __forceinline__ void flush_wide(f4v acc[4][4], double wide[64]) {
#pragma unroll
    for (int x = 0; x < 4; x++)
#pragma unroll
        for (int y = 0; y < 4; y++) {
#pragma unroll
            for (int r = 0; r < 4; r++) wide[16 * x + 4 * y + r] += (double)acc[x][y][r];
            acc[x][y] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
        }
}

// WIDE: the FP32 sums are added into the FP64 accumulators `wide` every four
// slabs (64 k) and at the end of the segment, so that FP32 rounding grows
// with 64 rather than with the whole K
template <typename T, bool WIDE>
__device__ __forceinline__ void run_seg(f4v acc[4][4], double* wide, float* smem, const T* A, const T* B,
                                        const GemmSeg& S, bool active) {
    const bool ta = S.flags & 1, tb = (S.flags & 2) != 0;
    const float sgn = (S.flags & 4) ? -1.0f : 1.0f;
    const bool kca = ta, kcb = !tb;
    const int nh = (TS / KH) * S.nk;
    const int64_t ha = S.sa / (TS / KH), hb = S.sb / (TS / KH);
    if (nh <= 0) return;
    float* U0 = smem;
    float* U1 = smem + SLA + SLB;
    float a0[BM * KH / NT], b0[BN * KH / NT];
    float a1[BM * KH / NT], b1[BN * KH / NT];
    load_slab<BM, T>(a0, A, S.lda, kca);
    load_slab<BN, T>(b0, B, S.ldb, kcb);
    if (nh > 1) {
        load_slab<BM, T>(a1, A + ha, S.lda, kca);
        load_slab<BN, T>(b1, B + hb, S.ldb, kcb);
    }
    store_slab<BM, LDA>(a0, U0, kca, sgn);
    store_slab<BN, LDB>(b0, U0 + SLA, kcb, 1.0f);
    if (nh > 2) {
        load_slab<BM, T>(a0, A + 2 * ha, S.lda, kca);
        load_slab<BN, T>(b0, B + 2 * hb, S.ldb, kcb);
    }
    __syncthreads();
    for (int h = 0; h < nh; h += 2) {
        if (active) mma_slab(acc, U0, U0 + SLA);
        if (h + 1 < nh) {
            store_slab<BM, LDA>(a1, U1, kca, sgn);
            store_slab<BN, LDB>(b1, U1 + SLA, kcb, 1.0f);
            if (h + 3 < nh) {
                load_slab<BM, T>(a1, A + (h + 3) * ha, S.lda, kca);
                load_slab<BN, T>(b1, B + (h + 3) * hb, S.ldb, kcb);
            }
        }
        __syncthreads();
        if (h + 1 >= nh) break;
        if (active) mma_slab(acc, U1, U1 + SLA);
        if (WIDE && active && (h & 3) == 2) flush_wide(acc, wide);   // slabs h - 2 .. h + 1 done
        if (h + 2 < nh) {
            store_slab<BM, LDA>(a0, U0, kca, sgn);
            store_slab<BN, LDB>(b0, U0 + SLA, kcb, 1.0f);
            if (h + 4 < nh) {
                load_slab<BM, T>(a0, A + (h + 4) * ha, S.lda, kca);
                load_slab<BN, T>(b0, B + (h + 4) * hb, S.ldb, kcb);
            }
        }
        __syncthreads();
    }
    if (WIDE && active) flush_wide(acc, wide);
}

__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_gemm_tasks_f32(const GemmTask* __restrict__ tasks, int64_t n, float* F32) {
    __shared__ float smem[2 * (SLA + SLB)];
    const int64_t t = xcd_task32(n);
    if (t >= n) return;
    const GemmTask& T = tasks[t];
    const int nseg = (T.flags >> 4) & 3;
    if (nseg == 0) return;   // padding entry
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int qr = w >> 1, qc = w & 1;
    const int nqa = gt_rows(T.flags), nqb = (T.flags & GT_COLS2) ? 2 : 1;
    const bool mine = qr < nqa && qc < nqb && (!(T.flags & GT_LOWER) || gt_diag(T.flags) + qr - qc >= 0);
    f4v acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; x++)
#pragma unroll
        for (int y = 0; y < 4; y++) acc[x][y] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int q = 0; q < 2; q++) {
        if (q >= nseg) break;
        const GemmSeg& S = T.s[q];
        run_seg<float, false>(acc, nullptr, smem, F32 + S.a, F32 + S.b, S, mine);
    }
    if (!mine) return;
    const bool over = T.flags & 1, atom = (T.flags & 2) != 0;
    const int64_t rs = (T.flags & GT_TSTORE) ? T.ldc : 1, cs = (T.flags & GT_TSTORE) ? 1 : T.ldc;
    float* C = F32 + T.c + (qr * 64 + 4 * (lane >> 4)) * rs + (qc * 64 + (lane & 15)) * cs;
    // v_mfma_f32_16x16x4f32 output: lane l, item r -> row 4(l/16) + r, column l%16
    if (rs == 1 && !atom && ((T.c | T.ldc) & 3) == 0) {
        // the lane's four rows are contiguous and 16-byte aligned
#pragma unroll
        for (int x = 0; x < 4; x++)
#pragma unroll
            for (int y = 0; y < 4; y++) {
                f4v* p = (f4v*)(C + 16 * x + (16 * y) * cs);
                *p = over ? acc[x][y] : *p + acc[x][y];
            }
        return;
    }
#pragma unroll
    for (int x = 0; x < 4; x++)
#pragma unroll
        for (int y = 0; y < 4; y++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                float* p = C + (16 * x + r) * rs + (16 * y) * cs;
                if (atom) atomicAdd(p, acc[x][y][r]);
                else *p = over ? acc[x][y][r] : *p + acc[x][y][r];
            }
}

__device__ __forceinline__ double* buf64(const Bufs& b, int id) {
    return id == BUF_FRONTS ? b.fronts : (id == BUF_X ? b.X : b.W);
}

// The same tasks on the FP64 buffers with FP32 arithmetic (the selected
// inversion of precision SELINV32): operands and outputs are addressed as in
// the FP64 task kernel (buffer ids in the flags), the operand slabs are
// rounded to FP32 as they are loaded, the products accumulate in FP32 on
// v_mfma_f32_16x16x4f32 over 64 k at a time and those partial sums in FP64,
// and the results are stored in FP64.  The FP64 accumulators take the
// register file to 256 VGPRs (one block of eight waves per CU; a few spill).
__global__ __launch_bounds__(NT) void k_gemm_tasks_x32(const GemmTask* __restrict__ tasks, int64_t n, Bufs bufs) {
    __shared__ float smem[2 * (SLA + SLB)];
    const int64_t t = xcd_task32(n);
    if (t >= n) return;
    const GemmTask& T = tasks[t];
    const int nseg = (T.flags >> 4) & 3;
    if (nseg == 0) return;   // padding entry
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int qr = w >> 1, qc = w & 1;
    const int nqa = gt_rows(T.flags), nqb = (T.flags & GT_COLS2) ? 2 : 1;
    const bool mine = qr < nqa && qc < nqb && (!(T.flags & GT_LOWER) || gt_diag(T.flags) + qr - qc >= 0);
    f4v acc[4][4];
    double wide[64];
#pragma unroll
    for (int x = 0; x < 4; x++)
#pragma unroll
        for (int y = 0; y < 4; y++) acc[x][y] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int q = 0; q < 64; q++) wide[q] = 0.0;
#pragma unroll
    for (int q = 0; q < 2; q++) {
        if (q >= nseg) break;
        const GemmSeg& S = T.s[q];
        run_seg<double, true>(acc, wide, smem, buf64(bufs, (S.flags >> 8) & 3) + S.a,
                              buf64(bufs, (S.flags >> 10) & 3) + S.b, S, mine);
    }
    if (!mine) return;
    const bool over = T.flags & 1, atom = (T.flags & 2) != 0;
    const int64_t rs = (T.flags & GT_TSTORE) ? T.ldc : 1, cs = (T.flags & GT_TSTORE) ? 1 : T.ldc;
    double* C = buf64(bufs, (T.flags >> 8) & 3) + T.c + (qr * 64 + 4 * (lane >> 4)) * rs + (qc * 64 + (lane & 15)) * cs;
    // v_mfma_f32_16x16x4f32 output: lane l, item r -> row 4(l/16) + r, column l%16
#pragma unroll
    for (int x = 0; x < 4; x++)
#pragma unroll
        for (int y = 0; y < 4; y++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                double* p = C + (16 * x + r) * rs + (16 * y) * cs;
                const double v = wide[16 * x + 4 * y + r];
                if (atom) atomicAdd(p, v);
                else *p = over ? v : *p + v;
            }
}

}  // namespace

void launch_gemm_tasks_f32(hipStream_t st, const GemmTask* t, int64_t n, float* F32) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gemm_tasks_f32, dim3((unsigned)n), dim3(NT), 0, st, t, n, F32);
}

void launch_gemm_tasks_x32(hipStream_t st, const GemmTask* t, int64_t n, Bufs b) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gemm_tasks_x32, dim3((unsigned)n), dim3(NT), 0, st, t, n, b);
}

}  // namespace ep

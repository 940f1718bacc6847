// Elastic deformation on MFMA (gfx950).
//
// Line contact (Sec. 3.3.1, case 1): H_el = K P with K[i][j] = k[|i-j|],
//   k[m] = -(1/pi) * (F((m + 1/2) h) - F((m - 1/2) h)),  F(t) = t ln|t| - t,
// the exact integral of ln|x - x'| over the cell of node j (P piecewise
// constant).  P holds B instances on the same grid (column major, N x B), so
// the evaluation is a dense N x N by N x B contraction.  The Toeplitz matrix
// is never stored: the kernel vector (N doubles) is staged in LDS and every
// MFMA A-operand element is k[|i - j|].
//
// Point contact (case 2): H_el[i][j] = sum_{i',j'} k2[|i-i'|][|j-j'|] P[i'][j'],
// k2 = (2/pi^2) * (cell integral of 1/r, closed form with asinh terms).  For
// a fixed row offset d = i - i' the j-sum is a Toeplitz product, so an
// output tile accumulates MFMAs with A = T_|d| (16 j x 4 j') and
// B = P[i - d][j'] (4 j' x 16 i) over all d and j'; FP64 and FP32 use 32 x 32
// tiles per wave (two A and two B operands feed four MFMAs), split BF16
// 16 x 16.  The d range is split over workgroups (fixed partition, partial
// sums reduced in a fixed order), so the result is deterministic.
//
// Precisions: FP64 (v_mfma_f64_16x16x4f64), FP32 (v_mfma_f32_16x16x4f32),
// and split BF16: every operand x is split as x = hi + lo with hi = bf16(x),
// lo = bf16(x - hi); hi*hi + hi*lo + lo*hi are accumulated in FP32 by
// v_mfma_f32_16x16x16bf16_1k.
#include <type_traits>

#include "common.h"
#include "ehl_internal.h"

namespace pq {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short bf16x4 __attribute__((ext_vector_type(4)));

PQ_DEV double cell_log(double d, double h)
{
    auto F = [](double t) { return t == 0.0 ? 0.0 : t * log(fabs(t)) - t; };
    return F(d + 0.5 * h) - F(d - 0.5 * h);
}

PQ_DEV double asinh_term(double a, double b) { return a == 0.0 ? 0.0 : fabs(a) * asinh(b / a); }

PQ_DEV double cell_inv_r(double dx, double dy, double hx, double hy)
{
    const double xp = dx + 0.5 * hx, xm = dx - 0.5 * hx;
    const double yp = dy + 0.5 * hy, ym = dy - 0.5 * hy;
    return asinh_term(xp, yp) + asinh_term(yp, xp) - asinh_term(xm, yp) - asinh_term(yp, xm) -
           asinh_term(xp, ym) - asinh_term(ym, xp) + asinh_term(xm, ym) + asinh_term(ym, xm);
}

// k[m], m = 0..N-1
__global__ void line_kernel_vec(int N, double h, double* __restrict__ k)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < N) k[m] = -cell_log((double)m * h, h) / M_PI;
}

// k2[a][b], a < Nx, b < Ny (row major, stride Ny)
__global__ void point_kernel_tab(int Nx, int Ny, double hx, double hy, double* __restrict__ k2)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < Nx * Ny) {
        const int a = idx / Ny, b = idx % Ny;
        k2[idx] = 2.0 / (M_PI * M_PI) * cell_inv_r(a * hx, b * hy, hx, hy);
    }
}

// ---------------------------------------------------------------------------
// MFMA helpers: one 16x16 accumulator tile, K-step 4 (FP64/FP32) or 16 (BF16).
// Operand layout (16x16x4): lane l supplies A[l%16][l/16] and B[l/16][l%16]
// (BF16 16x16x16: four consecutive k per lane, k = 4*(l/16) + e).  Result
// element r of lane l holds D[4*(l/16) + r][l%16] for the FP32 forms and
// D[4*r + l/16][l%16] for the FP64 form (checked on the device).
// ---------------------------------------------------------------------------
PQ_DEV f64x4 mfma_f64(double a, double b, f64x4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

PQ_DEV f32x4 mfma_f32(float a, float b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

PQ_DEV f32x4 mfma_bf16(bf16x4 a, bf16x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

PQ_DEV short to_bf16(float x)
{
    // round to nearest even
    uint32_t u = __float_as_uint(x);
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    return (short)(u >> 16);
}

PQ_DEV float from_bf16(short s) { return __uint_as_float(((uint32_t)(uint16_t)s) << 16); }

PQ_DEV void split_bf16(float x, short& hi, short& lo)
{
    hi = to_bf16(x);
    lo = to_bf16(x - from_bf16(hi));
}

// ---------------------------------------------------------------------------
// Line contact: out[i + N*b] = sum_j k[|i-j|] P[j + N*b].
// Workgroup = 4 waves; a wave owns 16 rows i and 32 columns b (two 16x16
// accumulators); the workgroup covers 64 rows.  The whole kernel vector is
// staged in LDS (N <= LINE_LDS_MAX).
// ---------------------------------------------------------------------------
template <int PREC>
__global__ void __launch_bounds__(256) line_deform_kernel(int N, int B,
                                                          const double* __restrict__ kvec,
                                                          const double* __restrict__ P,
                                                          double* __restrict__ out)
{
    extern __shared__ double sk[];  // N doubles
    for (int t = threadIdx.x; t < N; t += blockDim.x) sk[t] = kvec[t];
    __syncthreads();
    const int wave = threadIdx.x / 64, l = threadIdx.x % 64;
    const int i0 = (blockIdx.x * 4 + wave) * 16;
    const int b0 = blockIdx.y * 32;
    const int li = l % 16, lk = l / 16;
    const int i = i0 + li;  // A row of this lane
    if (i0 >= N) return;    // whole wave out of range (uniform)
    if constexpr (PREC == PREC_FP64) {
        f64x4 c0 = {0, 0, 0, 0}, c1 = {0, 0, 0, 0};
        const int bA = b0 + li, bB = b0 + 16 + li;
        // U K-steps per pass: all their loads (clamped, valid addresses) are
        // issued before the MFMAs, which zero out-of-range operands (the MFMA
        // is convergent, so the compiler does not unroll a loop of unknown
        // trip count by itself)
        constexpr int U = 4;
        const double* PA = P + (int64_t)min(bA, B - 1) * N;
        const double* PB = P + (int64_t)min(bB, B - 1) * N;
        const int ic = min(i, N - 1);
        for (int jb = 0; jb < N; jb += 4 * U) {
            double ar[U], x0r[U], x1r[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int jc = min(jb + 4 * u + lk, N - 1);
                ar[u] = sk[abs(ic - jc)];
                x0r[u] = PA[jc];
                x1r[u] = PB[jc];
            }
#pragma unroll
            for (int u = 0; u < U; u++) {
                const bool jin = jb + 4 * u + lk < N;
                const double a = (i < N && jin) ? ar[u] : 0.0;
                const double x0 = (jin && bA < B) ? x0r[u] : 0.0;
                const double x1 = (jin && bB < B) ? x1r[u] : 0.0;
                c0 = mfma_f64(a, x0, c0);
                c1 = mfma_f64(a, x1, c1);
            }
        }
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int io = i0 + 4 * r + lk;  // f64 result: row 4*r + l/16
            if (io < N) {
                if (b0 + li < B) out[(int64_t)(b0 + li) * N + io] = c0[r];
                if (b0 + 16 + li < B) out[(int64_t)(b0 + 16 + li) * N + io] = c1[r];
            }
        }
    } else if constexpr (PREC == PREC_FP32) {
        f32x4 c0 = {0, 0, 0, 0}, c1 = {0, 0, 0, 0};
        const int bA = b0 + li, bB = b0 + 16 + li;
        constexpr int U = 4;  // as in the FP64 path
        const double* PA = P + (int64_t)min(bA, B - 1) * N;
        const double* PB = P + (int64_t)min(bB, B - 1) * N;
        const int ic = min(i, N - 1);
        for (int jb = 0; jb < N; jb += 4 * U) {
            double ar[U], x0r[U], x1r[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int jc = min(jb + 4 * u + lk, N - 1);
                ar[u] = sk[abs(ic - jc)];
                x0r[u] = PA[jc];
                x1r[u] = PB[jc];
            }
#pragma unroll
            for (int u = 0; u < U; u++) {
                const bool jin = jb + 4 * u + lk < N;
                const float a = (i < N && jin) ? (float)ar[u] : 0.0f;
                const float x0 = (jin && bA < B) ? (float)x0r[u] : 0.0f;
                const float x1 = (jin && bB < B) ? (float)x1r[u] : 0.0f;
                c0 = mfma_f32(a, x0, c0);
                c1 = mfma_f32(a, x1, c1);
            }
        }
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int io = i0 + 4 * lk + r;
            if (io < N) {
                if (b0 + li < B) out[(int64_t)(b0 + li) * N + io] = c0[r];
                if (b0 + 16 + li < B) out[(int64_t)(b0 + 16 + li) * N + io] = c1[r];
            }
        }
    } else {  // split BF16, K-step 16: lane supplies k-indices 4*lk .. 4*lk+3
        f32x4 c0 = {0, 0, 0, 0}, c1 = {0, 0, 0, 0};
        const int bA = b0 + li, bB = b0 + 16 + li;
        const double* PA = P + (int64_t)bA * N;
        const double* PB = P + (int64_t)bB * N;
        for (int j0 = 0; j0 < N; j0 += 16) {
            bf16x4 ah, al, xh0, xl0, xh1, xl1;
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int j = j0 + 4 * lk + e;
                const bool jin = j < N;
                const float a = (i < N && jin) ? (float)sk[abs(i - j)] : 0.0f;
                const float x0 = (jin && bA < B) ? (float)PA[j] : 0.0f;
                const float x1 = (jin && bB < B) ? (float)PB[j] : 0.0f;
                short h, lo;
                split_bf16(a, h, lo);
                ah[e] = h;
                al[e] = lo;
                split_bf16(x0, h, lo);
                xh0[e] = h;
                xl0[e] = lo;
                split_bf16(x1, h, lo);
                xh1[e] = h;
                xl1[e] = lo;
            }
            c0 = mfma_bf16(ah, xh0, c0);
            c0 = mfma_bf16(ah, xl0, c0);
            c0 = mfma_bf16(al, xh0, c0);
            c1 = mfma_bf16(ah, xh1, c1);
            c1 = mfma_bf16(ah, xl1, c1);
            c1 = mfma_bf16(al, xh1, c1);
        }
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int io = i0 + 4 * lk + r;
            if (io < N) {
                if (b0 + li < B) out[(int64_t)(b0 + li) * N + io] = c0[r];
                if (b0 + 16 + li < B) out[(int64_t)(b0 + 16 + li) * N + io] = c1[r];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Line contact, FP64 / FP32 MFMA: out[i + N*b] = sum_j k[|i-j|] P[j + N*b].
// A wave owns one 16x16 output tile (16 rows i, 16 columns b), a workgroup
// 4 waves along i (64 rows) with the same 16 columns; at N = 4097, B = 170
// that is about 2.8 workgroups per CU, which hide each other's operand work
// and barriers behind the matrix pipe (one wave per SIMD on larger tiles
// left a third of the CUs idle).  Two accumulators take the even and odd
// K-steps, so a wave's MFMAs do not wait on each other.  The K index is free
// inside a chunk of LKG K-steps (4 LKG rows j): lane k-slot lk of step u takes
// row j = j0 + LKG lk + u.  A = k[|i - j|] from the kernel vector in LDS
// (staged once, with a zero at index N that rows i >= N and rows j >= N
// read); where every row j of a chunk lies on one side of every row i of
// the tile, a lane's A entries are consecutive kernel-vector entries (read
// with immediate offsets, no index arithmetic), else entry by entry.  B: the
// workgroup stages each chunk of its 16 P columns through LDS once (one
// 16-byte load per thread, whole cache lines; rows j >= N and columns
// b >= B as zero), two buffers, the next chunk's loads issued before the
// current chunk's MFMAs.  Rows i >= N and columns b >= B are not stored.
// ---------------------------------------------------------------------------
// K-steps per chunk (even; rows j per chunk a multiple of 16)
template <int PREC>
constexpr int line_kg()
{
    return 16;
}
template <int PREC>
constexpr int line_pb()  // staged column stride (16-byte aligned rows)
{
    return 4 * line_kg<PREC>() + 2;
}

template <int PREC>
__global__ void __launch_bounds__(256) line_deform_tiled(int N, int B,
                                                         const double* __restrict__ kvec,
                                                         const double* __restrict__ P,
                                                         double* __restrict__ out)
{
    using T = typename std::conditional<PREC == PREC_FP64, double, float>::type;
    constexpr int LKG = line_kg<PREC>();
    constexpr int LGJ = 4 * LKG;         // rows j per chunk
    constexpr int LPB = line_pb<PREC>();
    constexpr int SPT = LGJ / 16;        // staged values per thread
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
    T* pt = reinterpret_cast<T*>(lds_raw);  // [2][16][LPB] staged B chunks
    T* sk = pt + 2 * 16 * LPB;              // N + 1 (zero at N)
    const int tid = threadIdx.x;
    // the kernel vector: batches of 8 loads per thread, all issued before
    // their LDS stores (a load-then-store loop waits on memory per entry)
    for (int t0 = 0; t0 <= N; t0 += 8 * 256) {
        double kv[8];
#pragma unroll
        for (int e = 0; e < 8; e++) kv[e] = kvec[min(t0 + e * 256 + tid, N - 1)];
#pragma unroll
        for (int e = 0; e < 8; e++) {
            const int t = t0 + e * 256 + tid;
            if (t <= N) sk[t] = t < N ? (T)kv[e] : (T)0;
        }
    }
    const int wave = tid / 64, l = tid % 64;
    const int li = l % 16, lk = l / 16;
    const int i0 = blockIdx.x * 64 + wave * 16;  // this wave's first row
    const int b0 = blockIdx.y * 16;
    const int ia = i0 + li;  // A row of this lane
    const bool ina = ia < N;
    const int nch = (N + LGJ - 1) / LGJ;
    // staging: thread t loads column b0 + t / 16, rows j0 + SPT (t % 16) ..
    const int sc = tid / 16, sj = SPT * (tid % 16);
    const bool scol = b0 + sc < B;
    const double* pcol = P + (int64_t)(scol ? b0 + sc : 0) * N;
    double stv[SPT];
    auto gload = [&](int c) {
        const int j = c * LGJ + sj;
#pragma unroll
        for (int e = 0; e < SPT; e++) stv[e] = pcol[min(j + e, N - 1)];
    };
    auto lstore = [&](int c) {
        const int j = c * LGJ + sj;
        T* d = pt + ((c & 1) * 16 + sc) * LPB + sj;
#pragma unroll
        for (int e = 0; e < SPT; e++) d[e] = (scol && j + e < N) ? (T)stv[e] : (T)0;
    };
    gload(0);
    lstore(0);
    __syncthreads();
    // kernel-vector index of this lane's A entry at step u of chunk c (N: zero)
    auto aidx = [&](int c, int u) {
        const int j = c * LGJ + LKG * lk + u;
        return (ina && j < N) ? abs(ia - j) : N;
    };
    typedef typename std::conditional<PREC == PREC_FP64, f64x4, f32x4>::type acc_t;
    acc_t ce = {0, 0, 0, 0}, co = {0, 0, 0, 0};
    const bool rows_in = i0 + 15 < N;
    // chunk ranges of the tile (wave-uniform): MODE 1 every j below every i,
    // MODE 2 every j above every i (and inside), MODE 0 the others
    const int gA = (rows_in && i0 >= LGJ - 1) ? (i0 - (LGJ - 1)) / LGJ + 1 : 0;
    const int gB = rows_in ? max(gA, (i0 + 15 + LGJ - 1) / LGJ) : 0;
    const int gC = rows_in ? max(gB, min(nch, N >= LGJ ? (N - LGJ) / LGJ + 1 : 0)) : 0;
    for (int c = 0; c < nch; c++) {
        if (c + 1 < nch) gload(c + 1);  // the next chunk in flight
        const int jg = c * LGJ;
        T av[LKG];
        if (i0 < N && c < gA) {
            const T* ap = sk + (ia - jg - LKG * lk - (LKG - 1));
#pragma unroll
            for (int u = 0; u < LKG; u++) av[u] = ap[LKG - 1 - u];
        } else if (i0 < N && c >= gB && c < gC) {
            const T* ap = sk + (jg + LKG * lk - ia);
#pragma unroll
            for (int u = 0; u < LKG; u++) av[u] = ap[u];
        } else {
#pragma unroll
            for (int u = 0; u < LKG; u++) av[u] = sk[aidx(c, u)];
        }
        const T* bp = pt + ((c & 1) * 16 + li) * LPB + LKG * lk;
#pragma unroll
        for (int u = 0; u < LKG; u++) {
            const T x = bp[u];
            if constexpr (PREC == PREC_FP64) {
                if (u % 2 == 0) ce = mfma_f64(av[u], x, ce);
                else co = mfma_f64(av[u], x, co);
            } else {
                if (u % 2 == 0) ce = mfma_f32(av[u], x, ce);
                else co = mfma_f32(av[u], x, co);
            }
        }
        if (c + 1 < nch) lstore(c + 1);
        __syncthreads();
    }
    // D element r of lane l: FP64 row 4 r + l/16, FP32 row 4 (l/16) + r; column l%16
    const int ca = b0 + li;
    if (ca < B && i0 < N) {
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int ro = i0 + (PREC == PREC_FP64 ? 4 * r + lk : 4 * lk + r);
            if (ro < N) out[(int64_t)ca * N + ro] = (double)ce[r] + (double)co[r];
        }
    }
}

// ---------------------------------------------------------------------------
// Point contact, one instance per blockIdx.z.  P, out: Nx x Ny row major
// (P[i*Ny + j]).  Tile: 16 j (MFMA rows) x 16 i (MFMA columns) per wave,
// 4 waves per workgroup along i.  blockIdx.y = segment s of the d range;
// partial sums go to part[s][inst][Nx*Ny] and are reduced by
// point_reduce_kernel.
// ---------------------------------------------------------------------------
template <int PREC>  // PREC_SPLIT_BF16
__global__ void __launch_bounds__(256) point_deform_kernel(int Nx, int Ny, int nseg, int B,
                                                           const double* __restrict__ k2,
                                                           const double* __restrict__ P,
                                                           double* __restrict__ part)
{
    const int wave = threadIdx.x / 64, l = threadIdx.x % 64;
    const int li = l % 16, lk = l / 16;
    const int ntj = (Ny + 15) / 16;
    const int tj = blockIdx.x % ntj;
    const int ti = (blockIdx.x / ntj) * 4 + wave;
    const int j0 = tj * 16, i0 = ti * 16;
    const int s = blockIdx.y, inst = blockIdx.z;
    if (i0 >= Nx) return;
    const double* Pi = P + (int64_t)inst * Nx * Ny;
    // d range covering i - i' for i in [i0, i0+16), i' in [0, Nx)
    const int dlo = i0 - (Nx - 1), dhi = i0 + 15;
    const int span = dhi - dlo + 1;
    const int per = (span + nseg - 1) / nseg;
    const int ds0 = dlo + s * per, ds1 = min(dhi, ds0 + per - 1);
    const int jrow = j0 + li;  // A row (output j) of this lane
    const int icol = i0 + li;  // B column (output i) of this lane
    f32x4 c32 = {0, 0, 0, 0};
    for (int d = ds0; d <= ds1; d++) {
        const int ad = abs(d);
        if (ad >= Nx) continue;
        const double* krow = k2 + (int64_t)ad * Ny;
        const int ip = icol - d;  // P row for this lane's B column
        const bool iok = icol < Nx && ip >= 0 && ip < Nx;
        const double* prow = Pi + (int64_t)(iok ? ip : 0) * Ny;
        for (int jp0 = 0; jp0 < Ny; jp0 += 16) {
            bf16x4 ah, al, xh, xl;
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int jp = jp0 + 4 * lk + e;
                const bool jok = jp < Ny;
                const float a = (jrow < Ny && jok) ? (float)krow[abs(jrow - jp)] : 0.0f;
                const float x = (iok && jok) ? (float)prow[jp] : 0.0f;
                short h, lo;
                split_bf16(a, h, lo);
                ah[e] = h;
                al[e] = lo;
                split_bf16(x, h, lo);
                xh[e] = h;
                xl[e] = lo;
            }
            c32 = mfma_bf16(ah, xh, c32);
            c32 = mfma_bf16(ah, xl, c32);
            c32 = mfma_bf16(al, xh, c32);
        }
    }
    double* dst = part + ((int64_t)s * B + inst) * Nx * Ny;
#pragma unroll
    for (int r = 0; r < 4; r++) {
        const int jo = j0 + 4 * lk + r;  // D row (output j): f32 result row 4*(l/16) + r
        const int io = i0 + li;          // D column = output i
        if (jo < Ny && io < Nx) dst[(int64_t)io * Ny + jo] = (double)c32[r];
    }
}

// FP64 / FP32 point contact with a 32 j x 32 i output tile per wave (four
// 16 x 16 accumulators): each K-step loads two A columns (T_|d| rows) and two
// B rows (P rows) for four MFMAs, half the operand loads per MFMA of the
// 16 x 16 tile, whose loads (L1 traffic) had bound it.  4 waves per
// workgroup along i; blockIdx.y = segment of the d range as above.
template <int PREC>
__global__ void __launch_bounds__(256) point_deform_kernel32(int Nx, int Ny, int nseg, int B,
                                                             const double* __restrict__ k2,
                                                             const double* __restrict__ P,
                                                             double* __restrict__ part)
{
    constexpr int U = 4;  // K-steps per pass, loads issued before the MFMAs
    const int wave = threadIdx.x / 64, l = threadIdx.x % 64;
    const int li = l % 16, lk = l / 16;
    const int ntj = (Ny + 31) / 32;
    const int tj = blockIdx.x % ntj;
    const int ti = (blockIdx.x / ntj) * 4 + wave;
    const int j0 = tj * 32, i0 = ti * 32;
    const int s = blockIdx.y, inst = blockIdx.z;
    if (i0 >= Nx) return;
    const double* Pi = P + (int64_t)inst * Nx * Ny;
    const int dlo = i0 - (Nx - 1), dhi = i0 + 31;
    const int span = dhi - dlo + 1;
    const int per = (span + nseg - 1) / nseg;
    const int ds0 = dlo + s * per, ds1 = min(dhi, ds0 + per - 1);
    const int jr0 = j0 + li, jr1 = j0 + 16 + li;    // A rows (output j)
    const int ic0 = i0 + li, ic1 = i0 + 16 + li;    // B columns (output i)
    const int jc0 = min(jr0, Ny - 1), jc1 = min(jr1, Ny - 1);
    f64x4 d00 = {0, 0, 0, 0}, d01 = d00, d10 = d00, d11 = d00;
    f32x4 f00 = {0, 0, 0, 0}, f01 = f00, f10 = f00, f11 = f00;
    for (int d = ds0; d <= ds1; d++) {
        const int ad = abs(d);
        if (ad >= Nx) continue;  // uniform over the wave
        const double* krow = k2 + (int64_t)ad * Ny;
        const int ip0 = ic0 - d, ip1 = ic1 - d;  // P rows of the two B column tiles
        const bool ok0 = ic0 < Nx && ip0 >= 0 && ip0 < Nx;
        const bool ok1 = ic1 < Nx && ip1 >= 0 && ip1 < Nx;
        const double* pr0 = Pi + (int64_t)min(max(ip0, 0), Nx - 1) * Ny;
        const double* pr1 = Pi + (int64_t)min(max(ip1, 0), Nx - 1) * Ny;
        for (int jb = 0; jb < Ny; jb += 4 * U) {
            double a0[U], a1[U], x0[U], x1[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int jp = min(jb + 4 * u + lk, Ny - 1);
                a0[u] = krow[abs(jc0 - jp)];
                a1[u] = krow[abs(jc1 - jp)];
                x0[u] = pr0[jp];
                x1[u] = pr1[jp];
            }
#pragma unroll
            for (int u = 0; u < U; u++) {
                const bool jok = jb + 4 * u + lk < Ny;
                const double A0 = (jr0 < Ny && jok) ? a0[u] : 0.0;
                const double A1 = (jr1 < Ny && jok) ? a1[u] : 0.0;
                const double X0 = (ok0 && jok) ? x0[u] : 0.0;
                const double X1 = (ok1 && jok) ? x1[u] : 0.0;
                if constexpr (PREC == PREC_FP64) {
                    d00 = mfma_f64(A0, X0, d00);
                    d01 = mfma_f64(A0, X1, d01);
                    d10 = mfma_f64(A1, X0, d10);
                    d11 = mfma_f64(A1, X1, d11);
                } else {
                    f00 = mfma_f32((float)A0, (float)X0, f00);
                    f01 = mfma_f32((float)A0, (float)X1, f01);
                    f10 = mfma_f32((float)A1, (float)X0, f10);
                    f11 = mfma_f32((float)A1, (float)X1, f11);
                }
            }
        }
    }
    double* dst = part + ((int64_t)s * B + inst) * Nx * Ny;
#pragma unroll
    for (int r = 0; r < 4; r++) {
        // D row (output j): f64 result row 4*r + l/16, f32 result row 4*(l/16) + r
        const int jo = (PREC == PREC_FP64 ? 4 * r + lk : 4 * lk + r);
        const double v00 = PREC == PREC_FP64 ? d00[r] : (double)f00[r];
        const double v01 = PREC == PREC_FP64 ? d01[r] : (double)f01[r];
        const double v10 = PREC == PREC_FP64 ? d10[r] : (double)f10[r];
        const double v11 = PREC == PREC_FP64 ? d11[r] : (double)f11[r];
        if (j0 + jo < Ny && ic0 < Nx) dst[(int64_t)ic0 * Ny + j0 + jo] = v00;
        if (j0 + jo < Ny && ic1 < Nx) dst[(int64_t)ic1 * Ny + j0 + jo] = v01;
        if (j0 + 16 + jo < Ny && ic0 < Nx) dst[(int64_t)ic0 * Ny + j0 + 16 + jo] = v10;
        if (j0 + 16 + jo < Ny && ic1 < Nx) dst[(int64_t)ic1 * Ny + j0 + 16 + jo] = v11;
    }
}

// ---------------------------------------------------------------------------
// Point contact, FP64 / FP32 MFMA, staged like the line kernel.  For each x
// offset d the product is a Toeplitz product along y,
//   out[i][j] += sum_jp k2[|d|][|j - jp|] P[i - d][jp],
// i.e. the line kernel with the kernel row k2[|d|] and the P rows shifted
// by d as its instances.  A workgroup: 4 waves along j (16 rows j each, 64
// in all) and 16 columns i; it runs the chunk loop of the line kernel (32
// rows jp per chunk) once per d of its segment of the d range, with the
// kernel row in LDS (two buffers by the parity of d, so the next row is
// stored while the current one is still read) and each chunk of its 16 P
// rows i - d staged once (two buffers).  The items (d, chunk) form one
// pipeline: the next item's loads, and at a d boundary the next kernel row,
// are issued before the current item's MFMAs; one barrier per item.  The
// partial sums of the segments (blockIdx.y) go to part as for the other
// point kernels.  Needs Ny + 1 <= 2048 (the kernel row in 8 loads per
// thread).
// ---------------------------------------------------------------------------
constexpr int kPtKG = 8;                // K-steps per chunk
constexpr int kPtGJ = 4 * kPtKG;        // rows jp per chunk
constexpr int kPtPB = 4 * kPtKG + 2;    // staged column stride
constexpr int kPtKV = 8;                // kernel-row loads per thread

template <int PREC>
__global__ void __launch_bounds__(256) point_deform_tiled(int Nx, int Ny, int nseg, int B,
                                                          const double* __restrict__ k2,
                                                          const double* __restrict__ P,
                                                          double* __restrict__ part)
{
    using T = typename std::conditional<PREC == PREC_FP64, double, float>::type;
    constexpr int LKG = kPtKG, LGJ = kPtGJ, LPB = kPtPB;
    constexpr int SPT = LGJ / 16;  // staged values per thread
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
    T* pt = reinterpret_cast<T*>(lds_raw);  // [2][16][LPB] staged P chunks
    T* skb = pt + 2 * 16 * LPB;             // [2][Ny + 1] kernel rows (zero at Ny)
    const int NS = Ny + 1;
    const int tid = threadIdx.x;
    const int wave = tid / 64, l = tid % 64;
    const int li = l % 16, lk = l / 16;
    const int nbj = (Ny + 63) / 64;
    const int tj = (int)blockIdx.x % nbj, ti = (int)blockIdx.x / nbj;
    const int jw0 = tj * 64 + wave * 16;  // this wave's first output row j
    const int i0 = ti * 16;               // the workgroup's output columns i
    const int s = blockIdx.y, inst = blockIdx.z;
    if (i0 >= Nx) return;  // the whole workgroup
    const double* Pi = P + (int64_t)inst * Nx * Ny;
    // offsets d with i - d in [0, Nx) for some i of the workgroup, split
    // into nseg segments
    const int dlo = i0 - (Nx - 1), dhi = min(i0 + 15, Nx - 1);
    const int per = (dhi - dlo + 1 + nseg - 1) / nseg;
    const int ds0 = dlo + s * per, ds1 = min(dhi, ds0 + per - 1);
    const int nd = ds1 >= ds0 ? ds1 - ds0 + 1 : 0;
    const int nch = (Ny + LGJ - 1) / LGJ;
    const int nitems = nd * nch;
    typedef typename std::conditional<PREC == PREC_FP64, f64x4, f32x4>::type acc_t;
    acc_t ce = {0, 0, 0, 0}, co = {0, 0, 0, 0};
    const int ja = jw0 + li;  // A row (output j) of this lane
    const bool ina = ja < Ny;
    const bool rows_in = jw0 + 15 < Ny;
    // chunk ranges of the wave's rows (uniform): every jp below every j,
    // every jp above (and inside), the others
    const int gA = (rows_in && jw0 >= LGJ - 1) ? (jw0 - (LGJ - 1)) / LGJ + 1 : 0;
    const int gB = rows_in ? max(gA, (jw0 + 15 + LGJ - 1) / LGJ) : 0;
    const int gC = rows_in ? max(gB, min(nch, Ny >= LGJ ? (Ny - LGJ) / LGJ + 1 : 0)) : 0;
    // staging of P: thread t takes column i0 + t / 16 (P row i - d), rows
    // jp = chunk start + SPT (t % 16) ..
    const int sc = tid / 16, sj = SPT * (tid % 16);
    const int icol = i0 + sc;
    double stv[SPT];
    bool sok = false;
    auto gload = [&](int d, int c) {
        const int ip = icol - d;
        sok = icol < Nx && ip >= 0 && ip < Nx;
        const double* pr = Pi + (int64_t)min(max(ip, 0), Nx - 1) * Ny;
        const int j = c * LGJ + sj;
#pragma unroll
        for (int e = 0; e < SPT; e++) stv[e] = pr[min(j + e, Ny - 1)];
    };
    auto lstore = [&](int buf, int c) {
        const int j = c * LGJ + sj;
        T* d = pt + (buf * 16 + sc) * LPB + sj;
#pragma unroll
        for (int e = 0; e < SPT; e++) d[e] = (sok && j + e < Ny) ? (T)stv[e] : (T)0;
    };
    double kv[kPtKV];
    auto kload = [&](int d) {
        const double* kr = k2 + (int64_t)abs(d) * Ny;
#pragma unroll
        for (int e = 0; e < kPtKV; e++) kv[e] = kr[min(tid + 256 * e, Ny - 1)];
    };
    auto kstore = [&](int buf) {
#pragma unroll
        for (int e = 0; e < kPtKV; e++) {
            const int t = tid + 256 * e;
            if (t <= Ny) skb[buf * NS + t] = t < Ny ? (T)kv[e] : (T)0;
        }
    };
    if (nitems > 0) {
        kload(ds0);
        gload(ds0, 0);
        kstore(0);
        lstore(0, 0);
        __syncthreads();
        int d = ds0, c = 0, dpar = 0;
        for (int it = 0; it < nitems; it++) {
            int dn = d, cn = c + 1;
            if (cn == nch) {
                cn = 0;
                dn = d + 1;
            }
            const bool more = it + 1 < nitems;
            const bool newd = more && cn == 0;
            if (more) gload(dn, cn);  // the next item in flight
            if (newd) kload(dn);
            if (jw0 < Ny) {
                const T* sk = skb + dpar * NS;
                const int jg = c * LGJ;
                T av[LKG];
                if (c < gA) {
                    const T* ap = sk + (ja - jg - LKG * lk - (LKG - 1));
#pragma unroll
                    for (int u = 0; u < LKG; u++) av[u] = ap[LKG - 1 - u];
                } else if (c >= gB && c < gC) {
                    const T* ap = sk + (jg + LKG * lk - ja);
#pragma unroll
                    for (int u = 0; u < LKG; u++) av[u] = ap[u];
                } else {
#pragma unroll
                    for (int u = 0; u < LKG; u++) {
                        const int jp = jg + LKG * lk + u;
                        av[u] = sk[(ina && jp < Ny) ? abs(ja - jp) : Ny];
                    }
                }
                const T* bp = pt + ((it & 1) * 16 + li) * LPB + LKG * lk;
#pragma unroll
                for (int u = 0; u < LKG; u++) {
                    const T x = bp[u];
                    if constexpr (PREC == PREC_FP64) {
                        if (u % 2 == 0) ce = mfma_f64(av[u], x, ce);
                        else co = mfma_f64(av[u], x, co);
                    } else {
                        if (u % 2 == 0) ce = mfma_f32(av[u], x, ce);
                        else co = mfma_f32(av[u], x, co);
                    }
                }
            }
            if (more) lstore((it + 1) & 1, cn);
            if (newd) kstore(dpar ^ 1);
            __syncthreads();
            if (newd) dpar ^= 1;
            d = dn;
            c = cn;
        }
    }
    // D element r of lane l: FP64 row 4 r + l/16, FP32 row 4 (l/16) + r (output
    // j), column l % 16 (output i); every segment writes its tile (the
    // reduction sums all of them)
    double* dst = part + ((int64_t)s * B + inst) * Nx * Ny;
    const int io = i0 + li;
    if (io < Nx && jw0 < Ny) {
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int jo = jw0 + (PREC == PREC_FP64 ? 4 * r + lk : 4 * lk + r);
            if (jo < Ny) dst[(int64_t)io * Ny + jo] = (double)ce[r] + (double)co[r];
        }
    }
}

template <int PREC>
static size_t point_tiled_lds(int Ny)
{
    return (size_t)(2 * 16 * kPtPB + 2 * (Ny + 1)) * (PREC == PREC_FP64 ? 8 : 4);
}

__global__ void point_reduce_kernel(int64_t count, int nseg, const double* __restrict__ part,
                                    double* __restrict__ out)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= count) return;
    double s = 0.0;
    for (int g = 0; g < nseg; g++) s += part[(int64_t)g * count + idx];
    out[idx] = s;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
int launch_line_kernel_vec(int N, double h, double* k, hipStream_t s)
{
    hipLaunchKernelGGL(line_kernel_vec, dim3((N + 255) / 256), dim3(256), 0, s, N, h, k);
    return hip_ok(hipGetLastError()) ? PAQIF_OK : PAQIF_EHIP;
}

int launch_point_kernel_tab(int Nx, int Ny, double hx, double hy, double* k2, hipStream_t s)
{
    hipLaunchKernelGGL(point_kernel_tab, dim3((Nx * Ny + 255) / 256), dim3(256), 0, s, Nx, Ny, hx,
                       hy, k2);
    return hip_ok(hipGetLastError()) ? PAQIF_OK : PAQIF_EHIP;
}

// ---------------------------------------------------------------------------
// Line contact, split BF16 on gfx950's v_mfma_f32_16x16x32_bf16: every
// operand x = hi + lo with hi = bf16(x), lo = bf16(x - hi), and the product
// hi*hi + hi*lo + lo*hi accumulated in FP32 (three MFMAs per 32 rows j).
// Same tiling as line_deform_tiled: a 16x16 output tile per wave, 4 waves
// along i per workgroup, 64-row chunks of the workgroup's 16 P columns
// staged through LDS once, split into hi and lo halves as they are stored
// (a lane's 8 consecutive rows are one aligned 16-byte read per half).  The
// kernel vector sits in LDS split and packed, hi | lo << 16 per entry (zero
// at index N), so a lane's 8 entries at any alignment are four 2-dword
// reads, separated into hi and lo operands by byte permutes.  Lane k-group
// lk, element e of step u takes row j = j0 + 16 lk + 8 u + e.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8v __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
constexpr int SBJ = 64;        // rows j per chunk
constexpr int SBP = SBJ + 8;   // staged column stride in bf16 (16-byte aligned)

PQ_DEV uint32_t bf16_hi_lo(float x)
{
    short h, lo;
    split_bf16(x, h, lo);
    return (uint32_t)(uint16_t)h | ((uint32_t)(uint16_t)lo << 16);
}

PQ_DEV f32x4 mfma_bf16x32(u32x4 a, u32x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8v, a),
                                                   __builtin_bit_cast(bf16x8v, b), c, 0, 0, 0);
}

__global__ void __launch_bounds__(256) line_deform_sbf16(int N, int B,
                                                         const double* __restrict__ kvec,
                                                         const double* __restrict__ P,
                                                         double* __restrict__ out)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
    uint16_t* ph = reinterpret_cast<uint16_t*>(lds_raw);  // [2][16][SBP] hi halves
    uint16_t* pl = ph + 2 * 16 * SBP;                      // [2][16][SBP] lo halves
    uint32_t* kv = reinterpret_cast<uint32_t*>(pl + 2 * 16 * SBP);  // N + 1 packed
    const int tid = threadIdx.x;
    for (int t0 = 0; t0 <= N; t0 += 8 * 256) {
        double k8[8];
#pragma unroll
        for (int e = 0; e < 8; e++) k8[e] = kvec[min(t0 + e * 256 + tid, N - 1)];
#pragma unroll
        for (int e = 0; e < 8; e++) {
            const int t = t0 + e * 256 + tid;
            if (t <= N) kv[t] = t < N ? bf16_hi_lo((float)k8[e]) : 0u;
        }
    }
    const int wave = tid / 64, l = tid % 64;
    const int li = l % 16, lk = l / 16;
    const int i0 = blockIdx.x * 64 + wave * 16;
    const int b0 = blockIdx.y * 16;
    const int ia = i0 + li;
    const bool ina = ia < N;
    const int nch = (N + SBJ - 1) / SBJ;
    constexpr int SPT = SBJ / 16;  // staged values per thread
    const int sc = tid / 16, sj = SPT * (tid % 16);
    const bool scol = b0 + sc < B;
    const double* pcol = P + (int64_t)(scol ? b0 + sc : 0) * N;
    double stv[SPT];
    auto gload = [&](int c) {
        const int j = c * SBJ + sj;
#pragma unroll
        for (int e = 0; e < SPT; e++) stv[e] = pcol[min(j + e, N - 1)];
    };
    auto lstore = [&](int c) {
        const int j = c * SBJ + sj;
        const int o = ((c & 1) * 16 + sc) * SBP + sj;
#pragma unroll
        for (int e = 0; e < SPT; e++) {
            const uint32_t hl = (scol && j + e < N) ? bf16_hi_lo((float)stv[e]) : 0u;
            ph[o + e] = (uint16_t)(hl & 0xFFFFu);
            pl[o + e] = (uint16_t)(hl >> 16);
        }
    };
    gload(0);
    lstore(0);
    __syncthreads();
    f32x4 c0 = {0, 0, 0, 0}, c1 = {0, 0, 0, 0};
    const bool rows_in = i0 + 15 < N;
    const int gA = (rows_in && i0 >= SBJ - 1) ? (i0 - (SBJ - 1)) / SBJ + 1 : 0;
    const int gB = rows_in ? max(gA, (i0 + 15 + SBJ - 1) / SBJ) : 0;
    const int gC = rows_in ? max(gB, min(nch, N >= SBJ ? (N - SBJ) / SBJ + 1 : 0)) : 0;
    for (int c = 0; c < nch; c++) {
        if (c + 1 < nch) gload(c + 1);
        const int jg = c * SBJ;
        const int bo = ((c & 1) * 16 + li) * SBP + 16 * lk;
#pragma unroll
        for (int u = 0; u < 2; u++) {
            const int jb = jg + 16 * lk + 8 * u;  // this lane's first row j of the step
            uint32_t av[8];
            if (i0 < N && c < gA) {  // every j below every i: k[i - j], index descending
                const uint32_t* ap = kv + (ia - jb - 7);
#pragma unroll
                for (int e = 0; e < 8; e++) av[e] = ap[7 - e];
            } else if (i0 < N && c >= gB && c < gC) {  // every j above every i: k[j - i]
                const uint32_t* ap = kv + (jb - ia);
#pragma unroll
                for (int e = 0; e < 8; e++) av[e] = ap[e];
            } else {
#pragma unroll
                for (int e = 0; e < 8; e++) {
                    const int j = jb + e;
                    av[e] = kv[(ina && j < N) ? abs(ia - j) : N];
                }
            }
            u32x4 ah, al;
#pragma unroll
            for (int q = 0; q < 4; q++) {
                // low halves of entries 2q, 2q+1 -> hi operand; high halves -> lo operand
                ah[q] = __builtin_amdgcn_perm(av[2 * q + 1], av[2 * q], 0x05040100u);
                al[q] = __builtin_amdgcn_perm(av[2 * q + 1], av[2 * q], 0x07060302u);
            }
            const u32x4 bh = *reinterpret_cast<const u32x4*>(ph + bo + 8 * u);
            const u32x4 bl = *reinterpret_cast<const u32x4*>(pl + bo + 8 * u);
            c0 = mfma_bf16x32(ah, bh, c0);
            c1 = mfma_bf16x32(ah, bl, c1);
            c1 = mfma_bf16x32(al, bh, c1);
        }
        if (c + 1 < nch) lstore(c + 1);
        __syncthreads();
    }
    const int ca = b0 + li;
    if (ca < B && i0 < N) {
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int ro = i0 + 4 * lk + r;
            if (ro < N) out[(int64_t)ca * N + ro] = (double)(c0[r] + c1[r]);
        }
    }
}

static size_t line_sbf16_lds(int N) { return (size_t)(4 * 16 * SBP) * 2 + (size_t)(N + 1) * 4; }

// ---------------------------------------------------------------------------
// Point contact, split BF16: the items (d, chunk of rows jp) of
// point_deform_tiled with the operands of line_deform_sbf16: the kernel row
// k2[|d|] packed hi | lo (two buffers by the parity of d), each staged chunk
// of the 16 shifted P rows as hi and lo halves, one K = 32 step per chunk
// (k-group lk of a lane takes rows jp = chunk start + 8 lk .. + 7), three
// products hi*hi + hi*lo + lo*hi.  Needs Ny + 1 <= 2048.
// ---------------------------------------------------------------------------
constexpr int kPsJ = 32;        // rows jp per chunk
constexpr int kPsP = kPsJ + 8;  // staged column stride in bf16 (16-byte aligned)

__global__ void __launch_bounds__(256) point_deform_sbf16(int Nx, int Ny, int nseg, int B,
                                                          const double* __restrict__ k2,
                                                          const double* __restrict__ P,
                                                          double* __restrict__ part)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
    uint16_t* ph = reinterpret_cast<uint16_t*>(lds_raw);  // [2][16][kPsP] hi halves
    uint16_t* pl = ph + 2 * 16 * kPsP;                     // [2][16][kPsP] lo halves
    uint32_t* skb = reinterpret_cast<uint32_t*>(pl + 2 * 16 * kPsP);  // [2][Ny + 1] packed
    const int NS = Ny + 1;
    const int tid = threadIdx.x;
    const int wave = tid / 64, l = tid % 64;
    const int li = l % 16, lk = l / 16;
    const int nbj = (Ny + 63) / 64;
    const int tj = (int)blockIdx.x % nbj, ti = (int)blockIdx.x / nbj;
    const int jw0 = tj * 64 + wave * 16;
    const int i0 = ti * 16;
    const int s = blockIdx.y, inst = blockIdx.z;
    if (i0 >= Nx) return;  // the whole workgroup
    const double* Pi = P + (int64_t)inst * Nx * Ny;
    const int dlo = i0 - (Nx - 1), dhi = min(i0 + 15, Nx - 1);
    const int per = (dhi - dlo + 1 + nseg - 1) / nseg;
    const int ds0 = dlo + s * per, ds1 = min(dhi, ds0 + per - 1);
    const int nd = ds1 >= ds0 ? ds1 - ds0 + 1 : 0;
    const int nch = (Ny + kPsJ - 1) / kPsJ;
    const int nitems = nd * nch;
    f32x4 c0 = {0, 0, 0, 0}, c1 = {0, 0, 0, 0};
    const int ja = jw0 + li;
    const bool ina = ja < Ny;
    const bool rows_in = jw0 + 15 < Ny;
    const int gA = (rows_in && jw0 >= kPsJ - 1) ? (jw0 - (kPsJ - 1)) / kPsJ + 1 : 0;
    const int gB = rows_in ? max(gA, (jw0 + 15 + kPsJ - 1) / kPsJ) : 0;
    const int gC = rows_in ? max(gB, min(nch, Ny >= kPsJ ? (Ny - kPsJ) / kPsJ + 1 : 0)) : 0;
    constexpr int SPT = kPsJ / 16;
    const int sc = tid / 16, sj = SPT * (tid % 16);
    const int icol = i0 + sc;
    double stv[SPT];
    bool sok = false;
    auto gload = [&](int d, int c) {
        const int ip = icol - d;
        sok = icol < Nx && ip >= 0 && ip < Nx;
        const double* pr = Pi + (int64_t)min(max(ip, 0), Nx - 1) * Ny;
        const int j = c * kPsJ + sj;
#pragma unroll
        for (int e = 0; e < SPT; e++) stv[e] = pr[min(j + e, Ny - 1)];
    };
    auto lstore = [&](int buf, int c) {
        const int j = c * kPsJ + sj;
        const int o = (buf * 16 + sc) * kPsP + sj;
#pragma unroll
        for (int e = 0; e < SPT; e++) {
            const uint32_t hl = (sok && j + e < Ny) ? bf16_hi_lo((float)stv[e]) : 0u;
            ph[o + e] = (uint16_t)(hl & 0xFFFFu);
            pl[o + e] = (uint16_t)(hl >> 16);
        }
    };
    double kv[kPtKV];
    auto kload = [&](int d) {
        const double* kr = k2 + (int64_t)abs(d) * Ny;
#pragma unroll
        for (int e = 0; e < kPtKV; e++) kv[e] = kr[min(tid + 256 * e, Ny - 1)];
    };
    auto kstore = [&](int buf) {
#pragma unroll
        for (int e = 0; e < kPtKV; e++) {
            const int t = tid + 256 * e;
            if (t <= Ny) skb[buf * NS + t] = t < Ny ? bf16_hi_lo((float)kv[e]) : 0u;
        }
    };
    if (nitems > 0) {
        kload(ds0);
        gload(ds0, 0);
        kstore(0);
        lstore(0, 0);
        __syncthreads();
        int d = ds0, c = 0, dpar = 0;
        for (int it = 0; it < nitems; it++) {
            int dn = d, cn = c + 1;
            if (cn == nch) {
                cn = 0;
                dn = d + 1;
            }
            const bool more = it + 1 < nitems;
            const bool newd = more && cn == 0;
            if (more) gload(dn, cn);
            if (newd) kload(dn);
            if (jw0 < Ny) {
                const uint32_t* sk = skb + dpar * NS;
                const int jb = c * kPsJ + 8 * lk;  // this lane's first row jp
                uint32_t av[8];
                if (c < gA) {
                    const uint32_t* ap = sk + (ja - jb - 7);
#pragma unroll
                    for (int e = 0; e < 8; e++) av[e] = ap[7 - e];
                } else if (c >= gB && c < gC) {
                    const uint32_t* ap = sk + (jb - ja);
#pragma unroll
                    for (int e = 0; e < 8; e++) av[e] = ap[e];
                } else {
#pragma unroll
                    for (int e = 0; e < 8; e++) {
                        const int jp = jb + e;
                        av[e] = sk[(ina && jp < Ny) ? abs(ja - jp) : Ny];
                    }
                }
                u32x4 ah, al;
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    ah[q] = __builtin_amdgcn_perm(av[2 * q + 1], av[2 * q], 0x05040100u);
                    al[q] = __builtin_amdgcn_perm(av[2 * q + 1], av[2 * q], 0x07060302u);
                }
                const int bo = ((it & 1) * 16 + li) * kPsP + 8 * lk;
                const u32x4 bh = *reinterpret_cast<const u32x4*>(ph + bo);
                const u32x4 bl = *reinterpret_cast<const u32x4*>(pl + bo);
                c0 = mfma_bf16x32(ah, bh, c0);
                c1 = mfma_bf16x32(ah, bl, c1);
                c1 = mfma_bf16x32(al, bh, c1);
            }
            if (more) lstore((it + 1) & 1, cn);
            if (newd) kstore(dpar ^ 1);
            __syncthreads();
            if (newd) dpar ^= 1;
            d = dn;
            c = cn;
        }
    }
    double* dst = part + ((int64_t)s * B + inst) * Nx * Ny;
    const int io = i0 + li;
    if (io < Nx && jw0 < Ny) {
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int jo = jw0 + 4 * lk + r;
            if (jo < Ny) dst[(int64_t)io * Ny + jo] = (double)(c0[r] + c1[r]);
        }
    }
}

static size_t point_sbf16_lds(int Ny) { return (size_t)(4 * 16 * kPsP) * 2 + (size_t)(Ny + 1) * 8; }

// LDS of line_deform_tiled: two staged B chunks, the kernel vector and a zero
template <int PREC>
static size_t line_tiled_lds(int N)
{
    return (size_t)(2 * 16 * line_pb<PREC>() + N + 1) * (PREC == PREC_FP64 ? 8 : 4);
}

int launch_line_deform(int N, int B, int prec, const double* k, const double* P, double* out,
                       hipStream_t s)
{
    if (N <= 0 || B <= 0) return PAQIF_OK;
    dim3 grid((N + 63) / 64, (B + 31) / 32), block(256);
    const size_t lds = (size_t)N * sizeof(double);
    const dim3 gridt((N + 63) / 64, (B + 15) / 16);
    // the tiled kernel where its LDS fits in 64 KB (FP32: every line grid,
    // nx <= 8192; FP64 up to about 6000 nodes), else the untiled one
    constexpr size_t kLdsMax = 65536;
    if (prec == PREC_FP64 && line_tiled_lds<PREC_FP64>(N) <= kLdsMax)
        hipLaunchKernelGGL((line_deform_tiled<PREC_FP64>), gridt, block,
                           line_tiled_lds<PREC_FP64>(N), s, N, B, k, P, out);
    else if (prec == PREC_FP64)
        hipLaunchKernelGGL((line_deform_kernel<PREC_FP64>), grid, block, lds, s, N, B, k, P, out);
    else if (prec == PREC_FP32 && line_tiled_lds<PREC_FP32>(N) <= kLdsMax)
        hipLaunchKernelGGL((line_deform_tiled<PREC_FP32>), gridt, block,
                           line_tiled_lds<PREC_FP32>(N), s, N, B, k, P, out);
    else if (prec == PREC_FP32)
        hipLaunchKernelGGL((line_deform_kernel<PREC_FP32>), grid, block, lds, s, N, B, k, P, out);
    else if (line_sbf16_lds(N) <= kLdsMax)
        hipLaunchKernelGGL(line_deform_sbf16, gridt, block, line_sbf16_lds(N), s, N, B, k, P, out);
    else
        hipLaunchKernelGGL((line_deform_kernel<PREC_SPLIT_BF16>), grid, block, lds, s, N, B, k, P,
                           out);
    return hip_ok(hipGetLastError()) ? PAQIF_OK : PAQIF_EHIP;
}

// segments of the d range: about 4096 waves of 32 x 32 tiles at one instance
// (four per SIMD, to hide the operand-load latency), at most 64
int point_segments(int Nx, int Ny)
{
    const int tiles = ((Nx + 31) / 32) * ((Ny + 31) / 32);
    return std::max(1, std::min(64, 4096 / std::max(1, tiles)));
}

size_t point_workspace_doubles(int Nx, int Ny, int B)
{
    return (size_t)Nx * Ny + (size_t)point_segments(Nx, Ny) * B * Nx * Ny;
}

int launch_point_deform(int Nx, int Ny, int B, int prec, const double* k2, const double* P,
                        double* out, double* part, hipStream_t s)
{
    if (Nx <= 0 || Ny <= 0 || B <= 0) return PAQIF_OK;
    int nseg = point_segments(Nx, Ny);
    const int ntj32 = (Ny + 31) / 32, nti32 = (Nx + 31) / 32;
    const dim3 grid32(ntj32 * ((nti32 + 3) / 4), nseg, B), block(256);
    const int ntj = (Ny + 15) / 16, nti = (Nx + 15) / 16;
    const dim3 grid(ntj * ((nti + 3) / 4), nseg, B);
    // the staged kernels (Ny + 1 <= 256 kPtKV); segments for about 4096
    // waves at one instance, within the workspace's nseg
    const bool tiled = Ny + 1 <= 256 * kPtKV;
    if (tiled) {
        const int nbj = (Ny + 63) / 64, nbi = (Nx + 15) / 16;
        nseg = std::max(1, std::min(nseg, 4096 / (4 * nbj * nbi)));
        const dim3 gridp(nbj * nbi, nseg, B);
        if (prec == PREC_FP64)
            hipLaunchKernelGGL((point_deform_tiled<PREC_FP64>), gridp, block,
                               point_tiled_lds<PREC_FP64>(Ny), s, Nx, Ny, nseg, B, k2, P, part);
        else if (prec == PREC_FP32)
            hipLaunchKernelGGL((point_deform_tiled<PREC_FP32>), gridp, block,
                               point_tiled_lds<PREC_FP32>(Ny), s, Nx, Ny, nseg, B, k2, P, part);
        else
            hipLaunchKernelGGL(point_deform_sbf16, gridp, block, point_sbf16_lds(Ny), s, Nx, Ny,
                               nseg, B, k2, P, part);
    } else if (prec == PREC_FP64)
        hipLaunchKernelGGL((point_deform_kernel32<PREC_FP64>), grid32, block, 0, s, Nx, Ny, nseg,
                           B, k2, P, part);
    else if (prec == PREC_FP32)
        hipLaunchKernelGGL((point_deform_kernel32<PREC_FP32>), grid32, block, 0, s, Nx, Ny, nseg,
                           B, k2, P, part);
    else
        hipLaunchKernelGGL((point_deform_kernel<PREC_SPLIT_BF16>), grid, block, 0, s, Nx, Ny, nseg,
                           B, k2, P, part);
    if (!hip_ok(hipGetLastError())) return PAQIF_EHIP;
    const int64_t count = (int64_t)B * Nx * Ny;
    hipLaunchKernelGGL(point_reduce_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s,
                       count, nseg, part, out);
    return hip_ok(hipGetLastError()) ? PAQIF_OK : PAQIF_EHIP;
}

}  // namespace pq

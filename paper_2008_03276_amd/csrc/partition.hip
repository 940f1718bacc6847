// Partitioned PAQIF solve of ONE long band system (Sec. 2.1 eqs. 15-18,
// Sec. 2.2 "PAQIF method", Steps 1-7), spread over many wavefronts.
//
// The system of order N, half-bandwidth q, is cut into r consecutive blocks,
// block m owning rows p_m .. p_{m+1}-1 with p_m = floor(m N / r).  Its first
// q and last q unknowns are the outer unknowns U_F, U_L; the rest, U_M, are
// inner.  Inner rows only touch unknowns of their own block, so
//   A_ii u_M = f_i - A_io u_o                                  (Step 6)
// and the outer rows, after the inner unknowns are eliminated, form the
// reduced system on the outer unknowns of all blocks                (Step 4)
//   S_m u_o^(m) + L-^(m) U_L^(m-1) + L+^(m) U_F^(m+1) = g_m,
//   S_m = A_oo - A_oi A_ii^{-1} A_io,  g_m = f_o - A_oi A_ii^{-1} f_i.
// The paper writes these rows after the centre-out factorisation of the
// block, i.e. multiplied on the left by the inverse of the outer 2q x 2q
// block of W0 (Steps 1-3); the solution is the same.  In the natural order
// (U_F^(1), U_L^(1), U_F^(2), ...) the reduced matrix is a band of
// half-bandwidth 2q - 1 and order 2 q r.
//
// GPU realisation, five launches on one stream:
//   1. part_rhs: the 2q+1 right-hand sides of every block's inner system:
//      f_i and the 2q columns of A_io (nonzero on q rows each);
//   2. one batched PAQIF launch (plain linear mode) over the (2q+1) r inner
//      systems -- all blocks and right-hand sides in parallel (Steps 1-2);
//      the 2q+1 systems of a block read the same rows of the caller's band
//      (the kernel ignores the entries whose column falls outside the inner
//      system, which are exactly the couplings A_io);
//   3. part_reduce: S_m, g_m from the solutions next to the outer rows, and
//      the reduced band rows with the couplings L-, L+ (Steps 3-4);
//   4. the reduced system (half-bandwidth 2q) solved directly, in place of
//      the paper's normal equations: one PAQIF launch on one wavefront or,
//      for q = 2 and at least 512 reduced rows, the same partitioned scheme
//      once more (half-bandwidth 4 over about sqrt(K/8) blocks, its own
//      reduced system of half-bandwidth 8 solved whole);
//   5. part_combine: the outer unknowns projected on bounded rows in clip
//      mode (Step 5), u_M = x_f - X_io u_o with those values (Step 6),
//      projected (Step 7).
#include <algorithm>
#include <climits>
#include <cmath>

#include "common.h"
#include "paqif_args.h"

namespace pq {
namespace {

struct PartGeo {
    int64_t N;
    int q, r;
    int64_t Ni;  // inner rows of all blocks, N - 2 q r
};

PQ_DEV int64_t pstart(const PartGeo& g, int64_t m) { return (m * g.N) / g.r; }
// first compacted inner row of block m
PQ_DEV int64_t ioff(const PartGeo& g, int64_t m) { return pstart(g, m) - 2 * (int64_t)g.q * m; }

// block owning global row `row`: largest m with p_m <= row
PQ_DEV int block_of_row(const PartGeo& g, int64_t row)
{
    int lo = 0, hi = g.r - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pstart(g, mid) <= row) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// block owning compacted inner row `ir`
PQ_DEV int block_of_inner(const PartGeo& g, int64_t ir)
{
    int lo = 0, hi = g.r - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ioff(g, mid) <= ir) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// a(row, col) of the band (0 outside the band or the matrix)
PQ_DEV double band_at(const PartGeo& g, const double* band, int64_t row, int64_t col)
{
    const int64_t d = col - row;
    if (col < 0 || col >= g.N || d < -g.q || d > g.q) return 0.0;
    return band[row * (2 * g.q + 1) + (d + g.q)];
}

// global column of outer unknown j (0..2q-1) of block m
PQ_DEV int64_t outer_col(const PartGeo& g, int m, int j)
{
    return j < g.q ? pstart(g, m) + j : pstart(g, m + 1) - 2 * g.q + j;
}

// system k = t r + m: rows of its right-hand side / solution in the
// expanded arrays, and its first band row in the caller's band
__global__ void part_offsets_kernel(PartGeo g, int64_t* eoffs, int64_t* eboff)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t cnt = (int64_t)(2 * g.q + 1) * g.r;
    if (k > cnt) return;
    if (k == cnt) {
        eoffs[k] = (2 * g.q + 1) * g.Ni;
        return;
    }
    const int64_t t = k / g.r, m = k % g.r;
    eoffs[k] = t * g.Ni + ioff(g, m);
    eboff[k] = pstart(g, m) + g.q;
}

// Expanded row e = t * Ni + ir: inner row ir of its block with right-hand
// side t (0: f, 1 + j: column of outer unknown j).
// With pins (the exact mode's active set): the inner systems' flags are
// set from them, and the column of a pinned outer unknown is zero.
__global__ void part_rhs_kernel(PartGeo g, const double* __restrict__ band,
                                const double* __restrict__ f, const uint8_t* __restrict__ pin,
                                double* __restrict__ erhs, uint8_t* __restrict__ eact)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int W = 2 * g.q + 1;
    if (e >= (int64_t)W * g.Ni) return;
    const int t = (int)(e / g.Ni);
    const int64_t ir = e - (int64_t)t * g.Ni;
    const int m = block_of_inner(g, ir);
    const int64_t row = ir + 2 * (int64_t)g.q * m + g.q;  // global row
    if (pin) eact[e] = pin[row];
    double v;
    if (t == 0) {
        v = f[row];
    } else {
        const int64_t col = outer_col(g, m, t - 1);
        v = (pin && pin[col]) ? 0.0 : band_at(g, band, row, col);
    }
    erhs[e] = v;
}

// Reduced row R = 2 q m + c: S_m and g_m from the inner solutions next to
// the outer row, plus the couplings to the neighbouring blocks.
// A pinned outer unknown gets an identity row, and its column is zero in
// the other rows (the inner solutions already vanish on pinned inner rows).
__global__ void part_reduce_kernel(PartGeo g, const double* __restrict__ band,
                                   const double* __restrict__ f, const uint8_t* __restrict__ bounded,
                                   const uint8_t* __restrict__ pin, const double* __restrict__ ex,
                                   double* __restrict__ rband, double* __restrict__ rrhs,
                                   uint8_t* __restrict__ rbnd)
{
    const int64_t R = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int q = g.q, N2 = 2 * q, RW = 4 * q + 1;
    if (R >= (int64_t)N2 * g.r) return;
    const int m = (int)(R / N2), c = (int)(R % N2);
    const int64_t row = outer_col(g, m, c);
    const int64_t in0 = pstart(g, m) + q, in1 = pstart(g, m + 1) - q;  // inner range
    const int64_t io = ioff(g, m);
    double* out = rband + R * RW;
    for (int s = 0; s < RW; s++) out[s] = 0.0;
    rbnd[R] = bounded ? (bounded[row] ? 1 : 0) : 1;
    if (pin && pin[row]) {
        out[N2] = 1.0;
        rrhs[R] = 0.0;
        return;
    }
    // S_m row c and g_m[c]
    double gv = f[row];
    for (int j = 0; j < N2; j++) {
        if (pin && pin[outer_col(g, m, j)]) continue;
        double s = band_at(g, band, row, outer_col(g, m, j));
        for (int d = -q; d <= q; d++) {
            const int64_t col = row + d;
            if (col < in0 || col >= in1) continue;
            s -= band_at(g, band, row, col) * ex[(int64_t)(1 + j) * g.Ni + io + (col - in0)];
        }
        out[(int64_t)N2 * m + j - R + N2] = s;
    }
    for (int d = -q; d <= q; d++) {
        const int64_t col = row + d;
        if (col < in0 || col >= in1) continue;
        gv -= band_at(g, band, row, col) * ex[io + (col - in0)];
    }
    // couplings: first q rows to U_L^(m-1), last q rows to U_F^(m+1)
    if (c < q && m > 0) {
        for (int j = 0; j < q; j++) {
            const int64_t col = pstart(g, m) - q + j;
            if (pin && pin[col]) continue;
            out[(int64_t)N2 * (m - 1) + q + j - R + N2] += band_at(g, band, row, col);
        }
    } else if (c >= q && m + 1 < g.r) {
        for (int j = 0; j < q; j++) {
            const int64_t col = pstart(g, m + 1) + j;
            if (pin && pin[col]) continue;
            out[(int64_t)N2 * (m + 1) + j - R + N2] += band_at(g, band, row, col);
        }
    }
    rrhs[R] = gv;
}

// outer unknown R of the reduced solution, projected in clip mode (Step 5)
PQ_DEV double outer_value(const double* rx, const uint8_t* rbnd, int clip, int64_t R)
{
    const double v = rx[R];
    return (clip && rbnd[R]) ? (v > 0.0 ? v : 0.0) : v;
}

__global__ void part_combine_kernel(PartGeo g, const uint8_t* __restrict__ bounded, int clip,
                                    const double* __restrict__ ex, const double* __restrict__ rx,
                                    const uint8_t* __restrict__ rbnd, double* __restrict__ u)
{
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= g.N) return;
    const int q = g.q, N2 = 2 * q;
    const int m = block_of_row(g, row);
    const int64_t p0 = pstart(g, m), p1 = pstart(g, m + 1);
    const int64_t base = (int64_t)N2 * m;
    if (row < p0 + q) {
        u[row] = outer_value(rx, rbnd, clip, base + (row - p0));
        return;
    }
    if (row >= p1 - q) {
        u[row] = outer_value(rx, rbnd, clip, base + q + (row - (p1 - q)));
        return;
    }
    // Step 6 with the projected outer unknowns, then Step 7
    const int64_t ir = ioff(g, m) + (row - p0 - q);
    double v = ex[ir];
    for (int j = 0; j < N2; j++)
        v -= ex[(int64_t)(1 + j) * g.Ni + ir] * outer_value(rx, rbnd, clip, base + j);
    if (clip && (!bounded || bounded[row])) v = v > 0.0 ? v : 0.0;
    u[row] = v;
}

// status = the largest code over the inner systems and the reduced system
// (pinned inner solves run one active-set pass whose "not converged" code
// carries no meaning here and is dropped)
__global__ void part_status_kernel(const int32_t* __restrict__ est, int cnt,
                                   const int32_t* __restrict__ rst, int drop_lcp,
                                   int32_t* __restrict__ status)
{
    __shared__ int32_t red[256];
    int32_t v = threadIdx.x == 0 ? rst[0] : 0;
    for (int k = threadIdx.x; k < cnt; k += blockDim.x) {
        const int32_t c = est[k];
        v = max(v, (drop_lcp && c == SYS_LCP_NOT_CONVERGED) ? SYS_OK : c);
    }
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) status[0] = red[0];
}

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

struct PartLayout {
    size_t eoffs, eboff, erhs, ex, est, eit, erec, eact;
    size_t roffs, rband, rrhs, rx, rbnd, rst, rit, rrec, ract, sub;
    size_t mask, cnt;  // exact mode (top level only)
    size_t total;
};

// q = 2: a reduced system of at least kNestRows rows (half-bandwidth 4) is
// itself solved by the partitioned scheme, over sub_blocks() blocks; its own
// reduced system (half-bandwidth 8) is solved whole.
constexpr int64_t kNestRows = 512;
bool nests(int q, int64_t K) { return q == 2 && K >= kNestRows; }
int32_t sub_blocks(int64_t K, int q2)
{
    // balance the block levels (K / r) / 2 against the reduced levels q2 r
    int64_t r = (int64_t)std::sqrt((double)K / (2.0 * q2));
    r = std::max<int64_t>(1, std::min<int64_t>(r, K / (2 * q2 + 1)));
    return (int32_t)r;
}

bool part_valid(int64_t N, int q, int32_t r)
{
    if (!(q == 2 || q == 4) || r < 1 || N < 1) return false;
    if (N / r < 2 * q + 1) return false;                    // every block >= 2q+1 rows
    if ((int64_t)(2 * q + 1) * r > INT_MAX - 1) return false;
    if (N > ((int64_t)1 << 31)) return false;                // keeps m * N in int64
    if (N / r + 1 > ((int64_t)1 << 30) || (int64_t)2 * q * r > ((int64_t)1 << 30)) return false;
    return true;
}

PartLayout part_layout(int64_t N, int q, int32_t r)
{
    const size_t W = 2 * q + 1, cnt = W * (size_t)r;
    const size_t Ni = (size_t)(N - 2 * (int64_t)q * r), E = W * Ni, K = 2 * (size_t)q * r;
    PartLayout L;
    size_t p = 0;
    auto take = [&](size_t bytes) {
        const size_t at = p;
        p += a256(bytes);
        return at;
    };
    L.eoffs = take((cnt + 1) * sizeof(int64_t));
    L.eboff = take(cnt * sizeof(int64_t));
    L.erhs = take(E * sizeof(double));
    L.ex = take(E * sizeof(double));
    L.est = take(cnt * sizeof(int32_t));
    L.eit = take(cnt * sizeof(int32_t));
    L.erec = take(((E + cnt) / 2 + 1) * (size_t)record_stride(q, true) * sizeof(double));
    L.eact = take(E);
    L.roffs = take(2 * sizeof(int64_t));
    L.rband = take(K * (4 * q + 1) * sizeof(double));
    L.rrhs = take(K * sizeof(double));
    L.rx = take(K * sizeof(double));
    L.rbnd = take(K);
    L.rst = take(sizeof(int32_t));
    L.rit = take(sizeof(int32_t));
    L.rrec = take(((K + 1) / 2 + 1) * (size_t)record_stride(2 * q, true) * sizeof(double));
    L.ract = take(K);
    L.sub = nests(q, (int64_t)K) ? take(part_layout((int64_t)K, 2 * q,
                                                    sub_blocks((int64_t)K, 2 * q)).total)
                                 : p;
    L.mask = take((size_t)N);
    L.cnt = take(sizeof(unsigned long long));
    L.total = p;
    return L;
}

__global__ void part_roffs_kernel(int64_t K, int64_t* roffs)
{
    if (threadIdx.x == 0) {
        roffs[0] = 0;
        roffs[1] = K;
    }
}

unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

LcpArgs lcp_args(int32_t count, const int64_t* offs, const double* band, const double* b,
                 const uint8_t* bounded, int mode, double* u, int32_t* st, int32_t* it, void* rec,
                 uint8_t* act)
{
    LcpArgs la;
    la.count = count;
    la.offsets = offs;
    la.order = nullptr;
    la.band = band;
    la.b = b;
    la.bounded = bounded;
    la.mode = mode;
    la.max_iter = 1;
    la.refine_tol = 0.0;
    la.u = u;
    la.w = nullptr;
    la.active_out = nullptr;
    la.status = st;
    la.iters = it;
    la.rec = rec;
    la.act = act;
    la.r = nullptr;
    la.skip = nullptr;
    la.warm = 0;
    return la;
}

// One partitioned solve.  pin (or null): rows fixed at 0 (identity rows and
// columns, right-hand side 0), the exact mode's current active set.
int part_run(paqif_handle handle, int64_t n, int q, int32_t r, const double* band,
             const double* b, const uint8_t* bounded, const uint8_t* pin, int mode, double* u,
             int32_t* status, char* ws, hipStream_t s)
{
    const PartLayout L = part_layout(n, q, r);
    PartGeo g;
    g.N = n;
    g.q = q;
    g.r = r;
    g.Ni = n - 2 * (int64_t)q * r;
    const int W = 2 * q + 1;
    const int32_t cnt = W * r;
    const int64_t E = (int64_t)W * g.Ni, K = 2 * (int64_t)q * r;
    int64_t* eoffs = reinterpret_cast<int64_t*>(ws + L.eoffs);
    int64_t* eboff = reinterpret_cast<int64_t*>(ws + L.eboff);
    double* erhs = reinterpret_cast<double*>(ws + L.erhs);
    double* ex = reinterpret_cast<double*>(ws + L.ex);
    int32_t* est = reinterpret_cast<int32_t*>(ws + L.est);
    int64_t* roffs = reinterpret_cast<int64_t*>(ws + L.roffs);
    double* rband = reinterpret_cast<double*>(ws + L.rband);
    double* rrhs = reinterpret_cast<double*>(ws + L.rrhs);
    double* rx = reinterpret_cast<double*>(ws + L.rx);
    uint8_t* rbnd = reinterpret_cast<uint8_t*>(ws + L.rbnd);
    int32_t* rst = reinterpret_cast<int32_t*>(ws + L.rst);

    hipLaunchKernelGGL(part_offsets_kernel, dim3(nblk(cnt + 1)), dim3(256), 0, s, g, eoffs, eboff);
    uint8_t* eact = reinterpret_cast<uint8_t*>(ws + L.eact);
    hipLaunchKernelGGL(part_rhs_kernel, dim3(nblk(E)), dim3(256), 0, s, g, band, b, pin, erhs,
                       eact);
    if (!hip_ok(hipGetLastError())) return PAQIF_EHIP;
    // Steps 1-2: every block's inner system with its 2q+1 right-hand sides
    LcpArgs li = lcp_args(cnt, eoffs, band, erhs, nullptr, LCP_LINEAR, ex, est,
                          reinterpret_cast<int32_t*>(ws + L.eit), ws + L.erec, eact);
    li.band_off = eboff;
    if (pin) {
        // the kernel's exact mode, one solve, started from the pins in eact:
        // the solve with those rows and columns replaced by the identity
        li.mode = LCP_EXACT;
        li.warm = 1;
    }
    int e = dispatch_lcp(q, li, PREC_FP64, handle->layout[q_index(q)][0], s);
    if (e != PAQIF_OK) return e;
    // Steps 3-4: reduced band rows
    hipLaunchKernelGGL(part_reduce_kernel, dim3(nblk(K)), dim3(256), 0, s, g, band, b, bounded, pin,
                       ex, rband, rrhs, rbnd);
    if (!hip_ok(hipGetLastError())) return PAQIF_EHIP;
    // Step 4: the reduced system (half-bandwidth 2q) in plain linear mode;
    // its projection (Step 5) is applied where its values are read
    if (nests(q, K)) {
        e = part_run(handle, K, 2 * q, sub_blocks(K, 2 * q), rband, rrhs, nullptr, nullptr,
                     LCP_LINEAR, rx, rst, ws + L.sub, s);
    } else {
        // one system: lane layout 0 (a whole wavefront on it)
        hipLaunchKernelGGL(part_roffs_kernel, dim3(1), dim3(64), 0, s, K, roffs);
        LcpArgs lr = lcp_args(1, roffs, rband, rrhs, nullptr, LCP_LINEAR, rx, rst,
                              reinterpret_cast<int32_t*>(ws + L.rit), ws + L.rrec,
                              reinterpret_cast<uint8_t*>(ws + L.ract));
        e = dispatch_lcp(2 * q, lr, PREC_FP64, 0, s);
    }
    if (e != PAQIF_OK) return e;
    // Steps 5-7: projected outer unknowns, inner unknowns, their projection
    hipLaunchKernelGGL(part_combine_kernel, dim3(nblk(n)), dim3(256), 0, s, g, bounded,
                       mode == LCP_CLIP ? 1 : 0, ex, rx, rbnd, u);
    hipLaunchKernelGGL(part_status_kernel, dim3(1), dim3(256), 0, s, est, cnt, rst,
                       pin ? 1 : 0, status);
    return hip_ok(hipGetLastError()) ? PAQIF_OK : PAQIF_EHIP;
}

// active flags of the linear / clip modes: clip mode marks the bounded rows
// whose value is 0 after the projection
__global__ void part_clipped_kernel(int64_t n, const uint8_t* __restrict__ bounded, int clip,
                                    const double* __restrict__ u, uint8_t* __restrict__ act)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    act[i] = (clip && (!bounded || bounded[i]) && u[i] == 0.0) ? 1 : 0;
}

// exact mode: A_0 = {bounded i : b_i <= 0}
__global__ void part_act0_kernel(int64_t n, const double* __restrict__ b,
                                 const uint8_t* __restrict__ bounded, uint8_t* __restrict__ mask)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    mask[i] = ((!bounded || bounded[i]) && b[i] <= 0.0) ? 1 : 0;
}

__global__ void part_zero_kernel(unsigned long long* __restrict__ cnt)
{
    if (threadIdx.x == 0) cnt[0] = 0ull;
}

// w = A u - b with the caller's band; on bounded rows the next active set
// {i in A : w_i > 0} u {i not in A : u_i < 0}; counts the changes and the
// non-finite u.
__global__ void part_update_kernel(PartGeo g, const double* __restrict__ band,
                                   const double* __restrict__ b, const uint8_t* __restrict__ bounded,
                                   const double* __restrict__ u, uint8_t* __restrict__ mask,
                                   unsigned long long* __restrict__ cnt)
{
    // low 32 bits: active-set changes, high 32 bits: non-finite u
    __shared__ unsigned long long red[256];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long ch = 0;
    if (i < g.N) {
        const int q = g.q;
        double w = -b[i];
        for (int d = -q; d <= q; d++) {
            const int64_t j = i + d;
            if (j >= 0 && j < g.N) w = __builtin_fma(band[i * (2 * q + 1) + d + q], u[j], w);
        }
        const double ui = u[i];
        if (!isfinite(ui)) ch += 1ull << 32;
        if (!bounded || bounded[i]) {
            const int cur = mask[i] != 0;
            const int nxt = cur ? (w > 0.0) : (ui < 0.0);
            if (nxt != cur) {
                ch += 1;
                mask[i] = (uint8_t)nxt;
            }
        }
    }
    red[threadIdx.x] = ch;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[0]) atomicAdd(cnt, red[0]);
}

__global__ void part_finish_kernel(int32_t* __restrict__ status, int32_t* __restrict__ iters,
                                   int it, int converged, int nonfinite)
{
    if (threadIdx.x != 0) return;
    int32_t st = status[0];
    if (st == SYS_OK && nonfinite) st = SYS_NONFINITE;
    if (st == SYS_OK && !converged) st = SYS_LCP_NOT_CONVERGED;
    status[0] = st;
    if (iters) iters[0] = it;
}

}  // namespace
}  // namespace pq

extern "C" {

size_t paqif_partitioned_workspace_bytes(int64_t n, int q, int32_t r)
{
    if (!pq::part_valid(n, q, r)) return 0;
    return pq::part_layout(n, q, r).total;
}

int paqif_solve_partitioned(paqif_handle handle, int64_t n, int q, int32_t r, const double* band,
                            const double* b, const uint8_t* bounded, int mode, int max_iter,
                            double* u, uint8_t* active_out, int32_t* status, int32_t* iters,
                            void* workspace, void* stream)
{
    if (!handle || !pq::part_valid(n, q, r) ||
        !(mode == LCP_LINEAR || mode == LCP_CLIP || mode == LCP_EXACT) ||
        (mode == LCP_EXACT && max_iter < 1) || !band || !b || !u || !status || !workspace)
        return PAQIF_EINVAL;
    char* ws = static_cast<char*>(workspace);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const pq::PartLayout L = pq::part_layout(n, q, r);
    uint8_t* mask = reinterpret_cast<uint8_t*>(ws + L.mask);
    if (mode != LCP_EXACT) {
        int e = pq::part_run(handle, n, q, r, band, b, bounded, nullptr, mode, u, status, ws, s);
        if (e != PAQIF_OK) return e;
        hipLaunchKernelGGL(pq::part_finish_kernel, dim3(1), dim3(64), 0, s, status, iters, 1, 1, 0);
        if (active_out) {  // clip mode: the rows projected to 0; linear: none
            hipLaunchKernelGGL(pq::part_clipped_kernel, dim3(pq::nblk(n)), dim3(256), 0, s, n,
                               bounded, mode == LCP_CLIP ? 1 : 0, u, active_out);
        }
        return pq::hip_ok(hipGetLastError()) ? PAQIF_OK : PAQIF_EHIP;
    }
    // exact mode: active-set iteration around the partitioned solve; the
    // host reads the number of changes after every solve (synchronises s)
    pq::PartGeo g;
    g.N = n;
    g.q = q;
    g.r = r;
    g.Ni = n - 2 * (int64_t)q * r;
    unsigned long long* cnt = reinterpret_cast<unsigned long long*>(ws + L.cnt);
    hipLaunchKernelGGL(pq::part_act0_kernel, dim3(pq::nblk(n)), dim3(256), 0, s, n, b, bounded,
                       mask);
    int it = 0, converged = 0, nonfinite = 0;
    while (it < max_iter) {
        int e = pq::part_run(handle, n, q, r, band, b, bounded, mask, LCP_LINEAR, u, status, ws, s);
        if (e != PAQIF_OK) return e;
        it++;
        hipLaunchKernelGGL(pq::part_zero_kernel, dim3(1), dim3(64), 0, s, cnt);
        hipLaunchKernelGGL(pq::part_update_kernel, dim3(pq::nblk(n)), dim3(256), 0, s, g, band, b,
                           bounded, u, mask, cnt);
        unsigned long long h = 0;
        if (!pq::hip_ok(hipMemcpyAsync(&h, cnt, sizeof(h), hipMemcpyDeviceToHost, s)) ||
            !pq::hip_ok(hipStreamSynchronize(s)))
            return PAQIF_EHIP;
        nonfinite = (h >> 32) != 0;
        if (nonfinite) break;
        if ((h & 0xffffffffull) == 0) {
            converged = 1;
            break;
        }
    }
    // the loop ends with the flags of the next iteration when not converged;
    // the solution u belongs to the last solve
    hipLaunchKernelGGL(pq::part_finish_kernel, dim3(1), dim3(64), 0, s, status, iters, it,
                       converged, nonfinite);
    if (active_out &&
        !pq::hip_ok(hipMemcpyAsync(active_out, mask, (size_t)n, hipMemcpyDeviceToDevice, s)))
        return PAQIF_EHIP;
    return pq::hip_ok(hipGetLastError()) ? PAQIF_OK : PAQIF_EHIP;
}

}  // extern "C"

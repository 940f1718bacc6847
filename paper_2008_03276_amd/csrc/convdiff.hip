// Linear convection-diffusion workload (numerical results of the paper,
// Example 1 with the linear case study): (a u)_x + (b u)_y - eps Lap u = f
// on [-1, 1]^2 with Dirichlet data, a, b > 0 constant, kappa-scheme
// convection (Sec. 3.1, eqs. 40-42), 5-point diffusion, solved by alternating line
// relaxation as a defect correction whose line systems are batched PAQIF
// solves (plain linear mode, half-bandwidth 2).
//
// Grid: n x n nodes, h = 2/(n-1), node (i, j) at (x_i, y_j), arrays row major
// [i * n + j].  Convective difference along a direction at interior index i:
//   c (u_{i+1/2} - u_{i-1/2}) / h,
//   u_{i+1/2} = u_i + (1+k)/4 (u_{i+1} - u_i) + (1-k)/4 (u_i - u_{i-1}),
// with the ghost value u_{-1} = 2 u_0 - u_1 at i = 1 (so u_{1/2} = (u_0 + u_1)/2).
// Half-step along `axis`: on every line l of that direction at once solve
// M sigma = f - L_h u, M = the whole along-line operator (kappa convection +
// diffusion) plus the diagonal of the across-line part, then u += omega sigma.
// Also the paper's x-line splittings Ls0 / Ls1 and the distributive Ls3.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "common.h"
#include "paqif_args.h"

namespace pq {
namespace {

struct CdArgs {
    int n;
    double kappa, eps, a, b, h;
    const double* f;
    const double* u;
};

// convective difference at index i (1..n-2) of a line v (v[0], v[n-1] boundary)
PQ_DEV double conv_line(double vm2, double vm1, double v0, double vp1, int i, double k)
{
    const double up = v0 + 0.25 * (1.0 + k) * (vp1 - v0) + 0.25 * (1.0 - k) * (v0 - vm1);
    const double um = i >= 2 ? vm1 + 0.25 * (1.0 + k) * (v0 - vm1) + 0.25 * (1.0 - k) * (vm1 - vm2)
                             : 0.5 * (vm1 + v0);
    return up - um;
}

// f - L_h u at interior node (i, j)
PQ_DEV double defect_at(const CdArgs& A, int i, int j)
{
    const int n = A.n;
    const double* u = A.u;
    auto U = [&](int ii, int jj) { return u[(int64_t)ii * n + jj]; };
    const double c = U(i, j);
    const double cx = conv_line(i >= 2 ? U(i - 2, j) : 0.0, U(i - 1, j), c, U(i + 1, j), i, A.kappa);
    const double cy = conv_line(j >= 2 ? U(i, j - 2) : 0.0, U(i, j - 1), c, U(i, j + 1), j, A.kappa);
    const double lap = (U(i + 1, j) + U(i - 1, j) + U(i, j + 1) + U(i, j - 1) - 4.0 * c) /
                       (A.h * A.h);
    return A.f[(int64_t)i * n + j] - (A.a * cx / A.h + A.b * cy / A.h - A.eps * lap);
}

// thread per interior node: defect into rhs and the node's row of M into band
// (line l, row r: x-lines l = j, r = i - 1; y-lines l = i, r = j - 1)
__global__ void cd_assemble_kernel(CdArgs A, int axis, double* band, double* rhs)
{
    const int m = A.n - 2;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)m * m) return;
    const int p = (int)(t / m) + 1, q = (int)(t % m) + 1;  // (i, j) = (p, q)
    const int l = axis == 0 ? q : p, i = axis == 0 ? p : q;  // line and along index
    const int r = i - 1;
    const int64_t row = (int64_t)(l - 1) * m + r;
    rhs[row] = defect_at(A, p, q);
    const double k = A.kappa, h = A.h, e2 = A.eps / (h * h);
    const double c_al = axis == 0 ? A.a : A.b, c_ac = axis == 0 ? A.b : A.a;
    const double across = c_ac / h * (l >= 2 ? 0.25 * (3.0 - 3.0 * k) : 0.5 * (1.0 - k)) + 2.0 * e2;
    double w[5];
    if (i >= 2) {
        w[0] = c_al / h * (0.25 * (1.0 - k));
        w[1] = c_al / h * (0.25 * (3.0 * k - 5.0));
        w[2] = c_al / h * (0.25 * (3.0 - 3.0 * k));
        w[3] = c_al / h * (0.25 * (1.0 + k));
    } else {
        w[0] = 0.0;
        w[1] = c_al / h * (-0.25 * (3.0 - k));
        w[2] = c_al / h * (0.5 * (1.0 - k));
        w[3] = c_al / h * (0.25 * (1.0 + k));
    }
    w[4] = 0.0;
    w[1] += -e2;
    w[2] += 2.0 * e2 + across;
    w[3] += -e2;
    double* b = band + row * 5;
#pragma unroll
    for (int s = 0; s < 5; s++) {
        const int c = r + s - 2;
        b[s] = (c >= 0 && c < m) ? w[s] : 0.0;
    }
}

__global__ void cd_update_kernel(int n, int axis, double omega, const double* sigma, double* u)
{
    const int m = n - 2;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)m * m) return;
    const int p = (int)(t / m) + 1, q = (int)(t % m) + 1;
    const int l = axis == 0 ? q : p, i = axis == 0 ? p : q;
    u[(int64_t)p * n + q] += omega * sigma[(int64_t)(l - 1) * m + (i - 1)];
}

// ---------------------------------------------------------------------------
// Distributive line relaxation (Ls3 of Sec. 3.1, eqs. 51-54): the change of a node
// is distributed, u += s - (sum of the four neighbours' s) / 4, and a line
// solves for ghost changes whose distributed pattern cancels its defect.
// Row (i, l) of the line matrix, column k: L_h applied to the pattern of a
// unit ghost change at the line's node k, read at (i, l) (half-bandwidth 3,
// stored as a band of half-bandwidth 4).  Lines of one direction run in two
// colours (line index parity): neighbouring lines' patterns overlap.
// ---------------------------------------------------------------------------

// L_h at interior node (i, j) of the field U(ii, jj)
template <class F>
PQ_DEV double op_at(const CdArgs& A, int i, int j, F U)
{
    const double c = U(i, j);
    const double cx = conv_line(i >= 2 ? U(i - 2, j) : 0.0, U(i - 1, j), c, U(i + 1, j), i, A.kappa);
    const double cy = conv_line(j >= 2 ? U(i, j - 2) : 0.0, U(i, j - 1), c, U(i, j + 1), j, A.kappa);
    const double lap = (U(i + 1, j) + U(i - 1, j) + U(i, j + 1) + U(i, j - 1) - 4.0 * c) /
                       (A.h * A.h);
    return A.a * cx / A.h + A.b * cy / A.h - A.eps * lap;
}

// thread per row of the colour's lines (line slot k: line l = first + 2k)
__global__ void cd_ls3_assemble_kernel(CdArgs A, int axis, int first, int cnt, double* band,
                                       double* rhs)
{
    const int n = A.n, m = n - 2;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)cnt * m) return;
    const int k = (int)(t / m), r = (int)(t % m);
    const int l = first + 2 * k, i = r + 1;
    const int p = axis == 0 ? i : l, q = axis == 0 ? l : i;
    rhs[t] = defect_at(A, p, q);
    double* b = band + t * 9;
    for (int s = 0; s < 9; s++) {
        const int c = r + s - 4;  // column: the line's node c + 1
        double v = 0.0;
        if (c >= 0 && c < m && c - r >= -3 && c - r <= 2) {
            const int ci = axis == 0 ? c + 1 : l, cj = axis == 0 ? l : c + 1;
            auto pat = [&](int x, int y) {
                if (x == ci && y == cj) return 1.0;
                const int dist = abs(x - ci) + abs(y - cj);
                const bool inner = x >= 1 && x <= n - 2 && y >= 1 && y <= n - 2;
                return (dist == 1 && inner) ? -0.25 : 0.0;
            };
            v = op_at(A, p, q, pat);
        }
        b[s] = v;
    }
}

// u += omega * (distributed ghost changes of the colour's lines)
__global__ void cd_ls3_update_kernel(int n, int axis, int first, double omega,
                                     const double* sigma, double* u)
{
    const int m = n - 2;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)m * m) return;
    const int p = (int)(t / m) + 1, q = (int)(t % m) + 1;
    auto g = [&](int x, int y) {
        if (x < 1 || x > n - 2 || y < 1 || y > n - 2) return 0.0;
        const int l = axis == 0 ? y : x, i = axis == 0 ? x : y;
        if (l < first || ((l - first) & 1)) return 0.0;
        return sigma[(int64_t)((l - first) / 2) * m + (i - 1)];
    };
    const double du = g(p, q) - 0.25 * (g(p + 1, q) + g(p - 1, q) + g(p, q + 1) + g(p, q - 1));
    u[(int64_t)p * n + q] += omega * du;
}

// ---------------------------------------------------------------------------
// x-line splittings Ls0 / Ls1 (Sec. 3.1, eqs. 48-49): the implicit operator
// of x-line j is tridiagonal, u_{i-1}: -eps/h^2 - w a/h, u_i: w a/h +
// 4 eps/h^2 + the line's own y-convection coefficient, u_{i+1}: -eps/h^2,
// w = (2-k)/2 (Ls1) or (2-k)/2 + (1-k)/4 (Ls0); the rest of L_h acts through
// the defect.  The x-lines run in two colours (odd, then even j), each
// colour's defect taken after the other's update.
// ---------------------------------------------------------------------------

// thread per row of the colour's x-lines (slot k: line j = first + 2k);
// the band has half-bandwidth 2 with its outer diagonals zero
__global__ void cd_split_assemble_kernel(CdArgs A, double w, int first, int cnt, double* band,
                                         double* rhs)
{
    const int n = A.n, m = n - 2;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)cnt * m) return;
    const int k = (int)(t / m), r = (int)(t % m);
    const int j = first + 2 * k, i = r + 1;
    rhs[t] = defect_at(A, i, j);
    const double h = A.h, e2 = A.eps / (h * h), kp = A.kappa;
    const double own_y = A.b / h * (j >= 2 ? 0.25 * (3.0 - 3.0 * kp) : 0.5 * (1.0 - kp));
    double* b = band + t * 5;
    b[0] = 0.0;
    b[1] = r >= 1 ? -e2 - w * A.a / h : 0.0;
    b[2] = w * A.a / h + 4.0 * e2 + own_y;
    b[3] = r <= m - 2 ? -e2 : 0.0;
    b[4] = 0.0;
}

// u += omega sigma on the colour's x-lines
__global__ void cd_split_update_kernel(int n, int first, int cnt, double omega,
                                       const double* sigma, double* u)
{
    const int m = n - 2;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)cnt * m) return;
    const int k = (int)(t / m), r = (int)(t % m);
    const int j = first + 2 * k, i = r + 1;
    u[(int64_t)i * n + j] += omega * sigma[t];
}

// max over the interior of |f - L_h u| (mode 0) or |f| (mode 1), as the bit
// pattern of a non-negative double (ordered like the value) into *out
__global__ void cd_norm_kernel(CdArgs A, int mode, unsigned long long* out)
{
    const int m = A.n - 2;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v = 0.0;
    if (t < (int64_t)m * m) {
        const int p = (int)(t / m) + 1, q = (int)(t % m) + 1;
        v = fabs(mode == 0 ? defect_at(A, p, q) : A.f[(int64_t)p * A.n + q]);
        if (!(v == v)) v = INFINITY;  // a NaN defect reads as infinite
    }
    __shared__ double sh[256];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(sh[0]));
}

__global__ void cd_zero_kernel(unsigned long long* out) { *out = 0ull; }

__global__ void cd_offsets_kernel(int m, int64_t* offs)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= m) offs[i] = (int64_t)i * m;
}

// f = a u_x + b u_y - eps Lap u for u = x^4 + y^4, and the start iterate
// (exact boundary values, zero inside)
__global__ void cd_example_kernel(int n, double eps, double a, double b, double* f, double* u)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * n) return;
    const int i = (int)(t / n), j = (int)(t % n);
    const double h = 2.0 / (n - 1);
    const double x = -1.0 + h * i, y = -1.0 + h * j;
    f[t] = a * 4.0 * x * x * x + b * 4.0 * y * y * y - eps * (12.0 * x * x + 12.0 * y * y);
    const bool bnd = i == 0 || j == 0 || i == n - 1 || j == n - 1;
    u[t] = bnd ? x * x * x * x + y * y * y * y : 0.0;
}

struct CdLayout {
    size_t offs, band, rhs, sigma, lst, lit, norm, rec, act, total;
};

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

CdLayout cd_layout(int n)
{
    const size_t m = (size_t)n - 2, rows = m * m;
    CdLayout L;
    size_t p = 0;
    auto take = [&](size_t bytes) {
        const size_t at = p;
        p += a256(bytes);
        return at;
    };
    L.offs = take((m + 1) * sizeof(int64_t));
    L.band = take(rows * 5 * sizeof(double));
    L.rhs = take(rows * sizeof(double));
    L.sigma = take(rows * sizeof(double));
    L.lst = take(m * sizeof(int32_t));
    L.lit = take(m * sizeof(int32_t));
    L.norm = take(2 * sizeof(unsigned long long));
    L.rec = take(((rows + m) / 2 + 1) * (size_t)record_stride(2, true) * sizeof(double));
    L.act = take(rows);
    L.total = p;
    return L;
}

// Ls3 workspace: the same arrays, a band of half-bandwidth 4 and its records
CdLayout cd3_layout(int n)
{
    const size_t m = (size_t)n - 2, rows = m * m;
    CdLayout L;
    size_t p = 0;
    auto take = [&](size_t bytes) {
        const size_t at = p;
        p += a256(bytes);
        return at;
    };
    L.offs = take((m + 1) * sizeof(int64_t));
    L.band = take(rows * 9 * sizeof(double));
    L.rhs = take(rows * sizeof(double));
    L.sigma = take(rows * sizeof(double));
    L.lst = take(m * sizeof(int32_t));
    L.lit = take(m * sizeof(int32_t));
    L.norm = take(2 * sizeof(unsigned long long));
    L.rec = take(((rows + m) / 2 + 1) * (size_t)record_stride(4, true) * sizeof(double));
    L.act = take(rows);
    L.total = p;
    return L;
}

bool cd_valid(int n, double kappa, double eps, double a, double b)
{
    return n >= 5 && n <= 16385 && kappa >= -1.0 && kappa < 1.0 && eps >= 0.0 && a > 0.0 &&
           b > 0.0 && std::isfinite(eps) && std::isfinite(a) && std::isfinite(b);
}

}  // namespace
}  // namespace pq

extern "C" {

size_t cd_workspace_bytes(int n)
{
    if (n < 5 || n > 16385) return 0;
    return pq::cd_layout(n).total;
}

int cd_example(int n, double eps, double a, double b, double* f, double* u, void* stream)
{
    if (!pq::cd_valid(n, 0.0, eps, a, b) || !f || !u) return PAQIF_EINVAL;
    const int64_t cnt = (int64_t)n * n;
    hipLaunchKernelGGL(pq::cd_example_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), n, eps, a, b, f, u);
    return pq::hip_ok(hipGetLastError()) ? PAQIF_OK : PAQIF_EHIP;
}

int cd_line_relax(paqif_handle handle, int n, double kappa, double eps, double a, double b,
                  double omega, double tol, int max_iter, const double* f, double* u,
                  int32_t* iters, double* defect, void* workspace, void* stream)
{
    if (!handle || !pq::cd_valid(n, kappa, eps, a, b) || !(omega > 0.0 && omega < 2.0) ||
        !(tol >= 0.0) || max_iter < 1 || !f || !u || !iters || !defect || !workspace)
        return PAQIF_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const pq::CdLayout L = pq::cd_layout(n);
    char* ws = static_cast<char*>(workspace);
    const int m = n - 2;
    const int64_t rows = (int64_t)m * m;
    int64_t* offs = reinterpret_cast<int64_t*>(ws + L.offs);
    double* band = reinterpret_cast<double*>(ws + L.band);
    double* rhs = reinterpret_cast<double*>(ws + L.rhs);
    double* sigma = reinterpret_cast<double*>(ws + L.sigma);
    unsigned long long* nrm = reinterpret_cast<unsigned long long*>(ws + L.norm);

    pq::CdArgs A;
    A.n = n;
    A.kappa = kappa;
    A.eps = eps;
    A.a = a;
    A.b = b;
    A.h = 2.0 / (n - 1);
    A.f = f;
    A.u = u;

    pq::LcpArgs la;
    la.count = m;
    la.offsets = offs;
    la.order = nullptr;
    la.band = band;
    la.b = rhs;
    la.bounded = nullptr;
    la.mode = LCP_LINEAR;
    la.max_iter = 1;
    la.refine_tol = 0.0;
    la.u = sigma;
    la.w = nullptr;
    la.active_out = nullptr;
    la.status = reinterpret_cast<int32_t*>(ws + L.lst);
    la.iters = reinterpret_cast<int32_t*>(ws + L.lit);
    la.rec = ws + L.rec;
    la.act = reinterpret_cast<uint8_t*>(ws + L.act);
    la.r = nullptr;
    la.skip = nullptr;
    la.warm = 0;

    const unsigned nb = (unsigned)((rows + 255) / 256);
    hipLaunchKernelGGL(pq::cd_offsets_kernel, dim3((m + 256) / 256), dim3(256), 0, s, m, offs);
    // |f| over the interior sets the scale of the stopping test
    hipLaunchKernelGGL(pq::cd_zero_kernel, dim3(1), dim3(1), 0, s, nrm + 1);
    hipLaunchKernelGGL(pq::cd_norm_kernel, dim3(nb), dim3(256), 0, s, A, 1, nrm + 1);
    if (!pq::hip_ok(hipGetLastError())) return PAQIF_EHIP;
    unsigned long long host[2];
    const int layout = handle->layout[0][0];
    int it = 0;
    double res = INFINITY, fmax = 0.0;
    for (it = 1; it <= max_iter; it++) {
        for (int axis = 0; axis < 2; axis++) {
            hipLaunchKernelGGL(pq::cd_assemble_kernel, dim3(nb), dim3(256), 0, s, A, axis, band,
                               rhs);
            if (!pq::hip_ok(hipGetLastError())) return PAQIF_EHIP;
            int e = pq::dispatch_lcp(2, la, PREC_FP64, layout, s);
            if (e) return e;
            hipLaunchKernelGGL(pq::cd_update_kernel, dim3(nb), dim3(256), 0, s, n, axis, omega,
                               sigma, u);
            if (!pq::hip_ok(hipGetLastError())) return PAQIF_EHIP;
        }
        hipLaunchKernelGGL(pq::cd_zero_kernel, dim3(1), dim3(1), 0, s, nrm);
        hipLaunchKernelGGL(pq::cd_norm_kernel, dim3(nb), dim3(256), 0, s, A, 0, nrm);
        if (!pq::hip_ok(hipGetLastError()) ||
            hipMemcpyAsync(host, nrm, sizeof(host), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return PAQIF_EHIP;
        double v;
        memcpy(&v, &host[0], sizeof v);
        res = v;
        memcpy(&fmax, &host[1], sizeof fmax);
        if (res <= tol * fmax || !std::isfinite(res)) break;
    }
    *iters = std::min(it, max_iter);
    *defect = res;
    return PAQIF_OK;
}

int cd_split_relax(paqif_handle handle, int n, int which, double kappa, double eps, double a,
                   double b, double omega, double tol, int max_iter, const double* f, double* u,
                   int32_t* iters, double* defect, void* workspace, void* stream)
{
    if (!handle || !pq::cd_valid(n, kappa, eps, a, b) || !(which == 0 || which == 1) ||
        !(omega > 0.0 && omega < 2.0) || !(tol >= 0.0) || max_iter < 1 || !f || !u || !iters ||
        !defect || !workspace)
        return PAQIF_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const pq::CdLayout L = pq::cd_layout(n);
    char* ws = static_cast<char*>(workspace);
    const int m = n - 2;
    const int64_t rows = (int64_t)m * m;
    int64_t* offs = reinterpret_cast<int64_t*>(ws + L.offs);
    double* band = reinterpret_cast<double*>(ws + L.band);
    double* rhs = reinterpret_cast<double*>(ws + L.rhs);
    double* sigma = reinterpret_cast<double*>(ws + L.sigma);
    unsigned long long* nrm = reinterpret_cast<unsigned long long*>(ws + L.norm);
    // implicit weight of the x-upwind difference (eq. 49: Ls1; eq. 48: Ls0)
    const double w = which == 1 ? 0.5 * (2.0 - kappa) : 0.5 * (2.0 - kappa) + 0.25 * (1.0 - kappa);

    pq::CdArgs A;
    A.n = n;
    A.kappa = kappa;
    A.eps = eps;
    A.a = a;
    A.b = b;
    A.h = 2.0 / (n - 1);
    A.f = f;
    A.u = u;

    pq::LcpArgs la;
    la.offsets = offs;
    la.order = nullptr;
    la.band = band;
    la.b = rhs;
    la.bounded = nullptr;
    la.mode = LCP_LINEAR;
    la.max_iter = 1;
    la.refine_tol = 0.0;
    la.u = sigma;
    la.w = nullptr;
    la.active_out = nullptr;
    la.status = reinterpret_cast<int32_t*>(ws + L.lst);
    la.iters = reinterpret_cast<int32_t*>(ws + L.lit);
    la.rec = ws + L.rec;
    la.act = reinterpret_cast<uint8_t*>(ws + L.act);
    la.r = nullptr;
    la.skip = nullptr;
    la.warm = 0;

    const unsigned nb = (unsigned)((rows + 255) / 256);
    hipLaunchKernelGGL(pq::cd_offsets_kernel, dim3((m + 256) / 256), dim3(256), 0, s, m, offs);
    hipLaunchKernelGGL(pq::cd_zero_kernel, dim3(1), dim3(1), 0, s, nrm + 1);
    hipLaunchKernelGGL(pq::cd_norm_kernel, dim3(nb), dim3(256), 0, s, A, 1, nrm + 1);
    if (!pq::hip_ok(hipGetLastError())) return PAQIF_EHIP;
    unsigned long long host[2];
    const int layout = handle->layout[0][0];
    int it = 0;
    double res = INFINITY, fmax = 0.0;
    for (it = 1; it <= max_iter; it++) {
        for (int color = 1; color >= 0; color--) {
            const int first = color == 1 ? 1 : 2;  // x-lines j = first, first + 2, ...
            if (first > m) continue;
            const int cnt = (m - first) / 2 + 1;
            la.count = cnt;
            const unsigned nbl = (unsigned)(((int64_t)cnt * m + 255) / 256);
            hipLaunchKernelGGL(pq::cd_split_assemble_kernel, dim3(nbl), dim3(256), 0, s, A, w,
                               first, cnt, band, rhs);
            if (!pq::hip_ok(hipGetLastError())) return PAQIF_EHIP;
            int e = pq::dispatch_lcp(2, la, PREC_FP64, layout, s);
            if (e) return e;
            hipLaunchKernelGGL(pq::cd_split_update_kernel, dim3(nbl), dim3(256), 0, s, n, first,
                               cnt, omega, sigma, u);
            if (!pq::hip_ok(hipGetLastError())) return PAQIF_EHIP;
        }
        hipLaunchKernelGGL(pq::cd_zero_kernel, dim3(1), dim3(1), 0, s, nrm);
        hipLaunchKernelGGL(pq::cd_norm_kernel, dim3(nb), dim3(256), 0, s, A, 0, nrm);
        if (!pq::hip_ok(hipGetLastError()) ||
            hipMemcpyAsync(host, nrm, sizeof(host), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return PAQIF_EHIP;
        double v;
        memcpy(&v, &host[0], sizeof v);
        res = v;
        memcpy(&fmax, &host[1], sizeof fmax);
        if (res <= tol * fmax || !std::isfinite(res)) break;
    }
    *iters = std::min(it, max_iter);
    *defect = res;
    return PAQIF_OK;
}

size_t cd_ls3_workspace_bytes(int n)
{
    if (n < 5 || n > 16385) return 0;
    return pq::cd3_layout(n).total;
}

int cd_distributive_relax(paqif_handle handle, int n, double kappa, double eps, double a,
                          double b, double omega, double tol, int max_iter, const double* f,
                          double* u, int32_t* iters, double* defect, void* workspace,
                          void* stream)
{
    if (!handle || !pq::cd_valid(n, kappa, eps, a, b) || !(omega > 0.0 && omega < 2.0) ||
        !(tol >= 0.0) || max_iter < 1 || !f || !u || !iters || !defect || !workspace)
        return PAQIF_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const pq::CdLayout L = pq::cd3_layout(n);
    char* ws = static_cast<char*>(workspace);
    const int m = n - 2;
    const int64_t rows = (int64_t)m * m;
    int64_t* offs = reinterpret_cast<int64_t*>(ws + L.offs);
    double* band = reinterpret_cast<double*>(ws + L.band);
    double* rhs = reinterpret_cast<double*>(ws + L.rhs);
    double* sigma = reinterpret_cast<double*>(ws + L.sigma);
    unsigned long long* nrm = reinterpret_cast<unsigned long long*>(ws + L.norm);

    pq::CdArgs A;
    A.n = n;
    A.kappa = kappa;
    A.eps = eps;
    A.a = a;
    A.b = b;
    A.h = 2.0 / (n - 1);
    A.f = f;
    A.u = u;

    pq::LcpArgs la;
    la.offsets = offs;
    la.order = nullptr;
    la.band = band;
    la.b = rhs;
    la.bounded = nullptr;
    la.mode = LCP_LINEAR;
    la.max_iter = 1;
    la.refine_tol = 0.0;
    la.u = sigma;
    la.w = nullptr;
    la.active_out = nullptr;
    la.status = reinterpret_cast<int32_t*>(ws + L.lst);
    la.iters = reinterpret_cast<int32_t*>(ws + L.lit);
    la.rec = ws + L.rec;
    la.act = reinterpret_cast<uint8_t*>(ws + L.act);
    la.r = nullptr;
    la.skip = nullptr;
    la.warm = 0;

    const unsigned nb = (unsigned)((rows + 255) / 256);
    hipLaunchKernelGGL(pq::cd_offsets_kernel, dim3((m + 256) / 256), dim3(256), 0, s, m, offs);
    hipLaunchKernelGGL(pq::cd_zero_kernel, dim3(1), dim3(1), 0, s, nrm + 1);
    hipLaunchKernelGGL(pq::cd_norm_kernel, dim3(nb), dim3(256), 0, s, A, 1, nrm + 1);
    if (!pq::hip_ok(hipGetLastError())) return PAQIF_EHIP;
    unsigned long long host[2];
    const int layout = handle->layout[pq::q_index(4)][0];
    int it = 0;
    double res = INFINITY, fmax = 0.0;
    for (it = 1; it <= max_iter; it++) {
        for (int axis = 0; axis < 2; axis++) {
            for (int color = 1; color >= 0; color--) {
                const int first = color == 1 ? 1 : 2;  // lines first, first + 2, ...
                if (first > m) continue;
                const int cnt = (m - first) / 2 + 1;
                la.count = cnt;
                const unsigned nbl = (unsigned)(((int64_t)cnt * m + 255) / 256);
                hipLaunchKernelGGL(pq::cd_ls3_assemble_kernel, dim3(nbl), dim3(256), 0, s, A,
                                   axis, first, cnt, band, rhs);
                if (!pq::hip_ok(hipGetLastError())) return PAQIF_EHIP;
                int e = pq::dispatch_lcp(4, la, PREC_FP64, layout, s);
                if (e) return e;
                hipLaunchKernelGGL(pq::cd_ls3_update_kernel, dim3(nb), dim3(256), 0, s, n, axis,
                                   first, omega, sigma, u);
                if (!pq::hip_ok(hipGetLastError())) return PAQIF_EHIP;
            }
        }
        hipLaunchKernelGGL(pq::cd_zero_kernel, dim3(1), dim3(1), 0, s, nrm);
        hipLaunchKernelGGL(pq::cd_norm_kernel, dim3(nb), dim3(256), 0, s, A, 0, nrm);
        if (!pq::hip_ok(hipGetLastError()) ||
            hipMemcpyAsync(host, nrm, sizeof(host), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return PAQIF_EHIP;
        double v;
        memcpy(&v, &host[0], sizeof v);
        res = v;
        memcpy(&fmax, &host[1], sizeof fmax);
        if (res <= tol * fmax || !std::isfinite(res)) break;
    }
    *iters = std::min(it, max_iter);
    *defect = res;
    return PAQIF_OK;
}

}  // extern "C"

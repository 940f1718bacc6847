// PAQIF: batched alternate quadrant interlocking factorisation and banded
// LCP solve on gfx950.
//
// Method (Singh & Dutt, Sec. 2.2): A = W0 Z0 is computed from the centre of
// the band outwards.  Level k takes the pivot pair (p1, p2) = (s-k, s+k-1)
// (n = 2s; for n = 2m+1 the centre row is a 1x1 pivot first and level k
// takes (m-k, m+k)); the two pivot rows of the reduced matrix become rows of
// Z0, the two W0 columns come from one 2x2 solve per remaining row, and the
// remaining rows get a rank-2 update.  Z0 x = y is then solved from both
// ends inwards, one 2x2 system per level.
//
// GPU formulation.  On a band of half-width q only a 2q x 2q "frontier"
// block of the reduced matrix is ever modified: the q not-yet-eliminated
// rows left of the eliminated centre and the q rows right of it.  Each
// level consumes the two innermost frontier rows as pivots and brings in one
// new band row at each end.  A frontier row keeps its slot for its whole
// lifetime: left index g lives in slot (P1_0 - g) mod q, right index g in
// q + (g - P2_0) mod q, so the pivots of level k sit in slots j and q+j
// with j = (k-1) mod q, and the new rows of level k take those same slots.
// Unrolling the level loop by q makes every slot index a compile-time
// constant and the frontier never moves between lanes.
//
// One system per 2q*2q lanes (q = 2: four systems per wave; q = 4: one per
// wave; q = 8: one per wave, four frontier elements per lane).  Per level a
// lane publishes its frontier element to LDS, reads back the pivot block,
// its row's two pivot-column entries and its column's two pivot-row
// entries, and applies the rank-2 update to its element.  New band entries
// are prefetched q levels ahead into registers.  The forward solve
// W0 y = b is fused into the elimination (the right-hand side rides along as
// one more column).  Per level one record is written:
//
//   rec[0      .. 2q)    Z0 row p1 over the 2q outer unknowns (frontier slots
//                        after the level), i.e. the coefficients the back
//                        solve needs
//   rec[2q     .. 4q)    Z0 row p2, same slots
//   rec[4q     .. 4q+4)  inverse of the 2x2 pivot block, row major
//                        (centre 1x1 level: [1/a, 0, 0, 0])
//   rec[4q+4   .. 4q+6)  y(p1), y(p2) of the forward solve
//   rec[4q+6   .. 8q+6)  (optional) W0 multipliers (w1, w2) of the row held
//                        by each frontier slot after the level
//
// The back solve (Z0 x = y, ends inwards) runs in the same wave: 2q lanes
// hold the solved outer unknowns of the frontier slots, each level forms two
// dot products with a DPP butterfly, applies the stored inverse pivot and
// drops the two new unknowns into slots j and q+j.
#include <type_traits>
#include <utility>

#include "common.h"
#include "paqif_args.h"

namespace pq {

// Lane layouts: each lane owns a TR x TC tile of the 2q x 2q frontier; a
// superblock of S blocks of q levels is prefetched one superblock ahead; WPE
// is the occupancy the launch of 4096 systems needs.
//   q=2: L0 1x1 (16 lanes/system, 4 per wave)   L1 1x2 (8 lanes, 8 per wave)
//   q=4: L0 1x1 (64 lanes, 1 per wave)          L1 1x2 (32 lanes, 2 per wave)
//        L2 2x2 (16 lanes, 4 per wave)
//   q=8: L0 2x2 (64 lanes, 1 per wave)          L1 2x4 (32 lanes, 2 per wave)
//        L2 1x4 (64 lanes, 1 per wave)
// q = 2: layout 2 is one system per lane (its own kernel below)
// layout 3 (FP64): one system per 16-lane row, a frontier row per lane, the
// pivot rows broadcast by DPP (paqif_lcp_rows_kernel below)
constexpr int layout_count(int q) { return 4; }

template <int Q, int L>
struct Geo {
    static constexpr int N2 = 2 * Q;
    static constexpr int E = N2 * N2;
    static constexpr int TR = Q == 8 ? (L == 2 ? 1 : 2) : (Q == 4 && L == 2 ? 2 : 1);
    static constexpr int TC = Q == 8 ? (L == 1 ? 4 : (L == 2 ? 4 : 2)) : (L == 0 ? 1 : 2);
    static constexpr int LPS = E / (TR * TC);  // lanes per system
    static constexpr int SPW = 64 / LPS;       // systems per wave
    static constexpr int CT = N2 / TC;         // column tiles per tile row
    static constexpr int S = Q == 8 ? 1 : 16 / Q;  // blocks of q levels per prefetch superblock
    static constexpr int SB = S * Q;               // levels per superblock
    static constexpr int WPE = SPW == 1 ? 2 : (SPW == 2 ? 2 : 1);
    static constexpr int BW = 2 * Q + 1;       // band width
    static constexpr int ZREC = 4 * Q + 6;     // record without W0
    static constexpr int WREC = 4 * Q;         // W0 part of a record
    static_assert(LPS <= 64 && 64 % LPS == 0, "lanes per system");
    static_assert(LPS >= N2, "back solve needs 2q lanes");
    static_assert(N2 % TC == 0 && N2 % TR == 0, "tile");
};

// Opaque copy of a lane-varying value: the compiler must recompute what is
// derived from it after this point, so per-lane constants of one phase are
// not hoisted out of the outer active-set loop (which would keep them live,
// in registers, across every other phase).
PQ_DEV int launder(int x)
{
    asm volatile("" : "+v"(x));
    return x;
}

PQ_DEV int64_t uniform64(int64_t x)
{
    const uint64_t u = (uint64_t)x;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Number of level records of a system of order n: ceil(n/2).
PQ_DEV int64_t level_base(int64_t row_offset, int sys) { return (row_offset + sys) >> 1; }

struct SysView {
    int n;
    int npair;  // number of 2x2 levels
    bool odd;
    int P1_0, P2_0;  // pivots of the first 2x2 level
    GLB_PTR(const double) band;
    GLB_PTR(const uint8_t) pin;
    GLB_PTR(const double) rhs;
};

// Zero block that an empty system's view points at: the prefetch loads from
// clamped addresses unconditionally, and an empty system (or a lane without
// a system) has no element of its own to clamp to (its offset may equal the
// array length).  Indices stay below 2q+1 <= 17.
__device__ const double kZeroBand[32] = {};
__device__ const uint8_t kZeroFlags[32] = {};
__device__ const uint8_t kOneFlags[32] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1,
                                          1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
// Target of the stores of lanes that have nothing to store, so that store
// instructions need no branch (its contents are never read).
__device__ double kSink[128];

// Two doubles moved as one 16-byte access.
typedef double dbl2 __attribute__((ext_vector_type(2)));

PQ_DEV SysView make_view(int64_t off, int64_t n, const double* band, const uint8_t* pin,
                         const double* rhs, int bw, int64_t boff)
{
    SysView v;
    if (n <= 0) {
        v.n = 0;
        v.npair = 0;
        v.odd = false;
        v.P1_0 = -1;
        v.P2_0 = 0;
        v.band = GLB(const double, kZeroBand);
        v.pin = pin ? GLB(const uint8_t, kZeroFlags) : nullptr;
        v.rhs = rhs ? GLB(const double, kZeroBand) : nullptr;
        return v;
    }
    v.n = (int)n;
    v.odd = (n & 1) != 0;
    if (v.odd) {
        int m = (int)((n - 1) / 2);
        v.npair = m;
        v.P1_0 = m - 1;
        v.P2_0 = m + 1;
    } else {
        int s = (int)(n / 2);
        v.npair = s;
        v.P1_0 = s - 1;
        v.P2_0 = s;
    }
    v.band = GLB(const double, band + boff * bw);
    v.pin = pin ? GLB(const uint8_t, pin + off) : nullptr;
    v.rhs = rhs ? GLB(const double, rhs + off) : nullptr;
    return v;
}

// Effective matrix entry: pinned rows/columns replaced by the identity.
template <int Q>
PQ_DEV double aeff(const SysView& v, int i, int j)
{
    if (i < 0 || j < 0 || i >= v.n || j >= v.n) return 0.0;
    int d = j - i;
    if (d < -Q || d > Q) return 0.0;
    if (v.pin && (v.pin[i] | v.pin[j])) return i == j ? 1.0 : 0.0;
    return v.band[(int64_t)i * (2 * Q + 1) + (d + Q)];
}

PQ_DEV double beff(const SysView& v, GLB_PTR(const double) rhs, int i)
{
    if (i < 0 || i >= v.n) return 0.0;
    if (v.pin && v.pin[i]) return 0.0;
    return rhs[i];
}

// beff without branches (clamped address, then selects)
PQ_DEV double beff_sel(const SysView& v, GLB_PTR(const double) rhs, int i)
{
    const bool in = (i >= 0) & (i < v.n);
    const int ic = min(max(i, 0), v.n > 0 ? v.n - 1 : 0);
    double val = rhs[ic];
    if (v.pin) val = v.pin[ic] ? 0.0 : val;
    return in ? val : 0.0;
}

// Global index held by frontier slot c after level k (pivot slot j).
template <int Q>
PQ_DEV int slot_index_post(int c, int j, int p1k, int p2k)
{
    if (c < Q) return p1k - 1 - ((c - j - 1 + Q) & (Q - 1));
    return p2k + 1 + ((c - Q - j - 1 + Q) & (Q - 1));
}

// Global index held by slot c before the first 2x2 level.
template <int Q>
PQ_DEV int slot_index_init(int c, const SysView& v)
{
    return c < Q ? v.P1_0 - c : v.P2_0 + (c - Q);
}

// --------------------------------------------------------------------------
// Factorisation (+ fused forward solve when FUSED).
// lF: LDS frontier (N2*N2), lY: LDS rhs column (N2), lX: LDS extras (6q).
// rec: this system's first record, `stride` elements per record.
// `kmax` = largest npair among the systems sharing the wave (loop bound).
// Returns true if a pivot was singular / non-finite.
//
// Prefetch: within a block of q levels (j = 0..q-1) frontier element
// (a, b) receives a new band entry exactly at j = a mod q (its row slot is
// refilled) and at j = b mod q (its column slot is refilled).  So each lane
// loads two values per element per block, one block ahead.  The six
// per-level scalars (the four band entries coupling the pivots with the
// incoming rows and the two incoming right-hand sides) are loaded by lanes
// 0..6q-1, one block ahead, and published through LDS at the block start.
// --------------------------------------------------------------------------
template <int Q>
PQ_DEV double level_extra(const SysView& v, GLB_PTR(const double) rhs, bool fused, int k,
                          int e)
{
    const int p1k = v.P1_0 - (k - 1), p2k = v.P2_0 + (k - 1);
    const int g1 = p1k - Q, g2 = p2k + Q;
    switch (e) {
    case 0: return aeff_sel<Q>(v, p1k, g1);
    case 1: return aeff_sel<Q>(v, g1, p1k);
    case 2: return aeff_sel<Q>(v, p2k, g2);
    case 3: return aeff_sel<Q>(v, g2, p2k);
    case 4: return fused ? beff_sel(v, rhs, g1) : 0.0;
    default: return fused ? beff_sel(v, rhs, g2) : 0.0;
    }
}

// aeff without branches for a live system (n >= 1): the address is clamped
// into the system so the load is always valid, then out-of-band and pinned
// entries are selected away.
template <int Q>
PQ_DEV double aeff_sel(const SysView& v, int i, int j)
{
    const int d = j - i;
    const bool in = (i >= 0) & (j >= 0) & (i < v.n) & (j < v.n) & (d >= -Q) & (d <= Q);
    const int nm = v.n > 0 ? v.n - 1 : 0;
    const int ic = min(max(i, 0), nm), jc = min(max(j, 0), nm);
    const int dc = min(max(d + Q, 0), 2 * Q);
    double val = v.band[(int64_t)ic * (2 * Q + 1) + dc];
    if (v.pin) {  // uniform
        const bool pinned = (v.pin[ic] | v.pin[jc]) != 0;
        val = pinned ? (i == j ? 1.0 : 0.0) : val;
    }
    return in ? val : 0.0;
}

// One effective entry split into its raw loads: the band value at a clamped
// (valid) address and the pin flags of its row and column.  The
// load-independent part of the selection is a 2-bit code (bit 0: the entry
// exists, inside the matrix and the band; bit 1: diagonal), packed by the
// caller into one word per superblock.  The consumer applies the selection
// (ent_value) one superblock later: a select on a freshly loaded value would
// make the compiler wait for that load on the spot and so serialise the
// prefetch.
struct RawEnt {
    double val;
    uint32_t pi, pj;
};

PQ_DEV double ent_value(const RawEnt& r, uint32_t code)
{
    const bool pinned = (r.pi | r.pj) != 0u;
    const double s = pinned ? ((code & 2u) ? 1.0 : 0.0) : r.val;
    return (code & 1u) ? s : 0.0;
}

template <int Q>
PQ_DEV RawEnt raw_ent(const SysView& v, int i, int j, bool use, uint32_t& code)
{
    RawEnt r;
    const int d = j - i;
    const bool in =
        use & (i >= 0) & (j >= 0) & (i < v.n) & (j < v.n) & (d >= -Q) & (d <= Q);
    const int nm = v.n > 0 ? v.n - 1 : 0;
    const int ic = min(max(i, 0), nm), jc = min(max(j, 0), nm);
    const int dc = min(max(d + Q, 0), 2 * Q);
    r.val = v.band[(int64_t)ic * (2 * Q + 1) + dc];
    r.pi = v.pin ? (uint32_t)v.pin[ic] : 0u;
    r.pj = v.pin ? (uint32_t)v.pin[jc] : 0u;
    code = (in ? 1u : 0u) | (i == j ? 2u : 0u);
    return r;
}

// Raw form of level_extra: one load per element, from the band (e < 4) or
// the right-hand side (e >= 4, pinned rows give 0), chosen by address.
template <int Q>
PQ_DEV RawEnt raw_extra(const SysView& v, GLB_PTR(const double) rhs, bool fused, int k, int e,
                        bool use, uint32_t& code)
{
    const int p1k = v.P1_0 - (k - 1), p2k = v.P2_0 + (k - 1);
    const bool right = (e == 2) | (e == 3) | (e == 5);
    const bool swap = (e == 1) | (e == 3);
    const bool isr = e >= 4;
    const int p = right ? p2k : p1k, g = right ? p2k + Q : p1k - Q;
    const int i = (isr | swap) ? g : p, j = (isr | !swap) ? g : p;
    const int d = j - i;
    const bool in = use & (!isr | fused) & (i >= 0) & (j >= 0) & (i < v.n) & (j < v.n);
    const int nm = v.n > 0 ? v.n - 1 : 0;
    const int ic = min(max(i, 0), nm), jc = min(max(j, 0), nm);
    const int dc = min(max(d + Q, 0), 2 * Q);
    const bool from_rhs = isr & fused;
    GLB_PTR(const double) src = from_rhs ? rhs : v.band;
    const int64_t idx = from_rhs ? (int64_t)ic : (isr ? 0 : (int64_t)ic * (2 * Q + 1) + dc);
    RawEnt r;
    r.val = src[idx];
    r.pi = v.pin ? (uint32_t)v.pin[ic] : 0u;
    r.pj = v.pin ? (uint32_t)v.pin[jc] : 0u;
    code = in ? 1u : 0u;  // never diagonal: |d| = q, or a pinned rhs row (0)
    return r;
}

// New entry of element (a, b) at level k (pivot slot j = (k-1) mod q).
template <int Q>
PQ_DEV double level_new(const SysView& v, int k, int a, int b)
{
    const int j = (k - 1) & (Q - 1);
    const int p1k = v.P1_0 - (k - 1), p2k = v.P2_0 + (k - 1);
    return aeff_sel<Q>(v, slot_index_post<Q>(a, j, p1k, p2k), slot_index_post<Q>(b, j, p1k, p2k));
}

template <int Q, int L, typename FT, bool STORE_W, bool FUSED>
PQ_DEV bool factor_system(SysView v, bool live, GLB_PTR(FT) rec, int stride, LDS_PTR(FT) lF,
                          LDS_PTR(FT) lY, LDS_PTR(FT) lX, int ls, int kmax)
{
    ls = launder(ls);
    using G = Geo<Q, L>;
    constexpr int N2 = G::N2;
    constexpr int TR = G::TR;
    constexpr int TC = G::TC;
    constexpr int RPL = (2 * N2 + G::LPS - 1) / G::LPS;  // Z0 record elements per lane
    const int ta = ls / G::CT, tb = ls % G::CT;
    int a[TR], jr[TR], b[TC], jc[TC];
#pragma unroll
    for (int u = 0; u < TR; u++) {
        a[u] = ta * TR + u;
        jr[u] = a[u] & (Q - 1);
    }
#pragma unroll
    for (int w = 0; w < TC; w++) {
        b[w] = tb * TC + w;
        jc[w] = b[w] & (Q - 1);
    }

    bool bad = false;
    FT f[TR][TC], y[TR];
    GLB_PTR(const double) rhs = v.rhs;

    // ---- initial frontier (and the odd-n centre level) ------------------
    int ib[TC];
#pragma unroll
    for (int w = 0; w < TC; w++) ib[w] = slot_index_init<Q>(b[w], v);
    if (v.odd) {
        const int m = v.npair;  // centre index (n = 2m+1)
        const double amm = live ? aeff<Q>(v, m, m) : 1.0;
        if (!(amm != 0.0 && isfinite(amm))) bad = true;
        const double ramm = 1.0 / amm;
        const double bm = (FUSED && live) ? beff(v, rhs, m) : 0.0;
        double amb[TC];
#pragma unroll
        for (int w = 0; w < TC; w++) amb[w] = aeff<Q>(v, m, ib[w]);
#pragma unroll
        for (int u = 0; u < TR; u++) {
            const int ia = slot_index_init<Q>(a[u], v);
            const double aim = aeff<Q>(v, ia, m) * ramm;
#pragma unroll
            for (int w = 0; w < TC; w++) f[u][w] = (FT)(aeff<Q>(v, ia, ib[w]) - aim * amb[w]);
            y[u] = FUSED ? (FT)(beff(v, rhs, ia) - aim * bm) : (FT)0;
            if (STORE_W && live && tb == 0) {
                rec[4 * Q + 6 + 2 * a[u]] = (FT)aim;
                rec[4 * Q + 6 + 2 * a[u] + 1] = (FT)0;
            }
        }
        if (live) {
            // centre record: Z0 row m over the frontier slots, 1x1 pivot
            if (ta == 0) {
#pragma unroll
                for (int w = 0; w < TC; w++) {
                    rec[b[w]] = (FT)amb[w];
                    rec[N2 + b[w]] = (FT)0;
                }
            }
            if (ls == 0) {
                rec[4 * Q + 0] = (FT)ramm;
                rec[4 * Q + 1] = (FT)0;
                rec[4 * Q + 2] = (FT)0;
                rec[4 * Q + 3] = (FT)0;
                rec[4 * Q + 4] = (FT)bm;
                rec[4 * Q + 5] = (FT)0;
            }
        }
        rec += stride;
    } else {
#pragma unroll
        for (int u = 0; u < TR; u++) {
            const int ia = slot_index_init<Q>(a[u], v);
#pragma unroll
            for (int w = 0; w < TC; w++) f[u][w] = (FT)aeff<Q>(v, ia, ib[w]);
            y[u] = FUSED ? (FT)beff(v, rhs, ia) : (FT)0;
        }
    }

    // ---- prefetch: within each block of q levels element (a, b) is refilled
    // at j = a mod q (row) and at j = b mod q (column); the values of a whole
    // superblock of S blocks are loaded one superblock ahead -----------------
    constexpr int S = G::S;
    constexpr int SB = G::SB;
    RawEnt nR[S][TR][TC], nC[S][TR][TC];
    constexpr int XPL = (6 * SB + G::LPS - 1) / G::LPS;  // extras per lane
    RawEnt nX[XPL];
    static_assert(S * TR * TC <= 16 && XPL <= 32, "selection codes fit one word");
    uint32_t cR, cC, cX;  // selection codes, 2 bits per entry (1 per extra)
    // The index a slot takes at its refill is linear in t = kb + sb q (the
    // first level of the block, minus one): left slots move down by one per
    // level, right slots up.  Bases, signs and the last valid t of every
    // prefetched entry are set once here.
    int sgA[TR], sgB[TC];  // -1 left slot, +1 right slot
#pragma unroll
    for (int u = 0; u < TR; u++) sgA[u] = a[u] < Q ? -1 : 1;
#pragma unroll
    for (int w = 0; w < TC; w++) sgB[w] = b[w] < Q ? -1 : 1;
    int iR0[TR], tR[TR], jR0[TR][TC], iC0[TR][TC], jC0[TC], tC[TC];
#pragma unroll
    for (int u = 0; u < TR; u++) {
        // row refill at level t + jr + 1: slots a[u] and b[w] after that level
        const int p1 = v.P1_0 - jr[u], p2 = v.P2_0 + jr[u];
        iR0[u] = slot_index_post<Q>(a[u], jr[u], p1, p2);
        tR[u] = v.npair - jr[u] - 1;  // the level exists while t <= tR
#pragma unroll
        for (int w = 0; w < TC; w++) jR0[u][w] = slot_index_post<Q>(b[w], jr[u], p1, p2);
    }
#pragma unroll
    for (int w = 0; w < TC; w++) {
        const int p1 = v.P1_0 - jc[w], p2 = v.P2_0 + jc[w];
        jC0[w] = slot_index_post<Q>(b[w], jc[w], p1, p2);
        tC[w] = v.npair - jc[w] - 1;
#pragma unroll
        for (int u = 0; u < TR; u++) iC0[u][w] = slot_index_post<Q>(a[u], jc[w], p1, p2);
    }
    auto load_super = [&](int kn) {
        cR = cC = cX = 0u;
#pragma unroll
        for (int sb = 0; sb < S; sb++) {
            const int t = kn + sb * Q;
#pragma unroll
            for (int u = 0; u < TR; u++)
#pragma unroll
                for (int w = 0; w < TC; w++) {
                    const int sh = 2 * ((sb * TR + u) * TC + w);
                    uint32_t code;
                    nR[sb][u][w] = raw_ent<Q>(v, iR0[u] + sgA[u] * t, jR0[u][w] + sgB[w] * t,
                                              live && t <= tR[u], code);
                    cR |= code << sh;
                    nC[sb][u][w] = raw_ent<Q>(v, iC0[u][w] + sgA[u] * t, jC0[w] + sgB[w] * t,
                                              live && t <= tC[w] && jc[w] != jr[u], code);
                    cC |= code << sh;
                }
        }
#pragma unroll
        for (int x = 0; x < XPL; x++) {
            const int e = ls + x * G::LPS;
            const int kx = kn + e / 6 + 1;
            uint32_t code;
            nX[x] = raw_extra<Q>(v, rhs, FUSED, kx, e % 6, live && e < 6 * SB && kx <= v.npair,
                                 code);
            cX |= code << x;
        }
    };
    load_super(0);

    // ---- level loop, unrolled by a superblock of S*q levels ---------------
    for (int kb = 0; kb < kmax; kb += SB) {
        FT vR[S][TR][TC], vC[S][TR][TC];
#pragma unroll
        for (int sb = 0; sb < S; sb++)
#pragma unroll
            for (int u = 0; u < TR; u++)
#pragma unroll
                for (int w = 0; w < TC; w++) {
                    const int sh = 2 * ((sb * TR + u) * TC + w);
                    vR[sb][u][w] = (FT)ent_value(nR[sb][u][w], (cR >> sh) & 3u);
                    vC[sb][u][w] = (FT)ent_value(nC[sb][u][w], (cC >> sh) & 3u);
                }
#pragma unroll
        for (int x = 0; x < XPL; x++) {
            const int e = ls + x * G::LPS;
            if (e < 6 * SB) lX[e] = (FT)ent_value(nX[x], (cX >> x) & 1u);
        }
        load_super(kb + SB);
        // the whole superblock is unrolled (prefetched registers and LDS
        // offsets are compile-time); a wave runs whole superblocks, levels
        // past a system's last one compute on zeros and store nothing
#pragma unroll
        for (int sb = 0; sb < S; sb++)
#pragma unroll
        for (int j = 0; j < Q; j++) {    // pivot slot
            const int jj = sb * Q + j;   // level within the superblock
            const int k = kb + jj + 1;  // level number (1-based)
            const bool act = live && (k <= v.npair);

            // publish the tile and the rhs column
#pragma unroll
            for (int u = 0; u < TR; u++)
#pragma unroll
                for (int w = 0; w < TC; w++) lF[a[u] * N2 + b[w]] = f[u][w];
            if (tb == 0) {
#pragma unroll
                for (int u = 0; u < TR; u++) lY[a[u]] = y[u];
            }
            wave_sync();
            const FT P11 = lF[j * N2 + j], P12 = lF[j * N2 + Q + j];
            const FT P21 = lF[(Q + j) * N2 + j], P22 = lF[(Q + j) * N2 + Q + j];
            const FT y1 = lY[j], y2 = lY[Q + j];
            FT c1[TC], c2[TC], r1[TR], r2[TR];
#pragma unroll
            for (int w = 0; w < TC; w++) {
                c1[w] = lF[j * N2 + b[w]];
                c2[w] = lF[(Q + j) * N2 + b[w]];
            }
#pragma unroll
            for (int u = 0; u < TR; u++) {
                r1[u] = lF[a[u] * N2 + j];
                r2[u] = lF[a[u] * N2 + Q + j];
            }
            const FT E0 = lX[6 * jj + 0], E1 = lX[6 * jj + 1], E2 = lX[6 * jj + 2];
            const FT E3 = lX[6 * jj + 3], E4 = lX[6 * jj + 4], E5 = lX[6 * jj + 5];
            // frontier rows j and q+j as published (the record's Z0 rows);
            // element e < 2 N2 of the record reads row (e < N2 ? j : q+j)
            FT rraw[RPL];
#pragma unroll
            for (int r = 0; r < RPL; r++) {
                const int e = ls + r * G::LPS;
                const int row = (e & N2) ? Q + j : j;  // valid address for every lane
                rraw[r] = lF[row * N2 + (e & (N2 - 1))];
            }
            wave_sync();

            const FT det = P11 * P22 - P12 * P21;
            if (act && !(det != (FT)0 && isfinite(det))) bad = true;
            // 1/det: hardware reciprocal and two Newton steps (each squares
            // the relative error: ~2^-23 -> below 2^-53), a shorter dependent
            // chain than the IEEE division sequence on the level's critical
            // path; a zero or non-finite det is flagged above
            FT rd;
            if constexpr (sizeof(FT) == 8) {
                const double r0 = __builtin_amdgcn_rcp(det);
                const double r1 = __builtin_fma(r0, __builtin_fma(-det, r0, 1.0), r0);
                rd = __builtin_fma(r1, __builtin_fma(-det, r1, 1.0), r1);
            } else {
                rd = (FT)1 / det;
            }
            const FT i11 = P22 * rd, i12 = -P12 * rd, i21 = -P21 * rd, i22 = P11 * rd;

            // record: Z0 rows p1, p2 over the slots after this level, the
            // inverse pivot and the forward values; one element per lane
            if (act) {
#pragma unroll
                for (int r = 0; r < RPL; r++) {
                    const int e = ls + r * G::LPS;
                    const bool row1 = e < N2;
                    const int col = e & (N2 - 1);
                    // Z0 rows: the pivot columns take E0 / E2 and 0
                    const FT at_j = row1 ? E0 : (FT)0;
                    const FT at_qj = row1 ? (FT)0 : E2;
                    const FT zval = col == j ? at_j : (col == Q + j ? at_qj : rraw[r]);
                    if (e < 2 * N2) rec[e] = zval;
                }
                if (ls == 0) {
                    rec[4 * Q + 0] = i11;
                    rec[4 * Q + 1] = i12;
                    rec[4 * Q + 2] = i21;
                    rec[4 * Q + 3] = i22;
                    rec[4 * Q + 4] = y1;
                    rec[4 * Q + 5] = y2;
                }
            }

            // pivot-row values at this lane's columns (after the shift)
            FT cA[TC], cB[TC];
#pragma unroll
            for (int w = 0; w < TC; w++) {
                cA[w] = (b[w] == j) ? E0 : ((b[w] == Q + j) ? (FT)0 : c1[w]);
                cB[w] = (b[w] == j) ? (FT)0 : ((b[w] == Q + j) ? E2 : c2[w]);
            }
#pragma unroll
            for (int u = 0; u < TR; u++) {
                FT w1, w2;
                if (a[u] == j) {
                    w1 = E1 * i11;
                    w2 = E1 * i12;
                } else if (a[u] == Q + j) {
                    w1 = E3 * i21;
                    w2 = E3 * i22;
                } else {
                    w1 = r1[u] * i11 + r2[u] * i21;
                    w2 = r1[u] * i12 + r2[u] * i22;
                }
#pragma unroll
                for (int w = 0; w < TC; w++) {
                    const FT base = (jr[u] == j) ? vR[sb][u][w]
                                                 : ((jc[w] == j) ? vC[sb][u][w] : f[u][w]);
                    f[u][w] = base - (w1 * cA[w] + w2 * cB[w]);
                }
                if (FUSED) {
                    const FT yb = (a[u] == j) ? E4 : ((a[u] == Q + j) ? E5 : y[u]);
                    y[u] = yb - (w1 * y1 + w2 * y2);
                }
                if (STORE_W && act && tb == 0) {
                    rec[4 * Q + 6 + 2 * a[u]] = w1;
                    rec[4 * Q + 6 + 2 * a[u] + 1] = w2;
                }
            }
            rec += stride;
        }
    }
    return bad;
}

// --------------------------------------------------------------------------
// Forward solve W0 y = rhs with stored multipliers; writes y(p1), y(p2) into
// the records (used when the forward solve was not fused).  2q lanes per
// system hold the running right-hand side of their frontier slot.
// --------------------------------------------------------------------------
template <int Q, typename FT>
PQ_DEV void wsolve_system(SysView v, bool live, GLB_PTR(const double) rhs,
                                           GLB_PTR(FT) rec, int stride, int ls, int kmax,
                                           int gbase)
{
    ls = launder(ls);
    constexpr int N2 = 2 * Q;
    const bool mine = ls < N2;
    const int c = mine ? ls : 0;
    double bc = 0.0;
    if (v.odd) {
        const int m = v.npair;
        const double ym = live ? beff(v, rhs, m) : 0.0;
        if (mine && live) {
            bc = beff(v, rhs, slot_index_init<Q>(c, v)) - (double)rec[4 * Q + 6 + 2 * c] * ym;
            if (ls == 0) rec[4 * Q + 4] = (FT)ym;
        }
        rec += stride;
    } else if (mine && live) {
        bc = beff(v, rhs, slot_index_init<Q>(c, v));
    }
    // one block of q levels is loaded a block ahead: the lane's multipliers
    // of every level and the right-hand side entering its slot (refilled at
    // j = c mod q), raw from clamped addresses and selected when used
    GLB_PTR(const double) rb = v.n > 0 ? rhs : GLB(const double, kZeroBand);
    const int nm = v.n > 0 ? v.n - 1 : 0;
    const int lastk = v.npair > 0 ? v.npair - 1 : 0;
    FT nw[Q][2];
    double nbv;
    uint32_t npin;
    auto load_blk = [&](int kb) {
#pragma unroll
        for (int j = 0; j < Q; j++) {
            const int kk = min(max(kb + j, 0), lastk);  // record index of level kb+j+1
            const int64_t e = (int64_t)kk * stride + 4 * Q + 6 + 2 * c;
            nw[j][0] = rec[e];
            nw[j][1] = rec[e + 1];
        }
        const int k = kb + (c & (Q - 1)) + 1;
        const int g = c < Q ? v.P1_0 - (k - 1) - Q : v.P2_0 + (k - 1) + Q;
        const int gc = min(max(g, 0), nm);
        nbv = rb[gc];
        npin = v.pin ? (uint32_t)v.pin[gc] : 0u;
    };
    load_blk(0);
    for (int kb = 0; kb < kmax; kb += Q) {
        FT cw[Q][2];
#pragma unroll
        for (int j = 0; j < Q; j++) {
            cw[j][0] = nw[j][0];
            cw[j][1] = nw[j][1];
        }
        const int kin = kb + (c & (Q - 1)) + 1;
        const int gin = c < Q ? v.P1_0 - (kin - 1) - Q : v.P2_0 + (kin - 1) + Q;
        const double bin = (gin >= 0 && gin < v.n && npin == 0u) ? nbv : 0.0;
        load_blk(kb + Q);
#pragma unroll
        for (int j = 0; j < Q; j++) {
            const int k = kb + j + 1;
            const bool act = live && (k <= v.npair);
            const double y1 = __shfl(bc, gbase + j);
            const double y2 = __shfl(bc, gbase + Q + j);
            const double base = (c == j || c == Q + j) ? bin : bc;
            const double nb = base - ((double)cw[j][0] * y1 + (double)cw[j][1] * y2);
            bc = (act && mine) ? nb : bc;
            if (act && c == 0 && mine) {
                rec[(int64_t)(k - 1) * stride + 4 * Q + 4] = (FT)y1;
                rec[(int64_t)(k - 1) * stride + 4 * Q + 5] = (FT)y2;
            }
        }
    }
}

// --------------------------------------------------------------------------
// Back solve Z0 x = y, from both ends inwards.  x written to `x` (system
// base).  2q lanes per system hold the outer unknowns of the frontier slots.
// The q records of a block are contiguous; the system's lanes load the next
// block (going inwards) into registers while the current one is solved from
// LDS.  If ADD, x += solution instead of x = solution.
// --------------------------------------------------------------------------
template <int Q, int L, typename FT, bool ADD>
PQ_DEV void back_system(SysView v, bool live, GLB_PTR(const FT) rec0,
                                         int stride, GLB_PTR(double) x, LDS_PTR(FT) lB, int ls,
                                         int kmax)
{
    ls = launder(ls);
    using G = Geo<Q, L>;
    constexpr int N2 = 2 * Q;
    constexpr int LPS = G::LPS;
    constexpr int SB = G::SB;
    const bool mine = ls < N2;
    const int c = mine ? ls : 0;
    const int blk = SB * stride;                 // elements per superblock of records
    const int per_lane = (blk + LPS - 1) / LPS;  // <= MAXPL
    constexpr int MAXPL = (SB * (8 * Q + 6) + LPS - 1) / LPS;
    double xs = 0.0;
    GLB_PTR(const FT) recp = rec0 + (v.odd ? stride : 0);  // first 2x2 level record
    const int kb_last = kmax > 0 ? ((kmax - 1) / SB) * SB : -SB;
    const int64_t lim = live ? (int64_t)v.npair * stride : 0;  // valid elements from recp

    // raw loads from clamped (valid) addresses; elements past the records
    // are zeroed when the block is consumed, so that no select waits on a
    // load in flight
    FT nb[MAXPL];
    const int64_t gmax = lim > 0 ? lim - 1 : 0;
    auto load_block = [&](int kb) {
#pragma unroll
        for (int r = 0; r < MAXPL; r++) {
            const int e = ls + LPS * r;
            const int64_t ge = (int64_t)kb * stride + e;
            nb[r] = recp[ge < 0 ? 0 : (ge > gmax ? gmax : ge)];
        }
    };
    load_block(kb_last);
    for (int kb = kb_last; kb >= 0; kb -= SB) {
#pragma unroll
        for (int r = 0; r < MAXPL; r++) {
            const int e = ls + LPS * r;
            const bool ok = (int64_t)kb * stride + e < lim;  // kb >= 0 here
            if (r < per_lane && e < blk) lB[e] = ok ? nb[r] : (FT)0;
        }
        wave_sync();
        load_block(kb - SB);
#pragma unroll
        for (int jj = SB - 1; jj >= 0; jj--) {  // levels past the last one are inert
            const int j = jj & (Q - 1);
            const int k = kb + jj + 1;
            const bool act = live && (k <= v.npair);
            LDS_PTR(FT) r = lB + jj * stride;
            const double z1 = (double)r[c], z2 = (double)r[N2 + c];
            const double i11 = (double)r[4 * Q + 0], i12 = (double)r[4 * Q + 1];
            const double i21 = (double)r[4 * Q + 2], i22 = (double)r[4 * Q + 3];
            const double y1 = (double)r[4 * Q + 4], y2 = (double)r[4 * Q + 5];
            const double s1 = group_sum<N2>(mine ? z1 * xs : 0.0);
            const double s2 = group_sum<N2>(mine ? z2 * xs : 0.0);
            const double r1 = y1 - s1, r2 = y2 - s2;
            const double x1 = i11 * r1 + i12 * r2;
            const double x2 = i21 * r1 + i22 * r2;
            xs = (act && c == j) ? x1 : ((act && c == Q + j) ? x2 : xs);
            if (j == 0) {
                // block of q levels done: lane c (< 2q) holds the unknown of
                // slot c for the block's level kc; one store per block
                const int kc = kb + jj + (c & (Q - 1)) + 1;
                if (mine && live && kc <= v.npair) {
                    const int g = c < Q ? v.P1_0 - (kc - 1) : v.P2_0 + (kc - 1);
                    if (ADD)
                        x[g] += xs;
                    else
                        x[g] = xs;
                }
            }
        }
        wave_sync();
    }
    if (v.odd && live) {
        GLB_PTR(const FT) r = rec0;
        const double z = (double)r[c];
        const double s = group_sum<N2>(mine ? z * xs : 0.0);
        const double xm = (double)r[4 * Q] * ((double)r[4 * Q + 4] - s);
        if (ls == 0) {
            if (ADD)
                x[v.npair] += xm;
            else
                x[v.npair] = xm;
        }
    }
}

// --------------------------------------------------------------------------
// Kernels
// --------------------------------------------------------------------------

template <int Q, int L, typename FT>
struct LdsBlock {
    FT F[Geo<Q, L>::SPW][Geo<Q, L>::E];
    FT Y[Geo<Q, L>::SPW][Geo<Q, L>::N2];
    FT X[Geo<Q, L>::SPW][6 * Geo<Q, L>::SB];
    FT B[Geo<Q, L>::SPW][Geo<Q, L>::SB * (8 * Q + 6)];
};

template <typename T>
PQ_DEV LDS_PTR(T) as_lds(T* p)
{
    return (LDS_PTR(T))p;
}

// Residual pass over one system: w = A u - b with the original band.
// Returns (in *changes) the number of active-set changes for LCP_EXACT.
template <int Q, int LPS>
PQ_DEV void residual_update(SysView v, bool live, const LcpArgs& A, int64_t off, int ls,
                            bool update, bool write_w, int& changes, int& nonfinite)
{
    ls = launder(ls);
    constexpr int BW = 2 * Q + 1;
    GLB_PTR(const double) u = GLB(const double, A.u + off);
    GLB_PTR(const double) bb = GLB(const double, A.b + off);
    GLB_PTR(const double) band = v.band;
    GLB_PTR(double) wout = A.w ? GLB(double, A.w + off) : nullptr;
    GLB_PTR(const uint8_t) bnds = A.bounded ? GLB(const uint8_t, A.bounded + off) : nullptr;
    GLB_PTR(uint8_t) act = GLB(uint8_t, A.act + off);
    int ch = 0, nf = 0;
    // R rows per lane per pass; all their loads (clamped, valid addresses)
    // are issued before any is used, so a pass waits for memory once
    constexpr int R = BW <= 5 ? 4 : (BW <= 9 ? 2 : 1);
    if (live && !update && !(write_w && wout)) {
        // nothing to store (plain linear solve without w): only the
        // finiteness check of u
        constexpr int RU = 8;
        const int nm = v.n - 1;
        for (int i0 = ls; i0 < v.n; i0 += RU * LPS) {
            double uv[RU];
#pragma unroll
            for (int r = 0; r < RU; r++) uv[r] = u[min(i0 + r * LPS, nm)];
#pragma unroll
            for (int r = 0; r < RU; r++)
                if (i0 + r * LPS < v.n && !isfinite(uv[r])) nf = 1;
        }
    } else if (live) {
        const int nm = v.n - 1;
        for (int i0 = ls; i0 < v.n; i0 += R * LPS) {
            double av[R][BW], uv[R][BW], bv[R];
            uint32_t cv[R], kv[R];
#pragma unroll
            for (int r = 0; r < R; r++) {
                const int i = min(i0 + r * LPS, nm);
#pragma unroll
                for (int d = 0; d < BW; d++) {
                    av[r][d] = band[(int64_t)i * BW + d];
                    uv[r][d] = u[min(max(i + d - Q, 0), nm)];
                }
                bv[r] = bb[i];
                cv[r] = act[i];
                kv[r] = bnds ? (uint32_t)bnds[i] : 1u;
            }
#pragma unroll
            for (int r = 0; r < R; r++) {
                const int i = i0 + r * LPS;
                if (i < v.n) {
                    double s = 0.0;
#pragma unroll
                    for (int d = 0; d < BW; d++) {
                        const int jcol = i + d - Q;
                        s = __builtin_fma(av[r][d], (jcol >= 0 && jcol < v.n) ? uv[r][d] : 0.0, s);
                    }
                    const double wi = s - bv[r];
                    const double ui = uv[r][Q];
                    if (!isfinite(ui)) nf = 1;
                    if (write_w && wout) wout[i] = wi;
                    if (update) {
                        const int bnd = kv[r] != 0u;
                        const int cur = cv[r] != 0u;
                        const int nxt = bnd ? (cur ? (wi > 0.0) : (ui < 0.0)) : 0;
                        ch += (nxt != cur);
                        act[i] = (uint8_t)nxt;
                    }
                }
            }
        }
    }
    changes = group_sum_int<LPS>(ch);
    nonfinite = group_max_int<LPS>(nf);
}

// Effective residual r = b_eff - A_eff u on one system (for refinement);
// returns the group max |r| and max |b_eff|.
template <int Q, int L>
PQ_DEV void eff_residual(SysView v, bool live, GLB_PTR(const double) bsys,
                                          GLB_PTR(const double) u, GLB_PTR(double) r, int ls,
                                          double& rmax, double& bmax)
{
    ls = launder(ls);
    using G = Geo<Q, L>;
    double rm = 0.0, bm = 0.0;
    constexpr int BW = G::BW;
    constexpr int R = BW <= 5 ? 2 : 1;  // rows per lane per pass, loads issued first
    if (live) {
        const int nm = v.n - 1;
        for (int i0 = ls; i0 < v.n; i0 += R * G::LPS) {
            double av[R][BW], uv[R][BW], bv[R];
            uint32_t pv[R][BW];
#pragma unroll
            for (int rr = 0; rr < R; rr++) {
                const int i = min(i0 + rr * G::LPS, nm);
#pragma unroll
                for (int d = 0; d < BW; d++) {
                    const int jc = min(max(i + d - Q, 0), nm);
                    av[rr][d] = v.band[(int64_t)i * BW + d];
                    uv[rr][d] = u[jc];
                    pv[rr][d] = v.pin ? (uint32_t)v.pin[jc] : 0u;
                }
                bv[rr] = bsys[i];
            }
#pragma unroll
            for (int rr = 0; rr < R; rr++) {
                const int i = i0 + rr * G::LPS;
                if (i < v.n) {
                    // pinned rows and columns of A_eff are those of the identity
                    const bool pin_i = pv[rr][Q] != 0u;
                    double s = 0.0;
#pragma unroll
                    for (int d = 0; d < BW; d++) {
                        const int jcol = i + d - Q;
                        const bool in = jcol >= 0 && jcol < v.n;
                        const double a =
                            (pin_i || pv[rr][d] != 0u) ? (d == Q ? 1.0 : 0.0) : av[rr][d];
                        s = __builtin_fma(a, in ? uv[rr][d] : 0.0, s);
                    }
                    const double be = pin_i ? 0.0 : bv[rr];
                    const double ri = be - s;
                    r[i] = ri;
                    rm = fmax(rm, fabs(ri));
                    bm = fmax(bm, fabs(be));
                }
            }
        }
    }
#pragma unroll
    for (int m = G::LPS / 2; m >= 1; m >>= 1) {
        rm = fmax(rm, __shfl_xor(rm, m, G::LPS));
        bm = fmax(bm, __shfl_xor(bm, m, G::LPS));
    }
    rmax = rm;
    bmax = bm;
}

// Sweeps per launch of paqif_sweep_kernel: a halo of at most 128 rows per
// side of the 512 rows a workgroup holds (at q = 8, 12 sweeps in one launch
// with 336-row cores took 0.57 ms on a batch of 4096 systems of 513-4097
// rows, in two launches of 3 and 9 sweeps 0.81 ms: another read of the band
// costs more than the larger halo).
template <int Q>
constexpr int sweep_pass_max()
{
    return 1 + 128 / Q;
}

// Starting iterate of the exact LCP's active-set loop: kp projected Jacobi
// sweeps, u_i <- (b_i - sum_{j != i} a_ij u_j) / a_ii, clipped at zero on
// bounded rows, from the iterate in src (null: u = 0, so that the first
// sweep gives b_i / a_ii); the solve kernels then start from
// A_0 = {bounded i : u_i <= 0}.  The sweeps are pure Jacobi, every row
// independent, so a workgroup takes SWR = 2 SWC consecutive rows of one
// system, two per thread, whose band rows stay in the thread's registers
// for all kp sweeps, and runs them with the iterates in LDS.  Sweep s is
// exact on the rows at least s q from the held range's ends (the others
// read stale values at the ends), so the workgroup writes the rows at least
// (kp - 1) q inside, its core of SWR - 2 (kp - 1) q rows (temporal
// blocking: one read of the band for kp sweeps).  Rows outside the system
// hold zero.  Systems with fewer than sweep_min elimination levels are
// left alone (grid: cores x systems).
template <int Q>
__global__ void __launch_bounds__(SWC) paqif_sweep_kernel(SweepArgs S)
{
    constexpr int BW = 2 * Q + 1;
    constexpr int R = 2;                // rows per thread
    constexpr int SWR = R * SWC;        // rows held by the workgroup
    constexpr int UB = SWR + 2 * Q;     // iterate buffer: held rows and q beyond each end
    __shared__ __attribute__((aligned(16))) double ubuf[2][UB];
    const int sys = blockIdx.y;
    const int64_t off = S.offsets[sys];
    const int n = (int)(S.offsets[sys + 1] - off);
    const int kp = S.kp;
    const int H = (kp - 1) * Q;         // rows of the held range outside the core
    const int C = SWR - 2 * H;          // core rows
    const int c0 = blockIdx.x * C;
    if (n / 2 < S.sweep_min || c0 >= n) return;  // the whole workgroup
    const int blo = c0 - H;                      // first held row (may be < 0)
    const int i0 = blo + R * (int)threadIdx.x;   // this thread's first row
    const int64_t boff = S.band_off ? S.band_off[sys] : off;
    const bool hasu = S.src != nullptr;

    // this thread's rows (clamped loads; rows outside the system are
    // computed from a real row and then replaced by zero), and the source
    // iterate on the buffer's rows blo - q .. blo + SWR + q - 1
    double a[R][BW], bv[R];
    uint32_t kb[R];
    constexpr int PU = (UB + SWC - 1) / SWC;
    double ru[PU];
    {
        GLB_PTR(const double) gb = GLB(const double, S.band + boff * BW);
        GLB_PTR(const double) gr = GLB(const double, S.b + off);
        GLB_PTR(const uint8_t) gk =
            S.bounded ? GLB(const uint8_t, S.bounded + off) : GLB(const uint8_t, kOneFlags);
        GLB_PTR(const double) gs = GLB(const double, (hasu ? S.src : S.b) + off);
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int ic = min(max(i0 + r, 0), n - 1);
#pragma unroll
            for (int d = 0; d < BW; d++) a[r][d] = gb[(int64_t)ic * BW + d];
            // band entries of columns outside the system (padding) are not
            // part of A
#pragma unroll
            for (int d = 0; d < BW; d++) {
                const int j = ic + d - Q;
                if (d != Q && (j < 0 || j >= n)) a[r][d] = 0.0;
            }
            bv[r] = gr[ic];
            kb[r] = (uint32_t)gk[S.bounded ? ic : 0];
        }
#pragma unroll
        for (int t = 0; t < PU; t++)
            ru[t] = gs[min(max(blo - Q + (int)threadIdx.x + t * SWC, 0), n - 1)];
    }
#pragma unroll
    for (int t = 0; t < PU; t++) {
        const int e = (int)threadIdx.x + t * SWC;
        const int i = blo - Q + e;
        if (e < UB) ubuf[0][e] = (hasu && i >= 0 && i < n) ? ru[t] : 0.0;
    }
    // rows outside the system hold zero
    bool in[R];
#pragma unroll
    for (int r = 0; r < R; r++) in[r] = i0 + r >= 0 && i0 + r < n;
    __syncthreads();
    int cur = 0;
    for (int sw = 0; sw < kp; sw++) {
        const double* up = ubuf[cur];
        double* un = ubuf[cur ^ 1];
        // window: rows i0 - q .. i0 + R - 1 + q (buffer index R t ..)
        double w[R + 2 * Q];
#pragma unroll
        for (int k = 0; k < R + 2 * Q; k += 2) {
            const double2 p = *reinterpret_cast<const double2*>(up + R * threadIdx.x + k);
            w[k] = p.x;
            w[k + 1] = p.y;
        }
        double x[R];
#pragma unroll
        for (int r = 0; r < R; r++) {
            double sum = bv[r];
#pragma unroll
            for (int d = 0; d < BW; d++)
                if (d != Q) sum = __builtin_fma(-a[r][d], w[r + d], sum);
            const double v = sum / a[r][Q];
            x[r] = in[r] ? (kb[r] != 0u ? fmax(v, 0.0) : v) : 0.0;
        }
        *reinterpret_cast<double2*>(un + Q + R * threadIdx.x) = make_double2(x[0], x[1]);
        __syncthreads();
        cur ^= 1;
    }
    // the core rows c0 .. c0 + C - 1 (within the system)
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int i = i0 + r;
        if (i >= c0 && i < c0 + C && i < n) S.dst[off + i] = ubuf[cur][Q + R * threadIdx.x + r];
    }
}

// All k sweeps: ceil(k / sweep_pass_max) launches of (nearly) equal sweep
// counts, alternating between tmp and u so that the last one writes u.
template <int Q>
static int launch_sweeps(const LcpArgs& a, int max_n, double* tmp, hipStream_t s)
{
    const int k = a.sweeps;
    if (k <= 0 || a.count <= 0 || max_n <= 0) return PAQIF_OK;
    constexpr int KP = sweep_pass_max<Q>();
    const int passes = (k + KP - 1) / KP;
    SweepArgs S;
    S.count = a.count;
    S.offsets = a.offsets;
    S.band_off = a.band_off;
    S.band = a.band;
    S.b = a.b;
    S.bounded = a.bounded;
    S.sweep_min = a.sweep_min;
    const double* src = nullptr;
    for (int p = 0; p < passes; p++) {
        const int kp = k / passes + (p < k % passes ? 1 : 0);
        double* dst = ((passes - 1 - p) % 2 == 0) ? a.u : tmp;
        S.src = src;
        S.dst = dst;
        S.kp = kp;
        const int core = 2 * SWC - 2 * (kp - 1) * Q;  // rows written per workgroup
        const dim3 grid((max_n + core - 1) / core, a.count);
        hipLaunchKernelGGL((paqif_sweep_kernel<Q>), grid, dim3(SWC), 0, s, S);
        if (!hip_ok(hipGetLastError())) return PAQIF_EHIP;
        src = dst;
    }
    return PAQIF_OK;
}

// Whole LCP solve, one wave per SPW systems.
template <int Q, int L, typename FT>
__global__ void __launch_bounds__(64)
    __attribute__((amdgpu_waves_per_eu(Geo<Q, L>::WPE, 8))) paqif_lcp_kernel(LcpArgs A)
{
    using G = Geo<Q, L>;
    __shared__ LdsBlock<Q, L, FT> lds;
    const int lane = threadIdx.x;
    const int grp = lane / G::LPS;
    const int ls = lane % G::LPS;
    const int gbase = grp * G::LPS;
    const int slot = blockIdx.x * G::SPW + grp;
    bool live = slot < A.count;
    int sys = live ? (A.order ? A.order[slot] : slot) : 0;
    if (live && A.skip && A.skip[sys]) live = false;
    int64_t off = live ? A.offsets[sys] : 0;
    int64_t n = live ? A.offsets[sys + 1] - off : 0;
    int64_t boff = live && A.band_off ? A.band_off[sys] : off;
    if constexpr (G::SPW == 1) {  // one system per wave: keep its scalars in SGPRs
        sys = __builtin_amdgcn_readfirstlane(sys);
        off = uniform64(off);
        n = uniform64(n);
        boff = uniform64(boff);
    }
    SysView v = make_view(off, n, A.band, A.act, A.b, G::BW, boff);
    if (!live) {
        v.n = 0;
        v.npair = 0;
    }
    int kmax = group_max_int<64>(v.npair);  // whole wave loops to the largest system
    constexpr bool MIXED = sizeof(FT) == 4;
    constexpr int stride = MIXED ? (G::ZREC + G::WREC) : G::ZREC;
    GLB_PTR(FT) rec = GLB(FT, reinterpret_cast<FT*>(A.rec) + level_base(off, sys) * stride);

    const bool exact = A.mode == LCP_EXACT;
    // working active set: exact mode starts from A_0 = {bounded i : u_i <= 0}
    // for u after A.sweeps projected Jacobi sweeps (one sweep or none: the
    // sign of b, which predicts the binding constraints of a diagonally
    // dominant system), or, warm, from the flags the caller left in act
    // restricted to bounded rows; the other modes start empty
    const bool warm = exact && A.warm;
    const bool swept = exact && !warm && A.sweeps > 0 && live && v.npair >= A.sweep_min;
    GLB_PTR(const double) us = GLB(const double, (swept ? A.u : A.b) + off);
    if (live) {
        // 8 rows per lane per pass, loads (clamped rows) issued before use
        constexpr int R = 8;
        const int nm = v.n - 1;
        for (int i0 = ls; i0 < v.n; i0 += R * G::LPS) {
            uint32_t bn[R], pa[R];
            double bv[R];
#pragma unroll
            for (int r = 0; r < R; r++) {
                const int64_t g = off + min(i0 + r * G::LPS, nm);
                bn[r] = A.bounded ? (uint32_t)A.bounded[g] : 1u;
                pa[r] = warm ? (uint32_t)A.act[g] : 0u;
                bv[r] = us[g - off];
            }
#pragma unroll
            for (int r = 0; r < R; r++) {
                const int i = i0 + r * G::LPS;
                const bool start = warm ? pa[r] != 0u : bv[r] <= 0.0;
                if (i < v.n) A.act[off + i] = (exact && bn[r] != 0u && start) ? 1 : 0;
            }
        }
    }
    __syncthreads();

    const int max_it = exact ? max(A.max_iter, 1) : 1;
    int st = SYS_OK;
    int it = 0;
    bool done = !live;
    for (; it < max_it;) {
        // ---- factor (+ forward) and back solve ----------------------------
        bool bad;
        if constexpr (!MIXED) {
            bad = factor_system<Q, L, FT, false, true>(v, live && !done, rec, stride,
                                                    as_lds(lds.F[grp]), as_lds(lds.Y[grp]),
                                                    as_lds(lds.X[grp]), ls, kmax);
            __syncthreads();
            back_system<Q, L, FT, false>(v, live && !done, rec, stride, GLB(double, A.u + off),
                                      as_lds(lds.B[grp]), ls, kmax);
        } else {
            bad = factor_system<Q, L, FT, true, false>(v, live && !done, rec, stride,
                                                    as_lds(lds.F[grp]), as_lds(lds.Y[grp]),
                                                    as_lds(lds.X[grp]), ls, kmax);
            __syncthreads();
            // u = 0, then refinement sweeps: r = b_eff - A_eff u; u += solve(r)
            if (live && !done)
                for (int i = ls; i < v.n; i += G::LPS) A.u[off + i] = 0.0;
            __syncthreads();
            double bmax = 0.0, rmax = 0.0;
            int steps = 0;
            bool conv = false;
            for (;;) {
                eff_residual<Q, L>(v, live && !done, GLB(const double, A.b + off),
                                GLB(const double, A.u + off), GLB(double, A.r + off), ls, rmax,
                                bmax);
                const double tol = A.refine_tol * fmax(bmax, 1.0);
                const bool ok_here = !(live && !done) || (rmax <= tol) || bad;
                const int need = group_max_int<64>(ok_here ? 0 : 1);
                conv = ok_here;
                if (need == 0 || steps >= 8) break;
                __syncthreads();
                wsolve_system<Q, FT>(v, live && !done && !ok_here, GLB(const double, A.r + off),
                                     rec, stride, ls,
                                     kmax, gbase);
                __syncthreads();
                back_system<Q, L, FT, true>(v, live && !done && !ok_here, rec, stride,
                                         GLB(double, A.u + off),
                                         as_lds(lds.B[grp]), ls, kmax);
                __syncthreads();
                steps++;
            }
            if (live && !done && !conv && !bad) st = SYS_REFINE_STALLED;
        }
        __syncthreads();
        if (live && !done) it++;
        const int badg = group_max_int<G::LPS>(bad ? 1 : 0);
        if (live && !done && badg) {
            st = SYS_ZERO_PIVOT;
            done = true;
        }

        // ---- projection / residual / active-set update --------------------
        int changes = 0, nonfinite = 0;
        if (A.mode == LCP_CLIP && live && !done) {
            for (int i = ls; i < v.n; i += G::LPS) {
                const int bnd = A.bounded ? (A.bounded[off + i] != 0) : 1;
                const double ui = A.u[off + i];
                if (bnd && ui < 0.0) {
                    A.u[off + i] = 0.0;
                    A.act[off + i] = 1;
                }
            }
        }
        __syncthreads();
        residual_update<Q, G::LPS>(v, live && !done, A, off, ls, exact, true, changes, nonfinite);
        __syncthreads();
        if (live && !done) {
            if (nonfinite) {
                st = SYS_NONFINITE;
                done = true;
            } else if (!exact || changes == 0) {
                done = true;
            } else if (it >= max_it) {
                st = SYS_LCP_NOT_CONVERGED;
                done = true;
            }
        }
        const int all_done = group_max_int<64>(done ? 0 : 1) == 0;
        if (all_done) break;
        // systems that are done keep their results; the loop continues for
        // the others in the wave
    }
    if (live) {
        if (A.active_out) {  // copy, 8 rows per lane per pass
            constexpr int R = 8;
            const int nm = v.n - 1;
            for (int i0 = ls; i0 < v.n; i0 += R * G::LPS) {
                uint8_t f[R];
#pragma unroll
                for (int r = 0; r < R; r++) f[r] = A.act[off + min(i0 + r * G::LPS, nm)];
#pragma unroll
                for (int r = 0; r < R; r++)
                    if (i0 + r * G::LPS < v.n) A.active_out[off + i0 + r * G::LPS] = f[r];
            }
        }
        if (ls == 0) {
            A.status[sys] = st;
            if (A.iters) A.iters[sys] = it;
        }
    }
}

// Factor only (records with W0), no right-hand side; records in FT (FP64, or
// FP32 at the layout of the FP32 + refinement LCP path).

template <int Q, typename FT>
__global__ void __launch_bounds__(64)
    __attribute__((amdgpu_waves_per_eu(Geo<Q, 0>::WPE, 8))) paqif_factor_kernel(FactorArgs A)
{
    constexpr int L = 0;
    using G = Geo<Q, L>;
    __shared__ LdsBlock<Q, L, FT> lds;
    const int lane = threadIdx.x;
    const int grp = lane / G::LPS;
    const int ls = lane % G::LPS;
    const int slot = blockIdx.x * G::SPW + grp;
    const bool live = slot < A.count;
    int sys = live ? (A.order ? A.order[slot] : slot) : 0;
    int64_t off = live ? A.offsets[sys] : 0;
    int64_t n = live ? A.offsets[sys + 1] - off : 0;
    if constexpr (G::SPW == 1) {  // one system per wave: keep its scalars in SGPRs
        sys = __builtin_amdgcn_readfirstlane(sys);
        off = uniform64(off);
        n = uniform64(n);
    }
    SysView v = make_view(off, n, A.band, A.pinned, nullptr, G::BW, off);
    if (!live) {
        v.n = 0;
        v.npair = 0;
    }
    const int kmax = group_max_int<64>(v.npair);
    constexpr int stride = G::ZREC + G::WREC;
    GLB_PTR(FT) rec = GLB(FT, reinterpret_cast<FT*>(A.rec) + level_base(off, sys) * stride);
    bool bad = factor_system<Q, L, FT, true, false>(v, live, rec, stride, as_lds(lds.F[grp]),
                                                 as_lds(lds.Y[grp]), as_lds(lds.X[grp]), ls,
                                                 kmax);
    const int badg = group_max_int<G::LPS>(bad ? 1 : 0);
    if (live && ls == 0) A.status[sys] = badg ? SYS_ZERO_PIVOT : SYS_OK;
}


template <int Q, typename FT>
__global__ void __launch_bounds__(64) paqif_solve_factored_kernel(SolveArgs A)
{
    constexpr int L = 0;
    using G = Geo<Q, L>;
    __shared__ LdsBlock<Q, L, FT> lds;
    const int lane = threadIdx.x;
    const int grp = lane / G::LPS;
    const int ls = lane % G::LPS;
    const int gbase = grp * G::LPS;
    const int slot = blockIdx.x * G::SPW + grp;
    const bool live = slot < A.count;
    int sys = live ? (A.order ? A.order[slot] : slot) : 0;
    int64_t off = live ? A.offsets[sys] : 0;
    int64_t n = live ? A.offsets[sys + 1] - off : 0;
    if constexpr (G::SPW == 1) {  // one system per wave: keep its scalars in SGPRs
        sys = __builtin_amdgcn_readfirstlane(sys);
        off = uniform64(off);
        n = uniform64(n);
    }
    SysView v = make_view(off, n, nullptr, A.pinned, nullptr, G::BW, off);
    if (!live) {
        v.n = 0;
        v.npair = 0;
    }
    const int kmax = group_max_int<64>(v.npair);
    constexpr int stride = G::ZREC + G::WREC;
    GLB_PTR(FT) rec = GLB(FT, reinterpret_cast<FT*>(A.rec) + level_base(off, sys) * stride);
    wsolve_system<Q, FT>(v, live, GLB(const double, A.rhs + off), rec, stride, ls, kmax, gbase);
    __syncthreads();
    back_system<Q, L, FT, false>(v, live, rec, stride, GLB(double, A.x + off), as_lds(lds.B[grp]),
                                 ls, kmax);
}

// --------------------------------------------------------------------------
// One system per lane (small q): the whole 2q x 2q frontier and the
// right-hand-side column live in the lane's registers, so a level needs no
// LDS exchange and no cross-lane step; 64 systems per wave.  Same records,
// active-set rule and outputs as paqif_lcp_kernel in FP64.
// --------------------------------------------------------------------------
template <int Q>
struct LaneLevel {  // values entering the frontier at one level
    double nw[2 * Q][2 * Q];  // new entries of refilled elements (others unused)
    double e[6];              // the level's six extras
};

// element (a, b) is refilled (takes a new band entry) at pivot slot j
template <int Q>
PQ_DEV constexpr bool lane_refill(int a, int b, int j)
{
    return (a & (Q - 1)) == j || (b & (Q - 1)) == j;
}

template <int Q>
PQ_DEV void lane_load_level(const SysView& v, bool live, int k, int j, LaneLevel<Q>& L)
{
    constexpr int N2 = 2 * Q;
    const bool ok = live && k <= v.npair;
#pragma unroll
    for (int a = 0; a < N2; a++)
#pragma unroll
        for (int b = 0; b < N2; b++)
            if (lane_refill<Q>(a, b, j)) {
                const double val = level_new<Q>(v, k, a, b);
                L.nw[a][b] = ok ? val : 0.0;
            }
#pragma unroll
    for (int e = 0; e < 6; e++) {
        const double val = level_extra<Q>(v, v.rhs, true, k, e);
        L.e[e] = ok ? val : 0.0;
    }
}

template <int Q>
PQ_DEV bool lane_factor(const SysView& v, bool live, GLB_PTR(double) rec)
{
    constexpr int N2 = 2 * Q, ZR = 4 * Q + 6;
    double F[N2][N2], y[N2];
    bool bad = false;
    if (v.odd) {
        const int m = v.npair;
        const double amm = live ? aeff<Q>(v, m, m) : 1.0;
        if (live && !(amm != 0.0 && isfinite(amm))) bad = true;
        const double ramm = 1.0 / amm;
        const double bm = live ? beff(v, v.rhs, m) : 0.0;
        double amb[N2];
#pragma unroll
        for (int b = 0; b < N2; b++) amb[b] = aeff<Q>(v, m, slot_index_init<Q>(b, v));
#pragma unroll
        for (int a = 0; a < N2; a++) {
            const int ia = slot_index_init<Q>(a, v);
            const double aim = aeff<Q>(v, ia, m) * ramm;
#pragma unroll
            for (int b = 0; b < N2; b++)
                F[a][b] = aeff<Q>(v, ia, slot_index_init<Q>(b, v)) - aim * amb[b];
            y[a] = beff(v, v.rhs, ia) - aim * bm;
        }
        if (live) {
#pragma unroll
            for (int b = 0; b < N2; b++) {
                rec[b] = amb[b];
                rec[N2 + b] = 0.0;
            }
            rec[4 * Q + 0] = ramm;
            rec[4 * Q + 1] = 0.0;
            rec[4 * Q + 2] = 0.0;
            rec[4 * Q + 3] = 0.0;
            rec[4 * Q + 4] = bm;
            rec[4 * Q + 5] = 0.0;
        }
        rec += ZR;
    } else {
#pragma unroll
        for (int a = 0; a < N2; a++) {
            const int ia = slot_index_init<Q>(a, v);
#pragma unroll
            for (int b = 0; b < N2; b++) F[a][b] = live ? aeff<Q>(v, ia, slot_index_init<Q>(b, v)) : 0.0;
            y[a] = live ? beff(v, v.rhs, ia) : 0.0;
        }
    }
    // the values of a block of q levels are loaded one block ahead
    LaneLevel<Q> nxt[Q];
#pragma unroll
    for (int j = 0; j < Q; j++) lane_load_level<Q>(v, live, j + 1, j, nxt[j]);
    const int np = live ? v.npair : 0;
    for (int kb = 0; kb < np; kb += Q) {
        LaneLevel<Q> cur[Q];
#pragma unroll
        for (int j = 0; j < Q; j++) cur[j] = nxt[j];
#pragma unroll
        for (int j = 0; j < Q; j++) lane_load_level<Q>(v, live, kb + Q + j + 1, j, nxt[j]);
#pragma unroll
        for (int j = 0; j < Q; j++) {
            const int k = kb + j + 1;
            if (k > np) break;
            const LaneLevel<Q>& L = cur[j];
            const double P11 = F[j][j], P12 = F[j][Q + j], P21 = F[Q + j][j],
                         P22 = F[Q + j][Q + j];
            const double y1 = y[j], y2 = y[Q + j];
            const double det = P11 * P22 - P12 * P21;
            if (!(det != 0.0 && isfinite(det))) bad = true;
            const double rd = 1.0 / det;
            const double i11 = P22 * rd, i12 = -P12 * rd, i21 = -P21 * rd, i22 = P11 * rd;
            // record: Z0 rows p1, p2 over the slots after this level
            double cA[N2], cB[N2];
#pragma unroll
            for (int b = 0; b < N2; b++) {
                cA[b] = b == j ? L.e[0] : (b == Q + j ? 0.0 : F[j][b]);
                cB[b] = b == j ? 0.0 : (b == Q + j ? L.e[2] : F[Q + j][b]);
                rec[b] = cA[b];
                rec[N2 + b] = cB[b];
            }
            rec[4 * Q + 0] = i11;
            rec[4 * Q + 1] = i12;
            rec[4 * Q + 2] = i21;
            rec[4 * Q + 3] = i22;
            rec[4 * Q + 4] = y1;
            rec[4 * Q + 5] = y2;
            double w1[N2], w2[N2];
#pragma unroll
            for (int a = 0; a < N2; a++) {
                if (a == j) {
                    w1[a] = L.e[1] * i11;
                    w2[a] = L.e[1] * i12;
                } else if (a == Q + j) {
                    w1[a] = L.e[3] * i21;
                    w2[a] = L.e[3] * i22;
                } else {
                    w1[a] = F[a][j] * i11 + F[a][Q + j] * i21;
                    w2[a] = F[a][j] * i12 + F[a][Q + j] * i22;
                }
            }
#pragma unroll
            for (int a = 0; a < N2; a++) {
#pragma unroll
                for (int b = 0; b < N2; b++) {
                    const double base = lane_refill<Q>(a, b, j) ? L.nw[a][b] : F[a][b];
                    F[a][b] = base - (w1[a] * cA[b] + w2[a] * cB[b]);
                }
                const double yb = a == j ? L.e[4] : (a == Q + j ? L.e[5] : y[a]);
                y[a] = yb - (w1[a] * y1 + w2[a] * y2);
            }
            rec += ZR;
        }
    }
    return bad;
}

template <int Q>
PQ_DEV void lane_back(const SysView& v, bool live, GLB_PTR(const double) rec0,
                      GLB_PTR(double) x)
{
    constexpr int N2 = 2 * Q, ZR = 4 * Q + 6;
    if (!live) return;
    double xs[N2];
#pragma unroll
    for (int c = 0; c < N2; c++) xs[c] = 0.0;
    GLB_PTR(const double) recp = rec0 + (v.odd ? ZR : 0);
    const int np = v.npair;
    const int kb_last = np > 0 ? ((np - 1) / Q) * Q : -Q;
    double nb[Q][ZR];
    auto load = [&](int kb) {
#pragma unroll
        for (int j = 0; j < Q; j++) {
            const int k = kb + j + 1;
            const int kc = k < 1 ? 1 : (k > np ? np : k);  // valid record
#pragma unroll
            for (int t = 0; t < ZR; t++) nb[j][t] = recp[(int64_t)(kc - 1) * ZR + t];
        }
    };
    if (np > 0) load(kb_last);
    for (int kb = kb_last; kb >= 0; kb -= Q) {
        double cur[Q][ZR];
#pragma unroll
        for (int j = 0; j < Q; j++)
#pragma unroll
            for (int t = 0; t < ZR; t++) cur[j][t] = nb[j][t];
        if (kb - Q >= 0) load(kb - Q);
#pragma unroll
        for (int j = Q - 1; j >= 0; j--) {
            const int k = kb + j + 1;
            if (k > np) continue;
            const double* r = cur[j];
            double s1 = 0.0, s2 = 0.0;
#pragma unroll
            for (int c = 0; c < N2; c++) {
                s1 += r[c] * xs[c];
                s2 += r[N2 + c] * xs[c];
            }
            const double r1 = r[4 * Q + 4] - s1, r2 = r[4 * Q + 5] - s2;
            const double x1 = r[4 * Q + 0] * r1 + r[4 * Q + 1] * r2;
            const double x2 = r[4 * Q + 2] * r1 + r[4 * Q + 3] * r2;
            xs[j] = x1;
            xs[Q + j] = x2;
            x[v.P1_0 - (k - 1)] = x1;
            x[v.P2_0 + (k - 1)] = x2;
        }
    }
    if (v.odd) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < N2; c++) s += rec0[c] * xs[c];
        x[v.npair] = rec0[4 * Q] * (rec0[4 * Q + 4] - s);
    }
}

template <int Q>
__global__ void __launch_bounds__(64) paqif_lcp_lane_kernel(LcpArgs A)
{
    constexpr int BW = 2 * Q + 1, ZR = 4 * Q + 6;
    const int slot = blockIdx.x * 64 + threadIdx.x;
    bool live = slot < A.count;
    const int sys = live ? (A.order ? A.order[slot] : slot) : 0;
    if (live && A.skip && A.skip[sys]) live = false;
    const int64_t off = live ? A.offsets[sys] : 0;
    const int64_t n = live ? A.offsets[sys + 1] - off : 0;
    const int64_t boff = live && A.band_off ? A.band_off[sys] : off;
    SysView v = make_view(off, n, A.band, A.act, A.b, BW, boff);
    if (!live) {
        v.n = 0;
        v.npair = 0;
    }
    GLB_PTR(double) rec = GLB(double, reinterpret_cast<double*>(A.rec) + level_base(off, sys) * ZR);
    GLB_PTR(double) u = GLB(double, A.u + off);
    GLB_PTR(const double) bb = GLB(const double, A.b + off);
    GLB_PTR(const double) band = v.band;
    GLB_PTR(uint8_t) act = GLB(uint8_t, A.act + off);
    GLB_PTR(const uint8_t) bnds = A.bounded ? GLB(const uint8_t, A.bounded + off) : nullptr;
    const bool exact = A.mode == LCP_EXACT;
    // working active set: exact mode starts from {bounded i : u_i <= 0} for
    // u after A.sweeps projected Jacobi sweeps (none: the sign of b), or warm
    // from the flags in act (bounded rows only)
    const bool swept = exact && !A.warm && A.sweeps > 0 && live && v.npair >= A.sweep_min;
    GLB_PTR(const double) us = swept ? GLB(const double, u) : bb;
    for (int i = 0; i < v.n; i++)
        act[i] = (exact && (bnds ? bnds[i] != 0 : true) && (A.warm ? act[i] != 0 : us[i] <= 0.0));
    const int max_it = exact ? max(A.max_iter, 1) : 1;
    int st = SYS_OK, it = 0;
    bool done = !live;
    while (!done) {
        const bool bad = lane_factor<Q>(v, true, rec);
        lane_back<Q>(v, true, rec, u);
        it++;
        if (bad) {
            st = SYS_ZERO_PIVOT;
            break;
        }
        if (A.mode == LCP_CLIP)
            for (int i = 0; i < v.n; i++)
                if ((bnds ? bnds[i] != 0 : true) && u[i] < 0.0) {
                    u[i] = 0.0;
                    act[i] = 1;
                }
        // w = A u - b with the original band; active-set update
        int changes = 0;
        bool nonfinite = false;
        for (int i = 0; i < v.n; i++) {
            double s = 0.0;
#pragma unroll
            for (int d = 0; d < BW; d++) {
                const int jc = i + d - Q;
                if (jc >= 0 && jc < v.n) s += band[(int64_t)i * BW + d] * u[jc];
            }
            const double wi = s - bb[i];
            const double ui = u[i];
            if (!isfinite(ui)) nonfinite = true;
            if (A.w) A.w[off + i] = wi;
            if (exact) {
                const int bnd = bnds ? (bnds[i] != 0) : 1;
                const int cur = act[i];
                const int nxt = bnd ? (cur ? (wi > 0.0) : (ui < 0.0)) : 0;
                changes += nxt != cur;
                act[i] = (uint8_t)nxt;
            }
        }
        if (nonfinite) {
            st = SYS_NONFINITE;
            break;
        }
        if (!exact || changes == 0) break;
        if (it >= max_it) {
            st = SYS_LCP_NOT_CONVERGED;
            break;
        }
    }
    if (live) {
        if (A.active_out)
            for (int i = 0; i < v.n; i++) A.active_out[off + i] = act[i];
        A.status[sys] = st;
        if (A.iters) A.iters[sys] = it;
    }
}

// --------------------------------------------------------------------------
// Row layout (lane layout 3, FP64): one system per 16-lane row of the
// wavefront, frontier row slot a held whole by lane a (a < 2q; the lanes
// beyond 2q of a row idle), four systems per wave.  A level needs, in every
// lane, the two pivot rows; they are taken straight from the pivot lanes'
// registers by the DPP row broadcast of gfx950 (row_newbcast), fused into
// the FMAs of the rank-2 update (v_fmac_f64 with a broadcast operand), so a
// level has no LDS round trip and no cross-lane reduction.
//
// Pinned rows (the working active set) are replaced by rows of the identity
// only, not columns: with u_i = 0 forced by its row, the pinned column
// multiplies zero, so the solution is the same as with rows and columns
// replaced, and each entering band row needs only its own flag.
//
// Refill.  Lane a (side L = a < q, phase c = a mod q) is the pivot of the
// levels with j = c; at such a level its row leaves (it is published as the
// record's Z0 row) and the lane takes the new band row g (g1 or g2).  The
// new row is written once, pins applied, into a per-lane LDS buffer (double
// buffered by block parity) and read back in slot order at lane-constant
// offsets (the rotation by c cannot be a register index).  The columns j,
// q+j take at level j the entry of the lane's own row in the entering
// column, index q -+ d of its band row, d = (j - c) mod q, also read from
// the buffer.  Every band row is loaded once per factorisation.
//
// The back solve keeps the 2q outer unknowns in every lane of the row
// (compile-time slots) and forms the two Z0 dot products by broadcast FMAs
// from the lanes holding the record entries.
// --------------------------------------------------------------------------
namespace rows {

constexpr int LPS = 16;  // lanes per system (one DPP row)
constexpr int SPW = 4;   // systems per wave

template <int Q>
struct RG {
    static constexpr int N2 = 2 * Q;
    static constexpr int BW = 2 * Q + 1;
    static constexpr int ZR = 4 * Q + 6;  // record: Z0 rows, inverse pivot, forward values
    static constexpr int S = Q == 2 ? 4 : (Q == 4 ? 2 : 1);  // blocks of q levels per superblock
    static constexpr int SB = S * Q;                          // levels per superblock (8)
    static constexpr int RB = 2 * Q + 2;  // LDS refill buffer: effective band row + a zero
    static constexpr int BSB = 8;         // back-solve levels per prefetch superblock
    // discard area of the staging writes: lane l's base is 2l doubles in,
    // and its writes reach up to DUM doubles past it (a pivot row's 2q
    // values, or the three extras pairs) into the next lanes' areas, which
    // is harmless since nothing reads it; one instruction's 64 stores stay
    // distinct and 16 bytes apart (no bank conflicts)
    static constexpr int DUM = N2 > 6 ? N2 : 6;
};

// Calls f(std::integral_constant<int, I>) for I = 0 .. N-1 (compile-time
// indices for the DPP lane selects and register slots).
template <typename F, int... I>
PQ_DEV void static_for_impl(F&& f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
PQ_DEV void static_for(F&& f)
{
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Value of lane N of this lane's 16-lane row (DPP row_newbcast, one v_mov_b64).
template <int N>
PQ_DEV double bcast(double v)
{
    return __longlong_as_double(
        __builtin_amdgcn_mov_dpp(__double_as_longlong(v), 0x150 + N, 0xF, 0xF, false));
}

// acc += (value of src in lane N of the row) * mul, one v_fmac_f64 with a
// DPP row-broadcast source.  A DPP read needs two wait states after a VALU
// write of its source, which the compiler does not add in front of inline
// asm: the first broadcast FMA of a sequence takes an s_nop 1 (NOP), the
// others read sources that no instruction of the sequence writes.
template <int N, bool NOP = false>
PQ_DEV void fmac_bcast(double& acc, double src, double mul)
{
    if constexpr (NOP)
        asm volatile("s_nop 1\n\tv_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
                     : "+v"(acc)
                     : "v"(src), "v"(mul), "n"(N));
    else
        asm volatile("v_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
                     : "+v"(acc)
                     : "v"(src), "v"(mul), "n"(N));
}

// acc -= (value of src in lane N of the row) * mul: the same instruction
// with the negation modifier on its DPP source (exactly fma(-src, mul, acc)).
template <int N, bool NOP = false>
PQ_DEV void fmsc_bcast(double& acc, double src, double mul)
{
    if constexpr (NOP)
        asm volatile("s_nop 1\n\tv_fmac_f64_dpp %0, -%1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
                     : "+v"(acc)
                     : "v"(src), "v"(mul), "n"(N));
    else
        asm volatile("v_fmac_f64_dpp %0, -%1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
                     : "+v"(acc)
                     : "v"(src), "v"(mul), "n"(N));
}

// Effective entry with pinned rows only replaced by the identity.
template <int Q>
PQ_DEV double arow(const SysView& v, int i, int j)
{
    if (i < 0 || j < 0 || i >= v.n || j >= v.n) return 0.0;
    const int d = j - i;
    if (d < -Q || d > Q) return 0.0;
    if (v.pin && v.pin[i]) return i == j ? 1.0 : 0.0;
    return v.band[(int64_t)i * (2 * Q + 1) + (d + Q)];
}

// Factorisation with the fused forward solve; writes one record per level
// (odd n: the centre record first).  lbuf: this lane's 2 refill buffers.
// Returns true if a pivot of a live level was singular / non-finite.
template <int Q>
PQ_DEV bool factor(const SysView& v, bool live, GLB_PTR(double) rec, LDS_PTR(double) lbuf,
                   LDS_PTR(double) lrec, LDS_PTR(double) ldum, int a, int kmax)
{
    using G = RG<Q>;
    constexpr int N2 = G::N2, BW = G::BW, ZR = G::ZR, S = G::S, SB = G::SB, RB = G::RB;
    a = launder(a);
    const bool slot = a < N2;
    const bool left = a < Q;
    const int c = a & (Q - 1);
    const double lmask = (slot && left) ? 1.0 : 0.0, rmask = (slot && !left) ? 1.0 : 0.0;
    GLB_PTR(const double) rhs = v.rhs;
    bool bad = false;

    // ---- initial frontier (after the centre 1x1 level for odd n) ---------
    double f[N2], y;
    const int ia = slot ? (left ? v.P1_0 - a : v.P2_0 + (a - Q)) : -1;
    auto bef = [&](int i) {
        if (i < 0 || i >= v.n) return 0.0;
        if (v.pin && v.pin[i]) return 0.0;
        return rhs[i];
    };
    if (v.odd) {
        const int m = v.npair;
        const double amm = live ? arow<Q>(v, m, m) : 1.0;
        if (live && !(amm != 0.0 && isfinite(amm))) bad = true;
        const double ramm = 1.0 / amm;
        const double bm = live ? bef(m) : 0.0;
        const double aim = arow<Q>(v, ia, m) * ramm;
#pragma unroll
        for (int cc = 0; cc < N2; cc++) {
            const int ib = cc < Q ? v.P1_0 - cc : v.P2_0 + (cc - Q);
            f[cc] = arow<Q>(v, ia, ib) - aim * arow<Q>(v, m, ib);
        }
        y = bef(ia) - aim * bm;
        if (live) {  // centre record: Z0 row m over the slots, 1x1 pivot
            if (slot) {
                rec[a] = arow<Q>(v, m, ia);
                rec[N2 + a] = 0.0;
            }
            if (a == 0) {
                rec[4 * Q + 0] = ramm;
                rec[4 * Q + 1] = 0.0;
                rec[4 * Q + 2] = 0.0;
                rec[4 * Q + 3] = 0.0;
                rec[4 * Q + 4] = bm;
                rec[4 * Q + 5] = 0.0;
            }
        }
        rec += ZR;
    } else {
#pragma unroll
        for (int cc = 0; cc < N2; cc++) {
            const int ib = cc < Q ? v.P1_0 - cc : v.P2_0 + (cc - Q);
            f[cc] = arow<Q>(v, ia, ib);
        }
        y = bef(ia);
    }
    // a frontier row outside the system is an identity row (1 in its own
    // slot): the levels past the system's last one then pivot on identity
    // blocks, so a singular pivot can only be a real one
    if (slot && !(ia >= 0 && ia < v.n)) {
#pragma unroll
        for (int cc = 0; cc < N2; cc++) f[cc] = cc == a ? 1.0 : 0.0;
    }
    // refill buffers: block r's row goes to buffer r mod (S+1), so the rows
    // of the S blocks of a superblock and the row before them coexist; the
    // lane's initial row is block -1's (buffer S)
    double epub;  // the row's coupling to the column entering when it is the pivot
    {
        LDS_PTR(double) b0 = lbuf + S * RB;
#pragma unroll
        for (int t = 0; t < BW; t++) b0[t] = arow<Q>(v, ia, ia - Q + t);
        b0[BW] = 0.0;
        epub = arow<Q>(v, ia, left ? ia - Q : ia + Q);
    }

    // lane-constant LDS offsets of the refilled row in slot order (the
    // own-side slots except the lane's own, whose value enters as the
    // column entry; every other slot reads the zero at index 2q+1)
    int nro[N2];
#pragma unroll
    for (int cc = 0; cc < N2; cc++) {
        int t = G::BW;  // zero
        if (slot && left && cc < Q && cc != c) t = 2 * Q - 1 - ((cc - c - 1 + Q) & (Q - 1));
        if (slot && !left && cc >= Q && cc != Q + c) t = 1 + ((cc - Q - c - 1 + Q) & (Q - 1));
        nro[cc] = t;
    }

    // ---- prefetch of the refill rows: block s of a superblock refills this
    // lane at level kb + s q + c + 1 with row g; raw loads from clamped
    // addresses, one superblock ahead ------------------------------------------
    const int nm = v.n > 0 ? v.n - 1 : 0;
    // flags read unconditionally (a zero array stands in for "no pins"): a
    // load behind a branch is waited for at once
    const bool haspin = v.pin != nullptr;
    GLB_PTR(const uint8_t) pinp = haspin ? v.pin : GLB(const uint8_t, kZeroFlags);
    double rband[S][BW], rb[S];
    uint32_t rpin[S];
    bool rval[S];
    auto load_super = [&](int kn) {
#pragma unroll
        for (int s = 0; s < S; s++) {
            const int t = kn + s * Q + c;  // refill level - 1
            const int g = left ? v.P1_0 - t - Q : v.P2_0 + t + Q;
            rval[s] = slot && live && (t + 1 <= v.npair) && g >= 0 && g < v.n;
            const int gc = min(max(g, 0), nm);
#pragma unroll
            for (int u = 0; u < BW; u++) rband[s][u] = v.band[(int64_t)gc * BW + u];
            rb[s] = rhs[gc];
            rpin[s] = (uint32_t)pinp[haspin ? gc : 0];
        }
    };
    load_super(0);

    // records are staged in LDS (lrec: SB x ZR per system) by the pivot
    // lanes and copied out at the end of the superblock by all lanes of the
    // row in full 16-byte stores: all LDS reads first, then (after the
    // refill preparation, whose LDS wait covers them) all stores.  No store
    // or LDS write sits behind a branch (lanes with nothing to write aim at
    // ldum / kSink), so every wait count is exact.
    constexpr int NPAIR = SB * ZR / 2;
    constexpr int NST = (NPAIR + LPS - 1) / LPS;  // copy pairs per lane per superblock
    GLB_PTR(double) sink = GLB(double, kSink) + 2 * (threadIdx.x & 63);
    LDS_PTR(double) dum = ldum + 2 * (threadIdx.x & 63);
    LDS_PTR(double) stg = lrec;

    // ---- refill rows of the superblock at level kn+1 (raw loads in rband):
    // pins and range applied, into the LDS refill buffers; the rows in slot
    // order (nr) and the lane's entries in the entering columns (cvl) read
    // back.  Called before the level loop and at the end of each superblock,
    // after the record stores, so that its wait for the raw loads does not
    // also wait for those stores.
    double nr[S][N2], ybs[S], eps[S], wjs[S], wqs[S], cvl[S][Q];
    auto prepare = [&](int kn) {
        const int bbase = (kn / Q) % (S + 1);  // buffer of block 0 of the superblock
#pragma unroll
        for (int s = 0; s < S; s++) {
            const bool ok = rval[s];
            const double keep = (ok && rpin[s] == 0u) ? 1.0 : 0.0;
            // pinned rows and rows outside the system: identity rows
            const double one = (!ok || rpin[s] != 0u) ? 1.0 : 0.0;
            int bi = bbase + s;
            bi = bi > S ? bi - (S + 1) : bi;
            LDS_PTR(double) buf = lbuf + bi * RB;
            double e[BW];
#pragma unroll
            for (int u = 0; u < BW; u++) e[u] = rband[s][u] * keep;
            e[Q] += one;
#pragma unroll
            for (int u = 0; u < BW; u++) buf[u] = e[u];
            buf[BW] = 0.0;
            ybs[s] = rb[s] * keep;
            eps[s] = left ? e[0] : e[2 * Q];
            wjs[s] = left ? e[2 * Q] : 0.0;
            wqs[s] = left ? 0.0 : e[0];
        }
        wave_sync();
        // the lane's entries in the columns entering its side, level by level:
        // level j of block s reads the row it holds then (the previous
        // block's before its refill at j = c, the block's own from there on),
        // index q -+ d, d = (j - c) mod q
#pragma unroll
        for (int s = 0; s < S; s++) {
            int bi = bbase + s;
            bi = bi > S ? bi - (S + 1) : bi;
            const int pbi = bi == 0 ? S : bi - 1;
            LDS_PTR(double) buf = lbuf + bi * RB;
#pragma unroll
            for (int cc = 0; cc < N2; cc++) nr[s][cc] = buf[nro[cc]];
#pragma unroll
            for (int j = 0; j < Q; j++) {
                const int d = (j - c + Q) & (Q - 1);
                const int bsel = (j < c) ? pbi : bi;
                cvl[s][j] = lbuf[bsel * RB + (left ? Q - d : Q + d)];
            }
        }
        // every LDS read of the superblock is done here (lgkmcnt 0), so the
        // level loop, whose only LDS accesses are the record writes, never
        // waits on LDS
        __builtin_amdgcn_s_waitcnt(0xC07F);
    };
    prepare(0);

    for (int kb = 0; kb < kmax; kb += SB) {
        load_super(kb + SB);

        static_for<S>([&](auto SS) {
            constexpr int s = decltype(SS)::value;
            static_for<Q>([&](auto JJ) {
                constexpr int j = decltype(JJ)::value;
                const bool isref = slot && c == j;
                const double cv = cvl[s][j];  // entry of the lane's row in the entering column
                // pivot data from lanes j and q+j
                const double P11 = bcast<j>(f[j]), P12 = bcast<j>(f[Q + j]);
                const double P21 = bcast<Q + j>(f[j]), P22 = bcast<Q + j>(f[Q + j]);
                const double y1 = bcast<j>(y), y2 = bcast<Q + j>(y);
                const double E0 = bcast<j>(epub), E2 = bcast<Q + j>(epub);
                const double det = P11 * P22 - P12 * P21;
                if (!(det != 0.0 && isfinite(det))) bad = true;
                // 1/det: hardware reciprocal refined by two Newton steps
                const double r0 = __builtin_amdgcn_rcp(det);
                const double r1 = __builtin_fma(r0, __builtin_fma(-det, r0, 1.0), r0);
                const double rd = __builtin_fma(r1, __builtin_fma(-det, r1, 1.0), r1);
                const double i11 = P22 * rd, i12 = -P12 * rd, i21 = -P21 * rd, i22 = P11 * rd;
                // multipliers of this lane's row (the refilled lane: of its new row)
                const double wj = isref ? wjs[s] : f[j];
                const double wq = isref ? wqs[s] : f[Q + j];
                // (negated multipliers: the update subtracts)
                const double n1 = wj * i11 + wq * i21;
                const double n2 = wj * i12 + wq * i22;
                // rank-2 update into g (base: own row, or the refilled row); the
                // next level's pivot columns first, so that its pivot block can be
                // formed while the other columns are updated
                double g[N2];
                constexpr int jn = (j + 1) & (Q - 1);
                static_for<N2>([&](auto CC) {
                    constexpr int t = decltype(CC)::value;
                    constexpr int cc = t == 0 ? jn : (t == 1 ? Q + jn : (t - 2 < jn ? t - 2 : (t - 2 < Q + jn - 1 ? t - 1 : t)));
                    if constexpr (cc != j && cc != Q + j) {
                        g[cc] = isref ? nr[s][cc] : f[cc];
                        fmsc_bcast<j, t == 0>(g[cc], f[cc], n1);
                        fmsc_bcast<Q + j>(g[cc], f[cc], n2);
                    }
                });
                g[j] = __builtin_fma(-E0, n1, cv * lmask);
                g[Q + j] = __builtin_fma(-E2, n2, cv * rmask);
                // record (staged): the pivot lanes write their rows (Z0 rows p1,
                // p2 over the slots after the level), lane 0 of the row the
                // inverse and y
                {
                    constexpr int jj = s * Q + j;
                    // one base per level (the staging row or the lane's own
                    // discard area), the pairs at constant offsets from it
                    LDS_PTR(double) zr = isref ? stg + jj * ZR + (left ? 0 : N2) : dum;
#pragma unroll
                    for (int t = 0; t < Q; t++) {
                        dbl2 zv;
                        zv.x = f[2 * t];
                        zv.y = f[2 * t + 1];
                        if (2 * t == j) zv.x = epub * lmask;
                        if (2 * t + 1 == j) zv.y = epub * lmask;
                        if (2 * t == Q + j) zv.x = epub * rmask;
                        if (2 * t + 1 == Q + j) zv.y = epub * rmask;
                        *reinterpret_cast<LDS_PTR(dbl2)>(zr + 2 * t) = zv;
                    }
                    const int xp = a % 3;
                    dbl2 xv;
                    xv.x = xp == 0 ? i11 : (xp == 1 ? i21 : y1);
                    xv.y = xp == 0 ? i12 : (xp == 1 ? i22 : y2);
                    *reinterpret_cast<LDS_PTR(dbl2)>(a < 3 ? stg + jj * ZR + 4 * Q + 2 * xp : dum) =
                        xv;
                }
                double gy = isref ? ybs[s] : y;
                gy = __builtin_fma(-y1, n1, gy);
                gy = __builtin_fma(-y2, n2, gy);
                epub = isref ? eps[s] : epub;
#pragma unroll
                for (int cc = 0; cc < N2; cc++) f[cc] = g[cc];
                y = gy;
            });
        });
        // the superblock's records: pair e of the staging area to rec + 2e
        // if its level exists, else to the sink
        dbl2 cp[NST];
#pragma unroll
        for (int r = 0; r < NST; r++) {
            const int e = a + LPS * r;
            cp[r] = *reinterpret_cast<LDS_PTR(const dbl2)>(stg + 2 * (e < NPAIR ? e : 0));
        }
        prepare(kb + SB);
#pragma unroll
        for (int r = 0; r < NST; r++) {
            const int e = a + LPS * r;
            const bool ok = e < NPAIR && live && kb + (2 * e) / ZR + 1 <= v.npair;
            GLB_PTR(double) dst = ok ? rec + 2 * e : sink;
            *reinterpret_cast<GLB_PTR(dbl2)>(dst) = cp[r];
        }
        rec += SB * ZR;
    }
    return bad;
}

// Back solve Z0 x = y from both ends inwards; x written to `x` (system
// base).  Every lane of the row keeps the 2q outer unknowns xs (slots after
// the level being solved); lane t < 2q holds the record's Z0 entries of
// slot t, lanes 0..2 the pairs (i11, i12), (i21, i22), (y1, y2).
template <int Q>
PQ_DEV void back(const SysView& v, bool live, GLB_PTR(const double) rec0, GLB_PTR(double) x,
                 int a, int kmax)
{
    using G = RG<Q>;
    constexpr int N2 = G::N2, ZR = G::ZR, BSB = G::BSB;
    a = launder(a);
    const bool slot = a < N2;
    const int zc = slot ? a : 0;
    const int ep = 4 * Q + 2 * (a % 3);
    GLB_PTR(const double) recp = rec0 + (v.odd ? ZR : 0);  // first 2x2 level
    const int64_t lim = live ? (int64_t)v.npair : 0;       // valid records from recp
    double xs[N2];
#pragma unroll
    for (int cc = 0; cc < N2; cc++) xs[cc] = 0.0;
    double mine = 0.0;
    double pz1[BSB], pz2[BSB], pe0[BSB], pe1[BSB];
    const int rmax = lim > 0 ? (int)lim - 1 : 0;
    GLB_PTR(double) sink = GLB(double, kSink) + 2 * (threadIdx.x & 63);
    auto load_block = [&](int kb) {  // levels kb+1 .. kb+BSB (clamped records)
#pragma unroll
        for (int t = 0; t < BSB; t++) {
            const int r = min(max(kb + t, 0), rmax);
            GLB_PTR(const double) p = recp + (int64_t)r * ZR;
            pz1[t] = p[zc];
            pz2[t] = p[N2 + zc];
            const dbl2 ex = *reinterpret_cast<GLB_PTR(const dbl2)>(p + ep);
            pe0[t] = ex.x;
            pe1[t] = ex.y;
        }
    };
    const int kb_last = kmax > 0 ? ((kmax - 1) / BSB) * BSB : -BSB;
    if (kb_last >= 0) load_block(kb_last);
    // Software pipeline: of a level's two dot products only the terms of the
    // two slots that the level solved just before changes (the "late" terms);
    // the others (E: "early" sums, carried in registers) are formed while
    // that previous level still finishes.  The first level sees xs = 0.
    double e1a = 0.0, e1b = 0.0, e2a = 0.0, e2b = 0.0;
    for (int kb = kb_last; kb >= 0; kb -= BSB) {
        double z1[BSB], z2[BSB], e0[BSB], e1[BSB];
#pragma unroll
        for (int t = 0; t < BSB; t++) {
            z1[t] = pz1[t];
            z2[t] = pz2[t];
            e0[t] = pe0[t];
            e1[t] = pe1[t];
        }
        load_block(kb - BSB);  // unconditional (clamped): no branch, exact wait counts
        static_for<BSB>([&](auto TT) {
            constexpr int t = BSB - 1 - decltype(TT)::value;
            constexpr int j = t & (Q - 1);  // kb is a multiple of BSB, a multiple of q
            const int k = kb + t + 1;
            const bool act = live && k <= v.npair;
            constexpr int jp = (j + 1) & (Q - 1);  // slots of the previous level solved
            // late terms of this level
            fmac_bcast<jp, true>(e1a, z1[t], xs[jp]);
            fmac_bcast<Q + jp>(e1b, z1[t], xs[Q + jp]);
            fmac_bcast<jp>(e2a, z2[t], xs[jp]);
            fmac_bcast<Q + jp>(e2b, z2[t], xs[Q + jp]);
            // early sums of the next level in processing order (t - 1, or the
            // next superblock's last level, still in the prefetch registers):
            // every slot but the two this level solves
            double zn1, zn2;
            if constexpr (t > 0) {
                zn1 = z1[t - 1];
                zn2 = z2[t - 1];
            } else {
                zn1 = pz1[BSB - 1];
                zn2 = pz2[BSB - 1];
            }
            double n1a = 0.0, n1b = 0.0, n2a = 0.0, n2b = 0.0;
            static_for<N2>([&](auto CC) {
                constexpr int cc = decltype(CC)::value;
                constexpr int first = (j == 0) ? 1 : 0;  // first slot in the sequence
                if constexpr (cc != j && cc != Q + j) {
                    if constexpr (cc % 2 == 0) {
                        fmac_bcast<cc, cc == first>(n1a, zn1, xs[cc]);
                        fmac_bcast<cc>(n2a, zn2, xs[cc]);
                    } else {
                        fmac_bcast<cc, cc == first>(n1b, zn1, xs[cc]);
                        fmac_bcast<cc>(n2b, zn2, xs[cc]);
                    }
                }
            });
            const double s1a = e1a, s1b = e1b, s2a = e2a, s2b = e2b;
            e1a = n1a;
            e1b = n1b;
            e2a = n2a;
            e2b = n2b;
            const double i11 = bcast<0>(e0[t]), i12 = bcast<0>(e1[t]);
            const double i21 = bcast<1>(e0[t]), i22 = bcast<1>(e1[t]);
            const double y1 = bcast<2>(e0[t]), y2 = bcast<2>(e1[t]);
            const double r1 = y1 - (s1a + s1b), r2 = y2 - (s2a + s2b);
            const double x1 = i11 * r1 + i12 * r2;
            const double x2 = i21 * r1 + i22 * r2;
            xs[j] = act ? x1 : xs[j];
            xs[Q + j] = act ? x2 : xs[Q + j];
            if (act && slot && (a & (Q - 1)) == j) mine = a < Q ? x1 : x2;
            if constexpr (j == 0) {
                // block of q levels done: lane a (< 2q) holds the unknown of
                // slot a, level kc = k + (a mod q)
                const int kc = k + (a & (Q - 1));
                const int gi = a < Q ? v.P1_0 - (kc - 1) : v.P2_0 + (kc - 1);
                GLB_PTR(double) dst = (slot && live && kc <= v.npair) ? x + gi : sink;
                *dst = mine;
            }
        });
    }
    if (v.odd && live) {
        // centre: x_m = (y_m - Z0 row m . xs) / a_mm
        const double zm = rec0[zc];
        double sa = 0.0, sb = 0.0;
        static_for<N2>([&](auto CC) {
            constexpr int cc = decltype(CC)::value;
            if constexpr (cc % 2 == 0)
                fmac_bcast<cc, cc == 0>(sa, zm, xs[cc]);
            else
                fmac_bcast<cc>(sb, zm, xs[cc]);
        });
        if (a == 0) x[v.npair] = rec0[4 * Q] * (rec0[4 * Q + 4] - (sa + sb));
    }
}

// Residual pass of the row layout: w = A u - b with the original band and
// the active-set update, as residual_update, but each lane takes R
// consecutive rows per stage, so its u window is R + 2q values and its band
// rows one contiguous run; the loads of a stage (clamped addresses) are
// issued together, the next stage's before the current one is used.
template <int Q>
PQ_DEV void residual(const SysView& v, bool live, const LcpArgs& A, int64_t off, int ls,
                     bool update, bool write_w, int& changes, int& nonfinite)
{
    ls = launder(ls);
    constexpr int BW = 2 * Q + 1;
    constexpr int R = Q == 8 ? 2 : (Q == 4 ? 4 : 8);  // rows per lane per stage
    constexpr int UW = R + 2 * Q;
    GLB_PTR(const double) u = GLB(const double, A.u + off);
    GLB_PTR(const double) bb = GLB(const double, A.b + off);
    GLB_PTR(const double) band = v.band;
    GLB_PTR(double) wout = A.w ? GLB(double, A.w + off) : nullptr;
    const bool ww = write_w && wout != nullptr;
    const bool hasb = A.bounded != nullptr;
    GLB_PTR(const uint8_t) bnds =
        hasb ? GLB(const uint8_t, A.bounded + off) : GLB(const uint8_t, kOneFlags);
    GLB_PTR(uint8_t) act = GLB(uint8_t, A.act + off);
    // stores of rows past the end (and w when it is not wanted) go to the
    // sink: no store sits behind a branch
    GLB_PTR(double) sinkd = GLB(double, kSink) + (threadIdx.x & 63);
    GLB_PTR(uint8_t) sinkb = GLB(uint8_t, reinterpret_cast<uint8_t*>(kSink)) + (threadIdx.x & 63);
    struct Stage {
        double a[R][BW], u[UW], b[R];
        uint32_t c[R], k[R];
    };
    int ch = 0, nf = 0;
    if (live && v.n > 0) {
        const int nm = v.n - 1;
        const int step = R * LPS;
        auto load = [&](int i0, Stage& g) {  // clamped rows: always valid addresses
#pragma unroll
            for (int t = 0; t < UW; t++) g.u[t] = u[min(max(i0 - Q + t, 0), nm)];
#pragma unroll
            for (int r = 0; r < R; r++) {
                const int i = min(i0 + r, nm);
#pragma unroll
                for (int d = 0; d < BW; d++) g.a[r][d] = band[(int64_t)i * BW + d];
                g.b[r] = bb[i];
                g.c[r] = act[i];
                g.k[r] = (uint32_t)bnds[hasb ? i : 0];
            }
        };
        auto apply = [&](int i0, const Stage& g) {
#pragma unroll
            for (int r = 0; r < R; r++) {
                const int i = i0 + r;
                const bool in = i < v.n;
                double sum = 0.0;
#pragma unroll
                for (int d = 0; d < BW; d++) {
                    const int jcol = i + d - Q;
                    sum = __builtin_fma(g.a[r][d], (jcol >= 0 && jcol < v.n) ? g.u[r + d] : 0.0,
                                        sum);
                }
                const double wi = sum - g.b[r];
                const double ui = g.u[r + Q];
                if (in && !isfinite(ui)) nf = 1;
                *((ww && in) ? wout + i : sinkd) = wi;
                if (update) {
                    const int bnd = g.k[r] != 0u;
                    const int cur = g.c[r] != 0u;
                    const int nxt = bnd ? (cur ? (wi > 0.0) : (ui < 0.0)) : 0;
                    ch += (in && nxt != cur) ? 1 : 0;
                    *(in ? act + i : sinkb) = (uint8_t)nxt;
                }
            }
        };
        // two stages in flight: the next stage's loads are issued before the
        // current one is used
        Stage S0, S1;
        int i0 = ls * R;
        load(i0, S0);
        while (i0 < v.n) {
            load(i0 + step, S1);
            apply(i0, S0);
            i0 += step;
            if (i0 >= v.n) break;
            load(i0 + step, S0);
            apply(i0, S1);
            i0 += step;
        }
    }
    changes = group_sum_int<LPS>(ch);
    nonfinite = group_max_int<LPS>(nf);
}

}  // namespace rows

template <int Q>
struct RowLds {
    // per lane: S+1 refill buffers; an odd lane stride (in doubles) spreads
    // the 64-bit accesses of 16 lanes over distinct LDS bank pairs
    double buf[64][(rows::RG<Q>::S + 1) * rows::RG<Q>::RB + 1];
    alignas(16) double rec[rows::SPW][rows::RG<Q>::SB * rows::RG<Q>::ZR];  // staged records
    alignas(16) double dum[2 * 64 + rows::RG<Q>::DUM];  // discarded writes
};

// Whole LCP solve in the row layout (FP64), four systems per wave: the
// systems of wave `wave` of the call A, with the wave's LDS in `lds`.
template <int Q>
PQ_DEV void lcp_rows_wave(const LcpArgs& A, int wave, RowLds<Q>& lds)
{
    using G = rows::RG<Q>;
    const int lane = threadIdx.x;
    const int grp = lane >> 4;
    const int ls = lane & 15;
    const int slot = wave * rows::SPW + grp;
    bool live = slot < A.count;
    int sys = live ? (A.order ? A.order[slot] : slot) : 0;
    if (live && A.skip && A.skip[sys]) live = false;
    int64_t off = live ? A.offsets[sys] : 0;
    int64_t n = live ? A.offsets[sys + 1] - off : 0;
    int64_t boff = live && A.band_off ? A.band_off[sys] : off;
    SysView v = make_view(off, n, A.band, A.act, A.b, G::BW, boff);
    if (!live) {
        v.n = 0;
        v.npair = 0;
    }
    const int kmax = group_max_int<64>(v.npair);
    GLB_PTR(double) rec = GLB(double, reinterpret_cast<double*>(A.rec) + level_base(off, sys) * G::ZR);
    LDS_PTR(double) lbuf = as_lds(&lds.buf[lane][0]);

    const bool exact = A.mode == LCP_EXACT;
    const bool warm = exact && A.warm;
    // starting active set as in paqif_lcp_kernel (from the start sweeps'
    // iterate in u for the systems they ran on)
    const bool swept = exact && !warm && A.sweeps > 0 && live && v.npair >= A.sweep_min;
    GLB_PTR(const double) us = GLB(const double, (swept ? A.u : A.b) + off);
    if (live) {
        constexpr int R = 8;
        const int nm = v.n - 1;
        for (int i0 = ls; i0 < v.n; i0 += R * rows::LPS) {
            uint32_t bn[R], pa[R];
            double bv[R];
#pragma unroll
            for (int r = 0; r < R; r++) {
                const int64_t g = off + min(i0 + r * rows::LPS, nm);
                bn[r] = A.bounded ? (uint32_t)A.bounded[g] : 1u;
                pa[r] = warm ? (uint32_t)A.act[g] : 0u;
                bv[r] = us[g - off];
            }
#pragma unroll
            for (int r = 0; r < R; r++) {
                const int i = i0 + r * rows::LPS;
                const bool start = warm ? pa[r] != 0u : bv[r] <= 0.0;
                if (i < v.n) A.act[off + i] = (exact && bn[r] != 0u && start) ? 1 : 0;
            }
        }
    }
    __syncthreads();

    const int max_it = exact ? max(A.max_iter, 1) : 1;
    int st = SYS_OK;
    int it = 0;
    bool done = !live;
    for (; it < max_it;) {
        const bool bad = rows::factor<Q>(v, live && !done, rec, lbuf, as_lds(&lds.rec[grp][0]),
                                         as_lds(&lds.dum[0]), ls, kmax);
        __syncthreads();
        rows::back<Q>(v, live && !done, rec, GLB(double, A.u + off), ls, kmax);
        __syncthreads();
        if (live && !done) it++;
        const int badg = group_max_int<rows::LPS>(bad ? 1 : 0);
        if (live && !done && badg) {
            st = SYS_ZERO_PIVOT;
            done = true;
        }
        int changes = 0, nonfinite = 0;
        if (A.mode == LCP_CLIP && live && !done) {
            for (int i = ls; i < v.n; i += rows::LPS) {
                const int bnd = A.bounded ? (A.bounded[off + i] != 0) : 1;
                const double ui = A.u[off + i];
                if (bnd && ui < 0.0) {
                    A.u[off + i] = 0.0;
                    A.act[off + i] = 1;
                }
            }
        }
        __syncthreads();
        rows::residual<Q>(v, live && !done, A, off, ls, exact, true, changes, nonfinite);
        __syncthreads();
        if (live && !done) {
            if (nonfinite) {
                st = SYS_NONFINITE;
                done = true;
            } else if (!exact || changes == 0) {
                done = true;
            } else if (it >= max_it) {
                st = SYS_LCP_NOT_CONVERGED;
                done = true;
            }
        }
        const int all_done = group_max_int<64>(done ? 0 : 1) == 0;
        if (all_done) break;
    }
    if (live) {
        if (A.active_out) {
            constexpr int R = 8;
            const int nm = v.n - 1;
            for (int i0 = ls; i0 < v.n; i0 += R * rows::LPS) {
                uint8_t fl[R];
#pragma unroll
                for (int r = 0; r < R; r++) fl[r] = A.act[off + min(i0 + r * rows::LPS, nm)];
#pragma unroll
                for (int r = 0; r < R; r++)
                    if (i0 + r * rows::LPS < v.n) A.active_out[off + i0 + r * rows::LPS] = fl[r];
            }
        }
        if (ls == 0) {
            A.status[sys] = st;
            if (A.iters) A.iters[sys] = it;
        }
    }
}

template <int Q>
__global__ void __launch_bounds__(64) paqif_lcp_rows_kernel(LcpArgs A)
{
    __shared__ RowLds<Q> lds;
    lcp_rows_wave<Q>(A, blockIdx.x, lds);
}

// Several calls in one launch (each of its own q): workgroup g takes wave
// g / n of call g mod n, so the calls' waves interleave and the first
// (largest, in LPT order) waves of every call start first.  The wave's LDS
// is one block sized for the largest q.
constexpr size_t kRowsLds = sizeof(RowLds<8>) > sizeof(RowLds<4>)
                                ? (sizeof(RowLds<8>) > sizeof(RowLds<2>) ? sizeof(RowLds<8>)
                                                                         : sizeof(RowLds<2>))
                                : (sizeof(RowLds<4>) > sizeof(RowLds<2>) ? sizeof(RowLds<4>)
                                                                         : sizeof(RowLds<2>));

__global__ void __launch_bounds__(64) paqif_lcp_rows_many_kernel(RowsManyArgs M)
{
    __shared__ __attribute__((aligned(16))) unsigned char raw[kRowsLds];
    const int c = (int)(blockIdx.x % (unsigned)M.n);
    const int wave = (int)(blockIdx.x / (unsigned)M.n);
    if (wave >= M.waves[c]) return;  // the whole workgroup
    switch (M.q[c]) {
    case 2: lcp_rows_wave<2>(M.a[c], wave, *reinterpret_cast<RowLds<2>*>(raw)); break;
    case 4: lcp_rows_wave<4>(M.a[c], wave, *reinterpret_cast<RowLds<4>*>(raw)); break;
    default: lcp_rows_wave<8>(M.a[c], wave, *reinterpret_cast<RowLds<8>*>(raw)); break;
    }
}

int dispatch_lcp_rows_many(const RowsManyArgs& m, hipStream_t s)
{
    if (m.n < 1 || m.n > kMaxManyCalls) return PAQIF_EINVAL;
    int wmax = 0;
    for (int c = 0; c < m.n; c++) {
        if (m.q[c] != 2 && m.q[c] != 4 && m.q[c] != 8) return PAQIF_EINVAL;
        wmax = m.waves[c] > wmax ? m.waves[c] : wmax;
    }
    if (wmax == 0) return PAQIF_OK;
    hipLaunchKernelGGL(paqif_lcp_rows_many_kernel, dim3(wmax * m.n), dim3(64), 0, s, m);
    return hip_ok(hipGetLastError()) ? PAQIF_OK : PAQIF_EHIP;
}

int rows_waves(int count) { return (count + rows::SPW - 1) / rows::SPW; }


// --------------------------------------------------------------------------
// Host launchers
// --------------------------------------------------------------------------
template <int Q, int L>
static int launch_lcp_l(const LcpArgs& a, int prec, hipStream_t s)
{
    const int grid = (a.count + Geo<Q, L>::SPW - 1) / Geo<Q, L>::SPW;
    if (grid == 0) return PAQIF_OK;
    if (prec == PREC_FP32_IR)
        hipLaunchKernelGGL((paqif_lcp_kernel<Q, L, float>), dim3(grid), dim3(64), 0, s, a);
    else
        hipLaunchKernelGGL((paqif_lcp_kernel<Q, L, double>), dim3(grid), dim3(64), 0, s, a);
    return hip_ok(hipGetLastError()) ? PAQIF_OK : PAQIF_EHIP;
}

template <int Q>
static int launch_lcp(const LcpArgs& a, int prec, int layout, hipStream_t s)
{
    if (layout == 3) {
        // row layout (FP64); the FP32 + refinement path keeps layout 0
        if (prec == PREC_FP32_IR) return launch_lcp_l<Q, 0>(a, prec, s);
        const int grid = (a.count + rows::SPW - 1) / rows::SPW;
        if (grid == 0) return PAQIF_OK;
        hipLaunchKernelGGL((paqif_lcp_rows_kernel<Q>), dim3(grid), dim3(64), 0, s, a);
        return hip_ok(hipGetLastError()) ? PAQIF_OK : PAQIF_EHIP;
    }
    switch (layout) {
    case 1: return launch_lcp_l<Q, 1>(a, prec, s);
    case 2:
        if constexpr (Q == 2) {
            // one system per lane (FP64; the FP32 + refinement path keeps layout 0)
            if (prec == PREC_FP32_IR) return launch_lcp_l<Q, 0>(a, prec, s);
            const int grid = (a.count + 63) / 64;
            if (grid == 0) return PAQIF_OK;
            hipLaunchKernelGGL((paqif_lcp_lane_kernel<Q>), dim3(grid), dim3(64), 0, s, a);
            return hip_ok(hipGetLastError()) ? PAQIF_OK : PAQIF_EHIP;
        } else {
            return launch_lcp_l<Q, 2>(a, prec, s);
        }
    default: return launch_lcp_l<Q, 0>(a, prec, s);
    }
}

template <int Q>
static int launch_factor(const FactorArgs& a, hipStream_t s)
{
    const int grid = (a.count + Geo<Q, 0>::SPW - 1) / Geo<Q, 0>::SPW;
    if (grid == 0) return PAQIF_OK;
    if (a.prec == PREC_FP32_IR)
        hipLaunchKernelGGL((paqif_factor_kernel<Q, float>), dim3(grid), dim3(64), 0, s, a);
    else
        hipLaunchKernelGGL((paqif_factor_kernel<Q, double>), dim3(grid), dim3(64), 0, s, a);
    return hip_ok(hipGetLastError()) ? PAQIF_OK : PAQIF_EHIP;
}

template <int Q>
static int launch_solve(const SolveArgs& a, hipStream_t s)
{
    const int grid = (a.count + Geo<Q, 0>::SPW - 1) / Geo<Q, 0>::SPW;
    if (grid == 0) return PAQIF_OK;
    if (a.prec == PREC_FP32_IR)
        hipLaunchKernelGGL((paqif_solve_factored_kernel<Q, float>), dim3(grid), dim3(64), 0, s, a);
    else
        hipLaunchKernelGGL((paqif_solve_factored_kernel<Q, double>), dim3(grid), dim3(64), 0, s,
                           a);
    return hip_ok(hipGetLastError()) ? PAQIF_OK : PAQIF_EHIP;
}

int record_stride(int q, bool with_w) { return (4 * q + 6) + (with_w ? 4 * q : 0); }

int layouts_for(int q) { return (q == 2 || q == 4 || q == 8) ? layout_count(q) : 0; }

int dispatch_lcp(int q, const LcpArgs& a, int prec, int layout, hipStream_t s)
{
    switch (q) {
    case 2: return launch_lcp<2>(a, prec, layout, s);
    case 4: return launch_lcp<4>(a, prec, layout, s);
    case 8: return launch_lcp<8>(a, prec, layout, s);
    default: return PAQIF_EINVAL;
    }
}

int dispatch_sweeps(int q, const LcpArgs& a, int max_n, double* tmp, hipStream_t s)
{
    switch (q) {
    case 2: return launch_sweeps<2>(a, max_n, tmp, s);
    case 4: return launch_sweeps<4>(a, max_n, tmp, s);
    case 8: return launch_sweeps<8>(a, max_n, tmp, s);
    default: return PAQIF_EINVAL;
    }
}

int dispatch_factor(int q, const FactorArgs& a, hipStream_t s)
{
    switch (q) {
    case 2: return launch_factor<2>(a, s);
    case 4: return launch_factor<4>(a, s);
    case 8: return launch_factor<8>(a, s);
    default: return PAQIF_EINVAL;
    }
}

int dispatch_solve(int q, const SolveArgs& a, hipStream_t s)
{
    switch (q) {
    case 2: return launch_solve<2>(a, s);
    case 4: return launch_solve<4>(a, s);
    case 8: return launch_solve<8>(a, s);
    default: return PAQIF_EINVAL;
    }
}

}  // namespace pq

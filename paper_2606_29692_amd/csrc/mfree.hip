// Matrix-free generators: a pool of excitation-type generators applied
// straight from their Pauli terms (Eq. 3), with no CSR and no pair table.
//
// Derivation (host).  Every term of generator A flips the same bits x, so
// column c holds the single entry A[c ^ x, c] = f(c) with
//     f(c) = sum_t w_t (-1)^{|z_t & c|},   w_t = c_t i^{|x & z_t|}.
// Writing z_t = z_0 ^ D_t and taking a reduced echelon basis beta_1..beta_d
// of span{D_t}, D_t = XOR_i lambda_ti beta_i, so
//     f(c) = (-1)^{|z_0 & c|} g(y),  y_i = |beta_i & c| mod 2,
//     g(y) = sum_t w_t (-1)^{lambda_t . y}.
// g is evaluated on all 2^d patterns in term order from +0.0, the sum the
// CSR builder forms (up to the common sign, which rounding respects); when
// one pattern k survives the drop rule the support is the coset
// {c : |beta_i & c| = k_i}, closed under c -> c ^ x when every beta_i . x = 0.
//
// Enumeration (device).  A pair {r, c = r ^ x} is owned by the row with bit
// h (the top bit of x) clear.  Fixing h, the screen's tile bits (bits outside
// x, so a pair never leaves its tile) and the pivots of the reduced
// constraints leaves free bits; owner rows are enumerated by depositing a
// counter into them and setting every pivot from its parity constraint.  All
// of it is XOR-linear, so the screen splits each row index into a per-lane
// part (the lowest free bits, computed once per generator) and a per-iteration
// part (wave-uniform, on the scalar unit): the inner loop is two XORs and two
// LDS reads per pair.
#include "kernels.hpp"
#include "step_fin.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <vector>

struct vqe_mf_pool {
    int32_t n_qubits = 0;
    std::vector<vqe_mf_desc> desc;
};

namespace {

inline int parity64(uint64_t v) { return __builtin_popcountll(v) & 1; }
inline int top_bit(uint64_t v) { return 63 - __builtin_clzll(v); }

// ------------------------------------------------------------------ derivation
int describe(int32_t n_qubits, int64_t n_terms, const uint64_t *xm, const uint64_t *zm,
             const double *coeff, double tol, vqe_mf_desc *out)
{
    if (n_qubits < 1 || n_qubits > 30 || n_terms < 1 || !xm || !zm || !coeff || !out ||
        !(tol >= 0.0))
        return VQE_EINVAL;
    const uint64_t lim = ((uint64_t)1 << n_qubits) - 1;
    const uint64_t x = xm[0];
    for (int64_t t = 0; t < n_terms; t++) {
        if ((xm[t] | zm[t]) & ~lim)
            return VQE_EINVAL;
        if (xm[t] != x)
            return VQE_ENOTSUP;
    }
    if (x == 0)
        return VQE_ENOTSUP;
    // reduced echelon basis of span{z_t ^ z_0}; pivot = highest bit
    const uint64_t z0 = zm[0];
    uint64_t basis[64];
    int piv[64];
    int d = 0;
    for (int64_t t = 1; t < n_terms; t++) {
        uint64_t v = zm[t] ^ z0;
        for (int i = 0; i < d; i++)
            if ((v >> piv[i]) & 1)
                v ^= basis[i];
        if (!v)
            continue;
        if (d == VQE_MF_MAX_CON)
            return VQE_ENOTSUP;
        const int p = top_bit(v);
        for (int i = 0; i < d; i++)
            if ((basis[i] >> p) & 1)
                basis[i] ^= v;
        basis[d] = v;
        piv[d] = p;
        d++;
    }
    // pattern sums g(y), y in [0, 2^d): lambda_t,i = bit piv_i of D_t
    std::vector<double> gre((size_t)1 << d, 0.0), gim((size_t)1 << d, 0.0);
    for (int64_t t = 0; t < n_terms; t++) {
        const uint64_t D = zm[t] ^ z0;
        uint32_t lam = 0;
        for (int i = 0; i < d; i++)
            lam |= (uint32_t)((D >> piv[i]) & 1) << i;
        // w_t = c_t i^{|x & z_t|}
        double wr = coeff[2 * t], wi = coeff[2 * t + 1];
        switch (__builtin_popcountll(x & zm[t]) & 3) {
        case 1: { const double a = wr; wr = -wi; wi = a; break; }
        case 2: wr = -wr; wi = -wi; break;
        case 3: { const double a = wr; wr = wi; wi = -a; break; }
        default: break;
        }
        for (uint32_t y = 0; y < ((uint32_t)1 << d); y++) {
            const bool neg = __builtin_popcount(lam & y) & 1;
            gre[y] += neg ? -wr : wr;
            gim[y] += neg ? -wi : wi;
        }
    }
    int found = -1;
    for (uint32_t y = 0; y < ((uint32_t)1 << d); y++) {
        if (std::fabs(gre[y]) <= tol && std::fabs(gim[y]) <= tol)
            continue;
        if (found >= 0)
            return VQE_ENOTSUP;   // several cosets
        found = (int)y;
    }
    if (found < 0)
        return VQE_ENOTSUP;       // the operator vanishes
    for (int i = 0; i < d; i++)
        if (parity64(basis[i] & x))
            return VQE_ENOTSUP;   // support not closed under c -> c ^ x
    vqe_mf_desc o{};
    o.x = x;
    o.zsign = z0;
    o.v_re = gre[found];
    o.v_im = gim[found];
    o.n_qubits = n_qubits;
    o.n_con = d;
    for (int i = 0; i < d; i++)
        o.beta[i] = basis[i];
    o.kbits = (uint32_t)found;
    *out = o;
    return VQE_OK;
}

// ------------------------------------------------------------------ host records
uint32_t compress_bits(uint32_t a, const uint8_t *tbpos, int ntb)
{
    for (int i = 0; i < ntb; i++) {   // descending positions
        const int p = tbpos[i];
        a = ((a >> (p + 1)) << p) | (a & ((1u << p) - 1u));
    }
    return a;
}

// Record of generator d on the row set with tile bits tb (value bits vbits).
// Returns false when the constraints leave no owner row on the set.
void make_rec(const vqe_mf_desc &d, int j, int n, uint32_t tb, uint32_t vbits, MfRec *rec)
{
    MfRec r{};
    r.x = (uint32_t)d.x;
    r.zsign = (uint32_t)d.zsign;
    r.ex = (uint32_t)parity64(d.zsign & d.x);
    r.base = vbits;
    r.j = j;
    r.v_re = d.v_re;
    r.v_im = d.v_im;
    r.antiherm = mf_antihermitian(d) ? 1 : 0;
    const int h = top_bit(d.x);
    // tile bit positions, descending
    r.ntb = 0;
    for (int p = n - 1; p >= 0; p--)
        if ((tb >> p) & 1)
            r.tbpos[r.ntb++] = (uint8_t)p;
    r.cx = compress_bits(r.x, r.tbpos, r.ntb);
    // constraints with bit h (= 0 on owner rows) and the tile bits substituted
    uint32_t beta[VQE_MF_MAX_CON];
    uint32_t kb[VQE_MF_MAX_CON];
    int m = 0;
    bool empty = false;
    for (int i = 0; i < d.n_con; i++) {
        uint32_t b = (uint32_t)d.beta[i] & ~(1u << h);
        uint32_t k = (d.kbits >> i) & 1u;
        k ^= (uint32_t)__builtin_popcount(b & vbits) & 1u;
        b &= ~tb;
        for (int q = 0; q < m; q++)
            if ((b >> r.piv[q]) & 1) {
                b ^= beta[q];
                k ^= kb[q];
            }
        if (!b) {
            if (k)
                empty = true;
            continue;
        }
        const int p = 31 - __builtin_clz(b);
        for (int q = 0; q < m; q++)
            if ((beta[q] >> p) & 1) {
                beta[q] ^= b;
                kb[q] ^= k;
            }
        beta[m] = b;
        kb[m] = k;
        r.piv[m] = (uint8_t)p;
        m++;
    }
    r.ncon = m;
    uint32_t pivmask = 0;
    for (int q = 0; q < m; q++) {
        r.beta[q] = beta[q];
        r.kbits |= kb[q] << q;
        pivmask |= 1u << r.piv[q];
    }
    const uint32_t all = n == 32 ? 0xffffffffu : ((1u << n) - 1u);
    r.free_mask = all & ~(1u << h) & ~tb & ~pivmask;
    r.nfree = empty ? -1 : __builtin_popcount(r.free_mask);
    r.nlow = empty ? 0 : std::min(r.nfree, MF_LANE_BITS);
    uint32_t low = 0;
    int c = 0;
    for (int p = 0; p < n && c < r.nlow; p++)
        if ((r.free_mask >> p) & 1) {
            r.lowpos[c++] = (uint8_t)p;
            low |= 1u << p;
        }
    r.hi_mask = r.free_mask & ~low;
    *rec = r;
}

// Screen index tables of a tile record, appended to tabs: for lane l < 64 the
// part of element e = l of the lowest free bits, for u < 4 the part of
// element e = 64 u, then the part of every loop iteration (the higher free
// bits, the pivots with their parities k_i and the tile's fixed bits).  An
// entry is the part's compressed (tile) row index with |zsign & r| mod 2 in
// bit 31.  Deposit, pivots, compression and parity are all XOR-linear, so
// the entry of element l + 64 u in iteration t is lane[l] ^ unroll[u] ^ iter[t],
// the row the enumeration of vqe_mf_owner_rows derives from the same record.
void rec_tables(MfRec &rec, std::vector<uint32_t> &tabs)
{
    rec.tab_off = (uint32_t)tabs.size();
    auto pivots = [&](uint32_t a, bool withk) {
        uint32_t p = 0;
        for (int i = 0; i < rec.ncon; i++)
            p |= ((uint32_t)(__builtin_popcount(rec.beta[i] & a) ^ (withk ? (rec.kbits >> i) : 0u)) & 1u)
                 << rec.piv[i];
        return p;
    };
    auto entry = [&](uint32_t R) {
        return compress_bits(R, rec.tbpos, rec.ntb) |
               ((uint32_t)(__builtin_popcount(rec.zsign & R) & 1) << 31);
    };
    auto low = [&](uint32_t e) {
        uint32_t L = 0;
        for (int b = 0; b < rec.nlow; b++)
            L |= ((e >> b) & 1u) << rec.lowpos[b];
        return L ^ pivots(L, false);
    };
    const uint32_t nel = rec.nfree >= 0 ? 1u << rec.nlow : 0u;
    for (uint32_t l = 0; l < 64; l++)
        tabs.push_back(l < nel ? entry(low(l)) : 0u);
    for (uint32_t u = 0; u < 4; u++)
        tabs.push_back(64 * u < nel ? entry(low(64 * u)) : 0u);
    if (rec.nfree < 0)
        return;
    const int n_it = 1 << (rec.nfree - rec.nlow);
    uint32_t H = 0;
    for (int it = 0; it < n_it; it++) {
        tabs.push_back(entry(H ^ pivots(H, true) ^ rec.base));
        H = ((H | ~rec.hi_mask) + 1u) & rec.hi_mask;
    }
}

}  // namespace

// Anti-Hermitian on every pair: A[c, r] = -conj(A[r, c]), i.e.
// v (-1)^{|zsign & x|} = -conj(v).
bool mf_antihermitian(const vqe_mf_desc &d)
{
    const double s = parity64(d.zsign & d.x) ? -1.0 : 1.0;
    return s * d.v_re == -d.v_re && s * d.v_im == d.v_im;
}

int mf_host_plan(const vqe_mf_pool *pool, int64_t tile_rows, MfHostPlan *out, char *err,
                 size_t n_err)
{
    const int n = pool->n_qubits;
    const int64_t dim = (int64_t)1 << n;
    const int M = (int)pool->desc.size();
    int kt = 0;
    while (((int64_t)tile_rows << kt) < dim)
        kt++;
    if (kt > MF_MAX_TB) {
        std::snprintf(err, n_err, "matrix-free screen: too many row tiles");
        return VQE_ENOTSUP;
    }
    const int ntile = 1 << kt;
    out->M = M;
    out->ntile = ntile;
    out->tile_rows = (int32_t)std::min<int64_t>(tile_rows, dim);
    out->tile_recs.assign((size_t)M * ntile, MfRec{});
    out->full_recs.assign((size_t)M, MfRec{});
    out->tabs.clear();
    out->lists.clear();
    out->list_info.clear();
    // Tile bits: kt bits outside a generator's flip mask (never bit 0: the
    // staging reads row pairs {2i, 2i + 1}).  Each generator's own choice is
    // its kt highest such bits; every distinct set is staged once per tile,
    // so when a greedy cover -- repeatedly the kt-subset of bits 1 .. n-1
    // that the most of the remaining generators can use (ties: the higher
    // bits) -- needs fewer sets, the generators take the cover's sets.
    std::vector<uint32_t> tbs(M, 0u), own(M, 0u);
    for (int j = 0; j < M; j++) {
        int got = 0;
        for (int p = n - 1; p >= 1 && got < kt; p--)
            if (!((pool->desc[j].x >> p) & 1)) {
                own[j] |= 1u << p;
                got++;
            }
        if (got < kt) {
            std::snprintf(err, n_err, "matrix-free screen: generator %d leaves no tile bit", j);
            return VQE_ENOTSUP;
        }
    }
    auto distinct = [](std::vector<uint32_t> v) {
        std::sort(v.begin(), v.end());
        return (size_t)(std::unique(v.begin(), v.end()) - v.begin());
    };
    if (kt > 0) {
        std::vector<uint32_t> cand;
        for (int64_t m = ((int64_t)1 << (n - 1)) - 1; m >= 0; m--)
            if (__builtin_popcountll((unsigned long long)m) == kt)
                cand.push_back((uint32_t)m << 1);
        // the generators as bit sets: those still without a set, and per
        // bit those whose flip mask holds it; a candidate's count is then the
        // remaining generators outside the union of its bits' sets
        const int W = (M + 63) / 64;
        std::vector<uint64_t> left((size_t)W, 0ull), hold((size_t)n * W, 0ull), blocked((size_t)W);
        for (int j = 0; j < M; j++) {
            left[j >> 6] |= 1ull << (j & 63);
            for (int p = 0; p < n; p++)
                if ((pool->desc[j].x >> p) & 1)
                    hold[(size_t)p * W + (j >> 6)] |= 1ull << (j & 63);
        }
        int64_t n_left = M;
        while (n_left > 0) {
            size_t best = 0;
            int64_t best_cnt = 0;
            for (size_t c = 0; c < cand.size(); c++) {
                std::fill(blocked.begin(), blocked.end(), 0ull);
                for (uint32_t m = cand[c]; m; m &= m - 1) {
                    const uint64_t *h = hold.data() + (size_t)__builtin_ctz(m) * W;
                    for (int w = 0; w < W; w++)
                        blocked[w] |= h[w];
                }
                int64_t cnt = 0;
                for (int w = 0; w < W; w++)
                    cnt += __builtin_popcountll(left[w] & ~blocked[w]);
                if (cnt > best_cnt) {
                    best_cnt = cnt;
                    best = c;
                }
            }
            if (best_cnt == 0) {
                std::snprintf(err, n_err, "matrix-free screen: a generator leaves no tile bit");
                return VQE_ENOTSUP;
            }
            for (int j = 0; j < M; j++)
                if (((left[j >> 6] >> (j & 63)) & 1) && (pool->desc[j].x & cand[best]) == 0) {
                    tbs[j] = cand[best];
                    left[j >> 6] &= ~(1ull << (j & 63));
                }
            n_left -= best_cnt;
        }
    }
    if (distinct(tbs) >= distinct(own))
        tbs = own;
    for (int j = 0; j < M; j++) {
        const vqe_mf_desc &d = pool->desc[j];
        const uint32_t tb = tbs[j];
        int64_t owners = 0;
        for (int v = 0; v < ntile; v++) {
            uint32_t vbits = 0;
            int b = 0;
            for (int p = 0; p < n; p++)
                if ((tb >> p) & 1) {
                    if ((v >> b) & 1)
                        vbits |= 1u << p;
                    b++;
                }
            MfRec &rec = out->tile_recs[(size_t)j * ntile + v];
            make_rec(d, j, n, tb, vbits, &rec);
            rec_tables(rec, out->tabs);
            if (rec.nfree >= 0)
                owners += (int64_t)1 << rec.nfree;
        }
        make_rec(d, j, n, 0u, 0u, &out->full_recs[j]);
        const int64_t expect = (int64_t)1 << (n - 1 - d.n_con);
        if (owners != expect || out->full_recs[j].nfree < 0 ||
            ((int64_t)1 << out->full_recs[j].nfree) != expect) {
            std::snprintf(err, n_err, "matrix-free records of generator %d are inconsistent", j);
            return VQE_ENOTSUP;
        }
    }
    // lists per (tile-bit group, tile): generators by descending cost
    std::vector<uint32_t> groups(tbs);
    std::sort(groups.begin(), groups.end());
    groups.erase(std::unique(groups.begin(), groups.end()), groups.end());
    for (uint32_t tb : groups)
        for (int v = 0; v < ntile; v++) {
            std::vector<int32_t> js;
            for (int j = 0; j < M; j++)
                if (tbs[j] == tb)
                    js.push_back(j);
            auto cost = [&](int32_t j) {
                const MfRec &r = out->tile_recs[(size_t)j * ntile + v];
                return r.nfree < 0 ? 0.0 : std::ldexp(1.0, r.nfree);
            };
            std::stable_sort(js.begin(), js.end(),
                             [&](int32_t a, int32_t b) { return cost(a) > cost(b); });
            double work = 0.0;
            for (int32_t j : js)
                work += cost(j) + 64.0;   // a generator costs at least one wave pass
            out->list_info.push_back({(int32_t)out->lists.size(), (int32_t)js.size(), v, work});
            out->lists.insert(out->lists.end(), js.begin(), js.end());
        }
    return VQE_OK;
}

// ------------------------------------------------------------------ kernels
namespace {

// A record's enumeration fields held in registers: every loop below runs to
// the compile-time maximum with a predicate, so no array is indexed
// dynamically (which would move it to scratch memory).
struct MfRegs {
    uint32_t beta[VQE_MF_MAX_CON];
    uint32_t piv[VQE_MF_MAX_CON];
    uint32_t tbpos[MF_MAX_TB];
    uint32_t lowpos[MF_LANE_BITS];
    uint32_t kbits;
    int ncon, ntb, nlow;
};

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ MfRegs load_regs(const MfRec &r)
{
    MfRegs m;
    m.ncon = (int)uni((uint32_t)r.ncon);
    m.ntb = (int)uni((uint32_t)r.ntb);
    m.nlow = (int)uni((uint32_t)r.nlow);
    m.kbits = uni(r.kbits);
#pragma unroll
    for (int i = 0; i < VQE_MF_MAX_CON; i++) {
        m.beta[i] = uni(r.beta[i]);
        m.piv[i] = uni(r.piv[i]);
    }
#pragma unroll
    for (int i = 0; i < MF_MAX_TB; i++)
        m.tbpos[i] = uni(r.tbpos[i]);
#pragma unroll
    for (int i = 0; i < MF_LANE_BITS; i++)
        m.lowpos[i] = uni(r.lowpos[i]);
    return m;
}

// remove the tile bits (descending positions) from a row index
__device__ __forceinline__ uint32_t dev_compress(uint32_t a, const MfRegs &m)
{
#pragma unroll
    for (int i = 0; i < MF_MAX_TB; i++)
        if (i < m.ntb) {
            const uint32_t p = m.tbpos[i];
            a = ((a >> (p + 1)) << p) | (a & ((1u << p) - 1u));
        }
    return a;
}

// pivot bits of a partial row index a (free bits only): sum_i (k_i ^ |beta_i & a|) << piv_i,
// with the k_i included when withk
__device__ __forceinline__ uint32_t dev_pivots(uint32_t a, const MfRegs &m, bool withk)
{
    uint32_t p = 0;
#pragma unroll
    for (int i = 0; i < VQE_MF_MAX_CON; i++)
        if (i < m.ncon) {
            const uint32_t bit =
                ((uint32_t)__popc(m.beta[i] & a) ^ (withk ? (m.kbits >> i) : 0u)) & 1u;
            p |= bit << m.piv[i];
        }
    return p;
}

// Tile element: psi and sigma of one row.
template <int DT> struct TileElem;
template <> struct TileElem<VQE_C64> {
    using T = float4;   // psi.re, psi.im, sigma.re, sigma.im
    static __device__ __forceinline__ T load(const void *psi, const void *sig, int64_t r)
    {
        const float2 a = ldg(reinterpret_cast<const float2 *>(psi), r);
        const float2 b = ldg(reinterpret_cast<const float2 *>(sig), r);
        return make_float4(a.x, a.y, b.x, b.y);
    }
    static __device__ __forceinline__ void get(const T *t, uint32_t i, double2 &p, double2 &s)
    {
        const float4 e = t[i];
        p = make_double2(e.x, e.y);
        s = make_double2(e.z, e.w);
    }
};
template <> struct TileElem<VQE_C128> {
    struct T { double2 p, s; };
    static __device__ __forceinline__ T load(const void *psi, const void *sig, int64_t r)
    {
        T e;
        e.p = ldg(reinterpret_cast<const double2 *>(psi), r);
        e.s = ldg(reinterpret_cast<const double2 *>(sig), r);
        return e;
    }
    static __device__ __forceinline__ void get(const T *t, uint32_t i, double2 &p, double2 &s)
    {
        p = t[i].p;
        s = t[i].s;
    }
};

// Sum over the owner rows of one generator on the staged tile of
// (-1)^{|zsign & r|} [(-1)^ex conj(s_r) psi_c + conj(s_c) psi_r],  s = sigma (+ shift psi).
// Lane l takes the elements e = l + 64 u (u < MF_LANE_UNROLL) of the lowest
// free bits; the wave-uniform parts of the row index for up to 64 loop
// iterations are computed once, one iteration per lane, and read back with
// readlane, so the inner loop issues no scalar arithmetic.
#define MF_LANE_UNROLL 4
// With RE_ONLY (generators whose value v is real) only the real part of the
// sum is formed: the generator's contribution v_re Re(S) - v_im Im(S) needs
// no more.
template <int DT, bool SHIFT, bool RE_ONLY>
__device__ __forceinline__ double2 mf_tile_sum(const typename TileElem<DT>::T *tile, const MfRec &rec,
                                               const uint32_t *tabs, double shift, int lane)
{
    // the lane, unroll and iteration parts of the row index come from the
    // record's tables (the host derives them once per record)
    const uint32_t cx = uni(rec.cx);
    const int nlow = (int)uni((uint32_t)rec.nlow);
    const uint32_t *__restrict__ t = tabs + uni(rec.tab_off);
    double sre = 0.0, sim = 0.0;
    constexpr int U = MF_LANE_UNROLL;
    uint32_t cl[U], sl[U];
    bool on[U];
    const uint32_t lv = gmem(t)[lane];
#pragma unroll
    for (int u = 0; u < U; u++) {
        const uint32_t ev = lv ^ uni(gmem(t)[64 + u]);
        cl[u] = ev & 0x7fffffffu;
        sl[u] = ev >> 31;
        on[u] = (uint32_t)lane + 64u * u < (1u << nlow);
    }
    const double e1 = uni(rec.ex) ? -1.0 : 1.0;
    const int n_it = 1 << ((int)uni((uint32_t)rec.nfree) - nlow);
    for (int c0 = 0; c0 < n_it; c0 += 64) {
        // iteration c0 + lane's part, read back per iteration with readlane
        const uint32_t hv = c0 + lane < n_it ? gmem(t)[MF_TAB_ITER + c0 + lane] : 0u;
        const int nin = n_it - c0 < 64 ? n_it - c0 : 64;
        for (int i = 0; i < nin; i++) {
            const uint32_t hi = __builtin_amdgcn_readlane(hv, i);
            const uint32_t ch = hi & 0x7fffffffu, sh = hi >> 31;
            double2 pr[U], sr[U], pc[U], sc[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                const uint32_t ir = on[u] ? (cl[u] ^ ch) : 0u, ic = on[u] ? (ir ^ cx) : 0u;
                TileElem<DT>::get(tile, ir, pr[u], sr[u]);
                TileElem<DT>::get(tile, ic, pc[u], sc[u]);
            }
#pragma unroll
            for (int u = 0; u < U; u++) {
                if (SHIFT) {
                    sr[u].x += shift * pr[u].x;
                    sr[u].y += shift * pr[u].y;
                    sc[u].x += shift * pc[u].x;
                    sc[u].y += shift * pc[u].y;
                }
                // conj(s_r) psi_c and conj(s_c) psi_r
                const double u1r = sr[u].x * pc[u].x + sr[u].y * pc[u].y;
                const double u2r = sc[u].x * pr[u].x + sc[u].y * pr[u].y;
                const double tr = e1 * u1r + u2r;
                const bool neg = (sl[u] ^ sh) & 1u;
                const double w = on[u] ? (neg ? -1.0 : 1.0) : 0.0;
                sre += w * tr;
                if (!RE_ONLY) {
                    const double u1i = sr[u].x * pc[u].y - sr[u].y * pc[u].x;
                    const double u2i = sc[u].x * pr[u].y - sc[u].y * pr[u].x;
                    const double ti = e1 * u1i + u2i;
                    sim += w * ti;
                }
            }
        }
    }
    return make_double2(sre, sim);
}

// The same sum for a real state: the tile holds (psi_r, sigma_r) as reals, so
// S = sum of (-1)^{|zsign & r|} [(-1)^ex s_r psi_c + s_c psi_r] (generators of
// real value, unshifted or anti-Hermitian).
template <typename R2>
__device__ __forceinline__ double mf_tile_sum_real(const R2 *tile, const MfRec &rec,
                                                   const uint32_t *tabs, int lane)
{
    const uint32_t cx = uni(rec.cx);
    const int nlow = (int)uni((uint32_t)rec.nlow);
    const uint32_t *__restrict__ t = tabs + uni(rec.tab_off);
    double sre = 0.0;
    constexpr int U = MF_LANE_UNROLL;
    uint32_t cl[U], sl[U];
    bool on[U];
    const uint32_t lv = gmem(t)[lane];
#pragma unroll
    for (int u = 0; u < U; u++) {
        const uint32_t ev = lv ^ uni(gmem(t)[64 + u]);
        cl[u] = ev & 0x7fffffffu;
        sl[u] = ev >> 31;
        on[u] = (uint32_t)lane + 64u * u < (1u << nlow);
    }
    const double e1 = uni(rec.ex) ? -1.0 : 1.0;
    const int n_it = 1 << ((int)uni((uint32_t)rec.nfree) - nlow);
    // two loop iterations per pass (their gathers in flight together), each
    // with its own accumulator
    double sre1 = 0.0;
    auto iter = [&](uint32_t hi, R2 er[U], R2 ec[U]) {
        const uint32_t ch = hi & 0x7fffffffu;
#pragma unroll
        for (int u = 0; u < U; u++) {
            const uint32_t ir = on[u] ? (cl[u] ^ ch) : 0u, ic = on[u] ? (ir ^ cx) : 0u;
            er[u] = tile[ir];
            ec[u] = tile[ic];
        }
    };
    auto acc = [&](uint32_t hi, const R2 er[U], const R2 ec[U], double &a) {
        const uint32_t sh = hi >> 31;
#pragma unroll
        for (int u = 0; u < U; u++) {
            const double tr = e1 * ((double)er[u].y * (double)ec[u].x) +
                              (double)ec[u].y * (double)er[u].x;
            const bool neg = (sl[u] ^ sh) & 1u;
            a += (on[u] ? (neg ? -1.0 : 1.0) : 0.0) * tr;
        }
    };
    for (int c0 = 0; c0 < n_it; c0 += 64) {
        const uint32_t hv = c0 + lane < n_it ? gmem(t)[MF_TAB_ITER + c0 + lane] : 0u;
        const int nin = n_it - c0 < 64 ? n_it - c0 : 64;
        int i = 0;
        for (; i + 1 < nin; i += 2) {
            const uint32_t h0 = __builtin_amdgcn_readlane(hv, i);
            const uint32_t h1 = __builtin_amdgcn_readlane(hv, i + 1);
            R2 er0[U], ec0[U], er1[U], ec1[U];
            iter(h0, er0, ec0);
            iter(h1, er1, ec1);
            acc(h0, er0, ec0, sre);
            acc(h1, er1, ec1, sre1);
        }
        if (i < nin) {
            const uint32_t h0 = __builtin_amdgcn_readlane(hv, i);
            R2 er0[U], ec0[U];
            iter(h0, er0, ec0);
            acc(h0, er0, ec0, sre);
        }
    }
    return sre + sre1;
}

// One list of the tiled screen (generators sharing their tile bits, on tile
// v of those bits) for one workgroup: stage the tile's psi and sigma in LDS,
// then one wave per generator of the workgroup's share (range, range +
// n_ranges, ...) writes that generator's tile partial.
template <int DT>
__device__ __forceinline__ void screen_list(const ScreenState &st, int off, int n, int range,
                                            int n_ranges, int v, unsigned char *smem)
{
    const MfTable &tb = *st.mf;
    const int32_t *list = tb.lists + off;
    using T = typename TileElem<DT>::T;
    T *tile = reinterpret_cast<T *>(smem);
    const MfRec &r0 = tb.tile_recs[(int64_t)list[0] * tb.ntile + v];
    const int64_t rows = tb.tile_rows;
    const int ntb = (int)uni((uint32_t)r0.ntb);
    const uint32_t base = uni(r0.base);
    uint32_t tbp[MF_MAX_TB];
#pragma unroll
    for (int q = 0; q < MF_MAX_TB; q++)
        tbp[q] = uni(r0.tbpos[q]);
    // staging: each thread issues the loads of SU rows before its LDS writes
    constexpr int SU = 8;
    for (int64_t i0 = threadIdx.x; i0 < rows; i0 += 1024 * SU) {
        typename TileElem<DT>::T e[SU];
#pragma unroll
        for (int u = 0; u < SU; u++) {
            const int64_t i = i0 + 1024 * u;
            if (i < rows) {
                // insert the tile bits (ascending positions) into i
                uint32_t r = (uint32_t)i;
#pragma unroll
                for (int q = MF_MAX_TB - 1; q >= 0; q--)
                    if (q < ntb) {
                        const uint32_t p = tbp[q];
                        r = ((r >> p) << (p + 1)) | (r & ((1u << p) - 1u)) | (base & (1u << p));
                    }
                e[u] = TileElem<DT>::load(st.psi, st.sigma, (int64_t)r);
            }
        }
#pragma unroll
        for (int u = 0; u < SU; u++)
            if (i0 + 1024 * u < rows)
                tile[i0 + 1024 * u] = e[u];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int idx = wid;; idx += 16) {
        const int e = range + idx * n_ranges;
        if (e >= n)
            break;
        const int j = __builtin_amdgcn_readfirstlane(gmem(list)[e]);
        const MfRec &rec = tb.tile_recs[(int64_t)j * tb.ntile + v];
        double part = 0.0;
        if (rec.nfree >= 0) {
            const bool shifted = st.shift != 0.0 && !rec.antiherm;
            if (rec.v_im == 0.0 && !shifted) {
                // a real generator value: only Re(S) enters (v_re Re(S) - 0 Im(S))
                const double2 S = mf_tile_sum<DT, false, true>(tile, rec, tb.tabs, 0.0, lane);
                part = rec.v_re * group_sum<64>(S.x) - rec.v_im * 0.0;
            } else {
                const double2 S = shifted ? mf_tile_sum<DT, true, false>(tile, rec, tb.tabs, st.shift, lane)
                                          : mf_tile_sum<DT, false, false>(tile, rec, tb.tabs, 0.0, lane);
                const double re = group_sum<64>(S.x), im = group_sum<64>(S.y);
                part = rec.v_re * re - rec.v_im * im;
            }
        }
        if (lane == 0)
            gmem(st.partials)[(int64_t)j * tb.ntile + v] = part;
    }
}


// One workgroup per (state, tile-bit group, tile, generator range).
template <int DT>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(4, 4)))
k_screen_mf(const ScreenState *__restrict__ states, const int4 *__restrict__ tasks)
{
    const int4 task = tasks[blockIdx.x];
    if (task.x < 0)
        return;
    const ScreenState st = states[task.x];
    if (VQE_SKIP(st))
        return;
    extern __shared__ unsigned char smem[];
    screen_list<DT>(st, task.y, task.z, task.w & 0xff, (task.w >> 8) & 0xff, task.w >> 16, smem);
}

// Real-state screen: one workgroup per (state, generator range) stages the
// whole state as (psi.re, sigma.re) pairs; when every imaginary part is zero
// one wave per generator forms its gradient in real arithmetic and writes it
// as the tiled screen's tile-0 partial (the other tiles' partials zero).  For
// a state with a nonzero imaginary part the state's workgroups run the tiled
// screen instead, every list of it, each taking its share of each list.
template <int DT>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(4, 4)))
k_screen_mf_real(const ScreenState *__restrict__ states, const int4 *__restrict__ tasks)
{
    const int4 task = tasks[blockIdx.x];
    if (task.x < 0)
        return;
    const ScreenState st = states[task.x];
    if (VQE_SKIP(st))
        return;
    using T = typename Elem<DT>::T;
    using R2 = typename std::conditional<DT == VQE_C64, float2, double2>::type;
    const MfTable tb = *st.mf1;
    const int32_t *list = tb.lists + task.y;
    const int n = task.z;
    const int range = task.w & 0xff, n_ranges = (task.w >> 8) & 0xff;
    extern __shared__ unsigned char smem[];
    R2 *tile = reinterpret_cast<R2 *>(smem);
    const T *psi = reinterpret_cast<const T *>(st.psi);
    const T *sig = reinterpret_cast<const T *>(st.sigma);
    const int64_t rows = st.dim;
    __shared__ int s_next;
    if (threadIdx.x == 0)
        s_next = 0;
    int cplx = 0;
    constexpr int SU = 8;
    if (DT == VQE_C64 && (rows & 1) == 0 &&
        ((reinterpret_cast<uintptr_t>(psi) | reinterpret_cast<uintptr_t>(sig)) & 15) == 0) {
        // two rows per 16-byte load
        const vqe_v4f *psi4 = reinterpret_cast<const vqe_v4f *>(psi);
        const vqe_v4f *sig4 = reinterpret_cast<const vqe_v4f *>(sig);
        const int64_t pairs = rows / 2;
        for (int64_t i0 = threadIdx.x; i0 < pairs; i0 += 1024 * SU) {
            vqe_v4f a[SU], b[SU];
#pragma unroll
            for (int u = 0; u < SU; u++) {
                const int64_t i = i0 + 1024 * u;
                if (i < pairs) {
                    a[u] = gmem(psi4)[i];
                    b[u] = gmem(sig4)[i];
                }
            }
#pragma unroll
            for (int u = 0; u < SU; u++) {
                const int64_t i = i0 + 1024 * u;
                if (i < pairs) {
                    R2 e0, e1;
                    e0.x = a[u].x;
                    e0.y = b[u].x;
                    e1.x = a[u].z;
                    e1.y = b[u].z;
                    tile[2 * i] = e0;
                    tile[2 * i + 1] = e1;
                    cplx |= (a[u].y != 0) | (a[u].w != 0) | (b[u].y != 0) | (b[u].w != 0);
                }
            }
        }
    } else {
        for (int64_t i0 = threadIdx.x; i0 < rows; i0 += 1024 * SU) {
            T a[SU], b[SU];
#pragma unroll
            for (int u = 0; u < SU; u++) {
                const int64_t i = i0 + 1024 * u;
                if (i < rows) {
                    a[u] = ldg(psi, i);
                    b[u] = ldg(sig, i);
                }
            }
#pragma unroll
            for (int u = 0; u < SU; u++) {
                const int64_t i = i0 + 1024 * u;
                if (i < rows) {
                    R2 e;
                    e.x = a[u].x;
                    e.y = b[u].x;
                    tile[i] = e;
                    cplx |= (a[u].y != 0) | (b[u].y != 0);
                }
            }
        }
    }
    cplx = __syncthreads_or(cplx);
    if (cplx) {
        const MfTable &tc = *st.mf;
        for (int i = 0; i < tc.nlists; i++) {
            const int4 L = tc.linfo[i];
            __syncthreads();      // every wave is done with the previous tile
            screen_list<DT>(st, L.x, L.y, range, n_ranges, L.z, smem);
        }
        return;
    }
    const int ntc = st.mf_ntile;
    const int lane = threadIdx.x & 63;
    // waves take the workgroup's generators from a counter, in the list's
    // descending-cost order, so that they finish together
    for (;;) {
        int idx = 0;
        if (lane == 0)
            idx = atomicAdd(&s_next, 1);
        idx = __builtin_amdgcn_readfirstlane(idx);
        const int e = range + idx * n_ranges;
        if (e >= n)
            break;
        const int j = __builtin_amdgcn_readfirstlane(gmem(list)[e]);
        const MfRec &rec = tb.tile_recs[j];
        double part = 0.0;
        if (rec.nfree >= 0)
            part = rec.v_re * group_sum<64>(mf_tile_sum_real<R2>(tile, rec, tb.tabs, lane));
        if (lane < ntc)
            gmem(st.partials)[(int64_t)j * ntc + lane] = lane == 0 ? part : 0.0;
    }
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// The update of one owner pair e of the record (Eq. 6-8 on the 2x2 block);
// returns the change of |psi_r|^2 + |psi_c|^2 between the stored values.
template <int DT>
__device__ __forceinline__ double taylor_pair(const TaylorState *stp, const MfRec &rec, uint32_t e,
                                              double theta)
{
    // deposit e into the free bits, then the pivots
    uint32_t a = 0, fm = rec.free_mask, ee = e;
    while (fm) {
        const uint32_t low = fm & (0u - fm);
        if (ee & 1u)
            a |= low;
        ee >>= 1;
        fm ^= low;
    }
    const uint32_t r = a ^ dev_pivots(a, load_regs(rec), true);
    const uint32_t c = r ^ rec.x;
    const double2 v = make_double2(rec.v_re, rec.v_im);
    // A[r, c] = v (-1)^{|zsign & c|}, A[c, r] = v (-1)^{|zsign & r|}
    const double sa = (__popc(rec.zsign & c) & 1) ? -1.0 : 1.0;
    const double sb = (__popc(rec.zsign & r) & 1) ? -1.0 : 1.0;
    const double2 A = make_double2(sa * v.x, sa * v.y), Bv = make_double2(sb * v.x, sb * v.y);
    double cf[6];
    cf[0] = 1.0;
#pragma unroll
    for (int q = 1; q <= 5; q++)
        cf[q] = cf[q - 1] * theta / (double)q;
    void *psi = stp->psi;
    double2 vr = Elem<DT>::ld(psi, r), vc = Elem<DT>::ld(psi, c);
    const double before = (vr.x * vr.x + vr.y * vr.y) + (vc.x * vc.x + vc.y * vc.y);
    double2 ar = vr, ac = vc;
#pragma unroll
    for (int q = 1; q <= 5; q++) {
        const double2 nr = cmul(A, vc);
        const double2 nc = cmul(Bv, vr);
        vr = nr;
        vc = nc;
        ar.x += cf[q] * vr.x;
        ar.y += cf[q] * vr.y;
        ac.x += cf[q] * vc.x;
        ac.y += cf[q] * vc.y;
    }
    Elem<DT>::st(psi, r, ar);
    Elem<DT>::st(psi, c, ac);
    if (DT == VQE_C64) {
        // the stored values: FP32 storage rounds
        ar = make_double2((double)(float)ar.x, (double)(float)ar.y);
        ac = make_double2((double)(float)ac.x, (double)(float)ac.y);
    }
    return (ar.x * ar.x + ar.y * ar.y) + (ac.x * ac.x + ac.y * ac.y) - before;
}

// Fused Taylor-5 update on the selected generator's pairs, one thread per
// owner row, enumerated from the generator's whole-state record.  With
// tay_partials set, each block also writes the change of |psi|^2 over its
// pairs (from the stored values), so that the renormalisation can take the
// norm as the pre-update norm plus these changes.  With FIN every workgroup
// first forms the step's finalisation for its state (energy, gradients,
// selection; stored by the state's first workgroup) and updates along the
// generator it selects.  With theta_row set the angle of state s is
// theta_row[s] (one row of a caller's angle schedule), which the state's
// first workgroup also stores as the state's angle.
template <int DT, bool FIN>
__global__ void __launch_bounds__(TAYLOR_ROWS_PER_BLOCK)
k_taylor_mf(const TaylorState *__restrict__ states, const int2 *__restrict__ tasks,
            const SpmvState *__restrict__ spmv, const ScreenState *__restrict__ screen,
            const PairTable *__restrict__ tables, const SelectState *__restrict__ sel,
            int do_select, double rel_tie, const double *__restrict__ theta_row)
{
    const int2 task = tasks[blockIdx.x];
    if (task.x < 0)
        return;
    const TaylorState *stp = states + task.x;
    if (VQE_SKIP(*stp))
        return;
    int32_t k;
    if (FIN) {
        const SpmvState hs = spmv[task.x];
        k = step_fin_block(hs, screen, tables, sel[task.x], task.x, true, do_select != 0,
                           rel_tie, task.y == 0);
        if (!do_select)
            k = *stp->k;
    } else {
        k = *stp->k;
    }
    double theta;
    if (theta_row) {
        theta = theta_row[task.x];
        if (task.y == 0 && threadIdx.x == 0)
            *const_cast<double *>(stp->theta) = theta;
    } else {
        theta = *stp->theta;
    }
    double dn = 0.0;
    if (k >= 0 && k < stp->M) {
        const MfRec &rec = stp->mf->full_recs[k];
        const int64_t e = (int64_t)task.y * TAYLOR_ROWS_PER_BLOCK + threadIdx.x;
        if (rec.nfree >= 0 && e < ((int64_t)1 << rec.nfree))
            dn = taylor_pair<DT>(stp, rec, (uint32_t)e, theta);
    }
    if (!stp->tay_partials)
        return;
    __shared__ double red[TAYLOR_ROWS_PER_BLOCK / 64];
    dn = wave_sum(dn);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = dn;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < TAYLOR_ROWS_PER_BLOCK / 64; w++)
            t += red[w];
        gmem(stp->tay_partials)[task.y] = t;
    }
}

// Renormalisation after the fused update: |psi'|^2 = |psi|^2 (from this
// step's H product) plus the update blocks' changes, summed in block order.
template <int DT>
__global__ void __launch_bounds__(1024)
k_norm_scale_mf(const TaylorState *__restrict__ states, const int2 *__restrict__ tasks)
{
    const int2 t = tasks[blockIdx.x];
    if (t.x < 0)
        return;
    const TaylorState *stp = states + t.x;
    if (VQE_SKIP(*stp))
        return;
    const int64_t r0 = (int64_t)t.y * NORM_ROWS_PER_BLOCK;
    const int64_t r1 = r0 + NORM_ROWS_PER_BLOCK < stp->dim ? r0 + NORM_ROWS_PER_BLOCK : stp->dim;
    // a block's rows in two passes of 1,024 threads, their loads issued
    // before the norm's (the rows do not depend on it)
    constexpr int NT = 1024, U = NORM_ROWS_PER_BLOCK / NT;
    const bool renorm = stp->renorm != 0;
    double2 p[U];
    if (renorm) {
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t r = r0 + threadIdx.x + (int64_t)u * NT;
            if (r < r1)
                p[u] = Elem<DT>::ld(stp->psi, r);
        }
    }
    __shared__ double s_n2;
    if (threadIdx.x < 64) {
        double d = 0.0;
        for (int b = threadIdx.x; b < stp->ntay; b += 64)
            d += gmem(stp->tay_partials)[b];
        d = wave_sum(d);
        if (threadIdx.x == 0)
            s_n2 = *stp->n2_prev + d;
    }
    __syncthreads();
    const double n2 = s_n2;
    if (t.y == 0 && threadIdx.x == 0 && stp->norm2_out)
        stp->norm2_out[0] = n2;
    if (!renorm)
        return;
    const double inv = 1.0 / sqrt(n2);
#pragma unroll
    for (int u = 0; u < U; u++) {
        const int64_t r = r0 + threadIdx.x + (int64_t)u * NT;
        if (r < r1)
            Elem<DT>::st(stp->psi, r, make_double2(p[u].x * inv, p[u].y * inv));
    }
}

}  // namespace

void launch_screen_mf(int dtype, const ScreenState *states, const int4 *tasks, unsigned grid,
                      size_t lds, hipStream_t s)
{
    if (dtype == VQE_C128) {
        (void)hipFuncSetAttribute((const void *)k_screen_mf<VQE_C128>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        k_screen_mf<VQE_C128><<<grid, 1024, lds, s>>>(states, tasks);
    } else {
        (void)hipFuncSetAttribute((const void *)k_screen_mf<VQE_C64>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        k_screen_mf<VQE_C64><<<grid, 1024, lds, s>>>(states, tasks);
    }
}

void launch_screen_mf_real(int dtype, const ScreenState *states, const int4 *tasks, unsigned grid,
                           size_t lds, hipStream_t s)
{
    if (dtype == VQE_C128) {
        (void)hipFuncSetAttribute((const void *)k_screen_mf_real<VQE_C128>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        k_screen_mf_real<VQE_C128><<<grid, 1024, lds, s>>>(states, tasks);
    } else {
        (void)hipFuncSetAttribute((const void *)k_screen_mf_real<VQE_C64>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        k_screen_mf_real<VQE_C64><<<grid, 1024, lds, s>>>(states, tasks);
    }
}

void launch_norm_mf(int dtype, const TaylorState *states, const int2 *tasks, unsigned grid,
                    hipStream_t s)
{
    if (dtype == VQE_C128)
        k_norm_scale_mf<VQE_C128><<<grid, 1024, 0, s>>>(states, tasks);
    else
        k_norm_scale_mf<VQE_C64><<<grid, 1024, 0, s>>>(states, tasks);
}

void launch_taylor_mf(int dtype, const TaylorState *states, const int2 *tasks, unsigned grid,
                      const double *theta_row, hipStream_t s)
{
    if (dtype == VQE_C128)
        k_taylor_mf<VQE_C128, false><<<grid, TAYLOR_ROWS_PER_BLOCK, 0, s>>>(
            states, tasks, nullptr, nullptr, nullptr, nullptr, 0, 0.0, theta_row);
    else
        k_taylor_mf<VQE_C64, false><<<grid, TAYLOR_ROWS_PER_BLOCK, 0, s>>>(
            states, tasks, nullptr, nullptr, nullptr, nullptr, 0, 0.0, theta_row);
}

void launch_taylor_mf_fin(int dtype, const TaylorState *states, const int2 *tasks, unsigned grid,
                          const SpmvState *spmv, const ScreenState *screen,
                          const PairTable *tables, const SelectState *sel, bool select,
                          double rel_tie, const double *theta_row, hipStream_t s)
{
    if (dtype == VQE_C128)
        k_taylor_mf<VQE_C128, true><<<grid, TAYLOR_ROWS_PER_BLOCK, 0, s>>>(
            states, tasks, spmv, screen, tables, sel, select ? 1 : 0, rel_tie, theta_row);
    else
        k_taylor_mf<VQE_C64, true><<<grid, TAYLOR_ROWS_PER_BLOCK, 0, s>>>(
            states, tasks, spmv, screen, tables, sel, select ? 1 : 0, rel_tie, theta_row);
}

// ------------------------------------------------------------------ C ABI
extern "C" int vqe_mf_describe(int32_t n_qubits, int64_t n_terms, const uint64_t *xmask,
                               const uint64_t *zmask, const double *coeff, double drop_tol,
                               vqe_mf_desc *out)
{
    return describe(n_qubits, n_terms, xmask, zmask, coeff, drop_tol, out);
}

extern "C" int vqe_mf_pool_create(int32_t n_qubits, int32_t M, const int64_t *term_offset,
                                  const uint64_t *xmask, const uint64_t *zmask,
                                  const double *coeff, const double *drop_tol, vqe_mf_pool **out)
{
    if (!out)
        return VQE_EINVAL;
    *out = nullptr;
    if (M < 1 || !term_offset || !xmask || !zmask || !coeff || n_qubits < 1 || n_qubits > 30)
        return VQE_EINVAL;
    vqe_mf_pool *p = new (std::nothrow) vqe_mf_pool();
    if (!p)
        return VQE_ENOMEM;
    p->n_qubits = n_qubits;
    p->desc.resize(M);
    for (int j = 0; j < M; j++) {
        const int64_t t0 = term_offset[j], t1 = term_offset[j + 1];
        if (t0 < 0 || t1 <= t0) {
            delete p;
            return VQE_EINVAL;
        }
        double tol;
        if (drop_tol) {
            tol = drop_tol[j];
        } else {
            double mx = 0.0;
            for (int64_t t = t0; t < t1; t++)
                mx = std::max(mx, std::hypot(coeff[2 * t], coeff[2 * t + 1]));
            tol = 1e-12 * mx;
        }
        const int rc = describe(n_qubits, t1 - t0, xmask + t0, zmask + t0, coeff + 2 * t0, tol,
                                &p->desc[j]);
        if (rc) {
            delete p;
            return rc;
        }
    }
    *out = p;
    return VQE_OK;
}

extern "C" int vqe_mf_pool_destroy(vqe_mf_pool *pool)
{
    delete pool;
    return VQE_OK;
}

extern "C" int vqe_mf_pool_get(const vqe_mf_pool *pool, int32_t j, vqe_mf_desc *out)
{
    if (!pool || !out || j < 0 || j >= (int32_t)pool->desc.size())
        return VQE_EINVAL;
    *out = pool->desc[j];
    return VQE_OK;
}

// Host mirror of the device enumeration (same record, same lane/iteration
// split), for tests without a GPU.
extern "C" int vqe_mf_owner_rows(const vqe_mf_pool *pool, int32_t j, int64_t tile_rows,
                                 int32_t tile, int64_t *count, uint32_t *rows_out,
                                 uint32_t *lds_index_out)
{
    if (!pool || !count || j < 0 || j >= (int32_t)pool->desc.size() || tile_rows < 1)
        return VQE_EINVAL;
    MfHostPlan hp;
    char err[160];
    int rc = mf_host_plan(pool, tile_rows, &hp, err, sizeof(err));
    if (rc)
        return rc;
    if (tile < -1 || tile >= hp.ntile)
        return VQE_EINVAL;
    const MfRec &rec = tile < 0 ? hp.full_recs[j] : hp.tile_recs[(size_t)j * hp.ntile + tile];
    if (rec.nfree < 0) {
        *count = 0;
        return VQE_OK;
    }
    auto pivots = [&](uint32_t a, bool withk) {
        uint32_t p = 0;
        for (int i = 0; i < rec.ncon; i++)
            p |= ((uint32_t)(__builtin_popcount(rec.beta[i] & a) ^ (withk ? (rec.kbits >> i) : 0u)) & 1u)
                 << rec.piv[i];
        return p;
    };
    const int64_t n = (int64_t)1 << rec.nfree;
    *count = n;
    if (!rows_out)
        return VQE_OK;
    int64_t o = 0;
    const int n_it = 1 << (rec.nfree - rec.nlow);
    uint32_t H = 0;
    for (int it = 0; it < n_it; it++) {
        const uint32_t RH = H ^ pivots(H, true) ^ rec.base;
        for (uint32_t e = 0; e < (1u << rec.nlow); e++) {
            uint32_t L = 0;
            for (int b = 0; b < rec.nlow; b++)
                L |= ((e >> b) & 1u) << rec.lowpos[b];
            const uint32_t RL = L ^ pivots(L, false);
            rows_out[o] = RL ^ RH;
            if (lds_index_out)
                lds_index_out[o] = compress_bits(RL, rec.tbpos, rec.ntb) ^
                                   compress_bits(RH, rec.tbpos, rec.ntb);
            o++;
        }
        H = ((H | ~rec.hi_mask) + 1u) & rec.hi_mask;
    }
    return VQE_OK;
}

int32_t vqe_mf_pool_size(const vqe_mf_pool *pool) { return (int32_t)pool->desc.size(); }
int32_t vqe_mf_pool_qubits(const vqe_mf_pool *pool) { return pool->n_qubits; }

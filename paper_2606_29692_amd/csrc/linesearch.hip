// Line search over the angle of the selected generator (parameter
// optimisation, which the adaptive loop of Sec. III-D leaves implicit).
//
// For a generator whose square is minus the projector on its support
// (A^3 = -A: every fermionic single or double excitation, Sec. III-C), the
// fifth-order update of Eq. 6-8 collapses to
//     T5(theta A) psi = psi + s(theta) A psi + c(theta) A^2 psi,
//     s = theta - theta^3/6 + theta^5/120,   c = theta^2/2 - theta^4/24,
// so the energy (Eq. 1) of the renormalised update is a ratio of two
// quadratic forms in (1, s, c):
//     E(theta) = sum_ij f_i f_j Re K_ij / sum_ij f_i f_j Re G_ij,
//     f = (1, s, c),  G_ij = <v_i|v_j>,  K_ij = <v_i|H|v_j>,  v = (psi, A psi, A^2 psi).
// The plan builds v1 = A psi and v2 = A^2 psi (pair by pair), takes the two
// products S v1 and S v2 with its H-product schedule, reduces the entries in
// FP64 and minimises E over [-theta_max, theta_max]: the best of a 256-point
// grid, refined by golden-section search on the grid interval around it.
#include "kernels.hpp"

namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ double re_dot(double2 a, double2 b)   // Re(conj(a) b)
{
    return a.x * b.x + a.y * b.y;
}

// Workgroup sum of N values per thread into out[0..N) (fixed order).
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double *out)
{
    __shared__ double s_part[4][N];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < N; q++)
        v[q] = wave_sum(v[q]);
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < N; q++)
            s_part[wid][q] = v[q];
    __syncthreads();
    if (threadIdx.x < N) {
        const int q = threadIdx.x;
        out[q] = ((s_part[0][q] + s_part[1][q]) + s_part[2][q]) + s_part[3][q];
    }
}

// v1 = A psi and v2 = A^2 psi over a block of rows, with the partial sums
// Re<psi|v1>, Re<psi|v2>, <v1|v1>, Re<v1|v2>, <v2|v2>, Re<S psi|v1>, Re<S psi|v2>.
template <int DT>
__global__ void __launch_bounds__(256)
k_ls_vectors(const LsState *__restrict__ states, const int2 *__restrict__ tasks)
{
    const int2 task = tasks[blockIdx.x];
    if (task.x < 0)
        return;
    const LsState &st = states[task.x];
    if (VQE_SKIP(st))
        return;
    const int32_t k = *gmem(st.k);
    const bool valid = k >= 0 && k < st.M;
    double acc[LS_NVEC] = {0, 0, 0, 0, 0, 0, 0};
    const int64_t r0 = (int64_t)task.y * LS_ROWS_PER_BLOCK;
    const int64_t r1 = r0 + LS_ROWS_PER_BLOCK < st.dim ? r0 + LS_ROWS_PER_BLOCK : st.dim;
    for (int64_t r = r0 + threadIdx.x; r < r1 && valid; r += 256) {
        const double2 p = Elem<DT>::ld(st.psi, r), sg = Elem<DT>::ld(st.sigma, r);
        double2 v1 = make_double2(0.0, 0.0), v2 = make_double2(0.0, 0.0);
        bool on = false;
        int64_t c = 0;
        double2 a, b;
        if (st.mf) {
            const vqe_mf_desc &d = st.mf[k];
            const uint64_t rr = (uint64_t)r;
            on = true;
            for (int i = 0; i < d.n_con; i++)
                on = on && (uint32_t)(__popcll(d.beta[i] & rr) & 1) == ((d.kbits >> i) & 1u);
            if (on) {
                c = (int64_t)(rr ^ d.x);
                // A[r, c] = v (-1)^{|zsign & c|},  A[c, r] = v (-1)^{|zsign & r|}
                const double sa = (__popcll(d.zsign & (uint64_t)c) & 1) ? -1.0 : 1.0;
                const double sb = (__popcll(d.zsign & rr) & 1) ? -1.0 : 1.0;
                a = make_double2(sa * d.v_re, sa * d.v_im);
                b = make_double2(sb * d.v_re, sb * d.v_im);
            }
        } else {
            const vqe_csr &op = st.ops[k];
            const int k0 = gmem(op.rowptr)[r];
            if (gmem(op.rowptr)[r + 1] - k0 == 1) {
                on = true;
                c = gmem(op.col)[k0];
                a = Elem<DT>::ld(op.val, k0);
                b = Elem<DT>::ld(op.val, gmem(op.rowptr)[c]);
            }
        }
        if (on) {
            v1 = cmul(a, Elem<DT>::ld(st.psi, c));
            v2 = cmul(cmul(a, b), p);
        }
        Elem<DT>::st(st.v1, r, v1);
        Elem<DT>::st(st.v2, r, v2);
        acc[0] += re_dot(p, v1);
        acc[1] += re_dot(p, v2);
        acc[2] += re_dot(v1, v1);
        acc[3] += re_dot(v1, v2);
        acc[4] += re_dot(v2, v2);
        acc[5] += re_dot(sg, v1);
        acc[6] += re_dot(sg, v2);
    }
    block_sum<LS_NVEC>(acc, st.part_vec + (int64_t)task.y * LS_NVEC);
}

// Re<v1 | S v2> over a block of rows.
template <int DT>
__global__ void __launch_bounds__(256)
k_ls_dot(const LsState *__restrict__ states, const int2 *__restrict__ tasks)
{
    const int2 task = tasks[blockIdx.x];
    if (task.x < 0)
        return;
    const LsState &st = states[task.x];
    if (VQE_SKIP(st))
        return;
    double acc[1] = {0.0};
    const int64_t r0 = (int64_t)task.y * LS_ROWS_PER_BLOCK;
    const int64_t r1 = r0 + LS_ROWS_PER_BLOCK < st.dim ? r0 + LS_ROWS_PER_BLOCK : st.dim;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += 256)
        acc[0] += re_dot(Elem<DT>::ld(st.v1, r), Elem<DT>::ld(st.w2, r));
    block_sum<1>(acc, st.part_dot + task.y);
}

struct LsForms {
    double K[3][3], G[3][3];
};

__device__ __forceinline__ double ls_energy(const LsForms &f, double t)
{
    const double t2 = t * t;
    const double s = t * (1.0 + t2 * (-1.0 / 6.0 + t2 / 120.0));
    const double c = t2 * (0.5 - t2 / 24.0);
    const double w[3] = {1.0, s, c};
    double num = 0.0, den = 0.0;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            num += w[i] * w[j] * f.K[i][j];
            den += w[i] * w[j] * f.G[i][j];
        }
    return num / den;
}

// fixed-order sum of a strided partial array over the wave
__device__ __forceinline__ double wave_total(const double *p, int n, int stride, int q)
{
    double v = 0.0;
    for (int b = (int)(threadIdx.x & 63); b < n; b += 64)
        v += p[(int64_t)b * stride + q];
    return wave_sum(v);
}

// Minimiser of E(theta) over [-tm, tm]: the lowest point of an LS_GRID-point
// grid (lane l evaluates points l, l + 64, ...; ties to the lower index),
// refined by golden-section search on the neighbouring grid interval (every
// lane runs the same arithmetic); t_alt wins when nothing is lower.
__device__ double ls_minimise(const LsForms &f, double tm, int lane, double t_alt)
{
    // coarse grid: lane l evaluates points l, l + 64, l + 128, l + 192
    const double step = 2.0 * tm / (double)(LS_GRID - 1);
    double best = 0.0;
    int bi = -1;
    for (int i = lane; i < LS_GRID; i += 64) {
        const double e = ls_energy(f, -tm + step * i);
        if (bi < 0 || e < best) {
            best = e;
            bi = i;
        }
    }
    // wave argmin (lowest energy, then lowest index)
    for (int o = 32; o > 0; o >>= 1) {
        const double eo = __shfl_xor(best, o, 64);
        const int io = __shfl_xor(bi, o, 64);
        if (eo < best || (eo == best && io < bi)) {
            best = eo;
            bi = io;
        }
    }
    // golden-section refinement on the neighbouring grid interval (every lane
    // runs the same arithmetic)
    double lo = -tm + step * (bi > 0 ? bi - 1 : 0);
    double hi = -tm + step * (bi < LS_GRID - 1 ? bi + 1 : LS_GRID - 1);
    const double gr = 0.6180339887498949;
    double x1 = hi - gr * (hi - lo), x2 = lo + gr * (hi - lo);
    double f1 = ls_energy(f, x1), f2 = ls_energy(f, x2);
    for (int it = 0; it < 80; it++) {
        if (f1 <= f2) {
            hi = x2;
            x2 = x1;
            f2 = f1;
            x1 = hi - gr * (hi - lo);
            f1 = ls_energy(f, x1);
        } else {
            lo = x1;
            x1 = x2;
            f1 = f2;
            x2 = lo + gr * (hi - lo);
            f2 = ls_energy(f, x2);
        }
    }
    double t_best = -tm + step * bi, e_best = best;
    const double xm = 0.5 * (lo + hi), em = ls_energy(f, xm);
    if (em < e_best) {
        t_best = xm;
        e_best = em;
    }
    if (ls_energy(f, t_alt) < e_best)
        t_best = t_alt;
    return t_best;
}

// One wave per state: assemble G and K, minimise E(theta), write theta.
__global__ void __launch_bounds__(64)
k_ls_solve(const LsState *__restrict__ states, int n_states)
{
    const int s = blockIdx.x;
    if (s >= n_states)
        return;
    const LsState &st = states[s];
    if (VQE_SKIP(st))
        return;
    const int32_t k = *gmem(st.k);
    if (k < 0 || k >= st.M)
        return;
    const int lane = threadIdx.x;
    double pv[LS_NVEC];
#pragma unroll
    for (int q = 0; q < LS_NVEC; q++)
        pv[q] = wave_total(st.part_vec, st.nb_rows, LS_NVEC, q);
    const double h1 = wave_total(st.part_h1, st.nb_spmv, 3, 0);
    const double h2 = wave_total(st.part_h2, st.nb_spmv, 3, 0);
    const double d12 = wave_total(st.part_dot, st.nb_rows, 1, 0);
    const double e0 = gmem(st.energy)[0], n0 = gmem(st.energy)[1];
    const double sh = st.shift;
    LsForms f;
    f.G[0][0] = n0;
    f.G[0][1] = f.G[1][0] = pv[0];
    f.G[0][2] = f.G[2][0] = pv[1];
    f.G[1][1] = pv[2];
    f.G[1][2] = f.G[2][1] = pv[3];
    f.G[2][2] = pv[4];
    // K = <v_i|S v_j> + shift G_ij
    f.K[0][0] = e0 * n0;
    f.K[0][1] = f.K[1][0] = pv[5] + sh * pv[0];
    f.K[0][2] = f.K[2][0] = pv[6] + sh * pv[1];
    f.K[1][1] = h1 + sh * pv[2];
    f.K[1][2] = f.K[2][1] = d12 + sh * pv[3];
    f.K[2][2] = h2 + sh * pv[4];
    const double t_best = ls_minimise(f, st.theta_max, lane, 0.0);
    if (lane == 0)
        gmem(st.theta)[0] = t_best;
}


// ------------------------------------------------------------ re-optimisation
// Every angle of the ansatz  psi = T5(t_{n-1} A_{n-1}) ... T5(t_0 A_0) ref  by
// cyclic coordinate line search.  For the visited update m, with L the state
// before it and R the later updates (linear maps), the ansatz is
//     R T5(t A_m) L = R L + s(t) R A_m L + c(t) R A_m^2 L   (A_m^3 = -A_m),
// so its energy is the same ratio of quadratic forms as the line search's,
// over w_i = R A_m^i L.  Per visit: the vectors L, A L, A^2 L; the later
// updates applied to all three; three H products; twelve inner products; the
// minimiser; then L advances by the new T5(t_m A_m).

// The entries of generator k on row r: the partner c and A[r, c], A[c, r]
// (false when the row is not in the support).
__device__ __forceinline__ bool ro_pair(const RoState &st, int32_t k, int64_t r, int64_t &c,
                                        double2 &a, double2 &b, int dt)
{
    if (st.mf) {
        const vqe_mf_desc &d = st.mf[k];
        const uint64_t rr = (uint64_t)r;
        for (int i = 0; i < d.n_con; i++)
            if ((uint32_t)(__popcll(d.beta[i] & rr) & 1) != ((d.kbits >> i) & 1u))
                return false;
        c = (int64_t)(rr ^ d.x);
        const double sa = (__popcll(d.zsign & (uint64_t)c) & 1) ? -1.0 : 1.0;
        const double sb = (__popcll(d.zsign & rr) & 1) ? -1.0 : 1.0;
        a = make_double2(sa * d.v_re, sa * d.v_im);
        b = make_double2(sb * d.v_re, sb * d.v_im);
        return true;
    }
    const vqe_csr &op = st.ops[k];
    const int k0 = gmem(op.rowptr)[r];
    if (gmem(op.rowptr)[r + 1] - k0 != 1)
        return false;
    c = gmem(op.col)[k0];
    if (dt == VQE_C128) {
        a = Elem<VQE_C128>::ld(op.val, k0);
        b = Elem<VQE_C128>::ld(op.val, gmem(op.rowptr)[c]);
    } else {
        a = Elem<VQE_C64>::ld(op.val, k0);
        b = Elem<VQE_C64>::ld(op.val, gmem(op.rowptr)[c]);
    }
    return true;
}

__device__ __forceinline__ bool ro_valid(const RoState &st, int m)
{
    const int32_t k = gmem(st.ks)[m];
    return k >= 0 && k < st.M;
}

// v1 = A_m L, v2 = A_m^2 L over a block of rows; w = (L, v1, v2).
template <int DT>
__global__ void __launch_bounds__(256)
k_ro_vectors(const RoState *__restrict__ states, const int2 *__restrict__ tasks, int m)
{
    const int2 task = tasks[blockIdx.x];
    if (task.x < 0)
        return;
    const RoState &st = states[task.x];
    if (VQE_SKIP(st))
        return;
    const bool valid = ro_valid(st, m);
    const int32_t k = valid ? gmem(st.ks)[m] : 0;
    const int64_t r0 = (int64_t)task.y * LS_ROWS_PER_BLOCK;
    const int64_t r1 = r0 + LS_ROWS_PER_BLOCK < st.dim ? r0 + LS_ROWS_PER_BLOCK : st.dim;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) {
        const double2 p = Elem<DT>::ld(st.L, r);
        double2 v1 = make_double2(0.0, 0.0), v2 = make_double2(0.0, 0.0);
        int64_t c;
        double2 a, b;
        if (valid && ro_pair(st, k, r, c, a, b, DT)) {
            v1 = cmul(a, Elem<DT>::ld(st.L, c));
            v2 = cmul(cmul(a, b), p);
        }
        Elem<DT>::st(st.v1, r, v1);
        Elem<DT>::st(st.v2, r, v2);
        Elem<DT>::st(st.w[0], r, p);
        Elem<DT>::st(st.w[1], r, v1);
        Elem<DT>::st(st.w[2], r, v2);
    }
}

// In place y <- T5(t_m A_m) y (Eq. 6-8: five products and the power sum) for
// NV vectors: the w triple (NV = 3, the later updates of a visit) or L
// (NV = 1, the advance after a visit).  Each pair {r, c} of the support is
// updated by its owner row, so no two threads touch one element.
template <int DT, int NV>
__global__ void __launch_bounds__(256)
k_ro_taylor(const RoState *__restrict__ states, const int2 *__restrict__ tasks, int m)
{
    const int2 task = tasks[blockIdx.x];
    if (task.x < 0)
        return;
    const RoState &st = states[task.x];
    if (VQE_SKIP(st) || !ro_valid(st, m))
        return;
    const int32_t k = gmem(st.ks)[m];
    const double theta = gmem(st.thetas)[m];
    double cf[6];
    cf[0] = 1.0;
#pragma unroll
    for (int q = 1; q <= 5; q++)
        cf[q] = cf[q - 1] * theta / (double)q;
    void *vec[3] = {NV == 1 ? st.L : st.w[0], st.w[1], st.w[2]};
    const int64_t r0 = (int64_t)task.y * LS_ROWS_PER_BLOCK;
    const int64_t r1 = r0 + LS_ROWS_PER_BLOCK < st.dim ? r0 + LS_ROWS_PER_BLOCK : st.dim;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) {
        int64_t c;
        double2 a, b;
        if (!ro_pair(st, k, r, c, a, b, DT) || c < r)
            continue;
        if (c == r) {
            // a diagonal entry: the 1 x 1 block (A^2 = a^2 = -1)
#pragma unroll
            for (int v = 0; v < NV; v++) {
                double2 vr = Elem<DT>::ld(vec[v], r), ar = vr;
#pragma unroll
                for (int q = 1; q <= 5; q++) {
                    vr = cmul(a, vr);
                    ar.x += cf[q] * vr.x;
                    ar.y += cf[q] * vr.y;
                }
                Elem<DT>::st(vec[v], r, ar);
            }
            continue;
        }
#pragma unroll
        for (int v = 0; v < NV; v++) {
            double2 vr = Elem<DT>::ld(vec[v], r), vc = Elem<DT>::ld(vec[v], c);
            double2 ar = vr, ac = vc;
#pragma unroll
            for (int q = 1; q <= 5; q++) {
                const double2 nr = cmul(a, vc);
                const double2 nc = cmul(b, vr);
                vr = nr;
                vc = nc;
                ar.x += cf[q] * vr.x;
                ar.y += cf[q] * vr.y;
                ac.x += cf[q] * vc.x;
                ac.y += cf[q] * vc.y;
            }
            Elem<DT>::st(vec[v], r, ar);
            Elem<DT>::st(vec[v], c, ac);
        }
    }
}

// Re<w_i|w_j> and Re<w_i|S w_j> (i <= j) over a block of rows.
template <int DT>
__global__ void __launch_bounds__(256)
k_ro_dots(const RoState *__restrict__ states, const int2 *__restrict__ tasks)
{
    const int2 task = tasks[blockIdx.x];
    if (task.x < 0)
        return;
    const RoState &st = states[task.x];
    if (VQE_SKIP(st))
        return;
    double acc[RO_NDOT] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t r0 = (int64_t)task.y * LS_ROWS_PER_BLOCK;
    const int64_t r1 = r0 + LS_ROWS_PER_BLOCK < st.dim ? r0 + LS_ROWS_PER_BLOCK : st.dim;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) {
        double2 w[3], h[3];
#pragma unroll
        for (int i = 0; i < 3; i++) {
            w[i] = Elem<DT>::ld(st.w[i], r);
            h[i] = Elem<DT>::ld(st.h[i], r);
        }
        int q = 0;
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = i; j < 3; j++) {
                acc[q] += re_dot(w[i], w[j]);
                acc[6 + q] += re_dot(w[i], h[j]);
                q++;
            }
    }
    block_sum<RO_NDOT>(acc, st.part + (int64_t)task.y * RO_NDOT);
}

// One wave per state: the forms of visit m, its new angle (the current angle
// is kept unless something is lower) and the energy there.
__global__ void __launch_bounds__(64)
k_ro_solve(const RoState *__restrict__ states, int n_states, int m)
{
    const int s = blockIdx.x;
    if (s >= n_states)
        return;
    const RoState &st = states[s];
    if (VQE_SKIP(st) || !ro_valid(st, m))
        return;
    const int lane = threadIdx.x;
    double t[RO_NDOT];
#pragma unroll
    for (int q = 0; q < RO_NDOT; q++)
        t[q] = wave_total(st.part, st.nb_rows, RO_NDOT, q);
    LsForms f;
    int q = 0;
    for (int i = 0; i < 3; i++)
        for (int j = i; j < 3; j++) {
            f.G[i][j] = f.G[j][i] = t[q];
            // K = <w_i|S w_j> + shift G_ij (S = H - shift: FP32 storage)
            f.K[i][j] = f.K[j][i] = t[6 + q] + st.shift * t[q];
            q++;
        }
    const double t_cur = gmem(st.thetas)[m];
    const double t_new = ls_minimise(f, st.theta_max, lane, t_cur);
    if (lane == 0) {
        gmem(st.thetas)[m] = t_new;
        if (st.e_out)
            st.e_out[0] = ls_energy(f, t_new);
    }
}

// psi <- L (the ansatz state at the final angles; renormalised afterwards).
template <int DT>
__global__ void __launch_bounds__(256)
k_ro_finish(const RoState *__restrict__ states, const int2 *__restrict__ tasks)
{
    const int2 task = tasks[blockIdx.x];
    if (task.x < 0)
        return;
    const RoState &st = states[task.x];
    if (VQE_SKIP(st))
        return;
    const int64_t r0 = (int64_t)task.y * LS_ROWS_PER_BLOCK;
    const int64_t r1 = r0 + LS_ROWS_PER_BLOCK < st.dim ? r0 + LS_ROWS_PER_BLOCK : st.dim;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += 256)
        Elem<DT>::st(st.psi, r, Elem<DT>::ld(st.L, r));
}
}  // namespace

void launch_ls_vectors(int dtype, const LsState *states, const int2 *tasks, unsigned grid,
                       hipStream_t s)
{
    if (dtype == VQE_C128)
        k_ls_vectors<VQE_C128><<<grid, 256, 0, s>>>(states, tasks);
    else
        k_ls_vectors<VQE_C64><<<grid, 256, 0, s>>>(states, tasks);
}

void launch_ls_dot(int dtype, const LsState *states, const int2 *tasks, unsigned grid,
                   hipStream_t s)
{
    if (dtype == VQE_C128)
        k_ls_dot<VQE_C128><<<grid, 256, 0, s>>>(states, tasks);
    else
        k_ls_dot<VQE_C64><<<grid, 256, 0, s>>>(states, tasks);
}

void launch_ls_solve(const LsState *states, unsigned n_states, hipStream_t s)
{
    k_ls_solve<<<n_states, 64, 0, s>>>(states, (int)n_states);
}

void launch_ro_vectors(int dtype, const RoState *states, const int2 *tasks, unsigned grid, int m,
                       hipStream_t s)
{
    if (dtype == VQE_C128)
        k_ro_vectors<VQE_C128><<<grid, 256, 0, s>>>(states, tasks, m);
    else
        k_ro_vectors<VQE_C64><<<grid, 256, 0, s>>>(states, tasks, m);
}

void launch_ro_taylor(int dtype, const RoState *states, const int2 *tasks, unsigned grid, int m,
                      bool advance, hipStream_t s)
{
    if (dtype == VQE_C128) {
        if (advance)
            k_ro_taylor<VQE_C128, 1><<<grid, 256, 0, s>>>(states, tasks, m);
        else
            k_ro_taylor<VQE_C128, 3><<<grid, 256, 0, s>>>(states, tasks, m);
    } else {
        if (advance)
            k_ro_taylor<VQE_C64, 1><<<grid, 256, 0, s>>>(states, tasks, m);
        else
            k_ro_taylor<VQE_C64, 3><<<grid, 256, 0, s>>>(states, tasks, m);
    }
}

void launch_ro_dots(int dtype, const RoState *states, const int2 *tasks, unsigned grid,
                    hipStream_t s)
{
    if (dtype == VQE_C128)
        k_ro_dots<VQE_C128><<<grid, 256, 0, s>>>(states, tasks);
    else
        k_ro_dots<VQE_C64><<<grid, 256, 0, s>>>(states, tasks);
}

void launch_ro_solve(const RoState *states, unsigned n_states, int m, hipStream_t s)
{
    k_ro_solve<<<n_states, 64, 0, s>>>(states, (int)n_states, m);
}

void launch_ro_finish(int dtype, const RoState *states, const int2 *tasks, unsigned grid,
                      hipStream_t s)
{
    if (dtype == VQE_C128)
        k_ro_finish<VQE_C128><<<grid, 256, 0, s>>>(states, tasks);
    else
        k_ro_finish<VQE_C64><<<grid, 256, 0, s>>>(states, tasks);
}

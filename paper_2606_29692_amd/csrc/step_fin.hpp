// End of a batched step's screen for one state, by one 256-thread workgroup:
// the energy from the H product's block partials (Eq. 1), the gradients from
// the screen's tile partials (Eq. 5), then the largest |g_j| with the lowest
// index among the near-ties.  The energy is summed exactly as the single-call
// energy finalisation sums it, and g_j adds its tile partials in tile order.
#pragma once

#include "kernels.hpp"

#define FIN_LDS_G 2048   // gradients per state kept in LDS for the selection
// the matrix-free update repeats its state's finalisation in every block while
// the screen leaves at most this many partial sums per state (generators x
// row tiles); beyond, one finalisation kernel per state runs before the update
#define FIN_FUSE_PARTIALS 4096

// With write false nothing is stored, so that every workgroup of a state's
// update can form the same selection.  Returns the selected index in every
// thread (-1 without selection).  Without write the gradients must fit LDS
// (M <= FIN_LDS_G).
__device__ __forceinline__ int step_fin_block(const SpmvState &hs, const ScreenState *screen,
                                              const PairTable *tables, const SelectState &ss,
                                              int s, bool do_grad, bool do_select,
                                              double rel_tie, bool write)
{
    const int tid = threadIdx.x;
    if (tid < 64) {
        double re = 0.0, im = 0.0, n2 = 0.0;
        for (int b = tid; b < hs.nblocks; b += 64) {
            re += hs.partials[(int64_t)b * 3 + 0];
            im += hs.partials[(int64_t)b * 3 + 1];
            n2 += hs.partials[(int64_t)b * 3 + 2];
        }
        re = wave_sum(re);
        im = wave_sum(im);
        n2 = wave_sum(n2);
        if (write && tid == 0 && hs.energy_out) {
            hs.energy_out[0] = hs.shift + re / n2;
            hs.energy_out[1] = n2;
            hs.energy_out[2] = im;
        }
    }
    // the gradients also go to LDS when they fit, for the selection below
    __shared__ double s_g[FIN_LDS_G];
    __shared__ int s_k;
    const bool in_lds = do_grad && ss.M <= FIN_LDS_G;
    if (do_grad) {
        const ScreenState st = screen[s];
        const PairTable tb = tables[st.table];
        for (int j = tid; j < tb.M; j += 256) {
            double acc = 0.0;
            for (int t = 0; t < tb.nt; t++)
                acc += st.partials[(int64_t)j * tb.nt + t];
            if (write)
                st.g_out[j] = 2.0 * acc;
            if (in_lds)
                s_g[j] = 2.0 * acc;
        }
    }
    if (!do_select)
        return -1;
    __syncthreads();      // the gradients written above are read below
    if (tid < 64) {
        const double *g = in_lds ? s_g : ss.g;
        double gmax = 0.0;
        for (int j = tid; j < ss.M; j += 64)
            gmax = fmax(gmax, fabs(g[j]));
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
            gmax = fmax(gmax, __shfl_xor(gmax, o, 64));
        const double thr = gmax * (1.0 - rel_tie);
        int best = 0x7fffffff;
        for (int j = tid; j < ss.M; j += 64)
            if (fabs(g[j]) >= thr && j < best)
                best = j;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
            best = min(best, __shfl_xor(best, o, 64));
        if (tid == 0) {
            s_k = best == 0x7fffffff ? 0 : best;
            if (write) {
                ss.k_out[0] = s_k;
                ss.gmax_out[0] = gmax;
            }
        }
    }
    __syncthreads();
    return s_k;
}

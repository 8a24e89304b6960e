// Exact top-k over every non-trivial pair for long series (Algorithm 1, last
// line: when no step stops, the answer is the exact one), as a sweep of the
// diagonals b = a + s (2 s > w, so no trivial match is formed).
//
// Along a diagonal the centred cross product of dimension f,
//   C_f(a, b) = sum_t (x_f[a+t] - mu_f(a)) (x_f[b+t] - mu_f(b)),
// follows C(a+1, b+1) = C(a, b) + df(a) dg(b) + df(b) dg(a) with
// df(i) = (x[i+w] - x[i]) / 2 and dg(i) = (x[i+w] - mu(i+1)) + (x[i] - mu(i))
// (exact algebra; mu(i+1) = mu(i) + (x[i+w] - x[i]) / w), re-seeded by the
// direct sum at the start of every chunk of Lc steps. With population
// standard deviations the z-normalised distance of Eq. zned is
//   dist_f^2 = w (s_a + s_b) - 2 C_f / (sigma_a sigma_b)
// (s = 1 for a window that is not flat, 0 for a flat one: its normal form is
// all zeros). That value only FILTERS: a pair is emitted when the sum of its
// d smallest per-dimension distances is below the cut theta, and every
// emitted pair is verified from the series by k_verify (FP64, the same
// arithmetic as every verified pair of the traversal).
//
// A wavefront handles one chunk of Lc consecutive pairs on each of G = 64 / Dp
// adjacent diagonals, lane (q, f) carrying dimension f of diagonal q (Dp =
// D rounded up to a power of two; above 64 dimensions one diagonal per wave
// and two dimensions per lane). Per step, two ballots count for every
// diagonal the dimensions below theta and below theta / d: a sum of d
// distances below theta needs d of them below theta and one below theta / d.
// Pairs passing that test (rare) rank their dimensions through LDS and add
// the d smallest distances.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "internal.h"

namespace mm {

__device__ inline void sweep_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T, int DL>
__global__ __launch_bounds__(256) void k_sweep(const T* __restrict__ x, const double* __restrict__ mu,
                                               const double* __restrict__ isig, SweepArgs g,
                                               Cand* __restrict__ cand, uint32_t cap, Counters* __restrict__ cnt)
{
    __shared__ double sh[4][64 * DL];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t item = g.item_lo + (int64_t)blockIdx.x * 4 + wave;
    if (item >= g.item_hi) return;                       // uniform across the wavefront
    const int64_t grp = item / g.chunks, ch = item - grp * g.chunks;
    const int64_t s0 = g.s_lo + grp * g.G;                // first diagonal of the group
    if (s0 >= g.ns) return;
    const int64_t len0 = g.ns - s0;                       // pairs on the group's longest diagonal
    const int64_t a0 = ch * g.Lc;
    if (a0 >= len0) return;
    const int64_t a1 = a0 + g.Lc < len0 ? a0 + g.Lc : len0;
    const int q = lane / g.Dp, fl = lane - q * g.Dp;
    const int64_t s = s0 + q;
    const int64_t len = g.ns - s;                         // pairs on this lane's diagonal (may be <= a0)
    const int w = g.w;
    const double wd = (double)w;
    const uint64_t gmask = (g.Dp == 64 ? ~0ull : ((1ull << g.Dp) - 1ull)) << (q * g.Dp);

    int f[DL];
    bool on[DL];
    double C[DL];
#pragma unroll
    for (int u = 0; u < DL; ++u) {
        f[u] = fl + 64 * u;
        on[u] = f[u] < g.D && a0 < len;
        C[u] = 0.0;
        if (on[u]) {
            // re-seed: the direct centred cross product at (a0, a0 + s)
            const T* xf = x + (int64_t)f[u] * g.n;
            const double ma = mu[(int64_t)f[u] * g.ns + a0], mb = mu[(int64_t)f[u] * g.ns + a0 + s];
            double acc = 0.0;
            for (int t = 0; t < w; ++t) acc = acc + ((double)xf[a0 + t] - ma) * ((double)xf[a0 + s + t] - mb);
            C[u] = acc;
        }
    }
    for (int64_t a = a0; a < a1; ++a) {
        const bool act = a < len;
        const int64_t b = a + s;
        double d2[DL];
#pragma unroll
        for (int u = 0; u < DL; ++u) {
            d2[u] = __builtin_huge_val();
            if (act && on[u]) {
                const T* xf = x + (int64_t)f[u] * g.n;
                const double* mf = mu + (int64_t)f[u] * g.ns;
                const double* sf = isig + (int64_t)f[u] * g.ns;
                if (a > a0) {
                    const double xa0 = (double)xf[a - 1], xaw = (double)xf[a - 1 + w];
                    const double xb0 = (double)xf[b - 1], xbw = (double)xf[b - 1 + w];
                    const double dfa = (xaw - xa0) * 0.5, dga = (xaw - mf[a]) + (xa0 - mf[a - 1]);
                    const double dfb = (xbw - xb0) * 0.5, dgb = (xbw - mf[b]) + (xb0 - mf[b - 1]);
                    C[u] = C[u] + (dfa * dgb + dfb * dga);
                }
                const double ia = sf[a], ib = sf[b];
                const double sa = ia != 0.0 ? 1.0 : 0.0, sb = ib != 0.0 ? 1.0 : 0.0;
                d2[u] = wd * (sa + sb) - 2.0 * C[u] * ia * ib;
            }
        }
        int below = 0, low = 0;
#pragma unroll
        for (int u = 0; u < DL; ++u) {
            below += __popcll(__ballot(d2[u] < g.th2) & gmask);
            low += __popcll(__ballot(d2[u] < g.low2) & gmask);
        }
        const bool pass = act && below >= g.d && low >= 1;
        if (!__ballot(pass)) continue;
        // the rare path: rank the diagonal's D distances, add the d smallest
#pragma unroll
        for (int u = 0; u < DL; ++u) sh[wave][64 * u + lane] = d2[u];
        sweep_sync();
        double part = 0.0;
        if (pass) {
            const int base = q * g.Dp;
#pragma unroll
            for (int u = 0; u < DL; ++u) {
                if (!on[u]) continue;
                const double v = d2[u];
                const int me = fl + 64 * u;
                int rank = 0;
                for (int uu = 0; uu < DL; ++uu)
                    for (int j = 0; j < g.Dp; ++j) {
                        const int other = j + 64 * uu;
                        const double o = sh[wave][64 * uu + base + j];
                        rank += (o < v) || (o == v && other < me);
                    }
                if (rank < g.d) part += sqrt(v > 0.0 ? v : 0.0);
            }
        }
        // sum over the diagonal's lanes (a group of Dp aligned lanes)
        for (int o = 1; o < g.Dp; o <<= 1) part += __shfl_xor(part, o, 64);
        if (pass && fl == 0 && part < g.theta &&
            (g.nparts <= 1 || pair_part((uint32_t)a, (uint32_t)b, g.nparts) == (uint32_t)g.part)) {
            const uint32_t pos = atomicAdd(&cnt->n_cand, 1u);
            if (pos < cap) cand[pos] = Cand{(uint32_t)a, (uint32_t)b, 0u, 0u};
        }
        sweep_sync();
    }
}

hipError_t launch_sweep(const void* x, int dtype, const double* mu, const double* isig, const SweepArgs& g,
                        Cand* cand, uint32_t cap, Counters* cnt, hipStream_t s)
{
    const int64_t items = g.item_hi - g.item_lo;
    if (items <= 0) return hipSuccess;
    const dim3 grid((unsigned)((items + 3) / 4));
    if (g.DL == 1) {
        if (dtype == 0)
            hipLaunchKernelGGL((k_sweep<double, 1>), grid, dim3(256), 0, s, (const double*)x, mu, isig, g, cand, cap, cnt);
        else
            hipLaunchKernelGGL((k_sweep<float, 1>), grid, dim3(256), 0, s, (const float*)x, mu, isig, g, cand, cap, cnt);
    } else {
        if (dtype == 0)
            hipLaunchKernelGGL((k_sweep<double, 2>), grid, dim3(256), 0, s, (const double*)x, mu, isig, g, cand, cap, cnt);
        else
            hipLaunchKernelGGL((k_sweep<float, 2>), grid, dim3(256), 0, s, (const float*)x, mu, isig, g, cand, cap, cnt);
    }
    return hipGetLastError();
}

}  // namespace mm

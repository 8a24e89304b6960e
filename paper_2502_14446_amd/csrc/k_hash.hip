// Index construction on gfx950 (Algorithm 1, first loop; section 6.1).
//
//  * k_stats     rolling mean / population standard deviation of every window
//                (Eq. zned needs mu and sigma of each subsequence), FP64.
//  * k_rsample   projections of sampled z-normalised windows on random vectors,
//                the input of the r heuristic (section 6.1), FP64, sequential
//                per window so that every value is reproducible bit for bit.
//  * k_proj_*    the random projections a . x_hat of Eq. drp for every window
//                and every hash column, as one contraction per dimension:
//                V[c][a] = sum_t R[t][c] * x_hat_a[t]. The right operand is a
//                Hankel matrix (x_hat_a[t] comes from x[a + t]), staged once
//                per tile in LDS and normalised on load; the contraction runs
//                on MFMA; the epilogue quantises floor(v / r + U) and packs the
//                four one-byte symbols of a half-function into one word.
#include <hip/hip_runtime.h>

#include <hip/hip_bf16.h>
#include <stdint.h>

#include "internal.h"

namespace mm {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

// LDS staging of the FP32 projection rows: chunks of kRT32 steps of t, each
// a row of MB * 32 columns padded by 4 floats; the series tile in front of
// them is rounded up to 16 bytes.
constexpr int kRT32 = 16;
template <typename T, int WB>
__host__ __device__ inline size_t f32_series_bytes(int wpad)
{
    return ((size_t)(WB + wpad) * sizeof(T) + 15) / 16 * 16;
}


// ---------------------------------------------------------------------------
// Rolling statistics. Each thread owns kStatsChunk consecutive windows: the
// first by a direct two-pass sum, the rest by the sliding update
//   mu'  = mu + (x_in - x_out) / w
//   M2'  = M2 + (x_in - x_out) * ((x_in - mu') + (x_out - mu)).
// Windows whose sliding sigma is near zero relative to |mu|, or whose M2 fell
// far below the chunk's peak (cancellation), are recomputed directly with the
// plain two-pass definition, so the flat-window decision (sigma <= 1e-8 |mu|,
// normal form all zeros) is taken on exactly the definition's value.
// ---------------------------------------------------------------------------
constexpr int kStatsChunk = 15;   // odd: conflict-free strided LDS reads
constexpr int kStatsThreads = 256;

template <typename T>
__device__ inline void direct_stats(const T* xl, int w, double& mu, double& m2, double& sigma)
{
    double s = 0.0;
    for (int t = 0; t < w; ++t) s = s + (double)xl[t];
    mu = s / (double)w;
    double q = 0.0;
    for (int t = 0; t < w; ++t) {
        double dl = (double)xl[t] - mu;
        q = q + dl * dl;
    }
    m2 = q;
    sigma = sqrt(q / (double)w);
}

template <typename T>
__global__ __launch_bounds__(kStatsThreads) void k_stats(const T* __restrict__ x, int64_t n,
                                                         int64_t ns, int w,
                                                         double* __restrict__ mu_out,
                                                         double* __restrict__ isig_out)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* xs = reinterpret_cast<T*>(smem_raw);
    const int f = blockIdx.y;
    const int64_t a_blk = (int64_t)blockIdx.x * (kStatsThreads * kStatsChunk);
    const int nx = kStatsThreads * kStatsChunk + w - 1;
    const T* xf = x + (int64_t)f * n;
    for (int q = threadIdx.x; q < nx; q += kStatsThreads) {
        int64_t g = a_blk + q;
        xs[q] = g < n ? xf[g] : T(0);
    }
    __syncthreads();
    const int64_t a0 = a_blk + (int64_t)threadIdx.x * kStatsChunk;
    if (a0 >= ns) return;
    const T* xl = xs + threadIdx.x * kStatsChunk;
    double mu, m2, sigma;
    direct_stats(xl, w, mu, m2, sigma);
    double peak = m2;
    const double inv_w = 1.0 / (double)w;
    for (int c = 0; c < kStatsChunk; ++c) {
        const int64_t a = a0 + c;
        if (a >= ns) break;
        if (c > 0) {
            double xo = (double)xl[c - 1], xi = (double)xl[c - 1 + w];
            double dl = xi - xo;
            double mn = mu + dl * inv_w;
            m2 = m2 + dl * ((xi - mn) + (xo - mu));
            mu = mn;
            peak = fmax(peak, m2);
            double var = m2 * inv_w;
            sigma = var > 0.0 ? sqrt(var) : 0.0;
            if (!(sigma > 1e-6 * fabs(mu)) || m2 < 1e-9 * peak) {
                direct_stats(xl + c, w, mu, m2, sigma);
                peak = m2;
            }
        }
        const bool flat = sigma <= kFlatRel * fabs(mu);
        mu_out[(int64_t)f * ns + a] = mu;
        isig_out[(int64_t)f * ns + a] = flat ? 0.0 : 1.0 / sigma;
    }
}

// The first value of the series in [D][n] order that is NaN or infinite
// (the method is defined on real values), or ~0 when all are finite. Each
// thread visits its values in increasing index order and stops at its first
// such value, so the minimum over threads is the first overall.
template <typename T>
__global__ __launch_bounds__(256) void k_first_nonfinite(const T* __restrict__ x, int64_t total,
                                                        unsigned long long* __restrict__ first)
{
    unsigned long long mine = ~0ull;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride)
        if (!isfinite(x[i])) {
            mine = (unsigned long long)i;
            break;
        }
    if (mine != ~0ull) atomicMin(first, mine);
}

hipError_t launch_first_nonfinite(const void* x, int dtype, int64_t total, unsigned long long* first,
                                  hipStream_t s)
{
    const int64_t want = (total + 255) / 256;
    const unsigned blocks = (unsigned)(want < 2048 ? (want > 0 ? want : 1) : 2048);
    if (dtype == 0)
        hipLaunchKernelGGL(k_first_nonfinite<double>, dim3(blocks), dim3(256), 0, s, (const double*)x, total, first);
    else
        hipLaunchKernelGGL(k_first_nonfinite<float>, dim3(blocks), dim3(256), 0, s, (const float*)x, total, first);
    return hipGetLastError();
}

hipError_t launch_stats(const void* x, int dtype, int64_t n, int64_t ns, int D, int w, double* mu,
                        double* isig, hipStream_t s)
{
    const int per = kStatsThreads * kStatsChunk;
    dim3 grid((unsigned)((ns + per - 1) / per), (unsigned)D);
    if (dtype == 0) {
        size_t lds = (size_t)(per + w - 1) * sizeof(double);
        if (lds > 65536)
            (void)hipFuncSetAttribute((const void*)k_stats<double>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(k_stats<double>, grid, dim3(kStatsThreads), lds, s, (const double*)x, n,
                           ns, w, mu, isig);
    } else {
        size_t lds = (size_t)(per + w - 1) * sizeof(float);
        hipLaunchKernelGGL(k_stats<float>, grid, dim3(kStatsThreads), lds, s, (const float*)x, n,
                           ns, w, mu, isig);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// r heuristic input: for sampled windows (f, a) compute mu, sigma by the
// two-pass definition, the normal form (x - mu) / sigma (zeros if flat), and
// its dot product with each sample vector, all sequential in t, without
// fused multiply-add (the library is built with -ffp-contract=off).
// One wavefront takes G sampled windows, staged in LDS with coalesced loads
// when they fit, and one lane per (window, vector): the lanes of a window
// walk the same LDS words (broadcast reads), each with its own vector.
// Every lane computes its window's statistics itself, in the same order.
// ---------------------------------------------------------------------------
constexpr int kRsLds = 48 * 1024;   // LDS for the staged windows of one wavefront

template <typename T, bool staged>
__global__ __launch_bounds__(64) void k_rsample(const T* __restrict__ x, int64_t n, int D, int w,
                                                const int64_t* __restrict__ win, int S,
                                                const double* __restrict__ vec, int nvec, int VT,
                                                int G, double* __restrict__ dots)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* xs = reinterpret_cast<T*>(smem_raw);
    const int64_t total = (int64_t)D * S;
    const int64_t id0 = (int64_t)blockIdx.x * G;
    const int lane = threadIdx.x, slot = lane / VT, vi = lane - slot * VT;
    if constexpr (staged) {
        for (int g = 0; g < G; ++g) {
            const int64_t id = id0 + g;
            if (id >= total) break;
            const T* src = x + (id / S) * n + win[id];
            for (int t = lane; t < w; t += 64) xs[(size_t)g * w + t] = src[t];
        }
        __syncthreads();
    }
    const int64_t id = id0 + slot;
    if (slot >= G || id >= total) return;
    // (the staged window is read through the LDS array itself, so that its
    // loads are LDS loads rather than generic ones)
    const T* xa;
    if constexpr (staged) xa = xs + (size_t)slot * w;
    else xa = x + (id / S) * n + win[id];
    double mu, m2, sigma;
    direct_stats(xa, w, mu, m2, sigma);
    const bool flat = sigma <= kFlatRel * fabs(mu);
    for (int v = vi; v < nvec; v += VT) {
        const double* vv = vec + (int64_t)v * w;
        double dot = 0.0;
        for (int t = 0; t < w; ++t) {
            double z = flat ? 0.0 : ((double)xa[t] - mu) / sigma;
            dot = dot + vv[t] * z;
        }
        dots[id * nvec + v] = dot;
    }
}

hipError_t launch_rsample(const void* x, int dtype, int64_t n, int D, int w, const int64_t* win,
                          int S, const double* vec, int nvec, double* dots, hipStream_t s)
{
    const int64_t total = (int64_t)D * S;
    const size_t elem = dtype == 0 ? 8 : 4;
    // lanes per window (one per vector, up to 64) and windows per wavefront
    const int VT = nvec < 64 ? nvec : 64;
    int G = 64 / VT;
    while (G > 1 && (size_t)G * w * elem > (size_t)kRsLds) --G;
    const bool staged = (size_t)G * w * elem <= (size_t)kRsLds;
    const size_t lds = staged ? (size_t)G * w * elem : 0;
    dim3 grid((unsigned)((total + G - 1) / G));
    if (dtype == 0) {
        if (staged)
            hipLaunchKernelGGL((k_rsample<double, true>), grid, dim3(64), lds, s, (const double*)x, n, D, w,
                               win, S, vec, nvec, VT, G, dots);
        else
            hipLaunchKernelGGL((k_rsample<double, false>), grid, dim3(64), lds, s, (const double*)x, n, D, w,
                               win, S, vec, nvec, VT, G, dots);
    } else {
        if (staged)
            hipLaunchKernelGGL((k_rsample<float, true>), grid, dim3(64), lds, s, (const float*)x, n, D, w,
                               win, S, vec, nvec, VT, G, dots);
        else
            hipLaunchKernelGGL((k_rsample<float, false>), grid, dim3(64), lds, s, (const float*)x, n, D, w,
                               win, S, vec, nvec, VT, G, dots);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Quantise-and-pack epilogue: symbol = (floor(v / r + U) + 128) mod 256, four
// positions of one half-function in one word, position 0 most significant.
// (v / r + U equals (v + b) / r of Eq. drp with b = r U.)
// ---------------------------------------------------------------------------
__device__ inline uint32_t sym_of(float u)
{
    float h = floorf(fminf(fmaxf(u, -1.0e9f), 1.0e9f));
    return (uint32_t)(((int)h + 128) & 255);
}
__device__ inline uint32_t sym_of(double u)
{
    double h = floor(fmin(fmax(u, -1.0e9), 1.0e9));
    return (uint32_t)(((int)h + 128) & 255);
}

// The per-window statistics of a lane's NB windows (a0 + WS nb), loaded at
// the kernel's start with clamped indices (no branch, so the loads overlap
// the tile's); windows past the end get 0.
template <int NB, int WS>
__device__ inline void window_stats(const double* __restrict__ mu, const double* __restrict__ isig,
                                    int64_t a0, int64_t ns, double (&m)[NB], double (&sg)[NB])
{
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int64_t a = a0 + nb * WS;
        const int64_t ac = a < ns ? a : ns - 1;
        m[nb] = mu[ac];
        sg[nb] = isig[ac];
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
        if (a0 + nb * WS >= ns) m[nb] = sg[nb] = 0.0;
}

// The offsets U_f (Cpad values) copied into LDS by the first Cpad threads;
// the epilogue reads them there, so no global load waits behind its stores
// (the vector memory counter counts both).
template <typename U_T>
__device__ inline void stage_offsets(const U_T* __restrict__ Uf, int Cpad, U_T* us)
{
    if ((int)threadIdx.x < Cpad) us[threadIdx.x] = Uf[threadIdx.x];
}

// ---------------------------------------------------------------------------
// FP64 projection: v_mfma_f64_16x16x4f64. A (16 x 4): lane l holds
// A[l % 16][l / 16]; B (4 x 16) = x_hat^T: lane l holds B[l / 16][l % 16];
// D (16 x 16): lane l holds rows (l / 16) + 4 q, q = 0..3, of column l % 16
// (measured on gfx950). Row i of A therefore carries hash column
// 4 (i % 4) + i / 4, so that the four accumulators of a lane are the four
// positions of hash function (c0 + 4 (l / 16)) / 4 of window l % 16 and
// packing needs no data movement.
// Wave tile: all Cpad = 16 MB16 columns x 16 NB windows; block: 4 waves.
// ---------------------------------------------------------------------------
template <typename T, int MB16, int NB>
__global__ __launch_bounds__(256) void k_proj_f64(const T* __restrict__ x, int64_t n, int64_t ns,
                                                  int w, int wpad, const double* __restrict__ mu,
                                                  const double* __restrict__ isig,
                                                  const double* __restrict__ R,
                                                  const double* __restrict__ U, int Cpad, int NF,
                                                  int K, double inv_r, uint32_t* __restrict__ H)
{
    constexpr int WB = 4 * 16 * NB;   // windows per block
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* xs = reinterpret_cast<T*>(smem_raw);
    const int f = blockIdx.y;
    const int64_t a_blk = (int64_t)blockIdx.x * WB;
    const T* xf = x + (int64_t)f * n;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = lane & 15, kq = lane >> 4;
    const int wbase = wave * 16 * NB;
    double m_[NB], s_[NB];
    window_stats<NB, 16>(mu + (int64_t)f * ns, isig + (int64_t)f * ns, a_blk + wbase + col, ns, m_, s_);
    // the tile's loads in batches of eight per thread before the first use
    for (int q0 = 0; q0 < WB + wpad; q0 += 8 * 256) {
        T v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int q = q0 + u * 256 + (int)threadIdx.x;
            v[u] = q < WB + wpad && a_blk + q < n ? xf[a_blk + q] : T(0);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int q = q0 + u * 256 + (int)threadIdx.x;
            if (q < WB + wpad) xs[q] = v[u];
        }
    }
    double* us = reinterpret_cast<double*>(smem_raw + ((size_t)(WB + wpad) * sizeof(T) + 15) / 16 * 16);   // [Cpad]
    stage_offsets(U + (int64_t)f * Cpad, Cpad, us);
    __syncthreads();
    const int acol = 4 * (col & 3) + (col >> 2);   // hash column carried by A row `col`
    doublex4 acc[MB16][NB];
#pragma unroll
    for (int mb = 0; mb < MB16; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = doublex4{0.0, 0.0, 0.0, 0.0};
    const double* Rf = R + (int64_t)f * wpad * Cpad;
    for (int t0 = 0; t0 < wpad; t0 += 4) {
        const int t = t0 + kq;
        double av[MB16], bv[NB];
#pragma unroll
        for (int mb = 0; mb < MB16; ++mb) av[mb] = Rf[(int64_t)t * Cpad + mb * 16 + acol];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
            bv[nb] = ((double)xs[wbase + nb * 16 + col + t] - m_[nb]) * s_[nb];
#pragma unroll
        for (int mb = 0; mb < MB16; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
                acc[mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[mb], bv[nb], acc[mb][nb], 0, 0, 0);
    }
    const int half = K / 2;
#pragma unroll
    for (int mb = 0; mb < MB16; ++mb) {
        const int c0 = mb * 16 + 4 * kq;
        const int F = c0 / 4;
        if (F >= NF) continue;
        const double* Uf = us + c0;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int64_t a = a_blk + wbase + nb * 16 + col;
            if (a >= ns) continue;
            uint32_t word = 0;
#pragma unroll
            for (int p = 0; p < 4; ++p)
                if (p < half) word |= sym_of(fma(acc[mb][nb][p], inv_r, Uf[p])) << (24 - 8 * p);
            H[((int64_t)f * NF + F) * ns + a] = word;
        }
    }
}

// ---------------------------------------------------------------------------
// FP32 projection: v_mfma_f32_32x32x2f32. A (32 x 2): lane l holds
// A[l % 32][l / 32]; B (2 x 32): B[l / 32][l % 32]; D (32 x 32): lane l holds
// D[8 (q / 4) + 4 (l / 32) + q % 4][l % 32], q = 0..15, so each group of four
// accumulators is the four positions of one hash function.
// The normal form is computed in FP64 and rounded once to FP32.
// ---------------------------------------------------------------------------
template <typename T, int MB, int NB>
__global__ __launch_bounds__(256, 2) void k_proj_f32(const T* __restrict__ x, int64_t n, int64_t ns,
                                                  int w, int wpad, const double* __restrict__ mu,
                                                  const double* __restrict__ isig,
                                                  const float* __restrict__ R,
                                                  const float* __restrict__ U, int Cpad, int NF,
                                                  int K, float inv_r, uint32_t* __restrict__ H)
{
    constexpr int WB = 4 * 32 * NB;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* xs = reinterpret_cast<T*>(smem_raw);
    const int f = blockIdx.y;
    const int64_t a_blk = (int64_t)blockIdx.x * WB;
    const T* xf = x + (int64_t)f * n;
    // the tile's loads in batches of eight per thread before the first use
    for (int q0 = 0; q0 < WB + wpad; q0 += 8 * 256) {
        T v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int q = q0 + u * 256 + (int)threadIdx.x;
            v[u] = q < WB + wpad && a_blk + q < n ? xf[a_blk + q] : T(0);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int q = q0 + u * 256 + (int)threadIdx.x;
            if (q < WB + wpad) xs[q] = v[u];
        }
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = lane & 31, kk = lane >> 5;
    const int wbase = wave * 32 * NB;
    double m_[NB], s_[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        int64_t a = a_blk + wbase + nb * 32 + col;
        m_[nb] = a < ns ? mu[(int64_t)f * ns + a] : 0.0;
        s_[nb] = a < ns ? isig[(int64_t)f * ns + a] : 0.0;
    }
    floatx16 acc[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[mb][nb][q] = 0.0f;
    // projection rows staged through LDS in chunks of kRT32 steps of t shared
    // by the block's waves, the next chunk fetched into registers meanwhile
    const float* Rf = R + (int64_t)f * wpad * Cpad;
    float* rs = reinterpret_cast<float*>(smem_raw + f32_series_bytes<T, WB>(wpad));   // 2 x [kRT32][MB*32 + 4]
    constexpr int RW = MB * 32 + 4;                          // padded row (floats)
    constexpr int PIECES = kRT32 * MB * 32 / 4;              // 16-byte pieces per chunk
    constexpr int ITEMS = (PIECES + 255) / 256;
    floatx4 pre[ITEMS];
    auto fetch = [&](int t0) {
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const int id = threadIdx.x + 256 * it, tr = id / (MB * 8), seg = id % (MB * 8);
            if (id < PIECES) pre[it] = *reinterpret_cast<const floatx4*>(Rf + (int64_t)(t0 + tr) * Cpad + 4 * seg);
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const int id = threadIdx.x + 256 * it, tr = id / (MB * 8), seg = id % (MB * 8);
            if (id < PIECES) *reinterpret_cast<floatx4*>(rs + ((size_t)buf * kRT32 + tr) * RW + 4 * seg) = pre[it];
        }
    };
    const int nchunks = wpad / kRT32;
    fetch(0);
    stash(0);
    __syncthreads();
    for (int c = 0; c < nchunks; ++c) {
        const int cur = c & 1;
        if (c + 1 < nchunks) fetch((c + 1) * kRT32);
        const float* rb = rs + (size_t)cur * kRT32 * RW;
#pragma unroll 2
        for (int tl0 = 0; tl0 < kRT32; tl0 += 2) {
            const int tl = tl0 + kk, t = c * kRT32 + tl;
            float av[MB], bv[NB];
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) av[mb] = rb[(size_t)tl * RW + mb * 32 + col];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
                bv[nb] = (float)(((double)xs[wbase + nb * 32 + col + t] - m_[nb]) * s_[nb]);
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[mb], bv[nb], acc[mb][nb], 0, 0, 0);
        }
        if (c + 1 < nchunks) stash(cur ^ 1);
        __syncthreads();
    }
    const int half = K / 2;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int c0 = mb * 32 + 8 * g + 4 * kk;
            const int F = c0 / 4;
            if (F >= NF) continue;
            const float* Uf = U + (int64_t)f * Cpad + c0;
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int64_t a = a_blk + wbase + nb * 32 + col;
                if (a >= ns) continue;
                uint32_t word = 0;
#pragma unroll
                for (int p = 0; p < 4; ++p)
                    if (p < half) word |= sym_of(fmaf(acc[mb][nb][4 * g + p], inv_r, Uf[p])) << (24 - 8 * p);
                H[((int64_t)f * NF + F) * ns + a] = word;
            }
        }
}

// ---------------------------------------------------------------------------
// Low-precision projections (BF16, FP8 e4m3) with FP32 accumulation. The
// normal form x_hat = (x - mu) / sigma is itself the per-window scaling: it is
// formed in FP32 from a tile-local offset (x - ref, mu - ref, so no large
// offset cancels) and rounded once to the MFMA input type. R is stored
// column-major ([c][t], t contiguous) in the same type.
//   bf16: v_mfma_f32_32x32x16_bf16, lane l holds k = 8 (l / 32) + q, q < 8;
//   fp8:  v_mfma_scale_f32_32x32x64_f8f6f4 (unit scales), lane l holds
//         k = 32 (l / 32) + q, q < 32;
// for row l % 32 of A and column l % 32 of B; D as in the FP32 kernel.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx2v __attribute__((ext_vector_type(2)));
typedef int intx8 __attribute__((ext_vector_type(8)));
typedef int intx4 __attribute__((ext_vector_type(4)));

// LDS staging of the low-precision projection rows: chunks of kRT (bf16) or
// kRT8 (fp8) steps of t, rows padded to kRS / kRS8 elements (16 bytes of
// padding against bank conflicts; every row start stays 16-byte aligned),
// followed by the Cpad offsets U_f.
constexpr int kRT = 64, kRS = kRT + 8;
constexpr int kRT8 = 64, kRS8 = kRT8 + 16;
__host__ __device__ inline size_t lowp_stage_bytes(int proj, int Cpad)
{
    return (proj == 2 ? (size_t)2 * Cpad * kRS * 2 : (size_t)2 * Cpad * kRS8) + (size_t)Cpad * sizeof(float);
}

// The series tile four times, copy s shifted left by s elements
// (xs4[s][i] = x[a_blk + i + s] - ref): the run of values x_hat_a[t .. t + 7]
// a lane needs starts at a multiple of four in copy a mod 4, so it arrives
// in aligned 16-byte reads. Copies lie XL apart, XL = WB + wpad rounded up to
// 8 mod 64 elements: the four lanes that read the same offset of different
// copies then hit different LDS banks.
__host__ __device__ inline int shifted_stride(int WB, int wpad) { return (WB + wpad + 63) / 64 * 64 + 8; }
// Loads are issued in batches of eight per thread before the first is
// used, so a work-group waits out one memory latency per batch rather than
// one per element it stages.
template <typename T>
__device__ inline double load_tile_shifted(const T* __restrict__ xf, int64_t n, int64_t a_blk, int XL, float* xs4)
{
    constexpr int PRE = 8;
    const double ref = (double)xf[a_blk < n ? a_blk : n - 1];
    for (int q0 = 0; q0 < XL; q0 += PRE * (int)blockDim.x) {
        T v[PRE];
#pragma unroll
        for (int u = 0; u < PRE; ++u) {
            const int q = q0 + u * (int)blockDim.x + (int)threadIdx.x;
            const int64_t g = a_blk + q;
            v[u] = q < XL && g < n ? xf[g] : T(0);
        }
#pragma unroll
        for (int u = 0; u < PRE; ++u) {
            const int q = q0 + u * (int)blockDim.x + (int)threadIdx.x;
            if (q >= XL) break;
            const float y = a_blk + q < n ? (float)((double)v[u] - ref) : 0.0f;
#pragma unroll
            for (int sh = 0; sh < 4; ++sh)
                if (q >= sh) xs4[sh * XL + q - sh] = y;
        }
    }
    return ref;
}

template <int MB, int NB>
__device__ inline void quantize_store(const floatx16 (&acc)[MB][NB], const float* Uf0,
                                      int64_t a0, int col, int kk, int64_t ns, int NF, int K,
                                      float inv_r, uint32_t* __restrict__ Hf)
{
    // sym_of for four positions at once, in few VALU operations: the clamp
    // is one median, floor and conversion one instruction, and since
    // (h + 128) mod 256 is the low byte of h with its top bit flipped, the
    // four low bytes are gathered by two byte permutes and flipped by one
    // XOR; positions past K / 2 are masked to zero.
    const int half = K / 2;
    const uint32_t keep = half >= 4 ? 0xFFFFFFFFu : ~(0xFFFFFFFFu >> (8 * half));
    const uint32_t flip = 0x80808080u & keep;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int c0 = mb * 32 + 8 * g + 4 * kk;
            const int F = c0 / 4;
            if (F >= NF) continue;
            const float4 u4 = *reinterpret_cast<const float4*>(Uf0 + c0);
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int64_t a = a0 + nb * 32 + col;
                if (a >= ns) continue;
                int h[4];
                const float uu[4] = {u4.x, u4.y, u4.z, u4.w};
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    const float v = __builtin_amdgcn_fmed3f(fmaf(acc[mb][nb][4 * g + p], inv_r, uu[p]), -1.0e9f, 1.0e9f);
                    h[p] = (int)floorf(v);
                }
                // byte 3 <- h0, byte 2 <- h1, byte 1 <- h2, byte 0 <- h3
                const uint32_t lo = __builtin_amdgcn_perm((uint32_t)h[2], (uint32_t)h[3], 0x0c0c0400u);
                const uint32_t hi = __builtin_amdgcn_perm((uint32_t)h[0], (uint32_t)h[1], 0x04000c0cu);
                Hf[(int64_t)F * ns + a] = ((lo | hi) & keep) ^ flip;
            }
        }
}

template <typename T, int MB, int NB, int WAVES>
__global__ __launch_bounds__(64 * WAVES, 8 / WAVES) void k_proj_bf16(const T* __restrict__ x, int64_t n, int64_t ns,
                                                   int w, int wpad, const double* __restrict__ mu,
                                                   const double* __restrict__ isig,
                                                   const __bf16* __restrict__ R,
                                                   const float* __restrict__ U, int Cpad, int NF,
                                                   int K, float inv_r, uint32_t* __restrict__ H)
{
    constexpr int WB = WAVES * 32 * NB, NT = 64 * WAVES;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float* xs4 = reinterpret_cast<float*>(smem_raw);
    const int XL = shifted_stride(WB, wpad);
    const int f = blockIdx.y;
    const int64_t a_blk = (int64_t)blockIdx.x * WB;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = lane & 31, kk = lane >> 5;
    const int wbase = wave * 32 * NB;
    double m_[NB], s_[NB];
    window_stats<NB, 32>(mu + (int64_t)f * ns, isig + (int64_t)f * ns, a_blk + wbase + col, ns, m_, s_);
    const double ref = load_tile_shifted<T>(x + (int64_t)f * n, n, a_blk, XL, xs4);
    float sc[NB], off[NB];
    const float* xb[NB];   // this lane's Hankel run: copy col mod 4, aligned
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        sc[nb] = (float)s_[nb];
        off[nb] = (float)(-(m_[nb] - ref) * s_[nb]);
        xb[nb] = xs4 + (col & 3) * XL + wbase + nb * 32 + (col & ~3) + 8 * kk;
    }
    floatx16 acc[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[mb][nb][q] = 0.0f;
    // The projection rows are staged through LDS in chunks of kRT steps of t,
    // shared by the block's four waves (each would otherwise re-read them
    // from L2 for its own 64 windows); the next chunk is fetched into
    // registers while the current one feeds the MFMAs.
    const __bf16* Rf = R + (int64_t)f * Cpad * wpad;
    __bf16* rs = reinterpret_cast<__bf16*>(xs4 + 4 * XL);      // 2 x [MB * 32][kRS]
    constexpr int PIECES = MB * 32 * (kRT / 8);                // 16-byte pieces per chunk
    constexpr int ITEMS = (PIECES + NT - 1) / NT;
    bf16x8 pre[ITEMS];
    auto fetch = [&](int t0) {
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const int id = threadIdx.x + NT * it, row = id / (kRT / 8), seg = id % (kRT / 8);
            if (id < PIECES) pre[it] = *reinterpret_cast<const bf16x8*>(Rf + (int64_t)row * wpad + t0 + 8 * seg);
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const int id = threadIdx.x + NT * it, row = id / (kRT / 8), seg = id % (kRT / 8);
            if (id < PIECES) *reinterpret_cast<bf16x8*>(rs + ((size_t)buf * MB * 32 + row) * kRS + 8 * seg) = pre[it];
        }
    };
    float* us = reinterpret_cast<float*>(rs + (size_t)2 * MB * 32 * kRS);   // [MB * 32]
    stage_offsets(U + (int64_t)f * Cpad, MB * 32, us);
    const int nchunks = wpad / kRT;
    fetch(0);
    stash(0);
    __syncthreads();
    constexpr int NST = kRT / 16;   // MFMA steps of 16 t per chunk
    // Hankel reuse: window block nb at step s reads the run of block 0 at
    // step s + 2 nb (its windows start 32 nb later), so one fragment
    // F(s) = 8 values at xb[0] + 16 s serves block 0 at step s and block 1 at
    // step s - 2. Fragments live in a ring of four (slot s mod 4); F(s + 3)
    // is read during step s.
    static_assert(NB == 2, "the fragment ring assumes two window blocks");
    const int S = nchunks * NST;   // steps in all; block 1 reads up to F(S + 1)
    float4 fr[4][2];
    auto load_frag = [&](int sg, int slot) {
        const float4* xp = reinterpret_cast<const float4*>(__builtin_assume_aligned(xb[0] + 16 * sg, 16));
        fr[slot][0] = xp[0];
        fr[slot][1] = xp[1];
    };
    load_frag(0, 0);
    load_frag(1, 1);
    load_frag(2, 2);
    for (int c = 0; c < nchunks; ++c) {
        const int cur = c & 1;
        if (c + 1 < nchunks) fetch((c + 1) * kRT);
        const __bf16* rb = rs + (size_t)cur * MB * 32 * kRS + (size_t)col * kRS + 8 * kk;
        // projection rows of step st + 1 are read from LDS while step st runs
        bf16x8 av[2][MB];
        auto load_rows = [&](int st, int slot) {
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
                av[slot][mb] = *reinterpret_cast<const bf16x8*>(rb + (size_t)mb * 32 * kRS + st * 16);
        };
        load_rows(0, 0);
#pragma unroll
        for (int st = 0; st < NST; ++st) {
            const int sl = st & 1;
            const int sg = c * NST + st;
            if (st + 1 < NST) load_rows(st + 1, sl ^ 1);
            if (sg + 3 <= S + 1) load_frag(sg + 3, (st + 3) & 3);
            bf16x8 bv[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                // x_hat in FP32, rounded to bf16 two at a time
                const int slot = (st + 2 * nb) & 3;
                const float4 lo = fr[slot][0], hi = fr[slot][1];
                const float s0 = sc[nb], o0 = off[nb];
                const bf16x2 p0 = __builtin_convertvector((floatx2v){fmaf(lo.x, s0, o0), fmaf(lo.y, s0, o0)}, bf16x2);
                const bf16x2 p1 = __builtin_convertvector((floatx2v){fmaf(lo.z, s0, o0), fmaf(lo.w, s0, o0)}, bf16x2);
                const bf16x2 p2 = __builtin_convertvector((floatx2v){fmaf(hi.x, s0, o0), fmaf(hi.y, s0, o0)}, bf16x2);
                const bf16x2 p3 = __builtin_convertvector((floatx2v){fmaf(hi.z, s0, o0), fmaf(hi.w, s0, o0)}, bf16x2);
                bv[nb] = __builtin_shufflevector(__builtin_shufflevector(p0, p1, 0, 1, 2, 3),
                                                 __builtin_shufflevector(p2, p3, 0, 1, 2, 3), 0, 1, 2, 3, 4, 5, 6, 7);
            }
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[sl][mb], bv[nb], acc[mb][nb], 0, 0, 0);
        }
        if (c + 1 < nchunks) stash(cur ^ 1);
        __syncthreads();
    }
    quantize_store<MB, NB>(acc, us, a_blk + wbase, col, kk, ns, NF, K, inv_r, H + (int64_t)f * NF * ns);
}

template <typename T, int MB, int NB, int WAVES>
__global__ __launch_bounds__(64 * WAVES, 8 / WAVES) void k_proj_fp8(const T* __restrict__ x, int64_t n, int64_t ns,
                                                  int w, int wpad, const double* __restrict__ mu,
                                                  const double* __restrict__ isig,
                                                  const uint8_t* __restrict__ R,
                                                  const float* __restrict__ U, int Cpad, int NF,
                                                  int K, float inv_r, uint32_t* __restrict__ H)
{
    constexpr int WB = WAVES * 32 * NB, NT = 64 * WAVES;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float* xs4 = reinterpret_cast<float*>(smem_raw);
    const int XL = shifted_stride(WB, wpad);
    const int f = blockIdx.y;
    const int64_t a_blk = (int64_t)blockIdx.x * WB;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = lane & 31, kk = lane >> 5;
    const int wbase = wave * 32 * NB;
    double m_[NB], s_[NB];
    window_stats<NB, 32>(mu + (int64_t)f * ns, isig + (int64_t)f * ns, a_blk + wbase + col, ns, m_, s_);
    const double ref = load_tile_shifted<T>(x + (int64_t)f * n, n, a_blk, XL, xs4);
    float sc[NB], off[NB];
    const float* xb[NB];   // this lane's Hankel run: copy col mod 4, aligned
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        sc[nb] = (float)s_[nb];
        off[nb] = (float)(-(m_[nb] - ref) * s_[nb]);
        xb[nb] = xs4 + (col & 3) * XL + wbase + nb * 32 + (col & ~3) + 32 * kk;
    }
    floatx16 acc[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[mb][nb][q] = 0.0f;
    // projection rows staged through LDS as in the bf16 kernel (kRT8 steps of
    // t per chunk, one byte each)
    const uint8_t* Rf = R + (int64_t)f * Cpad * wpad;
    uint8_t* rs = reinterpret_cast<uint8_t*>(xs4 + 4 * XL);     // 2 x [MB * 32][kRS8]
    constexpr int PIECES = MB * 32 * (kRT8 / 16);               // 16-byte pieces per chunk
    constexpr int ITEMS = (PIECES + NT - 1) / NT;
    intx4 pre[ITEMS];
    auto fetch = [&](int t0) {
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const int id = threadIdx.x + NT * it, row = id / (kRT8 / 16), seg = id % (kRT8 / 16);
            if (id < PIECES) pre[it] = *reinterpret_cast<const intx4*>(Rf + (int64_t)row * wpad + t0 + 16 * seg);
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const int id = threadIdx.x + NT * it, row = id / (kRT8 / 16), seg = id % (kRT8 / 16);
            if (id < PIECES) *reinterpret_cast<intx4*>(rs + ((size_t)buf * MB * 32 + row) * kRS8 + 16 * seg) = pre[it];
        }
    };
    float* us = reinterpret_cast<float*>(rs + (size_t)2 * MB * 32 * kRS8);   // [MB * 32]
    stage_offsets(U + (int64_t)f * Cpad, MB * 32, us);
    const int nchunks = wpad / kRT8;
    fetch(0);
    stash(0);
    __syncthreads();
    for (int c = 0; c < nchunks; ++c) {
        const int cur = c & 1;
        if (c + 1 < nchunks) fetch((c + 1) * kRT8);
        const uint8_t* rb = rs + (size_t)cur * MB * 32 * kRS8;
#pragma unroll
        for (int st = 0; st < kRT8 / 64; ++st) {
        const int tl = st * 64 + 32 * kk;
        intx8 av[MB], bv[NB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
            av[mb] = *reinterpret_cast<const intx8*>(rb + (size_t)(mb * 32 + col) * kRS8 + tl);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const float4* xp = reinterpret_cast<const float4*>(
                __builtin_assume_aligned(xb[nb] + c * kRT8 + st * 64, 16));
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float4 v4 = xp[q];
                int v = __builtin_amdgcn_cvt_pk_fp8_f32(fmaf(v4.x, sc[nb], off[nb]),
                                                        fmaf(v4.y, sc[nb], off[nb]), 0, false);
                v = __builtin_amdgcn_cvt_pk_fp8_f32(fmaf(v4.z, sc[nb], off[nb]),
                                                    fmaf(v4.w, sc[nb], off[nb]), v, true);
                bv[nb][q] = v;
            }
        }
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
                acc[mb][nb] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av[mb], bv[nb], acc[mb][nb],
                                                                             0, 0, 0, 127, 0, 127);
        }
        if (c + 1 < nchunks) stash(cur ^ 1);
        __syncthreads();
    }
    quantize_store<MB, NB>(acc, us, a_blk + wbase, col, kk, ns, NF, K, inv_r, H + (int64_t)f * NF * ns);
}

// Both low-precision kernels take four waves of 64 windows per work-group.
constexpr int kLowpWB = 4 * 32 * 2;

size_t lowp_lds_bytes(int proj, int Cpad, int wpad)
{
    return (size_t)4 * shifted_stride(kLowpWB, wpad) * sizeof(float) + lowp_stage_bytes(proj, Cpad);
}

template <typename T, int MB>
static hipError_t go_lowp(int proj, const T* x, int64_t n, int64_t ns, int D, int w, int wpad,
                          const double* mu, const double* isig, const void* R, const float* U,
                          int Cpad, int NF, int K, float inv_r, uint32_t* H, hipStream_t s)
{
    // windows per wave: 64 (two 32-wide MFMA columns share each projection
    // operand read from LDS); four waves per work-group and two work-groups
    // per CU: eight-wave groups and a lower occupancy measured slower, and
    // fp8 with 32 windows per wave and three work-groups per CU 4% slower
    constexpr int WAVES = 4;
    const size_t lds = lowp_lds_bytes(proj, MB * 32, wpad);
    if (lds > kMaxLdsBytes) return hipErrorInvalidValue;   // refused when the plan is made
    if (proj == 2) {
        constexpr int NB = 2, WB = WAVES * 32 * NB;
        static_assert(WB == kLowpWB, "tile width");
        dim3 grid((unsigned)((ns + WB - 1) / WB), (unsigned)D);
        if (lds > 65536)
            (void)hipFuncSetAttribute((const void*)k_proj_bf16<T, MB, NB, WAVES>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL((k_proj_bf16<T, MB, NB, WAVES>), grid, dim3(64 * WAVES), lds, s, x, n, ns, w, wpad, mu,
                           isig, (const __bf16*)R, U, Cpad, NF, K, inv_r, H);
    } else {
        constexpr int NB = 2, WB = WAVES * 32 * NB;
        static_assert(WB == kLowpWB, "tile width");
        dim3 grid((unsigned)((ns + WB - 1) / WB), (unsigned)D);
        if (lds > 65536)
            (void)hipFuncSetAttribute((const void*)k_proj_fp8<T, MB, NB, WAVES>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL((k_proj_fp8<T, MB, NB, WAVES>), grid, dim3(64 * WAVES), lds, s, x, n, ns, w, wpad, mu,
                           isig, (const uint8_t*)R, U, Cpad, NF, K, inv_r, H);
    }
    return hipGetLastError();
}

template <typename T, int MB16>
static hipError_t go_f64(const T* x, int64_t n, int64_t ns, int D, int w, int wpad, const double* mu,
                         const double* isig, const double* R, const double* U, int Cpad, int NF,
                         int K, double inv_r, uint32_t* H, hipStream_t s)
{
    constexpr int NB = 2, WB = 4 * 16 * NB;
    dim3 grid((unsigned)((ns + WB - 1) / WB), (unsigned)D);
    size_t lds = ((size_t)(WB + wpad) * sizeof(T) + 15) / 16 * 16 + (size_t)Cpad * sizeof(double);
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void*)k_proj_f64<T, MB16, NB>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k_proj_f64<T, MB16, NB>), grid, dim3(256), lds, s, x, n, ns, w, wpad, mu,
                       isig, R, U, Cpad, NF, K, inv_r, H);
    return hipGetLastError();
}

template <typename T, int MB>
static hipError_t go_f32(const T* x, int64_t n, int64_t ns, int D, int w, int wpad, const double* mu,
                         const double* isig, const float* R, const float* U, int Cpad, int NF,
                         int K, float inv_r, uint32_t* H, hipStream_t s)
{
    constexpr int NB = 2, WB = 4 * 32 * NB;
    dim3 grid((unsigned)((ns + WB - 1) / WB), (unsigned)D);
    size_t lds = f32_series_bytes<T, WB>(wpad) + (size_t)2 * kRT32 * (MB * 32 + 4) * sizeof(float);
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void*)k_proj_f32<T, MB, NB>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k_proj_f32<T, MB, NB>), grid, dim3(256), lds, s, x, n, ns, w, wpad, mu,
                       isig, R, U, Cpad, NF, K, inv_r, H);
    return hipGetLastError();
}

template <typename T>
static hipError_t dispatch(int proj, const T* x, int64_t n, int64_t ns, int D, int w,
                           const double* mu, const double* isig, const void* R, const void* U,
                           int Cpad, int wpad, int NF, int K, double inv_r, uint32_t* H,
                           hipStream_t s)
{
    const int MB = Cpad / 32;   // Cpad is a multiple of 32, at most 128
    if (proj == 0) {
        const double* Rd = (const double*)R;
        const double* Ud = (const double*)U;
        switch (MB) {
        case 1: return go_f64<T, 2>(x, n, ns, D, w, wpad, mu, isig, Rd, Ud, Cpad, NF, K, inv_r, H, s);
        case 2: return go_f64<T, 4>(x, n, ns, D, w, wpad, mu, isig, Rd, Ud, Cpad, NF, K, inv_r, H, s);
        case 3: return go_f64<T, 6>(x, n, ns, D, w, wpad, mu, isig, Rd, Ud, Cpad, NF, K, inv_r, H, s);
        case 4: return go_f64<T, 8>(x, n, ns, D, w, wpad, mu, isig, Rd, Ud, Cpad, NF, K, inv_r, H, s);
        }
    } else if (proj == 1) {
        const float* Rf = (const float*)R;
        const float* Uf = (const float*)U;
        const float ir = (float)inv_r;
        switch (MB) {
        case 1: return go_f32<T, 1>(x, n, ns, D, w, wpad, mu, isig, Rf, Uf, Cpad, NF, K, ir, H, s);
        case 2: return go_f32<T, 2>(x, n, ns, D, w, wpad, mu, isig, Rf, Uf, Cpad, NF, K, ir, H, s);
        case 3: return go_f32<T, 3>(x, n, ns, D, w, wpad, mu, isig, Rf, Uf, Cpad, NF, K, ir, H, s);
        case 4: return go_f32<T, 4>(x, n, ns, D, w, wpad, mu, isig, Rf, Uf, Cpad, NF, K, ir, H, s);
        }
    } else if (proj == 2 || proj == 3) {
        const float* Uf = (const float*)U;
        const float ir = (float)inv_r;
        switch (MB) {
        case 1: return go_lowp<T, 1>(proj, x, n, ns, D, w, wpad, mu, isig, R, Uf, Cpad, NF, K, ir, H, s);
        case 2: return go_lowp<T, 2>(proj, x, n, ns, D, w, wpad, mu, isig, R, Uf, Cpad, NF, K, ir, H, s);
        case 3: return go_lowp<T, 3>(proj, x, n, ns, D, w, wpad, mu, isig, R, Uf, Cpad, NF, K, ir, H, s);
        case 4: return go_lowp<T, 4>(proj, x, n, ns, D, w, wpad, mu, isig, R, Uf, Cpad, NF, K, ir, H, s);
        }
    }
    return hipErrorNotSupported;
}

hipError_t launch_proj(int proj, const void* x, int dtype, int64_t n, int64_t ns, int D, int w,
                       const double* mu, const double* isig, const void* R, const void* U,
                       int Cpad, int wpad, int NF, int K, double inv_r, uint32_t* H, hipStream_t s)
{
    if (dtype == 0)
        return dispatch<double>(proj, (const double*)x, n, ns, D, w, mu, isig, R, U, Cpad, wpad,
                                NF, K, inv_r, H, s);
    return dispatch<float>(proj, (const float*)x, n, ns, D, w, mu, isig, R, U, Cpad, wpad, NF, K,
                           inv_r, H, s);
}

}  // namespace mm

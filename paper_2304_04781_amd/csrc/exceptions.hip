// Exact storage of the largest-range patches alongside the autoencoder latents
// (error bounding): per compressed state, select the K patches with the largest
// e-field range r (resolved to bins 2^-5 wide in relative terms; within the bin
// that holds the K-th largest range, lower patch indices first), keep their e
// values, and restore them after decompression. The time scheme does the same
// per window and source with its e-only vectors (4^3 cells x 32 levels).

#include "ae_internal.h"

namespace wv {
namespace {

constexpr int SEL_THREADS = 1024;
constexpr int SEL_CHUNK = 16 * SEL_THREADS;  // keys staged in LDS per pass of the selector

// inclusive block scan of one int per thread: lane scans within each wave, one
// wave scans the wave totals (two barriers); ws holds SEL_THREADS / 64 ints
__device__ int block_scan_incl(int v, int* ws)
{
    constexpr int NW = SEL_THREADS / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) ws[wave] = x;
    __syncthreads();
    if (wave == 0) {
        const int w = lane < NW ? ws[lane] : 0;
        int t = w;
#pragma unroll
        for (int o = 1; o < NW; o <<= 1) {
            const int y = __shfl_up(t, o, 64);
            if (lane >= o) t += y;
        }
        if (lane < NW) ws[lane] = t - w;  // exclusive offsets of the waves
    }
    __syncthreads();
    const int r = x + ws[wave];
    __syncthreads();  // ws may be reused by the next scan
    return r;
}

// keys: r_e = meta[p*8 + 1] > 0, ordered as uint32 bit patterns; bin = top bits
// (bins 2^-5 wide in relative terms). One work-group: an LDS histogram of the
// bins, the bin b holding the K-th largest key, then a list, in increasing patch
// order, of every patch in a bin above b and the first K - #{bin > b} patches of
// bin b. Being a single work-group it is meant to run beside other work.
constexpr int BIN_SHIFT = EXC_BIN_SHIFT;
constexpr int NBIN = EXC_NBIN;

// r of row p sits at meta[p * ms + 1]: ms = 8 for patches ((lo, r) of 4 fields, e
// first), 2 for the e-only vectors of the time scheme; with 16-bit metadata at
// meta16[p * ms + 1] as bfloat16 bits (the upper half of the same float)
__device__ __forceinline__ unsigned bin_of(const float* meta, const uint16_t* meta16, int ms, int p)
{
    const unsigned u = meta16 ? (unsigned)meta16[(long long)p * ms + 1] << 16
                              : __float_as_uint(meta[(long long)p * ms + 1]);
    return u >> BIN_SHIFT;
}

__global__ void __launch_bounds__(SEL_THREADS) select_kernel(const float* __restrict__ meta,
                                                             const uint16_t* __restrict__ meta16, int ms, int P, int K,
                                                             int* __restrict__ out)
{
    constexpr int BPT = NBIN / SEL_THREADS;  // bins per thread, highest bins to thread 0
    constexpr int KPT = SEL_CHUNK / SEL_THREADS;
    __shared__ int ws[SEL_THREADS / 64];
    __shared__ int s_bin, s_rem, s_tot[2];
    __shared__ unsigned hist[NBIN];
    __shared__ unsigned skey[SEL_THREADS * (KPT + 1)];
    const int tid = threadIdx.x, lane = tid & 63;
#pragma unroll
    for (int q = 0; q < BPT; ++q) hist[q * SEL_THREADS + tid] = 0u;
    __syncthreads();
    // histogram; a wave whose keys all agree (typically the floor value) adds once
    for (int c0 = 0; c0 < P; c0 += SEL_CHUNK) {
        unsigned key[KPT];
#pragma unroll
        for (int q = 0; q < KPT; ++q) {
            const int p = c0 + q * SEL_THREADS + tid;
            key[q] = p < P ? bin_of(meta, meta16, ms, p) : 0xFFFFFFFFu;
        }
#pragma unroll
        for (int q = 0; q < KPT; ++q) {
            const unsigned k0 = __shfl(key[q], 0, 64);
            if (__all(key[q] == k0)) {
                if (lane == 0 && k0 != 0xFFFFFFFFu) atomicAdd(&hist[k0], 64u);
            } else if (key[q] != 0xFFFFFFFFu) {
                atomicAdd(&hist[key[q]], 1u);
            }
        }
    }
    __syncthreads();
    // threshold bin: the bin holding the K-th largest key
    const int top = NBIN - BPT * (tid + 1);  // lowest bin of this thread's range
    unsigned hv[BPT];
    int c = 0;
#pragma unroll
    for (int q = 0; q < BPT; ++q) {
        hv[q] = hist[top + q];
        c += (int)hv[q];
    }
    const int above = block_scan_incl(c, ws) - c;  // keys in bins above this thread's range
    if (above < K && above + c >= K) {
        int cum = above;
        bool done = false;
#pragma unroll
        for (int q = BPT - 1; q >= 0; --q) {
            if (!done && cum + (int)hv[q] >= K) {
                s_bin = top + q;
                s_rem = K - cum;
                done = true;
            }
            cum += (int)hv[q];
        }
    }
    __syncthreads();
    const unsigned b = (unsigned)s_bin;
    const int rem = s_rem;
    // list in patch order, chunk by chunk: keys are staged in LDS with coalesced
    // loads, then each thread takes a contiguous run of KPT of them (padded layout:
    // run t starts at word (KPT + 1) t, so the runs fall in different banks)
    int base = 0, eqs = 0;  // picks written and ties seen before the chunk
    for (int c0 = 0; c0 < P; c0 += SEL_CHUNK) {
#pragma unroll
        for (int q = 0; q < KPT; ++q) {
            const int i = q * SEL_THREADS + tid;  // coalesced
            const int p = c0 + i;
            skey[(i / KPT) * (KPT + 1) + i % KPT] = p < P ? bin_of(meta, meta16, ms, p) : 0u;
        }
        __syncthreads();
        const int r0 = tid * KPT;  // run of this thread within the chunk
        int gt = 0, eq = 0;
#pragma unroll
        for (int q = 0; q < KPT; ++q) {
            const bool ok = c0 + r0 + q < P;
            const unsigned bp = skey[tid * (KPT + 1) + q];
            gt += ok && bp > b;
            eq += ok && bp == b;
        }
        const int eq_all = block_scan_incl(eq, ws);  // ties of the chunk up to and including this run
        const int eq_before = eqs + eq_all - eq;
        const int take_eq = max(0, min(eq, rem - eq_before));
        const int sel = gt + take_eq;
        const int sel_incl = block_scan_incl(sel, ws);
        int pos = base + sel_incl - sel;
        int eq_seen = 0;
#pragma unroll
        for (int q = 0; q < KPT; ++q) {
            const int p = c0 + r0 + q;
            const unsigned bp = skey[tid * (KPT + 1) + q];
            bool pick = p < P && bp > b;
            if (p < P && bp == b) {
                pick = eq_seen < take_eq;
                ++eq_seen;
            }
            if (pick) out[pos++] = p;
        }
        // chunk totals from the last thread
        if (tid == SEL_THREADS - 1) {
            s_tot[0] = sel_incl;
            s_tot[1] = eq_all;
        }
        __syncthreads();
        base += s_tot[0];
        eqs += s_tot[1];
        __syncthreads();  // skey and s_tot are rewritten by the next chunk
    }
}

// exc[k][l] = e of patch idx[k] at local cell l (one block per patch)
__global__ void gather_kernel(const float* __restrict__ state, int ny, int nx, int Py, int Px, int P,
                              const int* __restrict__ idx, float* __restrict__ exc)
{
    const int k = blockIdx.x, l = threadIdx.x;
    const int p = idx[k];
    if (p < 0 || p >= P) return;
    const int px = p % Px, py = (p / Px) % Py, pz = p / (Px * Py);
    const long long z = pz * 8 + (l >> 6), y = py * 8 + ((l >> 3) & 7), x = px * 8 + (l & 7);
    exc[(long long)k * 512 + l] = state[(z * ny + y) * nx + x];
}

__global__ void scatter_kernel(float* __restrict__ e, int ny, int nx, int Py, int Px, int P,
                               const int* __restrict__ idx, const float* __restrict__ exc)
{
    const int k = blockIdx.x, l = threadIdx.x;
    const int p = idx[k];
    if (p < 0 || p >= P) return;
    const int px = p % Px, py = (p / Px) % Py, pz = p / (Px * Py);
    const long long z = pz * 8 + (l >> 6), y = py * 8 + ((l >> 3) & 7), x = px * 8 + (l & 7);
    e[(z * ny + y) * nx + x] = exc[(long long)k * 512 + l];
}

// time scheme: exc[k][t*64 + cell] = e of block idx[k] of source s at level t (the
// last valid level for t >= nvalid), one work-group of 256 per vector, thread i
// holding level i / 8 and cells 8 (i % 8) .. + 7 (the layout of the vectors)
__global__ void time_gather_kernel(const float* __restrict__ e_win, int S, int s, int ny, int nx, long long N,
                                   int By, int Bx, long long B, int nvalid, const int* __restrict__ idx,
                                   float* __restrict__ exc)
{
    const long long b = idx[blockIdx.x];
    if (b < 0 || b >= B) return;
    const int bx = (int)(b % Bx), by = (int)((b / Bx) % By), bz = (int)(b / ((long long)Bx * By));
    const int t = threadIdx.x >> 3, q = threadIdx.x & 7;
    const int tl = t < nvalid ? t : nvalid - 1;
    const int lz = q >> 1, ly0 = (q & 1) * 2;
    const float* src =
        e_win + ((long long)tl * S + s) * N + ((long long)(bz * 4 + lz) * ny + by * 4 + ly0) * nx + bx * 4;
    float* dst = exc + (long long)blockIdx.x * 2048 + t * 64 + q * 8;
    *reinterpret_cast<float4*>(dst) = *reinterpret_cast<const float4*>(src);
    *reinterpret_cast<float4*>(dst + 4) = *reinterpret_cast<const float4*>(src + nx);
}

// the inverse for levels t < nvalid: the exact values over the decoded window
__global__ void time_scatter_kernel(float* __restrict__ e_win, int S, int s, int ny, int nx, long long N, int By,
                                    int Bx, long long B, int nvalid, const int* __restrict__ idx,
                                    const float* __restrict__ exc)
{
    const long long b = idx[blockIdx.x];
    if (b < 0 || b >= B) return;
    const int t = threadIdx.x >> 3, q = threadIdx.x & 7;
    if (t >= nvalid) return;
    const int bx = (int)(b % Bx), by = (int)((b / Bx) % By), bz = (int)(b / ((long long)Bx * By));
    const int lz = q >> 1, ly0 = (q & 1) * 2;
    float* dst = e_win + ((long long)t * S + s) * N + ((long long)(bz * 4 + lz) * ny + by * 4 + ly0) * nx + bx * 4;
    const float* src = exc + (long long)blockIdx.x * 2048 + t * 64 + q * 8;
    *reinterpret_cast<float4*>(dst) = *reinterpret_cast<const float4*>(src);
    *reinterpret_cast<float4*>(dst + nx) = *reinterpret_cast<const float4*>(src + 4);
}

// rng[b] = lower bound of patch bm b in the increasing list idx [K]
__global__ void ranges_kernel(const int* __restrict__ idx, int K, int bm, int nb, int* __restrict__ rng)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b > nb) return;
    const long long target = (long long)b * bm;
    int lo = 0, hi = K;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (idx[mid] < target) lo = mid + 1;
        else hi = mid;
    }
    rng[b] = lo;
}

}  // namespace

void exceptions_select(const PatchGrid& pg, const float* meta, int K, int* idx, hipStream_t st,
                       const uint16_t* meta16)
{
    if (K <= 0) return;
    WV_REQUIRE(K <= pg.P, WV_EINVAL, "more exception patches than patches");
    WV_REQUIRE(pg.P < (1LL << 31), WV_EINVAL, "too many patches for the exception selector");
    hipLaunchKernelGGL(select_kernel, dim3(1), dim3(SEL_THREADS), 0, st, meta, meta16, 8, (int)pg.P, K, idx);
    WV_HIP(hipGetLastError());
}

void exceptions_gather(const PatchGrid& pg, const float* state, int K, const int* idx, float* exc, hipStream_t st)
{
    if (K <= 0) return;
    hipLaunchKernelGGL(gather_kernel, dim3(K), dim3(512), 0, st, state, pg.ny, pg.nx, pg.ny / 8, pg.nx / 8, (int)pg.P,
                       idx, exc);
    WV_HIP(hipGetLastError());
}

void exceptions_store(const PatchGrid& pg, const float* state, const float* meta, int K, int* idx, float* exc,
                      hipStream_t st, const uint16_t* meta16)
{
    if (K <= 0) return;
    exceptions_select(pg, meta, K, idx, st, meta16);
    exceptions_gather(pg, state, K, idx, exc, st);
}

void exceptions_ranges(const PatchGrid& pg, int K, const int* idx, int bm, int* rng, hipStream_t st)
{
    const int nb = (int)((pg.P + bm - 1) / bm);
    hipLaunchKernelGGL(ranges_kernel, dim3((nb + 1 + 255) / 256), dim3(256), 0, st, idx, K, bm, nb, rng);
    WV_HIP(hipGetLastError());
}

void exceptions_restore(const PatchGrid& pg, float* e, int K, const int* idx, const float* exc, hipStream_t st)
{
    if (K <= 0) return;
    hipLaunchKernelGGL(scatter_kernel, dim3(K), dim3(512), 0, st, e, pg.ny, pg.nx, pg.ny / 8, pg.nx / 8, (int)pg.P,
                       idx, exc);
    WV_HIP(hipGetLastError());
}

void time_exceptions_store(const TimeGrid& tg, const float* e_win, int s, int nvalid, const float* meta, int K,
                           int* idx, float* exc, hipStream_t st)
{
    if (K <= 0) return;
    WV_REQUIRE(K <= tg.B, WV_EINVAL, "more exception vectors than blocks");
    WV_REQUIRE(tg.B < (1LL << 31), WV_EINVAL, "too many blocks for the exception selector");
    hipLaunchKernelGGL(select_kernel, dim3(1), dim3(SEL_THREADS), 0, st, meta, nullptr, 2, (int)tg.B, K, idx);
    const long long N = (long long)tg.nz * tg.ny * tg.nx;
    hipLaunchKernelGGL(time_gather_kernel, dim3(K), dim3(256), 0, st, e_win, tg.S, s, tg.ny, tg.nx, N, tg.ny / 4,
                       tg.nx / 4, tg.B, nvalid, idx, exc);
    WV_HIP(hipGetLastError());
}

void time_exceptions_restore(const TimeGrid& tg, float* e_win, int s, int nvalid, int K, const int* idx,
                             const float* exc, hipStream_t st)
{
    if (K <= 0) return;
    const long long N = (long long)tg.nz * tg.ny * tg.nx;
    hipLaunchKernelGGL(time_scatter_kernel, dim3(K), dim3(256), 0, st, e_win, tg.S, s, tg.ny, tg.nx, N, tg.ny / 4,
                       tg.nx / 4, tg.B, nvalid, idx, exc);
    WV_HIP(hipGetLastError());
}

}  // namespace wv

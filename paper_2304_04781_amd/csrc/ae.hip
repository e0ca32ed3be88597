// Patch autoencoder on gfx950: per-vector normalisation, bfloat16 MFMA
// encoder/decoder with fused epilogues, FP8 latent quantisation, training
// (forward, backward, MSE loss, Adam) and the autoencoder C entry points.
//
// Network (paper Sec. 3.3, Eq. (single_layer), dense layers sigma(y W + b)):
//   encoder 2048 -> hid (GELU) -> lat,  decoder lat -> hid (GELU) -> 2048.
// Vectors (Sec. 3.1 space compression): one 8^3-cell patch of the 4 state
// fields, entry f*512 + lz*64 + ly*8 + lx; normalised per field slice by
// r = max(max - min, beta_f), y = (x - min)/r (Sec. 3.3.1).
//
// Precision: y, weights, hidden activations and latents are bfloat16 (RNE);
// products accumulate in float32 on the matrix cores; biases, GELU and the
// output are float32. FP8 latents are OCP E4M3FN codes with one float32 scale
// per patch, s = max|z| / 448; the decoder consumes bfloat16(code * s).

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "ae_internal.h"
#include "ae_math.h"

namespace wv {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// OCP E4M3FN, round to nearest even, saturating at 448
__device__ __forceinline__ uint8_t f2e4m3(float x)
{
    const uint32_t sign = (__float_as_uint(x) >> 24) & 0x80u;
    const float a = fabsf(x);
    uint32_t code;
    if (a >= 448.0f) {
        code = 0x7E;
    } else {
        const int e = (int)((__float_as_uint(a) >> 23) & 0xFF) - 127;
        if (e < -6) {
            code = (uint32_t)rintf(a * 512.0f);  // subnormal quantum 2^-9
        } else {
            const float q = rintf(ldexpf(a, 3 - e));  // in [8, 16]
            code = (uint32_t)((e + 7) << 3) + ((uint32_t)q - 8u);
        }
        if (code > 0x7E) code = 0x7E;
    }
    return (uint8_t)(code | sign);
}
__device__ __forceinline__ float e4m32f(uint8_t c)
{
    const int E = (c >> 3) & 0xF, m = c & 7;
    const float v = E == 0 ? (float)m * 0.001953125f : ldexpf(1.0f + (float)m * 0.125f, E - 7);
    return (c & 0x80) ? -v : v;
}

// ------------------------------------------------------------------------------------
// GEMM  C[M][N] = sum_k A(m, k) B(n, k), bf16 operands, fp32 accumulation.
// 256 threads = 4 waves; each wave owns a WM x WN block of 16x16 MFMA tiles.
// A and B tiles (BM x BK, BN x BK, k fastest) are staged through LDS by loaders
// that know the source layout; epilogues consume (row, col, value).
// ------------------------------------------------------------------------------------
constexpr int BK = 64;  // k per LDS stage: two 32-deep MFMA steps; depths below a multiple are zero-filled
// k-tiles in flight in the generic GEMM (128 x 128 work-group tiles, smaller ones)
#ifndef WV_GEMM_PF_BIG
#define WV_GEMM_PF_BIG 3
#endif
#ifndef WV_GEMM_PF_SMALL
#define WV_GEMM_PF_SMALL 4
#endif
constexpr int GEMM_PF_BIG = WV_GEMM_PF_BIG, GEMM_PF_SMALL = WV_GEMM_PF_SMALL;
static_assert(GEMM_PF_BIG >= 2 && GEMM_PF_SMALL >= 2, "at least the next k-tile in flight");
#ifndef WV_LDS_PAD
#define WV_LDS_PAD 8
#endif
constexpr int LDS_PAD = WV_LDS_PAD;  // bf16 elements of padding per LDS row

// registers holding one BR x BK tile between its global load and its LDS store:
// chunk c = tid + 256 i of 8 bf16 in v[i], kept where m[i] is all ones (zero elsewhere:
// past the last row or the depth limit); the mask is applied at the store, so the
// loaded registers are not waited for before then
template <int BR>
struct Frag {
    static constexpr int NC = (BR * (BK / 8) + 255) / 256;
    uint4 v[NC];
    unsigned m[NC];
};

// an epilogue with kTile = true takes the whole C tile from LDS: tile(m0, n0, rows, cols, C, ldc)
template <class E, class = void>
struct EpiHasTile {
    static constexpr bool value = false;
};
template <class E>
struct EpiHasTile<E, std::void_t<decltype(E::kTile)>> {
    static constexpr bool value = E::kTile;
};

// per-thread loader state of one work-group's tile rows, set before the k loop: the
// source row of each of its chunks (clamped to a valid row past the last one, with its
// bit in `ok` cleared), so every stage issues the same loads and only adds its k offset
template <int BR>
struct LoadState {
    const uint16_t* row[Frag<BR>::NC];
    unsigned ok;
};

// source stored [rows][ld] with k contiguous; optional row gather
struct LoadK {
    const uint16_t* p;
    long long ld;
    const int* rows;  // nullable: logical row r reads source row rows[r]
    int nrows;        // logical rows
    int k_total;
    template <int BR>
    __device__ __forceinline__ void prepare(int r0, int tid, LoadState<BR>& s) const
    {
        static_assert(BR * (BK / 8) % 256 == 0, "every thread owns whole chunks");
        s.ok = 0;
#pragma unroll
        for (int i = 0; i < Frag<BR>::NC; ++i) {
            const int c = tid + 256 * i;
            const int gr = r0 + c / (BK / 8);
            const bool ok = gr < nrows;
            const int rr = ok ? gr : 0;
            s.row[i] = p + (long long)(rows ? rows[rr] : rr) * ld;
            s.ok |= (unsigned)ok << i;
        }
    }
    // chunk (row, k0 + kc .. + 7) of every owned chunk, zero past the last row or at
    // depths >= klim; the load itself is always issued (at depth 0 of the row when the
    // chunk is out of range), so every stage has the same number of loads in flight
    template <int BR>
    __device__ __forceinline__ void fetch(const LoadState<BR>& s, int k0, int klim, int tid, Frag<BR>& f) const
    {
#pragma unroll
        for (int i = 0; i < Frag<BR>::NC; ++i) {
            const int kc = ((tid + 256 * i) % (BK / 8)) * 8;
            const bool in = ((s.ok >> i) & 1u) && k0 + kc < klim;
            f.v[i] = *reinterpret_cast<const uint4*>(s.row[i] + (in ? k0 + kc : 0));
            // the mask passes through an empty asm statement, so the compiler cannot tell
            // when the loaded value is unused and keeps the load unconditional
            unsigned m = in ? 0xFFFFFFFFu : 0u;
            asm volatile("" : "+v"(m));
            f.m[i] = m;
        }
    }
    template <int BR>
    __device__ __forceinline__ void store(const Frag<BR>& f, int tid, uint16_t (*lds)[BK + LDS_PAD]) const
    {
#pragma unroll
        for (int i = 0; i < Frag<BR>::NC; ++i) {
            const int c = tid + 256 * i;
            const unsigned m = f.m[i];
            *reinterpret_cast<uint4*>(&lds[c / (BK / 8)][(c % (BK / 8)) * 8]) =
                make_uint4(f.v[i].x & m, f.v[i].y & m, f.v[i].z & m, f.v[i].w & m);
        }
    }
};


template <int BM, int BN, int WM, int WN, class LA, class LB, class EPI>
__global__ void __launch_bounds__(256) gemm_kernel(int M, int N, int K, int k_per_split, LA la, LB lb, EPI epi)
{
    static_assert((BM / WM) * (BN / WN) == 4, "4 waves");
    constexpr int TM = WM / 16, TN = WN / 16;
    // two LDS stages: the next k-tile is loaded into registers while the MFMAs of the
    // current one run, and stored to the other stage after them. An epilogue that
    // writes whole tiles gets the C tile staged in the same memory afterwards.
    __shared__ __attribute__((aligned(16))) uint16_t smem[2 * (BM + BN) * (BK + LDS_PAD)];
    auto sA = reinterpret_cast<uint16_t(*)[BM][BK + LDS_PAD]>(smem);
    auto sB = reinterpret_cast<uint16_t(*)[BN][BK + LDS_PAD]>(smem + 2 * BM * (BK + LDS_PAD));

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wm0 = (wave / (BN / WN)) * WM, wn0 = (wave % (BN / WN)) * WN;
    // tiles in a 1D grid, column tiles fastest so the row tile of A is reused from L2 by
    // the work-groups that follow; with a multiple of 8 tiles each XCD (work-group id
    // mod 8) takes a contiguous run of tiles, so that reuse stays within one L2
    const int ntn = (N + BN - 1) / BN;
    const int ntiles = ntn * ((M + BM - 1) / BM);
    int bid = blockIdx.x;
    if (ntiles % 8 == 0) bid = (bid % 8) * (ntiles / 8) + bid / 8;
    const int m0 = (bid / ntn) * BM, n0 = (bid % ntn) * BN;
    const int kb = blockIdx.z * k_per_split;
    const int ke = min(K, kb + k_per_split);

    f32x4 acc[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int fr = lane & 15, fk = (lane >> 4) * 8;
    // PF k-tiles in flight: while tile i is multiplied from one LDS stage, tile i + 1 waits
    // in registers to be stored to the other and tiles up to i + PF - 1 are being loaded
    // (a ring of PF - 1 register fragments). Every stage issues the same loads (zeros past
    // this split's depth), so the compiler counts the loads in flight exactly and waits
    // only for the tile it stores.
    constexpr int PF = (BM >= 128 && BN >= 128) ? GEMM_PF_BIG : GEMM_PF_SMALL;
    Frag<BM> fa[PF - 1];
    Frag<BN> fb[PF - 1];
    LoadState<BM> sla;
    LoadState<BN> slb;
    la.template prepare<BM>(m0, tid, sla);
    lb.template prepare<BN>(n0, tid, slb);
    const int nkt = kb < ke ? (ke - kb + BK - 1) / BK : 0;
    {
        Frag<BM> f0;
        Frag<BN> g0;
        la.template fetch<BM>(sla, kb, ke, tid, f0);
        lb.template fetch<BN>(slb, kb, ke, tid, g0);
#pragma unroll
        for (int q = 0; q < PF - 1; ++q) {
            la.template fetch<BM>(sla, kb + (q + 1) * BK, ke, tid, fa[q]);
            lb.template fetch<BN>(slb, kb + (q + 1) * BK, ke, tid, fb[q]);
        }
        la.template store<BM>(f0, tid, sA[0]);
        lb.template store<BN>(g0, tid, sB[0]);
    }
    __syncthreads();
    // tile t waits in ring slot (t - 1) % (PF - 1); the loop runs whole rounds of the ring
    // (the tiles past the last are zeros and are not multiplied)
    const int nit = (nkt + PF - 2) / (PF - 1) * (PF - 1);
    for (int i0 = 0; i0 < nit; i0 += PF - 1) {
#pragma unroll
        for (int u = 0; u < PF - 1; ++u) {
            const int i = i0 + u;
            const int cur = i & 1;
            if (i < nkt) {
#pragma unroll
                for (int ks = 0; ks < BK; ks += 32) {
                    bf16x8 af[TM], bfr[TN];
#pragma unroll
                    for (int a = 0; a < TM; ++a)
                        af[a] = *reinterpret_cast<const bf16x8*>(&sA[cur][wm0 + a * 16 + fr][ks + fk]);
#pragma unroll
                    for (int b = 0; b < TN; ++b)
                        bfr[b] = *reinterpret_cast<const bf16x8*>(&sB[cur][wn0 + b * 16 + fr][ks + fk]);
#pragma unroll
                    for (int a = 0; a < TM; ++a)
#pragma unroll
                        for (int b = 0; b < TN; ++b)
                            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
                }
            }
            la.template store<BM>(fa[u], tid, sA[cur ^ 1]);
            lb.template store<BN>(fb[u], tid, sB[cur ^ 1]);
            la.template fetch<BM>(sla, kb + (i + PF) * BK, ke, tid, fa[u]);
            lb.template fetch<BN>(slb, kb + (i + PF) * BK, ke, tid, fb[u]);
            __syncthreads();
        }
    }
    // C layout of a 16x16 tile: lane holds column lane%16, rows 4*(lane/16) + r
    const int cc = lane & 15, cr = (lane >> 4) * 4;
    if constexpr (EpiHasTile<EPI>::value) {
        constexpr int LDC = BN + 4;
        static_assert(BM * LDC * 4 <= (int)sizeof(smem), "the C tile fits in the operand stages");
        float* C = reinterpret_cast<float*>(smem);  // the loop ended with a barrier: the stages are free
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
            for (int b = 0; b < TN; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) C[(wm0 + a * 16 + cr + r) * LDC + wn0 + b * 16 + cc] = acc[a][b][r];
        __syncthreads();
        epi.tile(m0, n0, min(BM, M - m0), min(BN, N - n0), C, LDC, BM);
        return;
    }
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
            const int col = n0 + wn0 + b * 16 + cc;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm0 + a * 16 + cr + r;
                if (row < M && col < N) epi(row, col, acc[a][b][r], blockIdx.z);
            }
        }
}

// ---- epilogues ----------------------------------------------------------------------
struct EpiF32 {  // out[z][row][col] = v (+ bias[col])
    static constexpr bool kTile = true;
    float* out;
    long long ld, zstride;
    const float* bias;
    __device__ __forceinline__ void operator()(int r, int c, float v, int z) const
    {
        out[z * zstride + (long long)r * ld + c] = v + (bias ? bias[c] : 0.f);
    }
    // 4 consecutive columns per thread, one float4 store (cols and ld are multiples of 4)
    __device__ __forceinline__ void tile(int m0, int n0, int rows, int cols, float* C, int ldc, int) const
    {
        const int nq = cols / 4;
        float* o = out + blockIdx.z * zstride;
        for (int idx = threadIdx.x; idx < rows * nq; idx += 256) {
            const int rr = idx / nq, q = idx % nq;
            const int c = n0 + q * 4;
            float4 v = *reinterpret_cast<const float4*>(C + rr * ldc + q * 4);
            if (bias) {
                v.x += bias[c];
                v.y += bias[c + 1];
                v.z += bias[c + 2];
                v.w += bias[c + 3];
            } else {
                v.x += 0.f;
                v.y += 0.f;
                v.z += 0.f;
                v.w += 0.f;
            }
            *reinterpret_cast<float4*>(o + (long long)(m0 + rr) * ld + c) = v;
        }
    }
};
struct EpiBF16 {  // bf16(v + bias), optional fp32 copy
    uint16_t* out;
    long long ld;
    const float* bias;
    float* f32out;
    __device__ __forceinline__ void operator()(int r, int c, float v, int) const
    {
        const float x = v + (bias ? bias[c] : 0.f);
        out[(long long)r * ld + c] = f2bf(x);
        if (f32out) f32out[(long long)r * ld + c] = x;
    }
};
// Column sums of a float32 C tile (rows x cols in LDS, row stride ldc) into
// colpart[m0 / bm][n0 + c]: the bias gradient of a training layer summed over the
// tile's batch rows (a fixed order; the partials of all row tiles are summed after).
// All 256 threads take part: column c's rows are split into 256 / cols contiguous
// ranges, each summed in row order with eight loads ahead of the adds, and the range
// sums are added in range order (cols <= 256).
__device__ __forceinline__ void tile_colsum(float* colpart, long long ldp, int m0, int n0, int rows, int cols,
                                            const float* C, int ldc, int bm)
{
    __shared__ float red[256];
    __syncthreads();
    const int parts = 256 / cols;
    if ((int)threadIdx.x < parts * cols) {
        const int c = threadIdx.x % cols, part = threadIdx.x / cols;
        const int r1 = (part + 1) * rows / parts;
        int r = part * rows / parts;
        float s = 0.f;
        for (; r + 8 <= r1; r += 8) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = C[(r + u) * ldc + c];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += v[u];
        }
        for (; r < r1; ++r) s += C[r * ldc + c];
        red[threadIdx.x] = s;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < cols; c += 256) {
        float t = 0.f;
        for (int p = 0; p < parts; ++p) t += red[p * cols + c];
        colpart[(long long)(m0 / bm) * ldp + n0 + c] = t;
    }
}

// bf16 copy of a float32 C tile (rows x cols in LDS), transposed: T[(n0 + c) tld + m0 + r].
// Thread item (column c, group of 8 rows): one 16-byte store; the 8 threads of a column
// write 128 contiguous bytes (rows is a multiple of 8, tld of 8).
__device__ __forceinline__ void tile_store_t(uint16_t* T, long long tld, int m0, int n0, int rows, int cols,
                                             const float* C, int ldc)
{
    __syncthreads();
    const int rg = rows / 8;
    for (int i = threadIdx.x; i < cols * rg; i += 256) {
        const int c = i / rg, g = i % rg;
        const float* q = C + (g * 8) * ldc + c;
        *reinterpret_cast<uint4*>(T + (long long)(n0 + c) * tld + m0 + g * 8) =
            make_uint4(f2bf2(q[0], q[ldc]), f2bf2(q[2 * ldc], q[3 * ldc]), f2bf2(q[4 * ldc], q[5 * ldc]),
                       f2bf2(q[6 * ldc], q[7 * ldc]));
    }
}

struct EpiGelu {  // a = v + bias -> (pre-activation), bf16(gelu(a)) [and its transpose]
    static constexpr bool kTile = true;
    uint16_t* out;
    long long ld;
    const float* bias;
    float* pre;
    uint16_t* tout = nullptr;  // optional [ld][tld]: the bf16 activations transposed
    long long tld = 0;
    __device__ __forceinline__ void operator()(int r, int c, float v, int) const
    {
        const float a = v + bias[c];
        if (pre) pre[(long long)r * ld + c] = a;
        out[(long long)r * ld + c] = f2bf(gelu(a));
    }
    // 8 consecutive columns per thread (cols is a multiple of 8): one 16-byte store of
    // bf16 activations, two float4 stores of the pre-activation; 16 threads write one
    // 128-column row segment in 256 contiguous bytes
    __device__ __forceinline__ void tile(int m0, int n0, int rows, int cols, float* C, int ldc, int) const
    {
        const int nq = cols / 8;
        for (int idx = threadIdx.x; idx < rows * nq; idx += 256) {
            const int rr = idx / nq, q = idx % nq;
            const int c = n0 + q * 8;
            const float4 v0 = *reinterpret_cast<const float4*>(C + rr * ldc + q * 8);
            const float4 v1 = *reinterpret_cast<const float4*>(C + rr * ldc + q * 8 + 4);
            const float4 b0 = *reinterpret_cast<const float4*>(bias + c);
            const float4 b1 = *reinterpret_cast<const float4*>(bias + c + 4);
            const float4 a0 = make_float4(v0.x + b0.x, v0.y + b0.y, v0.z + b0.z, v0.w + b0.w);
            const float4 a1 = make_float4(v1.x + b1.x, v1.y + b1.y, v1.z + b1.z, v1.w + b1.w);
            const long long o = (long long)(m0 + rr) * ld + c;
            if (pre) {
                *reinterpret_cast<float4*>(pre + o) = a0;
                *reinterpret_cast<float4*>(pre + o + 4) = a1;
            }
            const float4 g0 = make_float4(gelu(a0.x), gelu(a0.y), gelu(a0.z), gelu(a0.w));
            const float4 g1 = make_float4(gelu(a1.x), gelu(a1.y), gelu(a1.z), gelu(a1.w));
            *reinterpret_cast<uint4*>(out + o) =
                make_uint4(f2bf2(g0.x, g0.y), f2bf2(g0.z, g0.w), f2bf2(g1.x, g1.y), f2bf2(g1.z, g1.w));
            if (tout) {
                *reinterpret_cast<float4*>(C + rr * ldc + q * 8) = g0;
                *reinterpret_cast<float4*>(C + rr * ldc + q * 8 + 4) = g1;
            }
        }
        if (tout) tile_store_t(tout, tld, m0, n0, rows, cols, C, ldc);
    }
};
struct EpiGeluBack {  // d = v * gelu'(pre) -> bf16 [and its transpose], the tile's column sums of d
    static constexpr bool kTile = true;
    uint16_t* out;
    const float* pre;
    long long ld;
    float* colpart;            // [row tiles][ld] column sums of d
    uint16_t* tout = nullptr;  // optional [ld][tld]: bf16 d transposed
    long long tld = 0;
    __device__ __forceinline__ void operator()(int r, int c, float v, int) const
    {
        const long long o = (long long)r * ld + c;
        out[o] = f2bf(v * gelu_prime(pre[o]));
    }
    // 8 consecutive columns per thread: vector loads of pre, one 16-byte bf16 store
    // (cols and ld are multiples of 8); d goes back into the tile for the sums
    __device__ __forceinline__ void tile(int m0, int n0, int rows, int cols, float* C, int ldc, int bm) const
    {
        const int nq = cols / 8;
        for (int idx = threadIdx.x; idx < rows * nq; idx += 256) {
            const int rr = idx / nq, q = idx % nq;
            const long long o = (long long)(m0 + rr) * ld + n0 + q * 8;
            const float4 v0 = *reinterpret_cast<const float4*>(C + rr * ldc + q * 8);
            const float4 v1 = *reinterpret_cast<const float4*>(C + rr * ldc + q * 8 + 4);
            const float4 p0 = *reinterpret_cast<const float4*>(pre + o);
            const float4 p1 = *reinterpret_cast<const float4*>(pre + o + 4);
            const float4 d0 = make_float4(v0.x * gelu_prime(p0.x), v0.y * gelu_prime(p0.y), v0.z * gelu_prime(p0.z),
                                          v0.w * gelu_prime(p0.w));
            const float4 d1 = make_float4(v1.x * gelu_prime(p1.x), v1.y * gelu_prime(p1.y), v1.z * gelu_prime(p1.z),
                                          v1.w * gelu_prime(p1.w));
            *reinterpret_cast<float4*>(C + rr * ldc + q * 8) = d0;
            *reinterpret_cast<float4*>(C + rr * ldc + q * 8 + 4) = d1;
            *reinterpret_cast<uint4*>(out + o) = make_uint4(f2bf2(d0.x, d0.y), f2bf2(d0.z, d0.w), f2bf2(d1.x, d1.y),
                                                            f2bf2(d1.z, d1.w));
        }
        tile_colsum(colpart, ld, m0, n0, rows, cols, C, ldc, bm);
        if (tout) tile_store_t(tout, tld, m0, n0, rows, cols, C, ldc);
    }
};

// A narrow training product (the latent layer, 32 columns): x = v (+ bias) -> bf16
// [and its transpose], optionally the tile's column sums of x.
struct EpiBF16T {
    static constexpr bool kTile = true;
    uint16_t* out;
    long long ld;
    const float* bias;         // nullable
    float* colpart = nullptr;  // optional [row tiles][ld]
    uint16_t* tout = nullptr;  // optional [ld][tld]
    long long tld = 0;
    __device__ __forceinline__ void operator()(int r, int c, float v, int) const
    {
        out[(long long)r * ld + c] = f2bf(v + (bias ? bias[c] : 0.f));
    }
    __device__ __forceinline__ void tile(int m0, int n0, int rows, int cols, float* C, int ldc, int bm) const
    {
        const int nq = cols / 8;
        for (int idx = threadIdx.x; idx < rows * nq; idx += 256) {
            const int rr = idx / nq, q = idx % nq;
            const int c = n0 + q * 8;
            float x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                x[u] = C[rr * ldc + q * 8 + u] + (bias ? bias[c + u] : 0.f);
                C[rr * ldc + q * 8 + u] = x[u];
            }
            *reinterpret_cast<uint4*>(out + (long long)(m0 + rr) * ld + c) =
                make_uint4(f2bf2(x[0], x[1]), f2bf2(x[2], x[3]), f2bf2(x[4], x[5]), f2bf2(x[6], x[7]));
        }
        if (colpart) tile_colsum(colpart, ld, m0, n0, rows, cols, C, ldc, bm);
        if (tout) tile_store_t(tout, tld, m0, n0, rows, cols, C, ldc);
    }
};

// The decoder's output layer in training with the loss folded in: yhat = v + b4 never
// leaves the tile. d = 2 w_bf (yhat - y) / (512 W) goes out as bf16 (the operand of
// the next products), its column sums over the tile's rows as float32 partials (the
// b4 gradient), and each row's share of sum_f w_bf sum_i (yhat - y)^2 / (512 W) over
// the tile's columns as a float64 partial lossp[row][n0 / cols_per_tile].
struct EpiMse {
    static constexpr bool kTile = true;
    const float* bias;      // b4
    const uint16_t* y;      // normalised inputs [.][ld], batch row b at y[idx[b]]
    const int* idx;
    long long ld;
    const float* w;         // [B][4] per-sample field weights
    const double* wsum;     // their total
    uint16_t* dq;           // [B][ld]
    float* colpart;         // [row tiles][ld]
    double* lossp;          // [row tiles][column tiles]
    int ntn;                // column tiles
    uint16_t* tout = nullptr;  // optional [ld][tld]: bf16 d transposed
    long long tld = 0;
    __device__ __forceinline__ void operator()(int, int, float, int) const {}
    // 8 consecutive columns per thread; 16 threads cover a 128-column row segment
    __device__ __forceinline__ void tile(int m0, int n0, int rows, int cols, float* C, int ldc, int bm) const
    {
        const double inv = 1.0 / (512.0 * wsum[0]);
        const double inv2 = 2.0 * inv;  // d(loss)/d(yhat) per unit weight and difference
        const int nq = cols / 8;
        double tl = 0.0;  // this thread's rows (their q = 0 thread) of the tile's loss
        for (int idx8 = threadIdx.x; idx8 < rows * nq; idx8 += 256) {
            const int rr = idx8 / nq, q = idx8 % nq;
            const int b = m0 + rr, c = n0 + q * 8;
            const long long src = idx ? idx[b] : b;
            const float wf = w[b * 4 + (c >> 9)];
            const float f = (float)(wf * inv2);
            const uint4 yv = *reinterpret_cast<const uint4*>(y + src * ld + c);
            const uint32_t yw[4] = {yv.x, yv.y, yv.z, yv.w};
            float d[8];
            double acc = 0.0;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const float yh = C[rr * ldc + q * 8 + u] + bias[c + u];
                const float yi = bf2f((uint16_t)(u & 1 ? yw[u >> 1] >> 16 : yw[u >> 1] & 0xFFFFu));
                const float diff = yh - yi;
                acc += (double)wf * diff * diff;
                d[u] = f * diff;
                C[rr * ldc + q * 8 + u] = d[u];
            }
            *reinterpret_cast<uint4*>(dq + (long long)b * ld + c) =
                make_uint4(f2bf2(d[0], d[1]), f2bf2(d[2], d[3]), f2bf2(d[4], d[5]), f2bf2(d[6], d[7]));
            // the row's share over the tile's columns: the nq threads of a row are consecutive
            // and aligned (nq = cols / 8 is 8 or 16), so a width-nq shuffle sum closes it
            for (int o = nq / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, nq);
            if (q == 0) tl += acc;
        }
        // the tile's loss: rows summed per wave (fixed shuffle order), then the 4 waves in order
        for (int o = 32; o > 0; o >>= 1) tl += __shfl_xor(tl, o, 64);
        __shared__ double wsh[4];
        if ((threadIdx.x & 63) == 0) wsh[threadIdx.x >> 6] = tl;
        __syncthreads();
        if (threadIdx.x == 0) lossp[(long long)(m0 / bm) * ntn + n0 / cols] = ((wsh[0] + wsh[1]) + (wsh[2] + wsh[3])) * inv;
        tile_colsum(colpart, ld, m0, n0, rows, cols, C, ldc, bm);
        if (tout) tile_store_t(tout, tld, m0, n0, rows, cols, C, ldc);
    }
};
struct EpiDenorm {  // decoder output of field f -> lo + r (v + b) scattered into the state
    float* state;
    const float* meta;  // [P][4][2]
    const float* bias;  // b4 + f*512
    int f, Py, Px, ny, nx;
    long long N;
    __device__ __forceinline__ void operator()(int p, int c, float v, int) const
    {
        const float y = v + bias[c];
        const float lo = meta[(long long)p * 8 + 2 * f], rr = meta[(long long)p * 8 + 2 * f + 1];
        const int px = p % Px, py = (p / Px) % Py, pz = p / (Px * Py);
        const int lz = c >> 6, ly = (c >> 3) & 7, lx = c & 7;
        const long long z = pz * 8 + lz, yy = py * 8 + ly, x = px * 8 + lx;
        state[f * N + (z * ny + yy) * nx + x] = lo + rr * y;
    }
};

template <int BM, int BN, int WM, int WN, class LA, class LB, class EPI>
void gemm(int M, int N, int K, const LA& la, const LB& lb, const EPI& epi, hipStream_t st, int splits = 1)
{
    WV_REQUIRE(K % 32 == 0, WV_EINVAL, "GEMM depth must be a multiple of 32");
    const int kps = (((K + BK - 1) / BK + splits - 1) / splits) * BK;
    dim3 grid(((M + BM - 1) / BM) * ((N + BN - 1) / BN), 1, splits);
    hipLaunchKernelGGL((gemm_kernel<BM, BN, WM, WN, LA, LB, EPI>), grid, dim3(256), 0, st, M, N, K, kps, la, lb, epi);
    WV_HIP(hipGetLastError());
}

// wide N (>= 128) and narrow N (<= 32) tile shapes
struct EpiTimeDenorm {  // decoder output of a time vector -> lo + r (v + b) into levels t < nvalid
    static constexpr bool kTile = true;
    float* e_win;
    const float* meta;  // [S*B][2]
    const float* bias;  // b4
    int S, ny, nx, By, Bx, nvalid;
    long long B, N;
    __device__ __forceinline__ void operator()(int row, int c, float v, int) const
    {
        const int t = c >> 6;
        if (t >= nvalid) return;
        const float yv = v + bias[c];
        const float lo = meta[(long long)row * 2], rr = meta[(long long)row * 2 + 1];
        const int s = (int)(row / B);
        const long long b = row % B;
        const int bx = (int)(b % Bx), by = (int)((b / Bx) % By), bz = (int)(b / ((long long)Bx * By));
        const int cell = c & 63, lz = cell >> 4, ly = (cell >> 2) & 3, lx = cell & 3;
        e_win[((long long)t * S + s) * N + ((long long)(bz * 4 + lz) * ny + by * 4 + ly) * nx + bx * 4 + lx] =
            lo + rr * yv;
    }
    // The tile's rows are consecutive vectors, i.e. blocks along x. Thread i takes row
    // i % 128 and every other group of 4 columns from i / 128 on: 4 columns are the
    // 4 x-cells of one (t, lz, ly) row of the block, so each thread moves float4s
    // (one LDS read, one store), and a wave's store covers 64 consecutive blocks
    // (a contiguous run of x). The row's block and (lo, r) are resolved once.
    __device__ __forceinline__ void tile(int m0, int n0, int rows, int cols, float* C, int ldc, int) const
    {
        const int rr = threadIdx.x & 127;
        if (rr >= rows) return;
        const long long row = (long long)m0 + rr;
        const int s = (int)(row / B);
        const long long b = row % B;
        const int bx = (int)(b % Bx), by = (int)((b / Bx) % By), bz = (int)(b / ((long long)Bx * By));
        const float lo = meta[row * 2], rg = meta[row * 2 + 1];
        float* base = e_win + (long long)s * N + ((long long)bz * 4 * ny + by * 4) * nx + bx * 4;
        const float* crow = C + rr * ldc;
        for (int cq = threadIdx.x >> 7; cq < cols / 4; cq += 2) {
            const int c = n0 + cq * 4;
            const int t = c >> 6;
            if (t >= nvalid) break;  // columns ascend, so do the levels
            const int cell = c & 63, lz = cell >> 4, ly = (cell >> 2) & 3;
            const float4 v = *reinterpret_cast<const float4*>(crow + cq * 4);
            const float4 bb = *reinterpret_cast<const float4*>(bias + c);
            *reinterpret_cast<float4*>(base + (long long)t * S * N + ((long long)lz * ny + ly) * nx) =
                make_float4(lo + rg * (v.x + bb.x), lo + rg * (v.y + bb.y), lo + rg * (v.z + bb.z),
                            lo + rg * (v.w + bb.w));
        }
    }
};

// Work-group tile (rows, columns) that gemm_auto launches for an M x N product:
// 128 x 128 when that gives at least two work-groups per CU, else 64 x 64 (training
// batches of a few thousand rows); 128 x 32 for products 32 columns wide.
#ifndef WV_GEMM_BIG_MIN_WG
#define WV_GEMM_BIG_MIN_WG 512
#endif
inline int gemm_auto_bm(int M, int N, int splits = 1)
{
    const long long wg128 = (long long)((M + 127) / 128) * ((N + 127) / 128) * splits;
    return N <= 32 ? 128 : (wg128 < WV_GEMM_BIG_MIN_WG ? 64 : 128);
}
inline int gemm_auto_bn(int M, int N, int splits = 1)
{
    const long long wg128 = (long long)((M + 127) / 128) * ((N + 127) / 128) * splits;
    return N <= 32 ? 32 : (wg128 < WV_GEMM_BIG_MIN_WG ? 64 : 128);
}

template <class LA, class LB, class EPI>
void gemm_auto(int M, int N, int K, const LA& la, const LB& lb, const EPI& epi, hipStream_t st, int splits = 1)
{
    const int bm = gemm_auto_bm(M, N, splits), bn = gemm_auto_bn(M, N, splits);
    if (bn == 32)
        gemm<128, 32, 32, 32>(M, N, K, la, lb, epi, st, splits);
    else if (bm == 64)
        gemm<64, 64, 32, 32>(M, N, K, la, lb, epi, st, splits);
    else
        gemm<128, 128, 64, 64>(M, N, K, la, lb, epi, st, splits);
}

// ------------------------------------------------------------------------------------
// normalisation: one work-group per patch, one wave per field (8 values per lane)
// ------------------------------------------------------------------------------------
// one work-group per output row: patch p = rows ? rows[row] : row (rows checked on the host)
__global__ void __launch_bounds__(256) normalize_kernel(const float* __restrict__ state, int ny, int nx,
                                                       long long N, int Py, int Px, const float* __restrict__ beta,
                                                       const int32_t* __restrict__ rows,
                                                       uint16_t* __restrict__ y, float* __restrict__ meta)
{
    const long long row = blockIdx.x;
    const long long p = rows ? (long long)rows[row] : row;
    const int f = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int px = p % Px, py = (p / Px) % Py, pz = p / ((long long)Px * Py);
    const int lz = l >> 3, ly = l & 7;
    const float* src = state + f * N + ((long long)(pz * 8 + lz) * ny + (py * 8 + ly)) * nx + px * 8;
    const float4 a = *reinterpret_cast<const float4*>(src);
    const float4 b = *reinterpret_cast<const float4*>(src + 4);
    float v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
    float lo = v[0], hi = v[0];
    for (int t = 1; t < 8; ++t) {
        lo = fminf(lo, v[t]);
        hi = fmaxf(hi, v[t]);
    }
    for (int o = 32; o > 0; o >>= 1) {
        lo = fminf(lo, __shfl_xor(lo, o, 64));
        hi = fmaxf(hi, __shfl_xor(hi, o, 64));
    }
    const float r = fmaxf(hi - lo, beta[f]);
    const float rinv = 1.0f / r;
    const uint4 o8 = make_uint4(f2bf2((v[0] - lo) * rinv, (v[1] - lo) * rinv), f2bf2((v[2] - lo) * rinv, (v[3] - lo) * rinv),
                                f2bf2((v[4] - lo) * rinv, (v[5] - lo) * rinv), f2bf2((v[6] - lo) * rinv, (v[7] - lo) * rinv));
    *reinterpret_cast<uint4*>(y + row * 2048 + f * 512 + l * 8) = o8;
    if (l == 0) {
        meta[row * 8 + 2 * f] = lo;
        meta[row * 8 + 2 * f + 1] = r;
    }
}

// time vectors of G x-adjacent blocks per work-group (all vectors of a window in
// order): the 512 rows (t, lz, ly) of the window are read as G float4 runs each,
// G * 16 bytes contiguous, so a row of blocks is fetched in whole cache lines.
// Thread i holds block i % G and rows i / G + (256 / G) m, m < 2 G.
template <int G>
__global__ void __launch_bounds__(256) time_normalize_group_kernel(const float* __restrict__ e_win, int S, int ny,
                                                                  int nx, long long N, int By, int Bx, long long B,
                                                                  int nvalid, const float* __restrict__ beta,
                                                                  uint16_t* __restrict__ y, float* __restrict__ meta)
{
    constexpr int NR = 2 * G;             // rows per thread
    constexpr int RS = 256 / G;           // row stride between a thread's rows
    const long long v0 = (long long)blockIdx.x * G;  // first vector of the group
    const int s = (int)(v0 / B);
    const long long b0 = v0 % B;
    const int bx0 = (int)(b0 % Bx), by = (int)((b0 / Bx) % By), bz = (int)(b0 / ((long long)Bx * By));
    const int g = threadIdx.x % G, r0 = threadIdx.x / G;
    float4 v[NR];
    float lo = INFINITY, hi = -INFINITY;
#pragma unroll
    for (int m = 0; m < NR; ++m) {
        const int r = r0 + RS * m;        // row = t * 16 + lz * 4 + ly
        const int t = r >> 4, lz = (r >> 2) & 3, ly = r & 3;
        const int tl = t < nvalid ? t : nvalid - 1;
        v[m] = *reinterpret_cast<const float4*>(e_win + ((long long)tl * S + s) * N +
                                                ((long long)(bz * 4 + lz) * ny + by * 4 + ly) * nx + (bx0 + g) * 4);
        lo = fminf(lo, fminf(fminf(v[m].x, v[m].y), fminf(v[m].z, v[m].w)));
        hi = fmaxf(hi, fmaxf(fmaxf(v[m].x, v[m].y), fmaxf(v[m].z, v[m].w)));
    }
    // lanes of one block differ by multiples of G
    for (int o = G; o < 64; o <<= 1) {
        lo = fminf(lo, __shfl_xor(lo, o, 64));
        hi = fmaxf(hi, __shfl_xor(hi, o, 64));
    }
    __shared__ float slo[4][G], shi[4][G];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) < G) {
        slo[w][g] = lo;
        shi[w][g] = hi;
    }
    __syncthreads();
    lo = fminf(fminf(slo[0][g], slo[1][g]), fminf(slo[2][g], slo[3][g]));
    hi = fmaxf(fmaxf(shi[0][g], shi[1][g]), fmaxf(shi[2][g], shi[3][g]));
    const float rr = fmaxf(hi - lo, beta[0]);
    const float rinv = 1.0f / rr;
    uint16_t* yv = y + (v0 + g) * (TWIN * 64);
#pragma unroll
    for (int m = 0; m < NR; ++m) {
        const int r = r0 + RS * m;
        const uint2 o = make_uint2(f2bf2((v[m].x - lo) * rinv, (v[m].y - lo) * rinv),
                                   f2bf2((v[m].z - lo) * rinv, (v[m].w - lo) * rinv));
        *reinterpret_cast<uint2*>(yv + r * 4) = o;
    }
    if (threadIdx.x < G) {
        meta[(v0 + g) * 2] = lo;
        meta[(v0 + g) * 2 + 1] = rr;
    }
}

// time vectors: one work-group per vector; thread i holds level t = i / 8 (the
// last valid level for t >= nvalid) and cells 8 (i % 8) .. + 7 of the block, i.e.
// the x-rows (lz, ly0) and (lz, ly0 + 1) with lz = (i % 8) / 2, ly0 = 2 (i % 2)
__global__ void __launch_bounds__(256) time_normalize_kernel(const float* __restrict__ e_win, int S, int ny, int nx,
                                                            long long N, int By, int Bx, long long B, int nvalid,
                                                            const float* __restrict__ beta,
                                                            const int32_t* __restrict__ rows,
                                                            uint16_t* __restrict__ y, float* __restrict__ meta)
{
    const long long row = blockIdx.x;
    const long long vix = rows ? (long long)rows[row] : row;
    const int s = (int)(vix / B);
    const long long b = vix % B;
    const int bx = (int)(b % Bx), by = (int)((b / Bx) % By), bz = (int)(b / ((long long)Bx * By));
    const int t = threadIdx.x >> 3, q = threadIdx.x & 7;
    const int tl = t < nvalid ? t : nvalid - 1;
    const int lz = q >> 1, ly0 = (q & 1) * 2;
    const float* src =
        e_win + ((long long)tl * S + s) * N + ((long long)(bz * 4 + lz) * ny + by * 4 + ly0) * nx + bx * 4;
    const float4 a = *reinterpret_cast<const float4*>(src);
    const float4 c = *reinterpret_cast<const float4*>(src + nx);
    const float v[8] = {a.x, a.y, a.z, a.w, c.x, c.y, c.z, c.w};
    float lo = v[0], hi = v[0];
    for (int k = 1; k < 8; ++k) {
        lo = fminf(lo, v[k]);
        hi = fmaxf(hi, v[k]);
    }
    for (int o = 32; o > 0; o >>= 1) {
        lo = fminf(lo, __shfl_xor(lo, o, 64));
        hi = fmaxf(hi, __shfl_xor(hi, o, 64));
    }
    __shared__ float slo[4], shi[4];
    if ((threadIdx.x & 63) == 0) {
        slo[threadIdx.x >> 6] = lo;
        shi[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    lo = fminf(fminf(slo[0], slo[1]), fminf(slo[2], slo[3]));
    hi = fmaxf(fmaxf(shi[0], shi[1]), fmaxf(shi[2], shi[3]));
    const float r = fmaxf(hi - lo, beta[0]);
    const float rinv = 1.0f / r;
    const uint4 o8 = make_uint4(f2bf2((v[0] - lo) * rinv, (v[1] - lo) * rinv), f2bf2((v[2] - lo) * rinv, (v[3] - lo) * rinv),
                                f2bf2((v[4] - lo) * rinv, (v[5] - lo) * rinv), f2bf2((v[6] - lo) * rinv, (v[7] - lo) * rinv));
    *reinterpret_cast<uint4*>(y + row * (TWIN * 64) + t * 64 + q * 8) = o8;
    if (threadIdx.x == 0) {
        meta[row * 2] = lo;
        meta[row * 2 + 1] = r;
    }
}

// per-patch, per-field (min, range): one work-group per (pz, py) row of patches,
// threads along x, groups of 8 lanes reduce one patch
__global__ void __launch_bounds__(256) minmax_kernel(const float* __restrict__ state, int ny, int nx, long long N,
                                                    int Py, int Px, const float* __restrict__ beta,
                                                    float* __restrict__ meta)
{
    const int row = blockIdx.x;
    const int py = row % Py, pz = row / Py;
    for (int x = threadIdx.x; x < nx; x += blockDim.x) {
        float lo[4], hi[4];
        for (int f = 0; f < 4; ++f) {
            lo[f] = INFINITY;
            hi[f] = -INFINITY;
            const float* src = state + f * N + ((long long)(pz * 8) * ny + py * 8) * nx + x;
            for (int lz = 0; lz < 8; ++lz)
                for (int ly = 0; ly < 8; ++ly) {
                    const float v = src[((long long)lz * ny + ly) * nx];
                    lo[f] = fminf(lo[f], v);
                    hi[f] = fmaxf(hi[f], v);
                }
            for (int o = 1; o < 8; o <<= 1) {
                lo[f] = fminf(lo[f], __shfl_xor(lo[f], o, 64));
                hi[f] = fmaxf(hi[f], __shfl_xor(hi[f], o, 64));
            }
        }
        if ((x & 7) == 0) {
            const long long p = (long long)row * Px + x / 8;
            for (int f = 0; f < 4; ++f) {
                meta[p * 8 + 2 * f] = lo[f];
                meta[p * 8 + 2 * f + 1] = fmaxf(hi[f] - lo[f], beta[f]);
            }
        }
    }
}

// latent fp32 [P][L] -> e4m3 codes + per-patch scale; one wave per patch
__global__ void quantize_kernel(const float* __restrict__ z, long long P, int L, uint8_t* __restrict__ q,
                                float* __restrict__ scale)
{
    const long long p = blockIdx.x * 4LL + (threadIdx.x >> 6);
    const int l = threadIdx.x & 63;
    if (p >= P) return;
    const float v = l < L ? z[p * L + l] : 0.f;
    float m = fabsf(v);
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    const float s = m > 0.f ? m / 448.0f : 1.0f;
    if (l < L) q[p * L + l] = f2e4m3(v / s);
    if (l == 0) scale[p] = s;
}

// e4m3 codes + scale -> bf16(code * s)
__global__ void dequantize_kernel(const uint8_t* __restrict__ q, const float* __restrict__ scale, long long P,
                                  int L, uint16_t* __restrict__ zb)
{
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= P * L) return;
    zb[i] = f2bf(e4m32f(q[i]) * scale[i / L]);
}

// ------------------------------------------------------------------------------------
// training helpers
// ------------------------------------------------------------------------------------
// per-sample field weights w[b][f] = (r / beta_f)^2 (weighting = 1) or 1, and
// their float64 total
__global__ void batch_weights_kernel(const float* __restrict__ meta, const int* __restrict__ idx, int B,
                                     const float* __restrict__ beta, int weighting, float* __restrict__ w,
                                     double* __restrict__ wsum)
{
    __shared__ double sh[256];
    double acc = 0.0;
    for (int q = threadIdx.x; q < 4 * B; q += 256) {
        const int b = q >> 2, f = q & 3;
        float v = 1.0f;
        if (weighting) {
            const long long src = idx ? idx[b] : b;
            const float t = meta[src * 8 + 2 * f + 1] / beta[f];
            v = t * t;
        }
        w[q] = v;
        acc += v;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) wsum[0] = sh[0];
}

__global__ void sum_partials_kernel(const double* __restrict__ partial, int n, double scale, double* __restrict__ out,
                                    int accumulate)
{
    __shared__ double sh[256];
    double a = 0.0;
    for (int q = threadIdx.x; q < n; q += 256) a += partial[q];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = (accumulate ? out[0] : 0.0) + scale * sh[0];
}

// Several split sums in one launch: segment g sums part[g] ([splits[g]][4 n4[g]]) into
// out[g], four consecutive elements per thread, eight partials loaded ahead of their
// sums, each element summed in the order z = 0, 1, ...
struct SumSegs {
    const float* part[8];
    float* out[8];
    long long n4[8];
    int splits[8];
    long long first[9];  // first float4 of each segment in the launch
    int nseg;
};
__global__ void __launch_bounds__(256) sums_kernel(const SumSegs g)
{
    const long long q = blockIdx.x * 256LL + threadIdx.x;
    if (q >= g.first[g.nseg]) return;
    int sg = 0;
    while (sg + 1 < g.nseg && q >= g.first[sg + 1]) ++sg;
    const long long j = q - g.first[sg];
    const long long n4 = g.n4[sg];
    const int splits = g.splits[sg];
    const float4* p = reinterpret_cast<const float4*>(g.part[sg]) + j;
    float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
    int z = 0;
    for (; z + 8 <= splits; z += 8) {
        float4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = p[(long long)(z + u) * n4];
#pragma unroll
        for (int u = 0; u < 8; ++u) s = make_float4(s.x + v[u].x, s.y + v[u].y, s.z + v[u].z, s.w + v[u].w);
    }
    for (; z < splits; ++z) {
        const float4 v = p[(long long)z * n4];
        s = make_float4(s.x + v.x, s.y + v.y, s.z + v.z, s.w + v.w);
    }
    reinterpret_cast<float4*>(g.out[sg])[j] = s;
}


__global__ void adam_kernel(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, long long n, float lr, float b1, float b2, float eps,
                            float c1, float c2)
{
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    w[i] = w[i] - lr * mh / (sqrtf(vh) + eps);
}

// fp32 W_l [fi][fo] -> bf16 W_l [fi][fo] and bf16 W_l^T [fo][fi] for the 4 layers in one
// launch: a work-group converts a 64 x 64 tile of one layer and writes its transpose
// through LDS, so both outputs are written in whole rows
struct ConvLayers {
    const float* w[4];
    uint16_t* wb[4];
    uint16_t* wt[4];
    int fi[4], fo[4];
    int first[5];  // first work-group of each layer
    int tx[4];     // column tiles of each layer
};
__global__ void __launch_bounds__(256) convert_kernel(const ConvLayers a)
{
    __shared__ uint16_t s[64][64 + 2];
    int t = blockIdx.x, l = 0;
    while (l < 3 && t >= a.first[l + 1]) ++l;
    t -= a.first[l];
    const int fi = a.fi[l], fo = a.fo[l];
    const int r0 = (t / a.tx[l]) * 64, c0 = (t % a.tx[l]) * 64;
    for (int i = threadIdx.x; i < 64 * 16; i += 256) {
        const int r = i >> 4, c = (i & 15) * 4;
        if (r0 + r < fi && c0 + c < fo) {
            const float4 v = *reinterpret_cast<const float4*>(a.w[l] + (long long)(r0 + r) * fo + c0 + c);
            const uint16_t b0 = f2bf(v.x), b1 = f2bf(v.y), b2 = f2bf(v.z), b3 = f2bf(v.w);
            *reinterpret_cast<uint2*>(a.wb[l] + (long long)(r0 + r) * fo + c0 + c) =
                make_uint2(b0 | (uint32_t)b1 << 16, b2 | (uint32_t)b3 << 16);
            s[r][c] = b0;
            s[r][c + 1] = b1;
            s[r][c + 2] = b2;
            s[r][c + 3] = b3;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 64 * 16; i += 256) {
        const int c = i >> 4, r = (i & 15) * 4;
        if (c0 + c < fo && r0 + r < fi)
            *reinterpret_cast<uint2*>(a.wt[l] + (long long)(c0 + c) * fi + r0 + r) =
                make_uint2(s[r][c] | (uint32_t)s[r + 1][c] << 16, s[r + 2][c] | (uint32_t)s[r + 3][c] << 16);
    }
}

int blocks(long long n, int bs) { return (int)std::max<long long>(1, (n + bs - 1) / bs); }



}  // namespace
}  // namespace wv

using namespace wv;

// ======================================================================================
struct ae_net {
    int in = 2048, hid = 512, lat = 32;
    long long nparam = 0;
    long long oW[4] = {0, 0, 0, 0}, ob[4] = {0, 0, 0, 0};
    int fi[4] = {0, 0, 0, 0}, fo[4] = {0, 0, 0, 0};
    float* master = nullptr;
    float* m1 = nullptr;
    float* m2 = nullptr;
    float* grad = nullptr;
    uint16_t* wb[4] = {nullptr, nullptr, nullptr, nullptr};  // bf16 W   [fi][fo]
    uint16_t* wt[4] = {nullptr, nullptr, nullptr, nullptr};  // bf16 W^T [fo][fi]
    uint16_t* wp1 = nullptr;  // W1^T and W4^T in MFMA fragment order (fused kernels only)
    uint16_t* wp4 = nullptr;
    float* beta_d = nullptr;
    double* loss_d = nullptr;
    double beta[4] = {1e-7, 1e-7, 1e-7, 1e-7};
    long long step = 0;
    // workspaces, one per stream (grown on demand): codec calls queued on different
    // streams (the forward and the incremental history) may run at the same time
    struct Workspace {
        hipStream_t st;
        void* p;
        size_t bytes;
    };
    std::vector<Workspace> ws;

    const float* bias(int l) const { return master + ob[l]; }
};

namespace wv {
namespace {

template <class T>
T* dalloc(size_t n)
{
    void* p = nullptr;
    const hipError_t e = hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error{e == hipErrorOutOfMemory ? WV_ENOMEM : WV_EDEVICE,
                    "autoencoder allocation of " + std::to_string(n * sizeof(T)) + " bytes failed"};
    }
    return static_cast<T*>(p);
}

void layout(ae_net* a)
{
    const int dims[5] = {a->in, a->hid, a->lat, a->hid, a->in};
    long long o = 0;
    for (int l = 0; l < 4; ++l) {
        a->fi[l] = dims[l];
        a->fo[l] = dims[l + 1];
        a->oW[l] = o;
        o += (long long)a->fi[l] * a->fo[l];
        a->ob[l] = o;
        o += a->fo[l];
    }
    a->nparam = o;
}

void pack_fused(ae_net* a, hipStream_t st)
{
    if (a->wp1) {
        fused_pack(a->wt[0], a->hid, a->in, a->wp1, st);
        fused_pack(a->wt[3], a->in, a->hid, a->wp4, st);
    }
}

// bf16 copies of the weights after a change of the fp32 masters; with pack, also the
// fragment-ordered copies of the fused encode and decode (training skips them until
// its last step: only the inference kernels read them)
void refresh_bf16(ae_net* a, hipStream_t st, bool pack = true)
{
    ConvLayers c{};
    int n = 0;
    for (int l = 0; l < 4; ++l) {
        c.w[l] = a->master + a->oW[l];
        c.wb[l] = a->wb[l];
        c.wt[l] = a->wt[l];
        c.fi[l] = a->fi[l];
        c.fo[l] = a->fo[l];
        c.tx[l] = (a->fo[l] + 63) / 64;
        c.first[l] = n;
        n += c.tx[l] * ((a->fi[l] + 63) / 64);
    }
    c.first[4] = n;
    hipLaunchKernelGGL(convert_kernel, dim3(n), dim3(256), 0, st, c);
    WV_HIP(hipGetLastError());
    if (pack) pack_fused(a, st);
}

void upload_beta(ae_net* a)
{
    float b[4];
    for (int f = 0; f < 4; ++f) b[f] = (float)a->beta[f];
    WV_HIP(hipMemcpy(a->beta_d, b, sizeof(b), hipMemcpyHostToDevice));
}

// the work buffer of the calls queued on stream st; calls on one stream run in
// order, so they share it
void* workspace(const ae_net* ac, size_t bytes, hipStream_t st)
{
    ae_net* a = const_cast<ae_net*>(ac);
    ae_net::Workspace* w = nullptr;
    for (auto& q : a->ws)
        if (q.st == st) w = &q;
    if (!w) {
        a->ws.push_back({st, nullptr, 0});
        w = &a->ws.back();
    }
    if (bytes > w->bytes) {
        WV_HIP(hipDeviceSynchronize());
        if (w->p) (void)hipFree(w->p);
        w->p = nullptr;
        w->bytes = 0;
        w->p = dalloc<uint8_t>(bytes);
        w->bytes = bytes;
    }
    return w->p;
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

void check_grid(const wv_grid* g)
{
    WV_REQUIRE(g, WV_EINVAL, "null grid");
    WV_REQUIRE(g->ny > 1 && g->nz % 8 == 0 && g->ny % 8 == 0 && g->nx % 8 == 0, WV_ESHAPE,
               "autoencoder needs a 3D grid divisible into 8^3 patches");
}

void normalize_state(const ae_net* a, const PatchGrid& pg, const float* state, uint16_t* y, float* meta,
                     hipStream_t st)
{
    const long long N = (long long)pg.nz * pg.ny * pg.nx;
    hipLaunchKernelGGL(normalize_kernel, dim3((unsigned)pg.P), dim3(256), 0, st, state, pg.ny, pg.nx, N, pg.ny / 8,
                       pg.nx / 8, a->beta_d, (const int32_t*)nullptr, y, meta);
    WV_HIP(hipGetLastError());
}

void normalize_rows(const ae_net* a, const PatchGrid& pg, const float* state, const int32_t* rows, int nrows,
                    uint16_t* y, float* meta, hipStream_t st)
{
    const long long N = (long long)pg.nz * pg.ny * pg.nx;
    hipLaunchKernelGGL(normalize_kernel, dim3((unsigned)nrows), dim3(256), 0, st, state, pg.ny, pg.nx, N, pg.ny / 8,
                       pg.nx / 8, a->beta_d, rows, y, meta);
    WV_HIP(hipGetLastError());
}

void check_time_grid(const wv_grid* g)
{
    WV_REQUIRE(g, WV_EINVAL, "null grid");
    WV_REQUIRE(g->ny > 1 && g->nz % 4 == 0 && g->ny % 4 == 0 && g->nx % 4 == 0 && g->nsrc >= 1, WV_ESHAPE,
               "time compression needs a 3D grid divisible into 4^3 blocks");
}


template <class F>
int guarded_ae(F&& f)
{
    try {
        return f();
    } catch (const Error& e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::exception& e) {
        set_error(e.what());
        return WV_EDEVICE;
    }
}

}  // namespace

int ae_latent_dim(const ae_net* net) { return net->lat; }
int ae_input_dim(const ae_net* net) { return net->in; }

long long ae_latent_bytes_per_patch(const ae_net* net, int fmt)
{
    return (long long)net->lat * (fmt == AE_LATENT_FP8 ? 1 : 2);
}

void ae_encode_state(const ae_net* a, const PatchGrid& pg, const float* state, int fmt, void* latent, float* meta,
                     float* qscale, hipStream_t st)
{
    WV_REQUIRE(a && state && latent && meta && (fmt == AE_LATENT_BF16 || qscale), WV_EINVAL,
               "encode: null buffer");
    const long long P = pg.P;
    if (fused_supported(a->hid, a->lat)) {
        const long long N = (long long)pg.nz * pg.ny * pg.nx;
        const int rows = (pg.nz / 8) * (pg.ny / 8);
        hipLaunchKernelGGL(minmax_kernel, dim3(rows), dim3(std::min(256, ((pg.nx + 63) / 64) * 64)), 0, st, state,
                           pg.ny, pg.nx, N, pg.ny / 8, pg.nx / 8, a->beta_d, meta);
        WV_HIP(hipGetLastError());
        if (fmt == AE_LATENT_BF16) {
            fused_encode(pg, state, meta, nullptr, 0, a->beta_d, a->wp1, a->bias(0), a->wt[1], a->bias(1),
                         (uint16_t*)latent, nullptr, st);
        } else {
            float* z = (float*)workspace(a, align256(P * (size_t)a->lat * 4), st);
            fused_encode(pg, state, meta, nullptr, 0, a->beta_d, a->wp1, a->bias(0), a->wt[1], a->bias(1), nullptr,
                         z, st);
            hipLaunchKernelGGL(quantize_kernel, dim3(blocks(P, 4)), dim3(256), 0, st, z, P, a->lat, (uint8_t*)latent,
                               qscale);
            WV_HIP(hipGetLastError());
        }
        return;
    }
    const size_t oy = 0, oh = align256(oy + P * 2048 * 2), oz = align256(oh + P * (size_t)a->hid * 2);
    uint8_t* ws = (uint8_t*)workspace(a, align256(oz + P * (size_t)a->lat * 4), st);
    uint16_t* y = (uint16_t*)(ws + oy);
    uint16_t* h = (uint16_t*)(ws + oh);
    float* z = (float*)(ws + oz);
    normalize_state(a, pg, state, y, meta, st);
    gemm_auto((int)P, a->hid, a->in, LoadK{y, a->in, nullptr, (int)P, a->in},
              LoadK{a->wt[0], a->in, nullptr, a->hid, a->in}, EpiGelu{h, a->hid, a->bias(0), nullptr}, st);
    const LoadK lh{h, a->hid, nullptr, (int)P, a->hid};
    const LoadK lw{a->wt[1], a->hid, nullptr, a->lat, a->hid};
    if (fmt == AE_LATENT_BF16) {
        gemm_auto((int)P, a->lat, a->hid, lh, lw, EpiBF16{(uint16_t*)latent, a->lat, a->bias(1), nullptr}, st);
    } else {
        gemm_auto((int)P, a->lat, a->hid, lh, lw, EpiF32{z, a->lat, 0, a->bias(1)}, st);
        hipLaunchKernelGGL(quantize_kernel, dim3(blocks(P, 4)), dim3(256), 0, st, z, P, a->lat, (uint8_t*)latent,
                           qscale);
        WV_HIP(hipGetLastError());
    }
}

void ae_encode_state_mm(const ae_net* a, const PatchGrid& pg, const float* state, const float* mm, int H, int fmt,
                        void* latent, float* meta, float* qscale, hipStream_t st, uint16_t* meta16)
{
    if (!fused_supported(a->hid, a->lat)) {
        WV_REQUIRE(!meta16, WV_EINVAL, "16-bit metadata needs the fused network shape (hidden 512, latent 32)");
        ae_encode_state(a, pg, state, fmt, latent, meta, qscale, st);
        return;
    }
    WV_REQUIRE(a && state && mm && latent && (meta || meta16) && (fmt == AE_LATENT_BF16 || qscale), WV_EINVAL,
               "encode: null buffer");
    const long long P = pg.P;
    if (fmt == AE_LATENT_BF16) {
        fused_encode(pg, state, meta, mm, H, a->beta_d, a->wp1, a->bias(0), a->wt[1], a->bias(1),
                     (uint16_t*)latent, nullptr, st, meta16);
    } else {
        float* z = (float*)workspace(a, align256(P * (size_t)a->lat * 4), st);
        fused_encode(pg, state, meta, mm, H, a->beta_d, a->wp1, a->bias(0), a->wt[1], a->bias(1), nullptr, z, st,
                     meta16);
        hipLaunchKernelGGL(quantize_kernel, dim3(blocks(P, 4)), dim3(256), 0, st, z, P, a->lat, (uint8_t*)latent,
                           qscale);
        WV_HIP(hipGetLastError());
    }
}

void ae_time_normalize_rows(const ae_net* a, const TimeGrid& tg, const float* e_win, int nvalid,
                            const int32_t* rows, long long nrows, uint16_t* y, float* meta, hipStream_t st)
{
    WV_REQUIRE(a->in == TWIN * 64, WV_EINVAL, "time compression needs an input width of 2048");
    WV_REQUIRE(nvalid >= 1 && nvalid <= TWIN, WV_EINVAL, "nvalid must lie in [1, 32]");
    if (nrows == 0) return;
    const long long N = (long long)tg.nz * tg.ny * tg.nx;
    const int Bx = tg.nx / 4;
    if (!rows) {
        // whole window: groups of x-adjacent blocks (a group never crosses a row of blocks)
        const long long M = nrows;
        auto launch = [&](auto kern, int G) {
            hipLaunchKernelGGL(kern, dim3((unsigned)(M / G)), dim3(256), 0, st, e_win, tg.S, tg.ny, tg.nx, N,
                               tg.ny / 4, Bx, tg.B, nvalid, a->beta_d, y, meta);
        };
        if (Bx % 8 == 0) launch(time_normalize_group_kernel<8>, 8);
        else if (Bx % 4 == 0) launch(time_normalize_group_kernel<4>, 4);
        else if (Bx % 2 == 0) launch(time_normalize_group_kernel<2>, 2);
        else launch(time_normalize_group_kernel<1>, 1);
        WV_HIP(hipGetLastError());
        return;
    }
    hipLaunchKernelGGL(time_normalize_kernel, dim3((unsigned)nrows), dim3(256), 0, st, e_win, tg.S, tg.ny, tg.nx, N,
                       tg.ny / 4, tg.nx / 4, tg.B, nvalid, a->beta_d, rows, y, meta);
    WV_HIP(hipGetLastError());
}

void ae_time_encode(const ae_net* a, const TimeGrid& tg, const float* e_win, int nvalid, uint16_t* latent,
                    float* meta, hipStream_t st)
{
    const long long M = tg.B * tg.S;
    const size_t oh = align256(M * (size_t)a->in * 2);
    uint8_t* ws = (uint8_t*)workspace(a, align256(oh + M * (size_t)a->hid * 2), st);
    uint16_t* y = (uint16_t*)ws;
    uint16_t* h = (uint16_t*)(ws + oh);
    ae_time_normalize_rows(a, tg, e_win, nvalid, nullptr, M, y, meta, st);
    gemm_auto((int)M, a->hid, a->in, LoadK{y, a->in, nullptr, (int)M, a->in},
              LoadK{a->wt[0], a->in, nullptr, a->hid, a->in}, EpiGelu{h, a->hid, a->bias(0), nullptr}, st);
    gemm_auto((int)M, a->lat, a->hid, LoadK{h, a->hid, nullptr, (int)M, a->hid},
              LoadK{a->wt[1], a->hid, nullptr, a->lat, a->hid}, EpiBF16{latent, a->lat, a->bias(1), nullptr}, st);
}

void ae_time_decode(const ae_net* a, const TimeGrid& tg, const uint16_t* latent, const float* meta, int nvalid,
                    float* e_win, hipStream_t st)
{
    WV_REQUIRE(a->in == TWIN * 64, WV_EINVAL, "time compression needs an input width of 2048");
    WV_REQUIRE(nvalid >= 1 && nvalid <= TWIN, WV_EINVAL, "nvalid must lie in [1, 32]");
    const long long M = tg.B * tg.S;
    uint16_t* h = (uint16_t*)workspace(a, align256(M * (size_t)a->hid * 2), st);
    gemm_auto((int)M, a->hid, a->lat, LoadK{latent, a->lat, nullptr, (int)M, a->lat},
              LoadK{a->wt[2], a->lat, nullptr, a->hid, a->lat}, EpiGelu{h, a->hid, a->bias(2), nullptr}, st);
    const long long N = (long long)tg.nz * tg.ny * tg.nx;
    gemm_auto((int)M, a->in, a->hid, LoadK{h, a->hid, nullptr, (int)M, a->hid},
              LoadK{a->wt[3], a->hid, nullptr, a->in, a->hid},
              EpiTimeDenorm{e_win, meta, a->bias(3), tg.S, tg.ny, tg.nx, tg.ny / 4, tg.nx / 4, nvalid, tg.B, N}, st);
}

void ae_decode_state(const ae_net* a, const PatchGrid& pg, const void* latent, const float* meta,
                     const float* qscale, int fmt, uint32_t mask, float* state, hipStream_t st,
                     const ExcPatches* exc, const uint16_t* meta16, long long grid)
{
    WV_REQUIRE(a && state && latent && (meta || meta16) && (fmt == AE_LATENT_BF16 || qscale), WV_EINVAL,
               "decode: null buffer");
    WV_REQUIRE(!meta16 || fused_supported(a->hid, a->lat), WV_EINVAL,
               "16-bit metadata needs the fused network shape (hidden 512, latent 32)");
    const long long P = pg.P;
    if (fused_supported(a->hid, a->lat)) {
        const uint16_t* zb = (const uint16_t*)latent;
        if (fmt == AE_LATENT_FP8) {
            uint16_t* zq = (uint16_t*)workspace(a, align256(P * (size_t)a->lat * 2), st);
            hipLaunchKernelGGL(dequantize_kernel, dim3(blocks(P * a->lat, 256)), dim3(256), 0, st,
                               (const uint8_t*)latent, qscale, P, a->lat, zq);
            WV_HIP(hipGetLastError());
            zb = zq;
        }
        for (int f = 0; f < 4; ++f)
            if (mask & (1u << f))
                fused_decode(pg, zb, meta, a->wt[2], a->bias(2), a->wp4, a->bias(3), f, state, st,
                             (exc && exc->K > 0 && f == 0) ? exc : nullptr, meta16, grid);
        return;
    }
    const size_t oh = 0, ozb = align256(oh + P * (size_t)a->hid * 2);
    uint8_t* ws = (uint8_t*)workspace(a, align256(ozb + P * (size_t)a->lat * 2), st);
    uint16_t* h = (uint16_t*)(ws + oh);
    const uint16_t* zb = (const uint16_t*)latent;
    if (fmt == AE_LATENT_FP8) {
        uint16_t* zq = (uint16_t*)(ws + ozb);
        hipLaunchKernelGGL(dequantize_kernel, dim3(blocks(P * a->lat, 256)), dim3(256), 0, st, (const uint8_t*)latent,
                           qscale, P, a->lat, zq);
        WV_HIP(hipGetLastError());
        zb = zq;
    }
    gemm_auto((int)P, a->hid, a->lat, LoadK{zb, a->lat, nullptr, (int)P, a->lat},
              LoadK{a->wt[2], a->lat, nullptr, a->hid, a->lat}, EpiGelu{h, a->hid, a->bias(2), nullptr}, st);
    const long long N = (long long)pg.nz * pg.ny * pg.nx;
    for (int f = 0; f < 4; ++f) {
        if (!(mask & (1u << f))) continue;
        gemm_auto((int)P, 512, a->hid, LoadK{h, a->hid, nullptr, (int)P, a->hid},
                  LoadK{a->wt[3] + (long long)f * 512 * a->hid, a->hid, nullptr, 512, a->hid},
                  EpiDenorm{state, meta, a->bias(3) + f * 512, f, pg.ny / 8, pg.nx / 8, pg.ny, pg.nx, N}, st);
    }
    if (exc && exc->K > 0 && (mask & 1u)) exceptions_restore(pg, state, exc->K, exc->idx, exc->exc, st);
}

namespace {

// One Adam step on a batch. Returns (device) the batch loss in *dloss (added if accumulate).
struct TrainBufs {
    float *a1, *a3, *w;  // pre-activations of layers 1 and 3; sample weights
    float* wpart[4];     // per layer: weight-gradient partials of the batch splits [splits][fi][fo]
    float* bpart[4];     // per layer: bias-gradient partials, column sums per row tile [ceil(B/64)][fo]
    double* lossp;   // [row tiles][column tiles] loss partials of the output layer
    uint16_t *h1, *zb, *h3, *d4, *d3, *dz, *d1;
    // the same [width][batch] (written transposed by the epilogues: the weight gradients'
    // operands), and the batch's input rows transposed
    uint16_t *h1t, *zbt, *h3t, *d4t, *d3t, *dzt, *d1t, *yt;
    double* wsum;
    bool w_const = false;  // w and wsum hold the unweighted loss's constant weights
};

TrainBufs train_buffers(const ae_net* a, int B, int splits, hipStream_t st)
{
    const size_t in = a->in, hid = a->hid, lat = a->lat;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o = align256(o + bytes);
        return r;
    };
    const size_t nb = B;
    size_t o_wp[4], o_bp[4];
    for (int l = 0; l < 4; ++l) {
        o_wp[l] = take((size_t)splits * a->fi[l] * a->fo[l] * 4);
        o_bp[l] = take(((nb + 63) / 64) * a->fo[l] * 4);
    }
    const size_t o_a1 = take(nb * hid * 4), o_a3 = take(nb * hid * 4),
                 o_loss = take(((nb + 63) / 64) * (in / 32) * 8),
                 o_h1 = take(nb * hid * 2), o_zb = take(nb * lat * 2), o_h3 = take(nb * hid * 2),
                 o_d4 = take(nb * in * 2), o_d3 = take(nb * hid * 2), o_dz = take(nb * lat * 2),
                 o_d1 = take(nb * hid * 2), o_h1t = take(nb * hid * 2), o_zbt = take(nb * lat * 2),
                 o_h3t = take(nb * hid * 2), o_d4t = take(nb * in * 2), o_d3t = take(nb * hid * 2),
                 o_dzt = take(nb * lat * 2), o_d1t = take(nb * hid * 2), o_yt = take(nb * in * 2),
                 o_w = take(nb * 16), o_ws = take(8);
    uint8_t* w = (uint8_t*)workspace(a, o, st);
    TrainBufs t;
    t.a1 = (float*)(w + o_a1);
    t.a3 = (float*)(w + o_a3);
    for (int l = 0; l < 4; ++l) {
        t.wpart[l] = (float*)(w + o_wp[l]);
        t.bpart[l] = (float*)(w + o_bp[l]);
    }
    t.lossp = (double*)(w + o_loss);
    t.h1 = (uint16_t*)(w + o_h1);
    t.zb = (uint16_t*)(w + o_zb);
    t.h3 = (uint16_t*)(w + o_h3);
    t.d4 = (uint16_t*)(w + o_d4);
    t.d3 = (uint16_t*)(w + o_d3);
    t.dz = (uint16_t*)(w + o_dz);
    t.d1 = (uint16_t*)(w + o_d1);
    t.h1t = (uint16_t*)(w + o_h1t);
    t.zbt = (uint16_t*)(w + o_zbt);
    t.h3t = (uint16_t*)(w + o_h3t);
    t.d4t = (uint16_t*)(w + o_d4t);
    t.d3t = (uint16_t*)(w + o_d3t);
    t.dzt = (uint16_t*)(w + o_dzt);
    t.d1t = (uint16_t*)(w + o_d1t);
    t.yt = (uint16_t*)(w + o_yt);
    t.w = (float*)(w + o_w);
    t.wsum = (double*)(w + o_ws);
    return t;
}

// weight gradient dW[fi][fo] = X^T D with split-K over the batch
// dst [C][R] = src rows transposed: dst[c][r] = src[rows ? rows[r] : r][c] for a bf16
// matrix of R rows (R % 8 == 0) and C columns (C % 8 == 0) with row stride ld; 64 x 64
// tiles through LDS, 16-byte loads and stores
__global__ void __launch_bounds__(256) transpose_kernel(const uint16_t* __restrict__ src, long long ld,
                                                        const int* __restrict__ rows, int R, int C,
                                                        uint16_t* __restrict__ dst)
{
    __shared__ uint16_t tile[64][64 + 2];
    const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int k = threadIdx.x + 256 * q;
        const int r = k >> 3, c8 = (k & 7) * 8;
        uint16_t v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (r0 + r < R && c0 + c8 < C) {
            const long long sr = rows ? rows[r0 + r] : r0 + r;
            const uint4 w = *reinterpret_cast<const uint4*>(src + sr * ld + c0 + c8);
            memcpy(v, &w, 16);
        }
        for (int i = 0; i < 8; ++i) tile[r][c8 + i] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int k = threadIdx.x + 256 * q;
        const int c = k >> 3, r8 = (k & 7) * 8;
        if (c0 + c < C && r0 + r8 < R) {
            uint16_t v[8];
            for (int i = 0; i < 8; ++i) v[i] = tile[r8 + i][c];
            uint4 w;
            memcpy(&w, v, 16);
            *reinterpret_cast<uint4*>(dst + (long long)(c0 + c) * R + r0 + r8) = w;
        }
    }
}

void transpose_rows(const uint16_t* src, long long ld, const int* rows, int R, int C, uint16_t* dst, hipStream_t st)
{
    hipLaunchKernelGGL(transpose_kernel, dim3((C + 63) / 64, (R + 63) / 64), dim3(256), 0, st, src, ld, rows, R, C,
                       dst);
    WV_HIP(hipGetLastError());
}

// dW_l = X^T D over the batch, from both operands stored transposed ([width][batch], so
// the GEMM streams whole k-contiguous rows): the batch is split `splits` ways and the
// partials are summed at the end of the batch (sum_grads)
void weight_grad(ae_net* a, int l, int B, const uint16_t* Xt, const uint16_t* Dt, TrainBufs& t, int splits,
                 hipStream_t st)
{
    const int fi = a->fi[l], fo = a->fo[l];
    gemm_auto(fi, fo, B, LoadK{Xt, B, nullptr, fi, B}, LoadK{Dt, B, nullptr, fo, B},
              EpiF32{t.wpart[l], fo, (long long)fi * fo, nullptr}, st, splits);
}

// every gradient of the batch from its partials, in one launch: the 4 weight gradients
// (split sums) and the 4 bias gradients (row-tile column sums of width fo_l, from
// work-group tiles of bm[l] rows), each summed in a fixed order
void sum_grads(ae_net* a, int B, int splits, const int* bm, TrainBufs& t, hipStream_t st)
{
    SumSegs g{};
    long long q = 0;
    int sg = 0;
    for (int l = 0; l < 4; ++l)
        for (int b = 0; b < 2; ++b) {
            const long long n = b ? a->fo[l] : (long long)a->fi[l] * a->fo[l];
            WV_REQUIRE(n % 4 == 0, WV_EINVAL, "gradient sums need layer widths that are multiples of 4");
            g.part[sg] = b ? t.bpart[l] : t.wpart[l];
            g.out[sg] = a->grad + (b ? a->ob[l] : a->oW[l]);
            g.n4[sg] = n / 4;
            g.splits[sg] = b ? (B + bm[l] - 1) / bm[l] : splits;
            g.first[sg] = q;
            q += n / 4;
            ++sg;
        }
    g.first[sg] = q;
    g.nseg = sg;
    hipLaunchKernelGGL(sums_kernel, dim3(blocks(q, 256)), dim3(256), 0, st, g);
}

void train_batch(ae_net* a, const uint16_t* y, const float* meta, int weighting, const int* idx, int B,
                 TrainBufs& t, int splits, double* dloss, int accumulate, hipStream_t st)
{
    const int in = a->in, hid = a->hid, lat = a->lat;
    // forward; the epilogues also write the transposed activations the weight gradients read
    gemm_auto(B, hid, in, LoadK{y, in, idx, B, in}, LoadK{a->wt[0], in, nullptr, hid, in},
              EpiGelu{t.h1, hid, a->bias(0), t.a1, t.h1t, B}, st);
    gemm_auto(B, lat, hid, LoadK{t.h1, hid, nullptr, B, hid}, LoadK{a->wt[1], hid, nullptr, lat, hid},
              EpiBF16T{t.zb, lat, a->bias(1), nullptr, t.zbt, B}, st);
    gemm_auto(B, hid, lat, LoadK{t.zb, lat, nullptr, B, lat}, LoadK{a->wt[2], lat, nullptr, hid, lat},
              EpiGelu{t.h3, hid, a->bias(2), t.a3, t.h3t, B}, st);
    // output layer with the loss: d4 (bf16 and transposed), the b4 gradient's row-tile
    // partials, the loss per tile
    // (the plain loss's weights are all 1, the same for every batch: set once)
    if (weighting || !t.w_const) {
        hipLaunchKernelGGL(batch_weights_kernel, dim3(1), dim3(256), 0, st, meta, idx, B, a->beta_d, weighting, t.w,
                           t.wsum);
        t.w_const = !weighting;
    }
    // rows of the work-group tiles whose column sums make each layer's bias gradient
    const int bm[4] = {gemm_auto_bm(B, hid), gemm_auto_bm(B, lat), gemm_auto_bm(B, hid), gemm_auto_bm(B, in)};
    const int bn4 = gemm_auto_bn(B, in);
    gemm_auto(B, in, hid, LoadK{t.h3, hid, nullptr, B, hid}, LoadK{a->wt[3], hid, nullptr, in, hid},
              EpiMse{a->bias(3), y, idx, in, t.w, t.wsum, t.d4, t.bpart[3], t.lossp, in / bn4, t.d4t, B}, st);
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, st, t.lossp,
                       ((B + bm[3] - 1) / bm[3]) * (in / bn4), 1.0, dloss, accumulate);
    // backward: layer 4
    weight_grad(a, 3, B, t.h3t, t.d4t, t, splits, st);
    gemm_auto(B, hid, in, LoadK{t.d4, in, nullptr, B, in}, LoadK{a->wb[3], in, nullptr, hid, in},
              EpiGeluBack{t.d3, t.a3, hid, t.bpart[2], t.d3t, B}, st);
    // layer 3
    weight_grad(a, 2, B, t.zbt, t.d3t, t, splits, st);
    gemm_auto(B, lat, hid, LoadK{t.d3, hid, nullptr, B, hid}, LoadK{a->wb[2], hid, nullptr, lat, hid},
              EpiBF16T{t.dz, lat, nullptr, t.bpart[1], t.dzt, B}, st);
    // layer 2
    weight_grad(a, 1, B, t.h1t, t.dzt, t, splits, st);
    gemm_auto(B, hid, lat, LoadK{t.dz, lat, nullptr, B, lat}, LoadK{a->wb[1], lat, nullptr, hid, lat},
              EpiGeluBack{t.d1, t.a1, hid, t.bpart[0], t.d1t, B}, st);
    // layer 1: the batch's input rows, gathered and transposed
    transpose_rows(y, in, idx, B, in, t.yt, st);
    weight_grad(a, 0, B, t.yt, t.d1t, t, splits, st);
    sum_grads(a, B, splits, bm, t, st);
    WV_HIP(hipGetLastError());
}

// split of the batch (the GEMM depth) in the weight gradients: enough work-groups to
// fill the CUs, partials summed in a fixed order
#ifndef WV_TRAIN_SPLITS_MAX
#define WV_TRAIN_SPLITS_MAX 8
#endif
int train_splits(int B) { return std::max(1, std::min(WV_TRAIN_SPLITS_MAX, B / 512)); }

void adam_update(ae_net* a, double lr, const ae_train_cfg& cfg, hipStream_t st, bool pack = true)
{
    a->step += 1;
    const double c1 = 1.0 - std::pow(cfg.beta1, (double)a->step);
    const double c2 = 1.0 - std::pow(cfg.beta2, (double)a->step);
    hipLaunchKernelGGL(adam_kernel, dim3(blocks(a->nparam, 256)), dim3(256), 0, st, a->master, a->m1, a->m2, a->grad,
                       a->nparam, (float)lr, (float)cfg.beta1, (float)cfg.beta2, (float)cfg.eps, (float)c1, (float)c2);
    WV_HIP(hipGetLastError());
    refresh_bf16(a, st, pack);
}

ae_net* new_net(int in, int hid, int lat)
{
    WV_REQUIRE(in == 2048, WV_EINVAL, "in_dim must be 2048 (4 fields x 8^3 cells)");
    WV_REQUIRE(hid >= 64 && hid % 64 == 0, WV_EINVAL, "hidden must be a positive multiple of 64");
    WV_REQUIRE(lat >= 16 && lat <= 64 && lat % 16 == 0, WV_EINVAL, "latent must be 16, 32, 48 or 64");
    std::unique_ptr<ae_net> a(new ae_net());
    a->in = in;
    a->hid = hid;
    a->lat = lat;
    layout(a.get());
    a->master = dalloc<float>(a->nparam);
    a->m1 = dalloc<float>(a->nparam);
    a->m2 = dalloc<float>(a->nparam);
    a->grad = dalloc<float>(a->nparam);
    WV_HIP(hipMemset(a->m1, 0, a->nparam * 4));
    WV_HIP(hipMemset(a->m2, 0, a->nparam * 4));
    WV_HIP(hipMemset(a->grad, 0, a->nparam * 4));
    for (int l = 0; l < 4; ++l) {
        a->wb[l] = dalloc<uint16_t>((size_t)a->fi[l] * a->fo[l]);
        a->wt[l] = dalloc<uint16_t>((size_t)a->fi[l] * a->fo[l]);
    }
    if (fused_supported(hid, lat)) {
        a->wp1 = dalloc<uint16_t>((size_t)in * hid);
        a->wp4 = dalloc<uint16_t>((size_t)in * hid);
    }
    a->beta_d = dalloc<float>(4);
    a->loss_d = dalloc<double>(1);
    upload_beta(a.get());
    return a.release();
}

void free_net(ae_net* a)
{
    if (!a) return;
    (void)hipDeviceSynchronize();
    for (float* p : {a->master, a->m1, a->m2, a->grad, a->beta_d})
        if (p) (void)hipFree(p);
    if (a->loss_d) (void)hipFree(a->loss_d);
    for (int l = 0; l < 4; ++l) {
        if (a->wb[l]) (void)hipFree(a->wb[l]);
        if (a->wt[l]) (void)hipFree(a->wt[l]);
    }
    if (a->wp1) (void)hipFree(a->wp1);
    if (a->wp4) (void)hipFree(a->wp4);
    for (auto& q : a->ws)
        if (q.p) (void)hipFree(q.p);
    delete a;
}

}  // namespace

// ---- the allocation-free encode ----------------------------------------------------
// ae_encode_noalloc stages the float32 latents of an FP8 encode (P x latent floats)
// in this file-scope device array instead of the per-stream work buffer. Each device
// holds its own copy; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device (the array's name is a host-side
// stand-in, not a device address).
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(16) << 20;
__device__ __align__(256) uint8_t scratch[NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// device address of `scratch` on the current device, looked up once per device
void* noalloc_scratch()
{
    int dev = -1;
    WV_HIP(hipGetDevice(&dev));
    WV_REQUIRE(dev >= 0 && dev < NOALLOC_MAX_DEVICES, WV_EDEVICE, "device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            throw Error{WV_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace
}  // namespace wv

// ======================================================================================
extern "C" {

int ae_create(int32_t in_dim, int32_t hidden, int32_t latent, const float* h_init, const double* h_beta, ae_net** out)
{
    return guarded_ae([&]() -> int {
        WV_REQUIRE(out && h_init, WV_EINVAL, "null argument");
        ae_net* a = new_net(in_dim, hidden, latent);
        try {
            WV_HIP(hipMemcpy(a->master, h_init, a->nparam * 4, hipMemcpyHostToDevice));
            if (h_beta)
                for (int f = 0; f < 4; ++f) a->beta[f] = h_beta[f];
            upload_beta(a);
            refresh_bf16(a, nullptr);
            WV_HIP(hipDeviceSynchronize());
        } catch (...) {
            free_net(a);
            throw;
        }
        *out = a;
        return WV_OK;
    });
}

void ae_destroy(ae_net* net) { free_net(net); }

int ae_param_count(const ae_net* a, int64_t* n)
{
    if (!a || !n) {
        set_error("null argument");
        return WV_EINVAL;
    }
    *n = a->nparam;
    return WV_OK;
}

int ae_get_params(const ae_net* a, float* h_out)
{
    return guarded_ae([&]() -> int {
        WV_REQUIRE(a && h_out, WV_EINVAL, "null argument");
        WV_HIP(hipDeviceSynchronize());
        WV_HIP(hipMemcpy(h_out, a->master, a->nparam * 4, hipMemcpyDeviceToHost));
        return WV_OK;
    });
}

int ae_set_params(ae_net* a, const float* h_in)
{
    return guarded_ae([&]() -> int {
        WV_REQUIRE(a && h_in, WV_EINVAL, "null argument");
        WV_HIP(hipDeviceSynchronize());
        WV_HIP(hipMemcpy(a->master, h_in, a->nparam * 4, hipMemcpyHostToDevice));
        refresh_bf16(a, nullptr);
        WV_HIP(hipDeviceSynchronize());
        return WV_OK;
    });
}

int ae_set_beta(ae_net* a, const double* h_beta)
{
    return guarded_ae([&]() -> int {
        WV_REQUIRE(a && h_beta, WV_EINVAL, "null argument");
        for (int f = 0; f < 4; ++f) {
            WV_REQUIRE(h_beta[f] > 0 && std::isfinite(h_beta[f]), WV_EINVAL, "beta must be positive");
            a->beta[f] = h_beta[f];
        }
        upload_beta(a);
        return WV_OK;
    });
}

int ae_get_beta(const ae_net* a, double* h_beta)
{
    if (!a || !h_beta) {
        set_error("null argument");
        return WV_EINVAL;
    }
    for (int f = 0; f < 4; ++f) h_beta[f] = a->beta[f];
    return WV_OK;
}

int ae_fit_beta(ae_net* a, const wv_grid* g, const float* states, int64_t nstates, double rel, void* stream)
{
    return guarded_ae([&]() -> int {
        WV_REQUIRE(a && g && states && nstates > 0 && rel > 0, WV_EINVAL, "bad argument");
        hipStream_t st = (hipStream_t)stream;
        const long long N = (long long)g->nz * g->ny * g->nx;
        double* d = dalloc<double>(4);
        launch_absmax_fields(states, nstates, N, d, st);
        double h[4];
        WV_HIP(hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, st));
        WV_HIP(hipStreamSynchronize(st));
        (void)hipFree(d);
        for (int f = 0; f < 4; ++f) a->beta[f] = h[f] > 0 ? rel * h[f] : rel;
        upload_beta(a);
        return WV_OK;
    });
}

int ae_save(const ae_net* a, const char* path)
{
    return guarded_ae([&]() -> int {
        WV_REQUIRE(a && path, WV_EINVAL, "null argument");
        WV_HIP(hipDeviceSynchronize());
        std::vector<float> buf(a->nparam);
        FILE* f = fopen(path, "wb");
        WV_REQUIRE(f, WV_EINVAL, std::string("cannot open ") + path);
        const char magic[8] = {'W', 'V', 'A', 'E', '0', '0', '0', '1'};
        const int32_t dims[3] = {a->in, a->hid, a->lat};
        fwrite(magic, 1, 8, f);
        fwrite(dims, sizeof(int32_t), 3, f);
        fwrite(&a->step, sizeof(long long), 1, f);
        fwrite(a->beta, sizeof(double), 4, f);
        for (const float* p : {a->master, a->m1, a->m2}) {
            WV_HIP(hipMemcpy(buf.data(), p, a->nparam * 4, hipMemcpyDeviceToHost));
            fwrite(buf.data(), 4, a->nparam, f);
        }
        const bool ok = fclose(f) == 0;
        WV_REQUIRE(ok, WV_EINVAL, "write failed");
        return WV_OK;
    });
}

int ae_load(const char* path, ae_net** out)
{
    return guarded_ae([&]() -> int {
        WV_REQUIRE(path && out, WV_EINVAL, "null argument");
        FILE* f = fopen(path, "rb");
        WV_REQUIRE(f, WV_EINVAL, std::string("cannot open ") + path);
        char magic[8];
        int32_t dims[3];
        long long step;
        double beta[4];
        bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, "WVAE0001", 8) == 0 &&
                  fread(dims, sizeof(int32_t), 3, f) == 3 && fread(&step, sizeof(long long), 1, f) == 1 &&
                  fread(beta, sizeof(double), 4, f) == 4;
        if (!ok) {
            fclose(f);
            throw Error{WV_EINVAL, "not an autoencoder file"};
        }
        ae_net* a = new_net(dims[0], dims[1], dims[2]);
        std::vector<float> buf(a->nparam);
        for (float* p : {a->master, a->m1, a->m2}) {
            if (fread(buf.data(), 4, a->nparam, f) != (size_t)a->nparam) {
                fclose(f);
                free_net(a);
                throw Error{WV_EINVAL, "truncated autoencoder file"};
            }
            WV_HIP(hipMemcpy(p, buf.data(), a->nparam * 4, hipMemcpyHostToDevice));
        }
        fclose(f);
        a->step = step;
        for (int q = 0; q < 4; ++q) a->beta[q] = beta[q];
        upload_beta(a);
        refresh_bf16(a, nullptr);
        WV_HIP(hipDeviceSynchronize());
        *out = a;
        return WV_OK;
    });
}

int ae_normalize(const ae_net* a, const wv_grid* g, const float* state, uint16_t* y, float* meta, void* stream)
{
    return guarded_ae([&]() -> int {
        WV_REQUIRE(a && state && y && meta, WV_EINVAL, "null argument");
        check_grid(g);
        normalize_state(a, patch_grid(g->nz, g->ny, g->nx), state, y, meta, (hipStream_t)stream);
        return WV_OK;
    });
}

int ae_normalize_rows(const ae_net* a, const wv_grid* g, const float* state, const int32_t* rows, int32_t nrows,
                      uint16_t* y, float* meta, void* stream)
{
    return guarded_ae([&]() -> int {
        WV_REQUIRE(a && state && (nrows == 0 || (rows && y && meta)), WV_EINVAL, "null argument");
        WV_REQUIRE(nrows >= 0, WV_EINVAL, "nrows must be >= 0");
        check_grid(g);
        const PatchGrid pg = patch_grid(g->nz, g->ny, g->nx);
        if (nrows == 0) return WV_OK;
        // every row must name a patch of the grid before the kernel reads it
        std::vector<int32_t> h((size_t)nrows);
        const hipStream_t st = (hipStream_t)stream;
        WV_HIP(hipMemcpyAsync(h.data(), rows, sizeof(int32_t) * nrows, hipMemcpyDeviceToHost, st));
        WV_HIP(hipStreamSynchronize(st));
        for (int32_t v : h) WV_REQUIRE(v >= 0 && v < pg.P, WV_EINVAL, "row index outside the patch grid");
        normalize_rows(a, pg, state, rows, nrows, y, meta, st);
        return WV_OK;
    });
}

int ae_time_fit_beta(ae_net* a, const wv_grid* g, const float* e, int64_t nlevels, double rel, void* stream)
{
    return guarded_ae([&]() -> int {
        WV_REQUIRE(a && g && e && nlevels > 0 && rel > 0, WV_EINVAL, "bad argument");
        check_time_grid(g);
        hipStream_t st = (hipStream_t)stream;
        const long long n = nlevels * g->nsrc * (long long)g->nz * g->ny * g->nx;
        constexpr int NB = 1024;
        double* d = dalloc<double>(3 * NB + 3);
        launch_range(e, n, d, NB, d + 3 * NB, st);
        double h[3];
        WV_HIP(hipMemcpyAsync(h, d + 3 * NB, sizeof(h), hipMemcpyDeviceToHost, st));
        WV_HIP(hipStreamSynchronize(st));
        (void)hipFree(d);
        WV_REQUIRE(h[2] == 0.0, WV_EINVAL, "e contains NaN");
        const double m = std::max(std::fabs(h[0]), std::fabs(h[1]));
        a->beta[0] = m > 0 ? rel * m : rel;
        upload_beta(a);
        return WV_OK;
    });
}

int ae_time_normalize(const ae_net* a, const wv_grid* g, const float* e_win, int32_t nvalid, const int32_t* rows,
                      int32_t nrows, uint16_t* y, float* meta, void* stream)
{
    return guarded_ae([&]() -> int {
        WV_REQUIRE(a && e_win && y && meta, WV_EINVAL, "null argument");
        check_time_grid(g);
        const TimeGrid tg = time_grid(g->nz, g->ny, g->nx, g->nsrc);
        const hipStream_t st = (hipStream_t)stream;
        long long n = tg.B * tg.S;
        if (rows) {
            WV_REQUIRE(nrows >= 0, WV_EINVAL, "nrows must be >= 0");
            std::vector<int32_t> h((size_t)nrows);
            if (nrows) {
                WV_HIP(hipMemcpyAsync(h.data(), rows, sizeof(int32_t) * nrows, hipMemcpyDeviceToHost, st));
                WV_HIP(hipStreamSynchronize(st));
            }
            for (int32_t v : h) WV_REQUIRE(v >= 0 && v < n, WV_EINVAL, "row index outside the block grid");
            n = nrows;
        }
        ae_time_normalize_rows(a, tg, e_win, nvalid, rows, n, y, meta, st);
        return WV_OK;
    });
}

int ae_time_encode(const ae_net* a, const wv_grid* g, const float* e_win, int32_t nvalid, uint16_t* latent,
                   float* meta, void* stream)
{
    return guarded_ae([&]() -> int {
        WV_REQUIRE(a && e_win && latent && meta, WV_EINVAL, "null argument");
        check_time_grid(g);
        wv::ae_time_encode(a, time_grid(g->nz, g->ny, g->nx, g->nsrc), e_win, nvalid, latent, meta,
                           (hipStream_t)stream);
        return WV_OK;
    });
}

int ae_time_decode(const ae_net* a, const wv_grid* g, const uint16_t* latent, const float* meta, int32_t nvalid,
                   float* e_win, void* stream)
{
    return guarded_ae([&]() -> int {
        WV_REQUIRE(a && latent && meta && e_win, WV_EINVAL, "null argument");
        check_time_grid(g);
        wv::ae_time_decode(a, time_grid(g->nz, g->ny, g->nx, g->nsrc), latent, meta, nvalid, e_win,
                           (hipStream_t)stream);
        return WV_OK;
    });
}

int ae_encode(const ae_net* a, const wv_grid* g, const float* state, int fmt, void* latent, float* meta,
              float* qscale, void* stream)
{
    return guarded_ae([&]() -> int {
        WV_REQUIRE(a && state && latent && meta, WV_EINVAL, "null argument");
        WV_REQUIRE(fmt == AE_LATENT_BF16 || (fmt == AE_LATENT_FP8 && qscale), WV_EINVAL, "bad latent format/scale");
        check_grid(g);
        ae_encode_state(a, patch_grid(g->nz, g->ny, g->nx), state, fmt, latent, meta, qscale, (hipStream_t)stream);
        return WV_OK;
    });
}

int ae_decode(const ae_net* a, const wv_grid* g, const void* latent, const float* meta, const float* qscale, int fmt,
              uint32_t mask, float* state, void* stream)
{
    return guarded_ae([&]() -> int {
        WV_REQUIRE(a && latent && meta && state, WV_EINVAL, "null argument");
        WV_REQUIRE(fmt == AE_LATENT_BF16 || (fmt == AE_LATENT_FP8 && qscale), WV_EINVAL, "bad latent format/scale");
        WV_REQUIRE((mask & ~0xFu) == 0, WV_EINVAL, "field mask has bits beyond the 4 fields");
        check_grid(g);
        ae_decode_state(a, patch_grid(g->nz, g->ny, g->nx), latent, meta, qscale, fmt, mask, state,
                        (hipStream_t)stream);
        return WV_OK;
    });
}

int ae_train_step(ae_net* a, const uint16_t* y, const float* meta, const int32_t* idx, int32_t B, double lr,
                  const ae_train_cfg* cfg, float* h_grads, double* h_loss, void* stream)
{
    return guarded_ae([&]() -> int {
        WV_REQUIRE(a && y && cfg && B > 0, WV_EINVAL, "bad argument");
        WV_REQUIRE(!cfg->weighting || meta, WV_EINVAL, "weighted loss needs meta");
        WV_REQUIRE(B % 32 == 0, WV_EINVAL, "batch must be a multiple of 32");
        hipStream_t st = (hipStream_t)stream;
        const int splits = train_splits(B);
        TrainBufs t = train_buffers(a, B, splits, st);
        double* dloss = a->loss_d;
        train_batch(a, y, meta, cfg->weighting, idx, B, t, splits, dloss, 0, st);
        if (h_grads) WV_HIP(hipMemcpyAsync(h_grads, a->grad, a->nparam * 4, hipMemcpyDeviceToHost, st));
        adam_update(a, lr, *cfg, st);
        double L = 0;
        WV_HIP(hipMemcpyAsync(&L, dloss, sizeof(double), hipMemcpyDeviceToHost, st));
        WV_HIP(hipStreamSynchronize(st));
        if (h_loss) *h_loss = L;
        return WV_OK;
    });
}

int ae_train(ae_net* a, const uint16_t* y, const float* meta, int64_t nsamples, const ae_train_cfg* cfg,
             const int32_t* perm, float* h_loss, void* stream)
{
    return guarded_ae([&]() -> int {
        WV_REQUIRE(a && y && cfg, WV_EINVAL, "null argument");
        WV_REQUIRE(!cfg->weighting || meta, WV_EINVAL, "weighted loss needs meta");
        WV_REQUIRE(cfg->batch > 0 && cfg->batch % 32 == 0, WV_EINVAL, "batch must be a positive multiple of 32");
        WV_REQUIRE(cfg->epochs >= 0 && nsamples >= cfg->batch, WV_EINVAL, "need at least one full batch");
        hipStream_t st = (hipStream_t)stream;
        const int B = cfg->batch;
        const int splits = train_splits(B);
        TrainBufs t = train_buffers(a, B, splits, st);
        double* dloss = a->loss_d;
        const long long nb = nsamples / B;
        std::vector<int> seq;
        int* dseq = nullptr;
        if (!perm) {
            seq.resize(nsamples);
            for (long long q = 0; q < nsamples; ++q) seq[q] = (int)q;
            dseq = dalloc<int>(nsamples);
            WV_HIP(hipMemcpyAsync(dseq, seq.data(), sizeof(int) * nsamples, hipMemcpyHostToDevice, st));
        }
        for (int e = 0; e < cfg->epochs; ++e) {
            const double lr = cfg->lr * std::pow(cfg->decay_factor, (double)(e / std::max(cfg->decay_every, 1)));
            const int* order = perm ? perm + (long long)e * nsamples : dseq;
            for (long long b = 0; b < nb; ++b) {
                train_batch(a, y, meta, cfg->weighting, order + b * B, B, t, splits, dloss, b > 0, st);
                adam_update(a, lr, *cfg, st, false);
            }
            double L = 0;
            WV_HIP(hipMemcpyAsync(&L, dloss, sizeof(double), hipMemcpyDeviceToHost, st));
            WV_HIP(hipStreamSynchronize(st));
            if (h_loss) h_loss[e] = (float)(L / (double)nb);
        }
        pack_fused(a, st);
        WV_HIP(hipStreamSynchronize(st));
        if (dseq) (void)hipFree(dseq);
        return WV_OK;
    });
}

int ae_encode_noalloc(const ae_net* a, const wv_grid* g, const float* state, int fmt, void* latent, float* meta,
                      float* qscale, void* stream)
{
    return guarded_ae([&]() -> int {
        WV_REQUIRE(a && state && latent && meta, WV_EINVAL, "null argument");
        WV_REQUIRE(fmt == AE_LATENT_BF16 || (fmt == AE_LATENT_FP8 && qscale), WV_EINVAL, "bad latent format/scale");
        check_grid(g);
        WV_REQUIRE(fused_supported(a->hid, a->lat), WV_EINVAL,
                   "ae_encode_noalloc needs the fused network shape (hidden 512, latent 32)");
        const PatchGrid pg = patch_grid(g->nz, g->ny, g->nx);
        const hipStream_t st = (hipStream_t)stream;
        const long long N = (long long)pg.nz * pg.ny * pg.nx;
        const int rows = (pg.nz / 8) * (pg.ny / 8);
        if (fmt == AE_LATENT_FP8) {
            const size_t need = (size_t)pg.P * a->lat * sizeof(float);
            WV_REQUIRE(need <= NOALLOC_SCRATCH_BYTES, WV_EINVAL,
                       "ae_encode_noalloc: FP8 staging needs " + std::to_string(need) + " bytes, beyond the " +
                           std::to_string(NOALLOC_SCRATCH_BYTES) + "-byte static scratch (at most " +
                           std::to_string(NOALLOC_SCRATCH_BYTES / (a->lat * sizeof(float))) + " patches)");
        }
        // the same kernels as ae_encode; only the FP8 staging buffer differs
        hipLaunchKernelGGL(minmax_kernel, dim3(rows), dim3(std::min(256, ((pg.nx + 63) / 64) * 64)), 0, st, state,
                           pg.ny, pg.nx, N, pg.ny / 8, pg.nx / 8, a->beta_d, meta);
        WV_HIP(hipGetLastError());
        if (fmt == AE_LATENT_BF16) {
            fused_encode(pg, state, meta, nullptr, 0, a->beta_d, a->wp1, a->bias(0), a->wt[1], a->bias(1),
                         (uint16_t*)latent, nullptr, st);
            return WV_OK;
        }
        float* z = (float*)noalloc_scratch();
        fused_encode(pg, state, meta, nullptr, 0, a->beta_d, a->wp1, a->bias(0), a->wt[1], a->bias(1), nullptr, z,
                     st);
        hipLaunchKernelGGL(quantize_kernel, dim3(blocks(pg.P, 4)), dim3(256), 0, st, z, pg.P, a->lat,
                           (uint8_t*)latent, qscale);
        WV_HIP(hipGetLastError());
        return WV_OK;
    });
}

}  // extern "C"

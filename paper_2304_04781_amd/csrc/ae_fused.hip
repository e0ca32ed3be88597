// Fused autoencoder inference kernels for the time loop (gfx950, bf16 MFMA).
//
// encode: one work-group of eight waves compresses 128 patches. The A operand (the
// normalised patch vectors) is built on the fly from the float32 state and the per-patch
// (min, range) metadata, rounded to bfloat16 and shared through LDS; each wave owns 64 of
// the 512 hidden units and keeps their W1 fragments in registers, loaded straight from L2.
// The second layer runs in the same work-group, split over the waves' hidden units.
// decode: the mirror image for one field: latent -> hidden (bias + GELU, LDS)
// -> 512 outputs of that field -> de-normalised float32 written into the state.
//
// Layout of a 16x16x32 bf16 MFMA (v_mfma_f32_16x16x32_bf16): A lane l holds
// row l%16, k = 8*(l/16)..+7; B lane l holds column l%16, same k; C lane l
// holds column l%16, rows 4*(l/16)..+3.

#include <algorithm>
#include <type_traits>

#include "ae_internal.h"
#include "ae_math.h"

namespace wv {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int BM = 128;       // patches per encode work-group
constexpr int NT = 512;       // threads (8 waves)
constexpr int HID = 512;      // hidden width handled by these kernels
constexpr int KB = 32;        // k per MFMA step
constexpr int HPAD = 8;       // bf16 padding per row of the decode's hidden layer

struct EncArgs {
    const float* state;   // [4][N]
    const float* meta;    // [P][4][2] (min, range); output when mm is given
    uint16_t* meta16;     // with mm: 16-bit output instead of meta (bfloat16 (lo, r), lo rounded
                          // down and r up, the values the normalisation then uses)
    const float* mm;      // optional [P][H][4][2] partial (min, max) from the forward step
    int H;
    const float* beta;    // [4] range floors (with mm)
    const uint16_t* w1p;  // W1^T [HID][2048] in fragment order
    const float* b1;      // [HID]
    const uint16_t* w2t;  // [L][HID]
    const float* b2;      // [L]
    uint16_t* zbf;        // [P][L] bf16 latent (or null)
    float* zf;            // [P][L] float32 latent (or null)
    long long P, N;
    int ny, nx, Py, Px;
    long long t0;         // first 128-patch tile of the launch
};

struct DecArgs {
    const uint16_t* z;    // [P][L] bf16
    const float* meta;
    const uint16_t* meta16;  // bfloat16 (lo, r) instead of meta when non-null
    const uint16_t* w3t;  // [HID][L]
    const float* b3;
    const uint16_t* w4p;  // W4^T [2048][HID] in fragment order, rows of field f at f*512
    const float* b4;      // [2048]
    float* state;         // [4][N]
    int f;
    long long P, N;
    int ny, nx, Py, Px;
    // exception patches (none when eidx is null): increasing indices, exact values
    // [K][512], per-work-group ranges into eidx
    const int* eidx;
    const float* exc;
    const int* erng;
    long long t0;  // first DEC_BM-patch tile of the launch
};

// Per-patch (lo, 1/r) of the work-group's bm patches into sMeta [bm][8] (threads
// tid < bm, one patch each). From the forward step's (min, max) partials the metadata is
// also computed here and published (float32, or bfloat16 with lo rounded down and r up);
// otherwise it is read from `meta`.
__device__ __forceinline__ void enc_meta(const EncArgs& a, long long m0, int tid, float* sMeta, int bm)
{
    if (tid < bm) {
        const long long p = m0 + tid;
        if (a.mm) {
            // combine the y sub-tile partials: r = max(max - min, beta_f); publish the metadata
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                float lo = 0.f, r = 1.f;
                if (p < a.P) {
                    lo = a.mm[(p * a.H) * 8 + 2 * f];
                    float hi = a.mm[(p * a.H) * 8 + 2 * f + 1];
                    for (int h = 1; h < a.H; ++h) {
                        lo = fminf(lo, a.mm[(p * a.H + h) * 8 + 2 * f]);
                        hi = fmaxf(hi, a.mm[(p * a.H + h) * 8 + 2 * f + 1]);
                    }
                    r = fmaxf(hi - lo, a.beta[f]);
                    if (a.meta16) {
                        // 16-bit metadata: lo_b <= lo and lo_b + r_b >= hi, so y stays in [0, 1]
                        // up to rounding and the decode reads the very values used here
                        const uint16_t lb = bf16_down(lo);
                        lo = bf2f(lb);
                        const uint16_t rb = bf16_up(fmaxf(hi - lo, a.beta[f]));
                        r = bf2f(rb);
                        a.meta16[p * 8 + 2 * f] = lb;
                        a.meta16[p * 8 + 2 * f + 1] = rb;
                    } else {
                        const_cast<float*>(a.meta)[p * 8 + 2 * f] = lo;
                        const_cast<float*>(a.meta)[p * 8 + 2 * f + 1] = r;
                    }
                }
                sMeta[tid * 8 + 2 * f] = lo;
                sMeta[tid * 8 + 2 * f + 1] = 1.0f / r;
            }
        } else {
            const float4 m01 = p < a.P ? *reinterpret_cast<const float4*>(a.meta + p * 8) : make_float4(0.f, 1.f, 0.f, 1.f);
            const float4 m23 = p < a.P ? *reinterpret_cast<const float4*>(a.meta + p * 8 + 4) : make_float4(0.f, 1.f, 0.f, 1.f);
            *reinterpret_cast<float4*>(sMeta + tid * 8) = make_float4(m01.x, 1.0f / m01.y, m01.z, 1.0f / m01.w);
            *reinterpret_cast<float4*>(sMeta + tid * 8 + 4) = make_float4(m23.x, 1.0f / m23.y, m23.z, 1.0f / m23.w);
        }
    }
}

// The encode work-group: eight waves over BM = 128 patches, wave w owning hidden units
// 64 w .. 64 w + 63. A wave loads the W1 fragments of its hidden units straight from L2
// into a register ring and each thread one raw state row of its patch into another; LDS
// holds only the normalised bfloat16 A double buffer, in the order the MFMA reads it (each
// fragment read is one contiguous 1 KiB per wave, free of bank conflicts), and the
// per-field (lo, 1/r). The second layer runs split over the waves' hidden units: each wave
// multiplies its 64 GELU outputs (staged per row tile through a private LDS area) by the
// matching columns of W2, and the eight partial latent blocks are summed in wave order
// through LDS. A work-group takes about 230 registers per lane of each wave, so one fills a
// CU's register file.
#ifndef WV_ENC_WD
#define WV_ENC_WD 3
#endif
#ifndef WV_ENC_RD
#define WV_ENC_RD 3
#endif
constexpr int ENC_WD = WV_ENC_WD, ENC_RD = WV_ENC_RD;  // register ring depths (W1, raw rows): 2 or 3
// Work-groups per encode launch (0: all tiles in one launch). An encode of more tiles is
// queued as several launches in a row on its stream, so it holds at most this many CUs at
// a time. The forward sweep needs one encode per step, and sliced encodes ran slower than
// the steps they left CUs to (128 work-groups per launch: 300 us per encode, against 182
// in one launch), so by default an encode is one launch.
#ifndef WV_ENC_GRID
#define WV_ENC_GRID 0
#endif
constexpr long long ENC_GRID = WV_ENC_GRID;
constexpr int ENC_HLD = 64 + 8;  // bf16 row of a wave's hidden staging tile [16][ENC_HLD]
constexpr int ENC_ZLD = 32 + 4;  // float row of the latent partial sums [BM][ENC_ZLD]
constexpr int ENC_R_BYTES = 8 * 16 * ENC_HLD * 2;  // the largest use of the shared region

template <int L, int WD, int RD>
__global__ void __launch_bounds__(NT) encode_kernel(const EncArgs a)
{
    static_assert(L == 32, "two latent column tiles");
    static_assert((WD == 2 || WD == 3) && (RD == 2 || RD == 3), "ring depths");
    constexpr int TI = BM / 16;             // row tiles
    constexpr int A_HALF = TI * 64 * 8;     // bf16 per A buffer: [TI][64 lanes][8]
    static_assert(NT == 4 * BM, "one thread per raw row of a step");
    static_assert(2 * A_HALF * 2 <= ENC_R_BYTES && BM * ENC_ZLD * 4 <= ENC_R_BYTES && BM * 8 * 4 <= ENC_R_BYTES,
                  "the A buffers, the second layer's staging and the metadata share one region");
    __shared__ __attribute__((aligned(16))) uint16_t sR[ENC_R_BYTES / 2];
    __shared__ __attribute__((aligned(16))) float2 sLR[4][BM];  // (lo, 1/r) per field and patch
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const long long m0 = (a.t0 + blockIdx.x) * BM;
    const int fr = lane & 15, fq = (lane >> 4) * 8, cr = (lane >> 4) * 4;

    // thread (am, aq) loads and normalises y row aq (of the four of a k-step) of patch am:
    // a wave covers one row of 64 patches. Rows of patches past P read patch 0 and are zeroed.
    const int am = tid & (BM - 1), aq = tid / BM;
    const long long pa = m0 + am;
    const bool a_ok = pa < a.P;
    long long abase = 0;
    if (a_ok) {
        const long long px = pa % a.Px, py = (pa / a.Px) % a.Py, pz = pa / ((long long)a.Px * a.Py);
        abase = ((pz * 8) * a.ny + py * 8 + aq) * a.nx + px * 8;
    }
    const float* rsrc = a.state + abase;
    const long long plane = (long long)a.ny * a.nx;
    // k-step kk: field kk / 16, z level (kk % 16) / 2, y rows 4 (kk % 2) .. + 3. Steps past
    // the last reload the last one, so every step issues the same loads.
    auto load_raw = [&](int kk, float4(&d)[2]) {
        const int k = kk < 64 ? kk : 63;
        const float* s = rsrc + ((k >> 4) * a.N + ((k & 15) >> 1) * plane + 4 * (k & 1) * a.nx);
        d[0] = *reinterpret_cast<const float4*>(s);
        d[1] = *reinterpret_cast<const float4*>(s + 4);
    };
    // fragment-ordered W1: block (kk, hidden tile t) of 64 lanes x 8 values at ((kk * 32 + t) * 64) * 8;
    // wave w owns hidden tiles 4 w .. 4 w + 3
    const uint16_t* wsrc = a.w1p + ((long long)(wave * 4) * 64 + lane) * 8;
    auto load_w = [&](int kk, uint4(&d)[4]) {
        const int k = kk < 64 ? kk : 63;
        const uint16_t* s = wsrc + (long long)k * (HID * KB);
#pragma unroll
        for (int j = 0; j < 4; ++j) d[j] = *reinterpret_cast<const uint4*>(s + j * 512);
    };
    // register rings: W1 of kk in slot kk % WD, loaded at the start of step kk - WD + 1; the
    // raw rows of kk in slot kk % RD, loaded at the start of step kk - RD and normalised at
    // the end of step kk - 1
    uint4 wb[WD][4];
    float4 rw[RD][2];
#pragma unroll
    for (int q = 0; q < RD; ++q) load_raw(q, rw[q]);
#pragma unroll
    for (int q = 0; q < WD - 1; ++q) load_w(q, wb[q]);

    {
        float* sMeta = reinterpret_cast<float*>(sR);  // [BM][8], free again once sLR is filled
        enc_meta(a, m0, tid, sMeta, BM);
        __syncthreads();
        if (tid < BM) {
            const float4 m01 = *reinterpret_cast<const float4*>(sMeta + tid * 8);
            const float4 m23 = *reinterpret_cast<const float4*>(sMeta + tid * 8 + 4);
            sLR[0][tid] = make_float2(m01.x, m01.y);
            sLR[1][tid] = make_float2(m01.z, m01.w);
            sLR[2][tid] = make_float2(m23.x, m23.y);
            sLR[3][tid] = make_float2(m23.z, m23.w);
        }
        __syncthreads();
    }
    // A fragment (row tile i, lane l) holds patch 16 i + l % 16, k 8 (l / 16) .. + 7, i.e. y row
    // l / 16 of the step: thread (am, aq) writes lane am % 16 + 16 aq of tile am / 16
    const uint32_t amask = a_ok ? 0xFFFFFFFFu : 0u;
    uint16_t* const a_dst = sR + ((am >> 4) * 64 + (am & 15) + 16 * aq) * 8;
    auto normalize = [&](int kk, const float4(&x)[2], int buf) {
        const int f = (kk < 64 ? kk : 63) >> 4;
        const float2 lr = sLR[f][am];
        const float l = lr.x, ri = lr.y;
        uint4 w;
        w.x = f2bf2((x[0].x - l) * ri, (x[0].y - l) * ri) & amask;
        w.y = f2bf2((x[0].z - l) * ri, (x[0].w - l) * ri) & amask;
        w.z = f2bf2((x[1].x - l) * ri, (x[1].y - l) * ri) & amask;
        w.w = f2bf2((x[1].z - l) * ri, (x[1].w - l) * ri) & amask;
        *reinterpret_cast<uint4*>(a_dst + buf * A_HALF) = w;
    };
    normalize(0, rw[0], 0);
    __syncthreads();

    f32x4 acc[TI][4];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const uint16_t* const a_src = sR + lane * 8;
    // step kk (q = kk mod the unroll period) refills the slots the previous steps freed (W1 of
    // kk + WD - 1, raw rows of kk + RD), multiplies the A tile of kk, normalises the rows of
    // kk + 1 into the other A buffer and ends with the one barrier that separates the
    // buffers' writes and reads
    auto step = [&](int kk, auto qc) {
        constexpr int q = decltype(qc)::value;
        load_w(kk + WD - 1, wb[(q + WD - 1) % WD]);
        load_raw(kk + RD, rw[q % RD]);
        const uint16_t* src = a_src + (kk & 1) * A_HALF;
#pragma unroll
        for (int i = 0; i < TI; ++i) {
            const bf16x8 fa = *reinterpret_cast<const bf16x8*>(src + i * 512);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, __builtin_bit_cast(bf16x8, wb[q % WD][j]),
                                                                    acc[i][j], 0, 0, 0);
        }
        normalize(kk + 1, rw[(q + 1) % RD], (kk + 1) & 1);
        __syncthreads();
    };
    // the loop is unrolled by the rings' common period U, so every slot index is a constant;
    // the 64 % U steps left over run after it
    using std::integral_constant;
    constexpr int U = WD == RD ? WD : 6;
    int k0 = 0;
#define WV_ENC_STEP(q) step(k0 + (q), integral_constant<int, (q)>{})
    for (; k0 + U <= 64; k0 += U) {
        WV_ENC_STEP(0);
        WV_ENC_STEP(1);
        if constexpr (U >= 3) WV_ENC_STEP(2);
        if constexpr (U == 6) {
            WV_ENC_STEP(3);
            WV_ENC_STEP(4);
            WV_ENC_STEP(5);
        }
    }
    if constexpr (64 % U >= 1) WV_ENC_STEP(0);
    if constexpr (64 % U >= 2) WV_ENC_STEP(1);
    if constexpr (64 % U >= 3) WV_ENC_STEP(2);
    if constexpr (64 % U >= 4) WV_ENC_STEP(3);
#undef WV_ENC_STEP

    // second layer, split over the waves' hidden units: H[:, 64 w .. 64 w + 63] W2[:, same]^T.
    // The loop ended with a barrier, so the region is free: wave w stages one row tile of its
    // GELU outputs at a time in its own [16][ENC_HLD] area (LDS accesses of one wave complete
    // in issue order, so no barrier is needed between its writes and reads).
    uint16_t* sHw = sR + wave * 16 * ENC_HLD;
    float bias1[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) bias1[j] = a.b1[wave * 64 + j * 16 + fr];
    // W2 fragments: B lane l = latent 16 jj + l % 16, hidden 64 w + 32 ks + 8 (l / 16) .. + 7
    bf16x8 w2f[2][2];
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
            w2f[ks][jj] = *reinterpret_cast<const bf16x8*>(a.w2t + (long long)(jj * 16 + fr) * HID + wave * 64 +
                                                           ks * 32 + fq);
    f32x4 zp[TI][2];
#pragma unroll
    for (int i = 0; i < TI; ++i) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) sHw[(cr + r) * ENC_HLD + j * 16 + fr] = f2bf(gelu(acc[i][j][r] + bias1[j]));
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        zp[i][0] = f32x4{0.f, 0.f, 0.f, 0.f};
        zp[i][1] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const bf16x8 ah = *reinterpret_cast<const bf16x8*>(sHw + fr * ENC_HLD + ks * 32 + fq);
#pragma unroll
            for (int jj = 0; jj < 2; ++jj)
                zp[i][jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, w2f[ks][jj], zp[i][jj], 0, 0, 0);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // the partial blocks summed in wave order: ((z_0 + z_1) + z_2) + ... in a [BM][ENC_ZLD] area
    float* sZ = reinterpret_cast<float*>(sR);
    __syncthreads();  // every wave is done with its staging area
    for (int w = 0; w < 8; ++w) {
        if (wave == w) {
#pragma unroll
            for (int i = 0; i < TI; ++i)
#pragma unroll
                for (int jj = 0; jj < 2; ++jj)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        float* z = sZ + (i * 16 + cr + r) * ENC_ZLD + jj * 16 + fr;
                        *z = w == 0 ? zp[i][jj][r] : *z + zp[i][jj][r];
                    }
        }
        __syncthreads();
    }
    // bias, then the latents: thread t writes 8 values of patch t / 4
    const int zr = tid >> 2, zc = (tid & 3) * 8;
    const long long p = m0 + zr;
    if (p < a.P) {
        float v[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) v[c] = sZ[zr * ENC_ZLD + zc + c] + a.b2[zc + c];
        if (a.zbf) {
            uint16_t* o = a.zbf + p * L + zc;
#pragma unroll
            for (int c = 0; c < 8; ++c) o[c] = f2bf(v[c]);
        }
        if (a.zf) {
            float* o = a.zf + p * L + zc;
#pragma unroll
            for (int c = 0; c < 8; ++c) o[c] = v[c];
        }
    }
}

// Decode: DEC_NW waves per work-group of DEC_BM patches; wave w owns hidden units
// and field-f outputs [OPW w, OPW w + OPW). W4 fragments are read from L2 PFD
// k-steps ahead of their use.
// 8 waves over 64 patches, at least 4 waves per SIMD: two work-groups share a CU (about
// 68 KB of LDS each), so one computes while the other writes its outputs, and a work-group
// also fits beside stencil work-groups (36 us alone at 256^3, against 42 us for 16 waves
// over 128 patches, one work-group per CU)
#ifndef WV_DEC_WAVES
#define WV_DEC_WAVES 8
#endif
#ifndef WV_DEC_PF
#define WV_DEC_PF 2
#endif
// minimum waves per SIMD asked of the register allocator (0: no request)
#ifndef WV_DEC_WPE
#define WV_DEC_WPE 4
#endif
constexpr int DEC_NW = WV_DEC_WAVES;
constexpr int DEC_NT = DEC_NW * 64;

template <int L>
__global__ void __launch_bounds__(DEC_NT) __attribute__((amdgpu_waves_per_eu(WV_DEC_WPE > 0 ? WV_DEC_WPE : 1)))
    decode_kernel(const DecArgs a)
{
    constexpr int BM = DEC_BM;         // patches per work-group
    constexpr int IT = BM / 16;        // 16-row tiles
    constexpr int OPW = HID / DEC_NW;  // hidden units / outputs per wave
    constexpr int JT = OPW / 16;       // 16-wide column tiles per wave
    constexpr int NK = HID / KB;       // k-steps of layer 4
    constexpr int PFD = WV_DEC_PF;
    extern __shared__ __attribute__((aligned(16))) uint16_t smem[];
    uint16_t(*sH)[HID + HPAD] = reinterpret_cast<uint16_t(*)[HID + HPAD]>(smem);
    // per-patch tables after the hidden layer: field offset of the patch origin, (min, range) of field f
    long long* sBase = reinterpret_cast<long long*>(smem + BM * (HID + HPAD));
    float* sLo = reinterpret_cast<float*>(sBase + BM);
    float* sRg = sLo + BM;
    int* sExc = reinterpret_cast<int*>(sRg + BM);  // exception slot of each patch, or -1
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int fr = lane & 15, fq = (lane >> 4) * 8, cr = (lane >> 4) * 4, q = lane >> 4;
    const long long tile = a.t0 + blockIdx.x;
    const long long m0 = tile * BM;
    const bool has_exc = a.eidx != nullptr;

    if (tid < BM) {
        sExc[tid] = -1;
        const long long p = m0 + tid;
        long long base = 0;
        float lo = 0.f, rg = 0.f;
        if (p < a.P) {
            const long long px = p % a.Px, py = (p / a.Px) % a.Py, pz = p / ((long long)a.Px * a.Py);
            base = (pz * 8 * a.ny + py * 8) * a.nx + px * 8;
            if (a.meta16) {
                lo = bf2f(a.meta16[p * 8 + 2 * a.f]);
                rg = bf2f(a.meta16[p * 8 + 2 * a.f + 1]);
            } else {
                lo = a.meta[p * 8 + 2 * a.f];
                rg = a.meta[p * 8 + 2 * a.f + 1];
            }
        }
        sBase[tid] = base;
        sLo[tid] = lo;
        sRg[tid] = rg;
    }

    // fragment-ordered W4: block (ks, r) at ((ks * 128 + r) * 64) * 8, rows of field f at r = 32 f
    const uint16_t* wb = a.w4p + ((long long)(a.f * 32 + wave * JT) * 64 + lane) * 8;
    bf16x8 bq[PFD + 1][JT];
    // the first W4 stages are in flight during layer 3
    #pragma unroll
    for (int u = 0; u < PFD; ++u)
        #pragma unroll
        for (int j = 0; j < JT; ++j)
            bq[u][j] = *reinterpret_cast<const bf16x8*>(wb + (long long)u * (128 * 512) + j * 512);

    // layer 3: H[BM][HID] = GELU(Z W3^T + b3) for this wave's hidden units
    {
        f32x4 acc[IT][JT];
        #pragma unroll
        for (int i = 0; i < IT; ++i)
            #pragma unroll
            for (int j = 0; j < JT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < L / KB; ++kk) {
            bf16x8 bw[JT];
            #pragma unroll
            for (int j = 0; j < JT; ++j)
                bw[j] = *reinterpret_cast<const bf16x8*>(a.w3t + (long long)(wave * OPW + j * 16 + fr) * L + kk * KB + fq);
            #pragma unroll
            for (int i = 0; i < IT; ++i) {
                const long long p = m0 + i * 16 + fr;
                bf16x8 az;
                if (p < a.P) {
                    az = *reinterpret_cast<const bf16x8*>(a.z + p * L + kk * KB + fq);
                } else {
                    const uint4 zero = make_uint4(0, 0, 0, 0);
                    az = *reinterpret_cast<const bf16x8*>(&zero);
                }
                #pragma unroll
                for (int j = 0; j < JT; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(az, bw[j], acc[i][j], 0, 0, 0);
            }
        }
        #pragma unroll
        for (int j = 0; j < JT; ++j) {
            const int n = wave * OPW + j * 16 + fr;
            const float bias = a.b3[n];
            #pragma unroll
            for (int i = 0; i < IT; ++i)
                #pragma unroll
                for (int r = 0; r < 4; ++r) sH[i * 16 + cr + r][n] = f2bf(gelu(acc[i][j][r] + bias));
        }
    }
    __syncthreads();
    if (has_exc) {
        const int e0 = a.erng[tile], e1 = a.erng[tile + 1];
        for (int t = e0 + tid; t < e1; t += DEC_NT) {
            const long long d = a.eidx[t] - m0;
            if (d >= 0 && d < BM) sExc[d] = t;
        }
    }
    // layer 4, rows of field f. A row m of tile i is patch 16 i + 4 (m % 4) + m / 4, so that the C rows
    // held for one r by the four lane groups are four x-adjacent patches: each store then covers whole
    // 128-byte rows.
    f32x4 acc[IT][JT];
    #pragma unroll
    for (int i = 0; i < IT; ++i)
        #pragma unroll
        for (int j = 0; j < JT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int arow = 4 * (fr & 3) + (fr >> 2);
    #pragma unroll
    for (int kk = 0; kk < NK; ++kk) {
        if (kk + PFD < NK)
            #pragma unroll
            for (int j = 0; j < JT; ++j)
                bq[(kk + PFD) % (PFD + 1)][j] =
                    *reinterpret_cast<const bf16x8*>(wb + (long long)(kk + PFD) * (128 * 512) + j * 512);
        bf16x8 af[IT];
        #pragma unroll
        for (int i = 0; i < IT; ++i) af[i] = *reinterpret_cast<const bf16x8*>(&sH[i * 16 + arow][kk * KB + fq]);
        #pragma unroll
        for (int i = 0; i < IT; ++i)
            #pragma unroll
            for (int j = 0; j < JT; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bq[kk % (PFD + 1)][j], acc[i][j], 0, 0, 0);
    }
    // de-normalise and write: output o = OPW wave + 16 j + fr of the patch -> (lz, ly, lx) = (o / 64, o / 8 % 8, o % 8)
    float bias[JT];
    long long off[JT];
    #pragma unroll
    for (int j = 0; j < JT; ++j) {
        const int o = wave * OPW + j * 16 + fr;
        bias[j] = a.b4[a.f * 512 + o];
        off[j] = ((long long)(o >> 6) * a.ny + ((o >> 3) & 7)) * a.nx + (o & 7);
    }
    float* out = a.state + a.f * a.N;
    if (has_exc) __syncthreads();  // sExc complete
    #pragma unroll
    for (int i = 0; i < IT; ++i)
        #pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int pl = i * 16 + 4 * r + q;
            if (m0 + pl >= a.P) continue;
            const long long base = sBase[pl];
            const float lo = sLo[pl], rg = sRg[pl];
            const int slot = has_exc ? sExc[pl] : -1;
            if (slot < 0) {
                #pragma unroll
                for (int j = 0; j < JT; ++j) out[base + off[j]] = lo + rg * (acc[i][j][r] + bias[j]);
            } else {
                #pragma unroll
                for (int j = 0; j < JT; ++j)
                    out[base + off[j]] = a.exc[(long long)slot * 512 + wave * OPW + j * 16 + fr];
            }
        }
}

__global__ void pack_kernel(const uint16_t* __restrict__ w, int rows, int K, uint16_t* __restrict__ out)
{
    const long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;  // 8-value chunk
    if (c >= (long long)rows * K / 8) return;
    const int lane = (int)(c & 63);
    const long long t = c >> 6;
    const int r16 = (int)(t % (rows / 16));
    const long long ks = t / (rows / 16);
    const long long row = r16 * 16 + (lane & 15), k = ks * 32 + (lane >> 4) * 8;
    *reinterpret_cast<uint4*>(out + c * 8) = *reinterpret_cast<const uint4*>(w + row * K + k);
}

template <class K>
void allow_smem(K kernel, size_t bytes)
{
    static bool done = false;
    if (!done) {
        WV_HIP(hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
        done = true;
    }
}

}  // namespace

bool fused_supported(int hid, int lat) { return hid == HID && lat == 32; }

void fused_pack(const uint16_t* w, int rows, int K, uint16_t* out, hipStream_t st)
{
    WV_REQUIRE(rows % 16 == 0 && K % 32 == 0, WV_EINVAL, "fragment packing needs rows % 16 == 0, K % 32 == 0");
    const long long chunks = (long long)rows * K / 8;
    hipLaunchKernelGGL(pack_kernel, dim3((unsigned)((chunks + 255) / 256)), dim3(256), 0, st, w, rows, K, out);
    WV_HIP(hipGetLastError());
}

void fused_encode(const PatchGrid& pg, const float* state, float* meta, const float* mm, int H, const float* beta,
                  const uint16_t* w1p, const float* b1, const uint16_t* w2t, const float* b2, uint16_t* zbf, float* zf,
                  hipStream_t st, uint16_t* meta16)
{
    WV_REQUIRE(!meta16 || mm, WV_EINVAL, "16-bit metadata is written from the step's (min, max) partials");
    EncArgs a{state, meta, meta16, mm, H, beta, w1p, b1, w2t, b2, zbf, zf, pg.P, (long long)pg.nz * pg.ny * pg.nx,
              pg.ny, pg.nx, pg.ny / 8, pg.nx / 8, 0};
    const long long tiles = (pg.P + BM - 1) / BM;
    const long long per = ENC_GRID > 0 ? ENC_GRID : tiles;
    for (a.t0 = 0; a.t0 < tiles; a.t0 += per) {
        hipLaunchKernelGGL((encode_kernel<32, ENC_WD, ENC_RD>), dim3((unsigned)std::min(per, tiles - a.t0)), dim3(NT), 0,
                           st, a);
        WV_HIP(hipGetLastError());
    }
}

void fused_decode(const PatchGrid& pg, const uint16_t* z, const float* meta, const uint16_t* w3t, const float* b3,
                  const uint16_t* w4p, const float* b4, int f, float* state, hipStream_t st, const ExcPatches* exc,
                  const uint16_t* meta16, long long grid)
{
    static_assert(DEC_BM % 16 == 0 && DEC_BM <= 512, "decode work-groups hold whole 16-patch tiles");
    DecArgs a{z, meta, meta16, w3t, b3, w4p, b4, state, f, pg.P, (long long)pg.nz * pg.ny * pg.nx, pg.ny, pg.nx,
              pg.ny / 8, pg.nx / 8, nullptr, nullptr, nullptr, 0};
    if (exc && exc->K > 0) {
        WV_REQUIRE(exc->idx && exc->exc && exc->rng, WV_EINVAL, "decode: null exception buffer");
        a.eidx = exc->idx;
        a.exc = exc->exc;
        a.erng = exc->rng;
    }
    const size_t sm = (size_t)DEC_BM * (HID + HPAD) * 2 + (size_t)DEC_BM * 20;
    allow_smem(decode_kernel<32>, sm);
    const long long tiles = (pg.P + DEC_BM - 1) / DEC_BM;
    const long long per = grid > 0 ? grid : tiles;
    for (a.t0 = 0; a.t0 < tiles; a.t0 += per) {
        hipLaunchKernelGGL(decode_kernel<32>, dim3((unsigned)std::min(per, tiles - a.t0)), dim3(DEC_NT), sm, st, a);
        WV_HIP(hipGetLastError());
    }
}

}  // namespace wv

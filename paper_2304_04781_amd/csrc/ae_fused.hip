// Fused autoencoder inference kernels for the time loop (gfx950, bf16 MFMA).
//
// encode: one work-group compresses 128 patches. The A operand (the normalised
// patch vectors) is built on the fly from the float32 state and the per-patch
// (min, range) metadata, rounded to bfloat16 and staged through LDS; the B
// operand (W1^T, k contiguous) goes straight from L2 into registers, each of the
// 8 waves owning 64 of the 512 hidden units. The hidden layer (bias + GELU,
// bfloat16) stays in LDS and the second layer runs in the same work-group.
// decode: the mirror image for one field: latent -> hidden (bias + GELU, LDS)
// -> 512 outputs of that field -> de-normalised float32 written into the state.
//
// Layout of a 16x16x32 bf16 MFMA (v_mfma_f32_16x16x32_bf16): A lane l holds
// row l%16, k = 8*(l/16)..+7; B lane l holds column l%16, same k; C lane l
// holds column l%16, rows 4*(l/16)..+3.

#include "ae_internal.h"

namespace wv {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }

constexpr int BM = 128;       // patches per work-group
constexpr int NT = 512;       // threads (8 waves)
constexpr int HID = 512;      // hidden width handled by these kernels
constexpr int KB = 32;        // k per MFMA step
constexpr int APAD = 8;       // bf16 padding per LDS row
constexpr int HPAD = 8;

struct EncArgs {
    const float* state;   // [4][N]
    const float* meta;    // [P][4][2] (min, range); output when mm is given
    const float* mm;      // optional [P][H][4][2] partial (min, max) from the forward step
    int H;
    const float* beta;    // [4] range floors (with mm)
    const uint16_t* w1t;  // [HID][2048]
    const float* b1;      // [HID]
    const uint16_t* w2t;  // [L][HID]
    const float* b2;      // [L]
    uint16_t* zbf;        // [P][L] bf16 latent (or null)
    float* zf;            // [P][L] float32 latent (or null)
    long long P, N;
    int ny, nx, Py, Px;
};

struct DecArgs {
    const uint16_t* z;    // [P][L] bf16
    const float* meta;
    const uint16_t* w3t;  // [HID][L]
    const float* b3;
    const uint16_t* w4t;  // [2048][HID], rows of field f at f*512
    const float* b4;      // [2048]
    float* state;         // [4][N]
    int f;
    long long P, N;
    int ny, nx, Py, Px;
};

template <int L>
__global__ void __launch_bounds__(NT) encode_kernel(const EncArgs a)
{
    extern __shared__ __attribute__((aligned(16))) uint16_t smem[];
    // phase 1: double-buffered A tiles [2][BM][KB + APAD]; phase 2: H [BM][HID + HPAD]
    uint16_t(*sA)[BM][KB + APAD] = reinterpret_cast<uint16_t(*)[BM][KB + APAD]>(smem);
    uint16_t(*sH)[HID + HPAD] = reinterpret_cast<uint16_t(*)[HID + HPAD]>(smem);

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const long long m0 = (long long)blockIdx.x * BM;

    // A staging: thread -> (patch row m, one of 4 ly rows of a k-step)
    const int am = tid >> 2, aq = tid & 3;
    const long long pa = m0 + am;
    const bool a_ok = pa < a.P;
    long long abase = 0;
    // per-field (min, range) of the block's patches, in LDS after the hidden-layer area
    float* sMeta = reinterpret_cast<float*>(smem + BM * (HID + HPAD));  // [BM][8]
    if (a_ok) {
        const int px = (int)(pa % a.Px), py = (int)((pa / a.Px) % a.Py), pz = (int)(pa / ((long long)a.Px * a.Py));
        abase = ((long long)pz * 8 * a.ny + py * 8) * a.nx + px * 8;
    }
    if (tid < BM) {
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
                    const_cast<float*>(a.meta)[p * 8 + 2 * f] = lo;
                    const_cast<float*>(a.meta)[p * 8 + 2 * f + 1] = r;
                }
                sMeta[tid * 8 + 2 * f] = lo;
                sMeta[tid * 8 + 2 * f + 1] = r;
            }
        } else {
            const float4 m01 = p < a.P ? *reinterpret_cast<const float4*>(a.meta + p * 8) : make_float4(0.f, 1.f, 0.f, 1.f);
            const float4 m23 = p < a.P ? *reinterpret_cast<const float4*>(a.meta + p * 8 + 4) : make_float4(0.f, 1.f, 0.f, 1.f);
            *reinterpret_cast<float4*>(sMeta + tid * 8) = m01;
            *reinterpret_cast<float4*>(sMeta + tid * 8 + 4) = m23;
        }
    }
    __syncthreads();
    // k-step kk covers field f = kk/16, lz = (kk%16)/2, ly = 4*(kk%2) + aq: rows of 8 x-cells
    const int fr = lane & 15, fq = (lane >> 4) * 8;
    const uint16_t* wb = a.w1t + (long long)(wave * 64 + fr) * 2048 + fq;  // B: hidden units of this wave

    f32x4 acc[8][4];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    float4 x0 = make_float4(0.f, 0.f, 0.f, 0.f), x1 = x0;
    bf16x8 b0, b1, b2, b3;          // B fragments of the current k-step
    bf16x8 n0, n1, n2, n3;          // prefetched B fragments of the next k-step
#define WV_LOAD_A(kk)                                                                              \
    if (a_ok) {                                                                                    \
        const int f_ = (kk) >> 4, lz_ = ((kk)&15) >> 1, ly_ = 4 * ((kk)&1) + aq;                   \
        const float* src_ = a.state + f_ * a.N + abase + ((long long)lz_ * a.ny + ly_) * a.nx;     \
        x0 = *reinterpret_cast<const float4*>(src_);                                               \
        x1 = *reinterpret_cast<const float4*>(src_ + 4);                                           \
    }
#define WV_STORE_A(buf, l, r)                                                                      \
    {                                                                                              \
        uint4 w_ = make_uint4(0, 0, 0, 0);                                                         \
        if (a_ok) {                                                                                \
            w_.x = (uint32_t)f2bf((x0.x - (l)) / (r)) | ((uint32_t)f2bf((x0.y - (l)) / (r)) << 16); \
            w_.y = (uint32_t)f2bf((x0.z - (l)) / (r)) | ((uint32_t)f2bf((x0.w - (l)) / (r)) << 16); \
            w_.z = (uint32_t)f2bf((x1.x - (l)) / (r)) | ((uint32_t)f2bf((x1.y - (l)) / (r)) << 16); \
            w_.w = (uint32_t)f2bf((x1.z - (l)) / (r)) | ((uint32_t)f2bf((x1.w - (l)) / (r)) << 16); \
        }                                                                                          \
        *reinterpret_cast<uint4*>(&sA[(buf)][am][aq * 8]) = w_;                                     \
    }
#define WV_LOAD_B(kk, d0, d1, d2, d3)                                                              \
    {                                                                                              \
        const uint16_t* q_ = wb + (kk) * KB;                                                       \
        d0 = *reinterpret_cast<const bf16x8*>(q_);                                                 \
        d1 = *reinterpret_cast<const bf16x8*>(q_ + 16 * 2048);                                     \
        d2 = *reinterpret_cast<const bf16x8*>(q_ + 32 * 2048);                                     \
        d3 = *reinterpret_cast<const bf16x8*>(q_ + 48 * 2048);                                     \
    }

    WV_LOAD_A(0);
    WV_STORE_A(0, sMeta[am * 8], sMeta[am * 8 + 1]);
    WV_LOAD_B(0, b0, b1, b2, b3);
    __syncthreads();
    for (int kk = 0; kk < 64; ++kk) {
        const int buf = kk & 1;
        const bool more = kk + 1 < 64;
        if (more) {
            WV_LOAD_A(kk + 1);
            WV_LOAD_B(kk + 1, n0, n1, n2, n3);
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const bf16x8 af = *reinterpret_cast<const bf16x8*>(&sA[buf][i * 16 + fr][fq]);
            acc[i][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, b0, acc[i][0], 0, 0, 0);
            acc[i][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, b1, acc[i][1], 0, 0, 0);
            acc[i][2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, b2, acc[i][2], 0, 0, 0);
            acc[i][3] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, b3, acc[i][3], 0, 0, 0);
        }
        if (more) {
            const int fn = (kk + 1) >> 4;
            WV_STORE_A(buf ^ 1, sMeta[am * 8 + 2 * fn], sMeta[am * 8 + 2 * fn + 1]);
            b0 = n0; b1 = n1; b2 = n2; b3 = n3;
        }
        __syncthreads();
    }
#undef WV_LOAD_A
#undef WV_STORE_A
#undef WV_LOAD_B
    // hidden layer: bias + GELU -> bf16 in LDS (aliases the A buffers)
    const int cr = (lane >> 4) * 4;
    #pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int n = wave * 64 + j * 16 + fr;
        const float bias = a.b1[n];
        #pragma unroll
        for (int i = 0; i < 8; ++i)
            #pragma unroll
            for (int r = 0; r < 4; ++r) sH[i * 16 + cr + r][n] = f2bf(gelu(acc[i][j][r] + bias));
    }
    __syncthreads();
    // second layer: Z[BM][L] = H W2^T; wave handles rows [16*wave, 16*wave+16), all L columns
    constexpr int TJ = L / 16;
    f32x4 z[TJ];
    #pragma unroll
    for (int j = 0; j < TJ; ++j) z[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int kk = 0; kk < HID / KB; ++kk) {
        const bf16x8 ah = *reinterpret_cast<const bf16x8*>(&sH[wave * 16 + fr][kk * KB + fq]);
        #pragma unroll
        for (int j = 0; j < TJ; ++j) {
            const bf16x8 bw = *reinterpret_cast<const bf16x8*>(a.w2t + (long long)(j * 16 + fr) * HID + kk * KB + fq);
            z[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bw, z[j], 0, 0, 0);
        }
    }
    #pragma unroll
    for (int j = 0; j < TJ; ++j) {
        const int n = j * 16 + fr;
        const float bias = a.b2[n];
        #pragma unroll
        for (int r = 0; r < 4; ++r) {
            const long long p = m0 + wave * 16 + cr + r;
            if (p < a.P) {
                const float v = z[j][r] + bias;
                if (a.zbf) a.zbf[p * L + n] = f2bf(v);
                if (a.zf) a.zf[p * L + n] = v;
            }
        }
    }
}

template <int L>
__global__ void __launch_bounds__(NT) decode_kernel(const DecArgs a)
{
    extern __shared__ __attribute__((aligned(16))) uint16_t smem[];
    uint16_t(*sH)[HID + HPAD] = reinterpret_cast<uint16_t(*)[HID + HPAD]>(smem);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int fr = lane & 15, fq = (lane >> 4) * 8, cr = (lane >> 4) * 4;
    const long long m0 = (long long)blockIdx.x * BM;

    // layer 3: H[BM][HID] = GELU(Z W3^T + b3); wave owns hidden units [64 wave, +64)
    {
        f32x4 acc[8][4];
        #pragma unroll
        for (int i = 0; i < 8; ++i)
            #pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < L / KB; ++kk) {
            bf16x8 bw[4];
            #pragma unroll
            for (int j = 0; j < 4; ++j)
                bw[j] = *reinterpret_cast<const bf16x8*>(a.w3t + (long long)(wave * 64 + j * 16 + fr) * L + kk * KB + fq);
            #pragma unroll
            for (int i = 0; i < 8; ++i) {
                const long long p = m0 + i * 16 + fr;
                bf16x8 az;
                if (p < a.P) {
                    az = *reinterpret_cast<const bf16x8*>(a.z + p * L + kk * KB + fq);
                } else {
                    const uint4 zero = make_uint4(0, 0, 0, 0);
                    az = *reinterpret_cast<const bf16x8*>(&zero);
                }
                #pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(az, bw[j], acc[i][j], 0, 0, 0);
            }
        }
        #pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = wave * 64 + j * 16 + fr;
            const float bias = a.b3[n];
            #pragma unroll
            for (int i = 0; i < 8; ++i)
                #pragma unroll
                for (int r = 0; r < 4; ++r) sH[i * 16 + cr + r][n] = f2bf(gelu(acc[i][j][r] + bias));
        }
    }
    __syncthreads();
    // layer 4, rows of field f: wave owns outputs [64 wave, +64) = the lz = wave plane of every patch
    f32x4 acc[8][4];
    #pragma unroll
    for (int i = 0; i < 8; ++i)
        #pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const uint16_t* wb = a.w4t + (long long)(a.f * 512 + wave * 64 + fr) * HID + fq;
    bf16x8 bcur[4], bnxt[4];
    #pragma unroll
    for (int j = 0; j < 4; ++j) bcur[j] = *reinterpret_cast<const bf16x8*>(wb + (long long)j * 16 * HID);
    for (int kk = 0; kk < HID / KB; ++kk) {
        const bool more = kk + 1 < HID / KB;
        if (more)
            #pragma unroll
            for (int j = 0; j < 4; ++j)
                bnxt[j] = *reinterpret_cast<const bf16x8*>(wb + (long long)j * 16 * HID + (kk + 1) * KB);
        bf16x8 af[8];
        #pragma unroll
        for (int i = 0; i < 8; ++i) af[i] = *reinterpret_cast<const bf16x8*>(&sH[i * 16 + fr][kk * KB + fq]);
        #pragma unroll
        for (int i = 0; i < 8; ++i)
            #pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bcur[j], acc[i][j], 0, 0, 0);
        if (more)
            #pragma unroll
            for (int j = 0; j < 4; ++j) bcur[j] = bnxt[j];
    }
    // de-normalise and write: column n = 64 wave + 16 j + fr -> (lz, ly, lx)
    #pragma unroll
    for (int i = 0; i < 8; ++i)
        #pragma unroll
        for (int r = 0; r < 4; ++r) {
            const long long p = m0 + i * 16 + cr + r;
            if (p >= a.P) continue;
            const float lo = a.meta[p * 8 + 2 * a.f], rg = a.meta[p * 8 + 2 * a.f + 1];
            const int px = (int)(p % a.Px), py = (int)((p / a.Px) % a.Py), pz = (int)(p / ((long long)a.Px * a.Py));
            #pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int c = j * 16 + fr;  // within the lz plane
                const int n = wave * 64 + c;
                const long long zz = pz * 8 + wave, yy = py * 8 + (c >> 3), xx = px * 8 + (c & 7);
                a.state[a.f * a.N + (zz * a.ny + yy) * a.nx + xx] = lo + rg * (acc[i][j][r] + a.b4[a.f * 512 + n]);
            }
        }
}

size_t enc_smem()
{
    const size_t a = 2 * BM * (KB + APAD) * 2, h = (size_t)BM * (HID + HPAD) * 2;
    return (a > h ? a : h) + (size_t)BM * 8 * 4;  // + per-patch (min, range) table
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

void fused_encode(const PatchGrid& pg, const float* state, float* meta, const float* mm, int H, const float* beta,
                  const uint16_t* w1t, const float* b1, const uint16_t* w2t, const float* b2, uint16_t* zbf, float* zf,
                  hipStream_t st)
{
    EncArgs a{state, meta, mm, H, beta, w1t, b1, w2t, b2, zbf, zf, pg.P, (long long)pg.nz * pg.ny * pg.nx, pg.ny,
              pg.nx, pg.ny / 8, pg.nx / 8};
    const size_t sm = enc_smem();
    allow_smem(encode_kernel<32>, sm);
    hipLaunchKernelGGL(encode_kernel<32>, dim3((unsigned)((pg.P + BM - 1) / BM)), dim3(NT), sm, st, a);
    WV_HIP(hipGetLastError());
}

void fused_decode(const PatchGrid& pg, const uint16_t* z, const float* meta, const uint16_t* w3t, const float* b3,
                  const uint16_t* w4t, const float* b4, int f, float* state, hipStream_t st)
{
    DecArgs a{z, meta, w3t, b3, w4t, b4, state, f, pg.P, (long long)pg.nz * pg.ny * pg.nx, pg.ny, pg.nx,
              pg.ny / 8, pg.nx / 8};
    const size_t sm = (size_t)BM * (HID + HPAD) * 2;
    allow_smem(decode_kernel<32>, sm);
    hipLaunchKernelGGL(decode_kernel<32>, dim3((unsigned)((pg.P + BM - 1) / BM)), dim3(NT), sm, st, a);
    WV_HIP(hipGetLastError());
}

}  // namespace wv

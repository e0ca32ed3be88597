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
#include "ae_math.h"

namespace wv {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// byte address of a shared-memory location, for inline-asm LDS instructions
template <class T>
__device__ __forceinline__ uint32_t lds_addr(T* p)
{
    return (uint32_t)(uintptr_t)(__attribute__((address_space(3))) T*)p;
}

constexpr int BM = 128;       // patches per work-group
constexpr int NT = 512;       // threads (8 waves)
constexpr int HID = 512;      // hidden width handled by these kernels
constexpr int KB = 32;        // k per MFMA step
constexpr int APAD = 8;       // bf16 padding per LDS row
constexpr int HPAD = 8;
constexpr int RS = 4;  // raw A stages in flight (encode); the wait counts below assume 4
// encode LDS: raw ring + two W1 fragment stages + bfloat16 double buffer, or the hidden layer
constexpr int ENC_PH1 = RS * BM * KB * 4 + 2 * HID * KB * 2 + 2 * BM * (KB + APAD) * 2;
constexpr int ENC_PH2 = BM * (HID + HPAD) * 2;
constexpr int ENC_META_OFF = ENC_PH1 > ENC_PH2 ? ENC_PH1 : ENC_PH2;  // bytes; [BM][8] floats follow

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
};

template <int L>
__global__ void __launch_bounds__(NT) encode_kernel(const EncArgs a)
{
    extern __shared__ __attribute__((aligned(16))) uint16_t smem[];
    // phase 1: a ring of RS raw float32 stages [RS][BM][KB] and two stages of W1
    // fragments [2][8 waves][4][64 lanes][8] (both filled by direct global->LDS
    // loads), then the normalised bfloat16 double buffer [2][BM][KB + APAD];
    // phase 2: H [BM][HID + HPAD] over the same bytes
    float(*sRaw)[BM * KB] = reinterpret_cast<float(*)[BM * KB]>(smem);
    uint16_t* sB = smem + RS * BM * KB * 2;                                    // 2 x 32 KiB
    uint16_t(*sA)[BM][KB + APAD] = reinterpret_cast<uint16_t(*)[BM][KB + APAD]>(sB + 2 * HID * KB);
    uint16_t(*sH)[HID + HPAD] = reinterpret_cast<uint16_t(*)[HID + HPAD]>(smem);

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const long long m0 = (long long)blockIdx.x * BM;

    // A staging: thread -> (patch row m, one of 4 ly rows of a k-step)
    const int am = tid >> 2, aq = tid & 3;
    const long long pa = m0 + am;
    const bool a_ok = pa < a.P;
    // per-field (min, 1/range) of the block's patches, in LDS after the hidden-layer area
    float* sMeta = reinterpret_cast<float*>(smem + ENC_META_OFF / 2);  // [BM][8]
    // direct loads: a stage holds 1024 pieces of 16 bytes, piece = 8 m + 2 row + half
    // (patch m, y row 4 (kk % 2) + row, x half); wave w loads pieces [128 w, 128 w + 128)
    // in two instructions, so a lane of instruction t owns piece 128 w + 64 t + lane.
    long long dbase[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int pc = 128 * wave + 64 * t + lane;
        const long long pm = m0 + (pc >> 3);
        dbase[t] = -1;
        if (pm < a.P) {
            const long long px = pm % a.Px, py = (pm / a.Px) % a.Py, pz = pm / ((long long)a.Px * a.Py);
            dbase[t] = (pz * 8 * a.ny + py * 8 + ((pc >> 1) & 3)) * a.nx + px * 8 + (pc & 1) * 4;
        }
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
    __syncthreads();
    // k-step kk covers field f = kk/16, lz = (kk%16)/2, ly = 4*(kk%2) + aq: rows of 8 x-cells
    const int fr = lane & 15, fq = (lane >> 4) * 8;

    f32x4 acc[8][4];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    // Pipeline over the 64 k-steps. All operands reach LDS by direct global->LDS
    // loads, whose completion is tracked by hand with vmcnt (loads finish in issue
    // order); every LDS access of the loop is inline asm that waits for its own
    // results, so the compiler adds no waits of its own. Per step kk:
    //   wait for this wave's W1 fragments of kk; read them into registers;
    //   load the W1 fragments of kk + 2 into the stage just read (4 loads);
    //   load the raw state rows of kk + RS into the raw stage converted last step (2);
    //   MFMAs on the bfloat16 A tile of kk;
    //   normalise the raw rows of kk + 1 into the other bfloat16 buffer;
    //   wait for this wave's raw loads of kk + 2; barrier.
    // Indices past the last step are clamped (harmless reloads), so the number of
    // loads per step, and with it every wait count, stays fixed.
    static_assert(RS == 4, "the wait counts assume four raw stages");
#define WV_WAIT_VM_LGKM0(n) __builtin_amdgcn_s_waitcnt(((n)&15) | (((n) >> 4) << 14) | (7 << 4))
#define WV_WAIT_VM(n) __builtin_amdgcn_s_waitcnt(((n)&15) | (((n) >> 4) << 14) | (7 << 4) | (15 << 8))
    // raw stage pieces: 1024 x 16 bytes, piece = 8 m + 2 row + half; wave w, load t owns 128 w + 64 t + lane
#define WV_DMA_A(kk)                                                                                \
    {                                                                                               \
        const int k_ = (kk) < 64 ? (kk) : 63;                                                       \
        const long long o_ = (k_ >> 4) * a.N + ((long long)((k_ & 15) >> 1) * a.ny + 4 * (k_ & 1)) * a.nx; \
        float* d_ = sRaw[(kk) % RS] + wave * 512;                                                   \
        __builtin_amdgcn_global_load_lds(a.state + (dbase[0] >= 0 ? o_ + dbase[0] : 0), d_, 16, 0, 0); \
        __builtin_amdgcn_global_load_lds(a.state + (dbase[1] >= 0 ? o_ + dbase[1] : 0), d_ + 256, 16, 0, 0); \
    }
    // W1 fragment stage of wave w: [4 tiles j][64 lanes] x 16 bytes in the order the MFMA reads them
    // (fragment-ordered W1: block (ks, r) of 64 x 8 values at ((ks * 32 + r) * 64) * 8)
    const uint16_t* wsrc = a.w1p + ((long long)(wave * 4) * 64 + lane) * 8;
#define WV_DMA_B(kk, st)                                                                            \
    {                                                                                               \
        const int k_ = (kk) < 64 ? (kk) : 63;                                                       \
        uint16_t* d_ = sB + (st) * (HID * KB) + wave * (64 * KB);                                   \
        _Pragma("unroll") for (int j_ = 0; j_ < 4; ++j_)                                            \
            __builtin_amdgcn_global_load_lds(wsrc + (long long)k_ * (HID * KB) + j_ * 512, d_ + j_ * 512, 16, 0, 0); \
    }
    const uint32_t b_addr = lds_addr(sB + wave * (64 * KB) + lane * 8);
    // A fragments of tile i: row 16 i + fr, k fq..fq+7 of a bfloat16 buffer
    const uint32_t af_addr = lds_addr(&sA[0][fr][fq]);
    // normalisation: thread (am, aq) converts row aq of patch am
    const uint32_t raw_addr = lds_addr(&sRaw[0][am * KB + aq * 8]);
    const uint32_t sa_addr = lds_addr(&sA[0][am][aq * 8]);
    const float4 mlo = *reinterpret_cast<const float4*>(sMeta + am * 8);      // (lo0, ri0, lo1, ri1)
    const float4 mhi = *reinterpret_cast<const float4*>(sMeta + am * 8 + 4);  // (lo2, ri2, lo3, ri3)
    __builtin_amdgcn_sched_barrier(0);
#define WV_CONVERT(kk, buf)                                                                         \
    {                                                                                               \
        const int k_ = (kk) < 64 ? (kk) : 63, f_ = k_ >> 4;                                         \
        f32x4 x0, x1;                                                                               \
        asm volatile("ds_read_b128 %0, %2\n\tds_read_b128 %1, %2 offset:16\n\ts_waitcnt lgkmcnt(0)"   \
                     : "=&v"(x0), "=&v"(x1)                                                           \
                     : "v"(raw_addr + (uint32_t)(k_ % RS) * (BM * KB * 4))                          \
                     : "memory");                                                                   \
        const float l_ = f_ == 0 ? mlo.x : f_ == 1 ? mlo.z : f_ == 2 ? mhi.x : mhi.z;              \
        const float ri_ = f_ == 0 ? mlo.y : f_ == 1 ? mlo.w : f_ == 2 ? mhi.y : mhi.w;             \
        u32x4 w_ = {0u, 0u, 0u, 0u};                                                                \
        if (a_ok) {                                                                                 \
            w_.x = f2bf2((x0.x - l_) * ri_, (x0.y - l_) * ri_);                                     \
            w_.y = f2bf2((x0.z - l_) * ri_, (x0.w - l_) * ri_);                                     \
            w_.z = f2bf2((x1.x - l_) * ri_, (x1.y - l_) * ri_);                                     \
            w_.w = f2bf2((x1.z - l_) * ri_, (x1.w - l_) * ri_);                                     \
        }                                                                                           \
        asm volatile("ds_write_b128 %0, %1 offset:%2"                                               \
                     :                                                                              \
                     : "v"(sa_addr), "v"(w_), "i"((buf) * BM * (KB + APAD) * 2)                     \
                     : "memory");                                                                   \
    }

    // prologue: the raw rows of steps 0 and 1, then as in steps -2 and -1 (W1 of 0
    // and 1, raw rows of 2 and 3); normalise step 0.
    WV_DMA_A(0);
    WV_DMA_A(1);
    WV_DMA_B(0, 0);
    WV_DMA_A(2);
    WV_DMA_B(1, 1);
    WV_DMA_A(3);
    __builtin_amdgcn_sched_barrier(0);
    WV_WAIT_VM(14);  // raw rows of step 0 (14 loads issued after them)
    __builtin_amdgcn_s_barrier();
    WV_CONVERT(0, 0);
    WV_WAIT_VM_LGKM0(12);  // raw rows of step 1
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
    // One step, in issue order (sched_barrier pins it): a single LDS read block for
    // the W1 fragments of kk, the raw rows of kk + 1 and A tiles 0-3; then the 32
    // MFMAs in row tiles, with the direct loads, the reads of A tiles 4-7 and the
    // normalisation of kk + 1 slotted between tiles so that they issue while the
    // matrix pipe is busy.
#define WV_TILE(t)                                                                                  \
    _Pragma("unroll") for (int j = 0; j < 4; ++j)                                                   \
        acc[t][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[t], bw[j], acc[t][j], 0, 0, 0);     \
    __builtin_amdgcn_sched_barrier(0);
    for (int k0 = 0; k0 < 64; k0 += 2) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int kk = k0 + u;
            const int kn = kk + 1 < 64 ? kk + 1 : 63;  // the step normalised at the end of this one
            WV_WAIT_VM(8);  // W1 fragments of kk: issued two steps ago, 8 loads since
            u32x4 g0, g1, g2, g3, r0, r1, f0, f1, f2, f3;
            asm volatile(
                "ds_read_b128 %0, %10 offset:%13\n\tds_read_b128 %1, %10 offset:%14\n\t"
                "ds_read_b128 %2, %10 offset:%15\n\tds_read_b128 %3, %10 offset:%16\n\t"
                "ds_read_b128 %4, %11\n\tds_read_b128 %5, %11 offset:16\n\t"
                "ds_read_b128 %6, %12 offset:%17\n\tds_read_b128 %7, %12 offset:%18\n\t"
                "ds_read_b128 %8, %12 offset:%19\n\tds_read_b128 %9, %12 offset:%20\n\t"
                "s_waitcnt lgkmcnt(0)"
                : "=&v"(g0), "=&v"(g1), "=&v"(g2), "=&v"(g3), "=&v"(r0), "=&v"(r1), "=&v"(f0), "=&v"(f1), "=&v"(f2), "=&v"(f3)
                : "v"(b_addr), "v"(raw_addr + (uint32_t)(kn % RS) * (BM * KB * 4)), "v"(af_addr),
                  "i"(u * HID * KB * 2), "i"(u * HID * KB * 2 + 1024), "i"(u * HID * KB * 2 + 2048),
                  "i"(u * HID * KB * 2 + 3072), "i"(u * BM * (KB + APAD) * 2),
                  "i"(u * BM * (KB + APAD) * 2 + 16 * (KB + APAD) * 2),
                  "i"(u * BM * (KB + APAD) * 2 + 32 * (KB + APAD) * 2),
                  "i"(u * BM * (KB + APAD) * 2 + 48 * (KB + APAD) * 2)
                : "memory");
            const bf16x8 bw[4] = {__builtin_bit_cast(bf16x8, g0), __builtin_bit_cast(bf16x8, g1),
                                  __builtin_bit_cast(bf16x8, g2), __builtin_bit_cast(bf16x8, g3)};
            bf16x8 fa[8];
            fa[0] = __builtin_bit_cast(bf16x8, f0);
            fa[1] = __builtin_bit_cast(bf16x8, f1);
            fa[2] = __builtin_bit_cast(bf16x8, f2);
            fa[3] = __builtin_bit_cast(bf16x8, f3);
            __builtin_amdgcn_sched_barrier(0);
            WV_TILE(0);
            WV_DMA_B(kk + 2, u);
            __builtin_amdgcn_sched_barrier(0);
            WV_TILE(1);
            WV_DMA_A(kk + RS);
            __builtin_amdgcn_sched_barrier(0);
            WV_TILE(2);
#pragma unroll
            for (int t = 4; t < 8; ++t) fa[t] = *reinterpret_cast<const bf16x8*>(&sA[u][t * 16 + fr][fq]);
            __builtin_amdgcn_sched_barrier(0);
            WV_TILE(3);
            // normalise the raw rows of kn (held in r0, r1)
            const int fn = kn >> 4;
            const float l_ = fn == 0 ? mlo.x : fn == 1 ? mlo.z : fn == 2 ? mhi.x : mhi.z;
            const float ri_ = fn == 0 ? mlo.y : fn == 1 ? mlo.w : fn == 2 ? mhi.y : mhi.w;
            const f32x4 x0 = __builtin_bit_cast(f32x4, r0), x1 = __builtin_bit_cast(f32x4, r1);
            u32x4 w_;
            w_.x = a_ok ? f2bf2((x0.x - l_) * ri_, (x0.y - l_) * ri_) : 0u;
            w_.y = a_ok ? f2bf2((x0.z - l_) * ri_, (x0.w - l_) * ri_) : 0u;
            __builtin_amdgcn_sched_barrier(0);
            WV_TILE(4);
            w_.z = a_ok ? f2bf2((x1.x - l_) * ri_, (x1.y - l_) * ri_) : 0u;
            w_.w = a_ok ? f2bf2((x1.z - l_) * ri_, (x1.w - l_) * ri_) : 0u;
            __builtin_amdgcn_sched_barrier(0);
            WV_TILE(5);
            asm volatile("ds_write_b128 %0, %1 offset:%2"
                         :
                         : "v"(sa_addr), "v"(w_), "i"((u ^ 1) * BM * (KB + APAD) * 2)
                         : "memory");
            __builtin_amdgcn_sched_barrier(0);
            WV_TILE(6);
            WV_TILE(7);
            WV_WAIT_VM_LGKM0(12);  // raw rows of kk + 2: issued at step kk - 2, 12 loads since
            __builtin_amdgcn_s_barrier();
            __builtin_amdgcn_sched_barrier(0);
        }
    }
#undef WV_TILE
    // no direct load may land in the ring once the hidden layer reuses its bytes
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
#undef WV_DMA_A
#undef WV_DMA_B
#undef WV_CONVERT
#undef WV_WAIT_VM
#undef WV_WAIT_VM_LGKM0
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
#pragma unroll
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
    const long long m0 = (long long)blockIdx.x * BM;
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
        const int e0 = a.erng[blockIdx.x], e1 = a.erng[blockIdx.x + 1];
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

size_t enc_smem() { return (size_t)ENC_META_OFF + (size_t)BM * 8 * 4; }

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
              pg.ny, pg.nx, pg.ny / 8, pg.nx / 8};
    const size_t sm = enc_smem();
    allow_smem(encode_kernel<32>, sm);
    hipLaunchKernelGGL(encode_kernel<32>, dim3((unsigned)((pg.P + BM - 1) / BM)), dim3(NT), sm, st, a);
    WV_HIP(hipGetLastError());
}

void fused_decode(const PatchGrid& pg, const uint16_t* z, const float* meta, const uint16_t* w3t, const float* b3,
                  const uint16_t* w4p, const float* b4, int f, float* state, hipStream_t st, const ExcPatches* exc,
                  const uint16_t* meta16)
{
    static_assert(DEC_BM % 16 == 0 && DEC_BM <= 512, "decode work-groups hold whole 16-patch tiles");
    DecArgs a{z, meta, meta16, w3t, b3, w4p, b4, state, f, pg.P, (long long)pg.nz * pg.ny * pg.nx, pg.ny, pg.nx,
              pg.ny / 8, pg.nx / 8, nullptr, nullptr, nullptr};
    if (exc && exc->K > 0) {
        WV_REQUIRE(exc->idx && exc->exc && exc->rng, WV_EINVAL, "decode: null exception buffer");
        a.eidx = exc->idx;
        a.exc = exc->exc;
        a.erng = exc->rng;
    }
    const size_t sm = (size_t)DEC_BM * (HID + HPAD) * 2 + (size_t)DEC_BM * 20;
    allow_smem(decode_kernel<32>, sm);
    hipLaunchKernelGGL(decode_kernel<32>, dim3((unsigned)((pg.P + DEC_BM - 1) / DEC_BM)), dim3(DEC_NT), sm, st, a);
    WV_HIP(hipGetLastError());
}

}  // namespace wv

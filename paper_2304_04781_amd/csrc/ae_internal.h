// Internal interface between the solver context and the autoencoder code.
#pragma once

#include "wv_internal.h"

namespace wv {

struct PatchGrid {
    int nz, ny, nx;
    long long P;  // patches = (nz/8)(ny/8)(nx/8)
};

inline PatchGrid patch_grid(int nz, int ny, int nx)
{
    return PatchGrid{nz, ny, nx, (long long)(nz / 8) * (ny / 8) * (nx / 8)};
}

// Time compression (paper Sec. 3.2): one vector holds e on a 4^3 block of cells
// over TWIN consecutive time levels, entry t*64 + lz*16 + ly*4 + lx, vector
// s*B + b for source s and block b = (bz*By + by)*Bx + bx. A window buffer holds
// levels [TWIN][S][N]; a window of nvalid < TWIN levels repeats its last level.
constexpr int TWIN = 32;
struct TimeGrid {
    int nz, ny, nx, S;
    long long B;  // blocks per source
};
inline TimeGrid time_grid(int nz, int ny, int nx, int S)
{
    return TimeGrid{nz, ny, nx, S, (long long)(nz / 4) * (ny / 4) * (nx / 4)};
}
// normalised bf16 vectors y [nrows][TWIN*64] and (lo, r) meta [nrows][2] of the
// vectors rows[0..nrows) (rows == nullptr: all S*B in order)
void ae_time_normalize_rows(const ae_net* net, const TimeGrid& tg, const float* e_win, int nvalid,
                            const int32_t* rows, long long nrows, uint16_t* y, float* meta, hipStream_t st);
// compress a window into bf16 latents [S*B][L] and meta [S*B][2]
void ae_time_encode(const ae_net* net, const TimeGrid& tg, const float* e_win, int nvalid, uint16_t* latent,
                    float* meta, hipStream_t st);
// decompress into the first nvalid levels of the window buffer
void ae_time_decode(const ae_net* net, const TimeGrid& tg, const uint16_t* latent, const float* meta, int nvalid,
                    float* e_win, hipStream_t st);

// exception vectors of the time scheme, per window and source s: the K vectors with
// the largest range r (meta [B][2] of source s, the same key and tie rule as the
// patches) in increasing block order into idx [K], their values [K][2048] into exc
// (gathered from the window buffer before it is refilled); restore writes levels
// t < nvalid of them back over a decoded window
void time_exceptions_store(const TimeGrid& tg, const float* e_win, int s, int nvalid, const float* meta, int K,
                           int* idx, float* exc, hipStream_t st);
void time_exceptions_restore(const TimeGrid& tg, float* e_win, int s, int nvalid, int K, const int* idx,
                             const float* exc, hipStream_t st);

int ae_latent_dim(const ae_net* net);
int ae_input_dim(const ae_net* net);
// bytes per patch of the latent store (latent codes only)
long long ae_latent_bytes_per_patch(const ae_net* net, int fmt);

// Compress one state [4][N] into latent [P][L] (+ meta [P][4][2], qscale [P] for FP8).
void ae_encode_state(const ae_net* net, const PatchGrid& pg, const float* state, int fmt,
                     void* latent, float* meta, float* qscale, hipStream_t st);
// Compress with the per-patch (min, max) partials [P][H][4][2] computed by the
// forward step (no separate pass over the state for the normalisation).
// meta16 (optional): bfloat16 (lo, r) written instead of meta, lo rounded down and
// r up to bfloat16 before the normalisation uses them.
void ae_encode_state_mm(const ae_net* net, const PatchGrid& pg, const float* state, const float* mm, int H, int fmt,
                        void* latent, float* meta, float* qscale, hipStream_t st, uint16_t* meta16 = nullptr);
// Exception patches of one stored state: K patch indices in increasing order,
// their exact e values [K][512] ((lz, ly, lx) order), and rng [ceil(P/DEC_BM) + 1]:
// the exceptions of patches [DEC_BM b, DEC_BM b + DEC_BM) are idx[rng[b] .. rng[b+1]).
struct ExcPatches {
    const int* idx;
    int K;
    const float* exc;
    const int* rng;
};
#ifndef WV_DEC_BM
#define WV_DEC_BM 64
#endif
constexpr int DEC_BM = WV_DEC_BM;  // patches per decode work-group
// Decompress the fields in field_mask into state [4][N]; with exc, the e values of
// its patches are the exact ones.
// meta16 (optional): bfloat16 (lo, r) read instead of meta.
void ae_decode_state(const ae_net* net, const PatchGrid& pg, const void* latent, const float* meta,
                     const float* qscale, int fmt, uint32_t field_mask, float* state, hipStream_t st,
                     const ExcPatches* exc = nullptr, const uint16_t* meta16 = nullptr, long long grid = 0);

// Fused inference kernels (hidden width 512, latent 32): meta must already hold
// the per-patch (min, range) of the state for encode.
bool fused_supported(int hid, int lat);
// Repack a bf16 matrix [rows][K] (rows % 16 == 0, K % 32 == 0) into MFMA fragment
// order [K/32][rows/16][64 lanes][8]: lane l of block (ks, r) holds row 16 r + l % 16,
// k = 32 ks + 8 (l / 16) .. +7, so one k-step of a row range is contiguous.
void fused_pack(const uint16_t* w, int rows, int K, uint16_t* out, hipStream_t st);
// meta: input (min, range), or output when the partial (min, max) table mm
// [P][H][4][2] of the forward step is given (then r = max(max - min, beta_f)).
// w1p: W1^T packed by fused_pack; w4p: W4^T packed by fused_pack.
void fused_encode(const PatchGrid& pg, const float* state, float* meta, const float* mm, int H, const float* beta,
                  const uint16_t* w1p, const float* b1, const uint16_t* w2t, const float* b2, uint16_t* zbf, float* zf,
                  hipStream_t st, uint16_t* meta16 = nullptr);
// exc (field 0 only): exception patches written with their exact values.
// grid > 0: the decode is queued as launches of at most grid work-groups, one after the
// other on st, so it holds fewer CUs at a time (0: one launch).
void fused_decode(const PatchGrid& pg, const uint16_t* z, const float* meta, const uint16_t* w3t, const float* b3,
                  const uint16_t* w4p, const float* b4, int f, float* state, hipStream_t st,
                  const ExcPatches* exc = nullptr, const uint16_t* meta16 = nullptr, long long grid = 0);

// Exception patches: the K largest-e-range patches of one compressed state are
// kept exactly. Ranges are compared by key = bits(r_e) >> EXC_BIN_SHIFT (bins 2^-5
// wide in relative terms); within the bin of the K-th largest, lower patch indices
// win.
constexpr int EXC_BIN_SHIFT = 18;
constexpr int EXC_NBIN = 1 << (32 - EXC_BIN_SHIFT);
// selection from meta [P][4][2] into idx [K] (increasing patch order); a single
// work-group kernel, cheap to overlap with other work
void exceptions_select(const PatchGrid& pg, const float* meta, int K, int* idx, hipStream_t st,
                       const uint16_t* meta16 = nullptr);
// copy the e values of the selected patches to exc [K][512]
void exceptions_gather(const PatchGrid& pg, const float* state, int K, const int* idx, float* exc, hipStream_t st);
// both
void exceptions_store(const PatchGrid& pg, const float* state, const float* meta, int K, int* idx, float* exc,
                      hipStream_t st, const uint16_t* meta16 = nullptr);
// rng [ceil(P/bm) + 1]: rng[b] = number of idx entries below patch bm b
void exceptions_ranges(const PatchGrid& pg, int K, const int* idx, int bm, int* rng, hipStream_t st);
// Write the stored e values back into an e field [N].
void exceptions_restore(const PatchGrid& pg, float* e, int K, const int* idx, const float* exc, hipStream_t st);

}  // namespace wv

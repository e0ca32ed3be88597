// Internal declarations shared by the HIP sources of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "plan.h"
#include "wavecomp.h"

namespace wv {

void set_error(const std::string& msg);

// HIP call whose failure throws (converted to WV_EDEVICE at the entry point)
#define WV_HIP(expr)                                                                   \
    do {                                                                               \
        hipError_t _e = (expr);                                                        \
        if (_e != hipSuccess)                                                          \
            throw ::wv::Error{WV_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)}; \
    } while (0)

// ---- stencil -----------------------------------------------------------------------

enum StepMode { MODE_FWD = 0, MODE_ADJ = 1, MODE_INC = 2, MODE_ADJQ = 3, MODE_ADJD = 4 };
// gradient accumulation phase of an adjoint step within its block of steps
enum AccPhase { ACC_EACH = 0, ACC_FIRST = 1, ACC_MID = 2, ACC_LAST = 3 };

// Tiling of the (y, x) plane and of z into chunks, plus the receiver list
// bucketed per (y, x) tile and sorted by depth.
struct Tiling {
    int bx = 64, by = 8;
    int tiles_x = 0, tiles_y = 0, chunks_z = 0, kc = 0;  // forward / incremental chunks
    int chunks_adj = 0, kc_adj = 0;                       // adjoint chunks
    // receivers of tile t at level k: rec_ent[rec_ptr[t (nz + 1) + k] ..
    // rec_ptr[t (nz + 1) + k + 1]), sorted by (local cell, receiver)
    int* rec_ptr = nullptr;   // [tiles][nz + 1]
    int4* rec_ent = nullptr;  // (k, local, r, 0)
};

struct StepArgs {
    int nz, ny, nx;
    long long N;         // cells per field
    long long sstride;   // floats between sources in a state array (4 N)
    float dtdx, dt;
    const float *wzc, *wzf, *wyc, *wyf, *wxc, *wxf;   // per-axis layer factors
    const float* m;      // c^2
    const float* in;     // state in  [S][4][N]
    float* out;          // state out [S][4][N]
    // sources (forward): centre face of each wavefield's source, box radius and
    // weights [(2R+1)^dims] (dk slowest)
    const int* src_kji;
    int src_radius;
    const float* src_w;
    const float* wavelet;  // [S][T]
    int nt, step;
    // receivers
    const int* rec_ptr;
    const int4* rec_ent;
    int nrec, tidx;        // time index into traces / residual
    float* traces;         // forward / incremental: [S][T][R]
    const float* resid;    // adjoint: [S][T][R]
    // adjoint: forward e at this level and the Kahan accumulators (per source)
    const float* ek;       // [S][ekstride]
    long long ekstride;
    float* acc;            // [S][2][N]: sum, compensation
    float* blk;            // [S][N]: float32 partial of the current block of steps
    int acc_phase;         // AccPhase of this step
    // full-Newton Hessian action: q of the mu step [S][N] (written by ADJQ, read by
    // ADJD), de^k of the dmu step
    float* qbuf;
    const float* dek;
    long long dekstride;
    // forward and incremental forward: e of the new state also written here ([S][N],
    // per-source stride N), the time-compression window slot of this level; null for none
    float* e_extra;
    // incremental forward: dm and forward e^n
    const float* dm;
    const float* en;
    long long enstride;
    int tiles_x, tiles_y, chunks_z, kc;
    int chunks_adj, kc_adj;
    // forward only: per-(patch, y sub-tile) min/max of the 4 new fields,
    // [S][P][8/BY][4][2] = (min, max), written when non-null (3D, grid of 8^3 patches)
    float* mm_out;
};

void launch_step(int mode, bool has_y, const StepArgs& a, int nsrc, hipStream_t st);
Tiling make_tiling(int nz, int ny, int nx, const std::vector<int>& rec_kji);
void free_tiling(Tiling& t);

// ---- reductions / elementwise -------------------------------------------------------

void launch_square(const float* c, float* m, long long n, hipStream_t st);
// J partial sums and residual; returns nothing (result in d_out[0] after finalize).
void launch_misfit(const float* p, const float* d, float* resid, long long n, double wres,
                   double wJ, double* partial, int nblocks, double* d_out, hipStream_t st);
void launch_scale_weights(const float* p, float* resid, long long n, double w, hipStream_t st);
void launch_grad_finish(const float* c, const float* acc, long long N, int nsrc, double scale,
                        float* g, hipStream_t st);
void launch_fill(float* p, long long n, float v, hipStream_t st);
// h = scale (dc * sum_s acc_s + c * sum_s dacc_s), acc/dacc [S][2][N] compensated pairs
void launch_newton_finish(const float* c, const float* dc, const float* acc, const float* dacc, long long N,
                          int nsrc, double scale, float* h, hipStream_t st);
void launch_compare(const float* a, const float* b, long long n, int* flag, hipStream_t st);
void launch_copy(float* dst, const float* src, long long n, hipStream_t st);
// d_out2[0] = sum (a - b)^2, d_out2[1] = sum b^2 (float64, fixed order)
void launch_err_norms(const float* a, const float* b, long long n, double* partial, int nblocks, double* d_out2,
                      hipStream_t st);
void launch_rel_err(const float* a, const float* b, long long n, double* partial, int nblocks,
                    double* d_out, hipStream_t st);
void launch_absmax_fields(const float* states, long long nstates, long long N, double* d_out4,
                          hipStream_t st);
// min, max and NaN count of x into d_out3 (float64)
void launch_range(const float* x, long long n, double* partial, int nblocks, double* d_out3,
                  hipStream_t st);
// dm = 2 c dc
void launch_dm(const float* c, const float* dc, float* dm, long long n, hipStream_t st);
// inverse-problem layer (inverse.hip)
void launch_prior(const float* u, const float* u0, float* out, int nz, int ny, int nx, double alpha, double cz,
                  double cy, double cx, double scale, bool accumulate, hipStream_t st);
void launch_axpby(float* y, const float* x, double a, double b, long long n, hipStream_t st);
void launch_lincomb(float* out, const float* x, double a, const float* y, long long n, hipStream_t st);
void launch_dot(const float* a, const float* b, long long n, double* partial, int nblocks, double* d_out,
                hipStream_t st);

}  // namespace wv

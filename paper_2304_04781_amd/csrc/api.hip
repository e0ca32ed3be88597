// Solver context, history storage policies, time loops and the C entry points
// of wavecomp.h (forward, adjoint, gradient, incremental forward, Hv).

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ae_internal.h"
#include "wv_internal.h"

namespace wv {

namespace {
thread_local std::string g_error;
}

void set_error(const std::string& msg) { g_error = msg; }

template <class F>
int guarded(F&& f)
{
    try {
        return f();
    } catch (const Error& e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return WV_ENOMEM;
    } catch (const std::exception& e) {
        set_error(e.what());
        return WV_EDEVICE;
    }
}

template <class T>
T* dev_alloc(size_t count)
{
    if (count == 0) count = 1;
    void* p = nullptr;
    const hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
        (void)hipGetLastError();
        throw Error{WV_ENOMEM, "device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed"};
    }
    if (e != hipSuccess) throw Error{WV_EDEVICE, std::string("hipMalloc: ") + hipGetErrorString(e)};
    // zero-filled: fields a mode never writes (v_y in 2D) read as zero in every state buffer
    WV_HIP(hipMemsetAsync(p, 0, count * sizeof(T), nullptr));
    WV_HIP(hipStreamSynchronize(nullptr));
    return static_cast<T*>(p);
}

template <class T>
void dev_free(T*& p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

// Sampled per-class kernel timing with HIP events recorded on the stream the
// timed work runs on (every `every`-th launch of each class).
struct KernelTimer {
    static constexpr int NCLS = 8;
    int every = 0;
    long long seen[NCLS] = {};
    double sum_ms[NCLS] = {};
    long long cnt[NCLS] = {};
    struct Rec {
        int cls;
        hipEvent_t a, b;
    };
    std::vector<hipEvent_t> pool;
    std::vector<Rec> recs;

    hipEvent_t get()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e;
        WV_HIP(hipEventCreate(&e));
        return e;
    }
    // fold finished records into the totals (waits for them)
    void collect()
    {
        for (const Rec& r : recs) {
            WV_HIP(hipEventSynchronize(r.b));
            float ms = 0.f;
            WV_HIP(hipEventElapsedTime(&ms, r.a, r.b));
            sum_ms[r.cls] += ms;
            cnt[r.cls] += 1;
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        recs.clear();
    }
    // returns the record index to close with end(), or -1 when this launch is not sampled
    int begin(int cls, hipStream_t st)
    {
        if (every <= 0 || (seen[cls]++ % every) != 0) return -1;
        if (recs.size() >= 4096) collect();
        Rec r{cls, get(), get()};
        WV_HIP(hipEventRecord(r.a, st));
        recs.push_back(r);
        return (int)recs.size() - 1;
    }
    void end(int idx, hipStream_t st)
    {
        if (idx >= 0) WV_HIP(hipEventRecord(recs[idx].b, st));
    }
    void reset(int ev)
    {
        collect();
        every = ev;
        for (int i = 0; i < NCLS; ++i) {
            seen[i] = cnt[i] = 0;
            sum_ms[i] = 0.0;
        }
    }
    void destroy()
    {
        for (const Rec& r : recs) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        recs.clear();
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
        pool.clear();
    }
};
enum {
    TM_FWD = 0,
    TM_ADJ = 1,
    TM_INC = 2,
    TM_ENCODE = 3,
    TM_DECODE = 4,
    TM_EXC_SELECT = 5,
    TM_EXC_RESTORE = 6,
    TM_EXC_GATHER = 7
};

}  // namespace wv

using namespace wv;

// Flags of the events that order the main and side streams. They are recorded and waited on
// within one device (the host only asks whether they completed), and every kernel releases
// its writes to the device when it ends, so the events need no system-scope fence: without
// it the 256^3 x 400 gradient and Gauss-Newton Hv ran about 1 % faster, results bit for bit
// unchanged (a device-scope release instead changed nothing).
#ifndef WV_SYNC_EVENT_FLAGS
#define WV_SYNC_EVENT_FLAGS (hipEventDisableTiming | hipEventDisableSystemFence)
#endif
constexpr unsigned SYNC_EVENT_FLAGS = WV_SYNC_EVENT_FLAGS;

// decoded-e slots: the decode of a state runs up to NEB - 1 steps ahead of its use
#ifndef WV_NEB
#define WV_NEB 3
#endif
constexpr int NEB = WV_NEB;
// Work-groups per decode launch in the reverse sweep of a gradient (0: one launch). A
// decode there runs two steps ahead of the adjoint step that reads it, so it may take
// longer than a step; queued as two launches (384 work-groups, then the rest at 256^3) it
// holds fewer CUs at a time, and the adjoint step beside it ran 184 us instead of 197.
// The incremental forward sweep of a Hessian action keeps one launch (its decodes run
// beside the encodes of the incremental states, and sliced they ran slower).
#ifndef WV_REV_DEC_GRID
#define WV_REV_DEC_GRID 384
#endif
constexpr long long REV_DEC_GRID = WV_REV_DEC_GRID;

// Latent store of the states x_1 .. x_{T-1} of every source (AE modes): latents,
// per-patch metadata, FP8 scales and the exact e values of the exception patches
struct LatStore {
    uint8_t* lat = nullptr;   // [T-1][S][P][L]
    float* meta = nullptr;    // [T-1][S][P][4][2] float32 (lo, r), or
    uint16_t* meta16 = nullptr;  // the same as bfloat16 (16-bit metadata)
    float* qs = nullptr;      // [T-1][S][P]
    int* exc_idx = nullptr;   // [T-1][S][K]
    float* exc = nullptr;     // [T-1][S][K][512]
    int* exc_rng = nullptr;   // [T-1][S][nbd + 1]: exceptions per decode work-group
};

// One time-compressed history (e^1..e^{T-1} of the forward solve, or de^1..de^{T-1}
// of the incremental forward): latents [nwin][S B][L] bf16, meta [nwin][S B][2]
// (lo, r), the K exact vectors per window and source, and two window buffers
// [2][TWIN][S][N]. The forward fills one buffer while the other is compressed on
// the store's side stream; the reverse-time sweeps read one while the next window
// is decompressed into the other.
struct TimeStore {
    uint16_t* lat = nullptr;
    float* meta = nullptr;
    float* win = nullptr;
    int* exc_idx = nullptr;      // [nwin][S][K] block indices, increasing
    float* exc = nullptr;        // [nwin][S][K][2048] their exact values
    int K = 0;
    int side = 0;                // side stream index of its codec work
    int buf_w[2] = {-1, -1};     // window held decoded in each buffer (-1: none)
    int cur_w = -1;              // window the main stream reads now
    hipEvent_t ev_fill[2] = {}, ev_enc[2] = {}, ev_ready[2] = {}, ev_free[2] = {};
};

// stored states checked by the accuracy guard per forward solve (plus the last)
constexpr int GUARD_CHECKS = 16;

struct wv_ctx {
    KernelTimer tm;
    wv_grid g{};
    bool has_y = true;
    long long N = 0;
    int S = 1, T = 1, R = 0;
    hipStream_t st = nullptr;

    float* tab = nullptr;  // wzc wzf wyc wyf wxc wxf
    float *wzc = nullptr, *wzf = nullptr, *wyc = nullptr, *wyf = nullptr, *wxc = nullptr, *wxf = nullptr;
    Tiling tl;

    int* src_kji = nullptr;      // [S][3]
    float* src_w = nullptr;      // source stencil weights
    int src_radius = 0;
    float* m = nullptr;
    float* c_last = nullptr;
    float* wavelet = nullptr;
    float* work[3] = {nullptr, nullptr, nullptr};  // [2]: only for autoencoder stores
    float* adj[2] = {nullptr, nullptr};
    float* incb[3] = {nullptr, nullptr, nullptr};  // the third only while an incremental store runs beside
    float* acc = nullptr;
    float* blk = nullptr;        // [S][N] float32 partial gradient of a block of adjoint steps
    float* ebuf = nullptr;       // [NEB][S][N]: decoded e, one slot per state in flight
    float* dm = nullptr;
    float* traces = nullptr;
    float* resid = nullptr;      // dt/sigma^2 (p - d) of the last gradient
    float* dtr = nullptr;
    float* dresid = nullptr;     // dt/sigma^2 dp of the last Hessian action
    // full-Newton Hessian action: second adjoint state, its sums, q of the mu step,
    // de history (full storage) and a decoded de^k (AE modes)
    float* adj2[2] = {nullptr, nullptr};
    float* dacc = nullptr;
    float* dblk = nullptr;
    float* qbuf = nullptr;
    float* dehist = nullptr;
    float* dbuf = nullptr;
    double* partial = nullptr;
    double* dscal = nullptr;
    int* dflag = nullptr;
    int nblk_red = 1024;

    // history store
    int mode = WV_STORE_NONE;
    int nslots = 0;
    ae_net* ae = nullptr;
    int64_t budget = 0;
    double guard_tol = 0.0;
    int fallback = WV_FALLBACK_NONE;
    float* slots = nullptr;      // checkpoint slots 1..nslots-1
    float* ehist = nullptr;      // full storage of e^1..e^{T-1}
    LatStore fs;                 // AE store of the forward states
    LatStore ds;                 // AE store of the incremental forward states (optional)
    bool store_delta = false;    // compress the incremental states in the AE modes
    bool delta_ok = false;       // ds holds the incremental states of the last incremental forward
    int64_t delta_bytes = 0;
    int exc_req = 0;             // requested exception patches per state
    int meta_req = 32;           // requested bits per (lo, r) value of the AE stores (32 or 16)
    bool m16 = false;            // the AE stores keep bfloat16 (lo, r)
    int K = 0;                   // active exception patches per state
    int nbd = 0;                 // decode work-groups per state
    long long pipe_grid = 0;     // work-groups per decode launch of the running decode pipeline (0: one launch)
    float* mmpart = nullptr;     // [3][S][P][H][4][2] (min, max) partials of the forward step
    int H = 1;                   // y sub-tiles per patch
    // Autoencoder stores and decodes run beside the stencil steps: `side` encodes
    // x_j (and decodes e^k for the reverse sweeps), `side2` selects and copies the
    // exception patches of x_j. Forward states rotate through three buffers, so
    // the store of x_j may take until the step that overwrites x_j, two later.
    // The incremental forward's latent store encodes dx_n on `side3` (the decodes of
    // e^n are on `side`) and selects and copies its exception patches on `side2`.
    // The three side streams belong to the device, not the context (shared_side).
    hipStream_t side = nullptr;
    hipStream_t side2 = nullptr;
    hipStream_t side3 = nullptr;
    hipEvent_t ev_step[3] = {};    // main: x_j written (j mod 3)
    hipEvent_t ev_enc[3] = {};     // side: x_j encoded
    hipEvent_t ev_stored[3] = {};  // x_j fully stored: its buffer and mmpart slot are free
    hipEvent_t ev_ready[NEB] = {};  // side: e^k decoded into ebuf slot
    hipEvent_t ev_free[NEB] = {};   // main: ebuf slot consumed
    hipEvent_t ev_join = nullptr;
    hipEvent_t ev_dstep[3] = {};    // main: dx_n written (n mod 3), incremental forward
    hipEvent_t ev_denc[3] = {};     // dx_n encoded
    hipEvent_t ev_dstored[3] = {};  // dx_n fully stored: its buffer and partial slot are free
    long long P = 0;
    long long lat_bytes = 0;     // per patch
    int64_t store_bytes = 0;

    bool store_ok = false;       // the store matches c_last
    bool degraded = false;       // accuracy guard tripped
    double guard_err = -1.0;
    // accuracy guard buffers (allocated with the AE store when guard_tol > 0): the
    // decoded e of a checked state [S][N], the reduction partials of its error and the
    // errors [GUARD_CHECKS + 1][S] of the checked states of the last forward solve
    float* gbuf = nullptr;
    double* gpart = nullptr;
    double* gres = nullptr;
    bool have_grad = false;
    double sigma = 1.0;
    long long last_fwd_steps = 0;

    // time compression: the forward history ts and (full-Newton products) the
    // incremental history tds, on one block layout
    TimeStore ts;
    TimeStore tds;
    long long TB = 0;            // 4^3 blocks per source
    int nwin = 0;
    int tlat_dim = 0;
    bool tdelta_ok = false;      // tds holds the incremental states of the last incremental forward

    // MAP layer: BiLaplacian prior and the Newton-CG work vectors
    double prior_alpha = 0.0;
    double prior_theta[3] = {0.0, 0.0, 0.0};
    float* prior_c0 = nullptr;
    float* prior_w = nullptr;    // A (c - c0) or A dc
    float* nvec = nullptr;       // [8][N]: g, trial g, trial c, p, r, d, H d, M r
    float* pvec = nullptr;       // [4][N]: the inner CG of the elliptic solves

    long long state_floats() const { return 4LL * N * S; }
    float* slot_ptr(int b) const { return slots + (long long)(b - 1) * state_floats(); }
};

namespace {

double axis_sigma(double pos, int n, bool low_absorbs, int ns, double smax)
{
    double s = 0.0;
    if (ns <= 0) return 0.0;
    if (low_absorbs && pos < ns) s += smax * std::pow((ns - pos) / ns, 2);
    const double w = n - pos;
    if (w < ns) s += smax * std::pow((ns - w) / ns, 2);
    return s;
}

void build_tables(wv_ctx* c)
{
    const wv_grid& g = c->g;
    const int ns = g.sponge;
    const double smax = ns > 0 ? 3.0 * g.c_ref * std::log(1000.0) / (2.0 * ns * g.dx) : 0.0;
    const int nz = g.nz, ny = g.ny, nx = g.nx;
    std::vector<float> h(2 * (size_t)(nz + ny + nx));
    float* wzc = h.data();
    float* wzf = wzc + nz;
    float* wyc = wzf + nz;
    float* wyf = wyc + ny;
    float* wxc = wyf + ny;
    float* wxf = wxc + nx;
    for (int k = 0; k < nz; ++k) {
        wzc[k] = (float)std::exp(-g.dt * axis_sigma(k + 0.5, nz, false, ns, smax));
        wzf[k] = (float)std::exp(-g.dt * axis_sigma(k, nz, false, ns, smax));
    }
    for (int j = 0; j < ny; ++j) {
        wyc[j] = c->has_y ? (float)std::exp(-g.dt * axis_sigma(j + 0.5, ny, true, ns, smax)) : 1.0f;
        wyf[j] = c->has_y ? (float)std::exp(-g.dt * axis_sigma(j, ny, true, ns, smax)) : 1.0f;
    }
    for (int i = 0; i < nx; ++i) {
        wxc[i] = (float)std::exp(-g.dt * axis_sigma(i + 0.5, nx, true, ns, smax));
        wxf[i] = (float)std::exp(-g.dt * axis_sigma(i, nx, true, ns, smax));
    }
    c->tab = dev_alloc<float>(h.size());
    WV_HIP(hipMemcpy(c->tab, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice));
    c->wzc = c->tab;
    c->wzf = c->wzc + nz;
    c->wyc = c->wzf + nz;
    c->wyf = c->wyc + ny;
    c->wxc = c->wyf + ny;
    c->wxf = c->wxc + nx;
}

StepArgs base_args(const wv_ctx* c)
{
    StepArgs a{};
    a.nz = c->g.nz;
    a.ny = c->g.ny;
    a.nx = c->g.nx;
    a.N = c->N;
    a.sstride = 4 * c->N;
    a.dtdx = (float)(c->g.dt / c->g.dx);
    a.dt = (float)c->g.dt;
    a.wzc = c->wzc; a.wzf = c->wzf; a.wyc = c->wyc; a.wyf = c->wyf; a.wxc = c->wxc; a.wxf = c->wxf;
    a.m = c->m;
    a.src_kji = c->src_kji;
    a.src_radius = c->src_radius;
    a.src_w = c->src_w;
    a.wavelet = c->wavelet;
    a.nt = c->T;
    a.rec_ptr = c->tl.rec_ptr;
    a.rec_ent = c->tl.rec_ent;
    a.nrec = c->R;
    a.tiles_x = c->tl.tiles_x;
    a.tiles_y = c->tl.tiles_y;
    a.chunks_z = c->tl.chunks_z;
    a.kc = c->tl.kc;
    a.chunks_adj = c->tl.chunks_adj;
    a.kc_adj = c->tl.kc_adj;
    a.mm_out = nullptr;
    return a;
}

// one forward step n: state in -> out; traces (nullptr: not recorded); mm: per-patch
// (min, max) partials of the new state (nullptr: not computed)
// e_extra: the new e is also written there ([S][N]), the time-compression window slot
void fwd_step(wv_ctx* c, const float* in, float* out, int n, float* traces, float* mm = nullptr,
              float* e_extra = nullptr)
{
    StepArgs a = base_args(c);
    a.in = in;
    a.out = out;
    a.step = n;
    a.tidx = n;
    a.traces = traces;
    a.mm_out = mm;
    a.e_extra = e_extra;
    if (!traces) a.nrec = 0;
    const int t = c->tm.begin(TM_FWD, c->st);
    launch_step(MODE_FWD, c->has_y, a, c->S, c->st);
    c->tm.end(t, c->st);
}

// adjoint launch k: (mu^{k+2}, eta^{k+1}) -> (mu^{k+1}, eta^k), consuming e^k
// Adjoint steps sum their gradient terms per block of WV_ACC_BLOCK consecutive
// steps in float32 and add each block to the compensated (Kahan) pair; the phase
// of the step at sweep position j (0 = the sweep's first step), the sweep ending at k = 1.
#ifndef WV_ACC_BLOCK
#define WV_ACC_BLOCK 8
#endif
int acc_phase(long long j, int k)
{
    const bool first = j % WV_ACC_BLOCK == 0, last = j % WV_ACC_BLOCK == WV_ACC_BLOCK - 1 || k == 1;
    return first ? (last ? ACC_EACH : ACC_FIRST) : (last ? ACC_LAST : ACC_MID);
}

// One adjoint step of `mode` (MODE_ADJ; MODE_ADJQ / MODE_ADJD for the two sweeps
// of the full-Newton Hessian action) accumulating into acc / blk.
void adj_step_x(wv_ctx* c, int mode, const float* in, float* out, int k, const float* resid, const float* ek,
                long long ekstride, int phase, float* acc, float* blk, const float* dek = nullptr)
{
    StepArgs a = base_args(c);
    a.blk = blk;
    a.acc_phase = phase;
    a.in = in;
    a.out = out;
    a.tidx = k;
    a.resid = resid;
    a.ek = ek;
    a.ekstride = ekstride;
    a.acc = acc;
    a.qbuf = c->qbuf;
    a.dek = dek;
    a.dekstride = c->N;
    a.dm = c->dm;
    const int t = c->tm.begin(TM_ADJ, c->st);
    launch_step(mode, c->has_y, a, c->S, c->st);
    c->tm.end(t, c->st);
}

void adj_step(wv_ctx* c, const float* in, float* out, int k, const float* resid, const float* ek,
              long long ekstride, int phase)
{
    adj_step_x(c, MODE_ADJ, in, out, k, resid, ek, ekstride, phase, c->acc, c->blk);
}

void inc_step(wv_ctx* c, const float* in, float* out, int n, const float* en, long long enstride,
              float* dtraces, float* e_extra = nullptr, float* mm = nullptr)
{
    StepArgs a = base_args(c);
    a.e_extra = e_extra;
    a.mm_out = mm;
    a.in = in;
    a.out = out;
    a.tidx = n;
    a.step = n;
    a.traces = dtraces;
    a.dm = c->dm;
    a.en = en;
    a.enstride = enstride;
    const int t = c->tm.begin(TM_INC, c->st);
    launch_step(MODE_INC, c->has_y, a, c->S, c->st);
    c->tm.end(t, c->st);
}

void ensure_inc(wv_ctx* c)
{
    if (!c->incb[0]) {
        c->incb[0] = dev_alloc<float>(c->state_floats());
        c->incb[1] = dev_alloc<float>(c->state_floats());
        c->dm = dev_alloc<float>(c->N);
    }
}

void free_latstore(LatStore& L)
{
    dev_free(L.lat);
    dev_free(L.meta);
    dev_free(L.meta16);
    dev_free(L.qs);
    dev_free(L.exc_idx);
    dev_free(L.exc);
    dev_free(L.exc_rng);
}

// frees the buffers of a time store; its events live as long as the context
void free_timestore(TimeStore& T)
{
    dev_free(T.lat);
    dev_free(T.meta);
    dev_free(T.win);
    dev_free(T.exc_idx);
    dev_free(T.exc);
    T.K = 0;
    T.buf_w[0] = T.buf_w[1] = -1;
    T.cur_w = -1;
}

void free_store(wv_ctx* c)
{
    dev_free(c->slots);
    dev_free(c->ehist);
    free_latstore(c->fs);
    free_latstore(c->ds);
    c->delta_ok = false;
    c->delta_bytes = 0;
    dev_free(c->mmpart);
    dev_free(c->work[2]);
    dev_free(c->gbuf);
    dev_free(c->gpart);
    dev_free(c->gres);
    free_timestore(c->ts);
    free_timestore(c->tds);
    c->tdelta_ok = false;
    c->K = 0;
    c->m16 = false;
    c->store_bytes = 0;
    c->store_ok = false;
}

void alloc_slots(wv_ctx* c, int nslots)
{
    if (nslots < 1) throw Error{WV_EINVAL, "checkpointing needs at least one slot"};
    const long long bytes = (long long)(nslots - 1) * c->state_floats() * 4;
    if (c->budget > 0 && bytes > c->budget) throw Error{WV_ENOMEM, "checkpoint slots exceed the memory budget"};
    dev_free(c->slots);
    c->nslots = nslots;
    if (nslots > 1) c->slots = dev_alloc<float>((size_t)(nslots - 1) * c->state_floats());
}

// check c: positive, finite and stable for leapfrog
void check_speed(wv_ctx* c, const float* cdev)
{
    launch_range(cdev, c->N, c->partial, c->nblk_red, c->dscal, c->st);
    double h[3];
    WV_HIP(hipMemcpyAsync(h, c->dscal, sizeof(h), hipMemcpyDeviceToHost, c->st));
    WV_HIP(hipStreamSynchronize(c->st));
    WV_REQUIRE(h[2] == 0.0, WV_EINVAL, "wave speed contains NaN");
    WV_REQUIRE(h[0] > 0.0, WV_EINVAL, "wave speed must be positive");
    const double dims = c->has_y ? 3.0 : 2.0;
    const double cfl = h[1] * c->g.dt / c->g.dx;
    WV_REQUIRE(cfl < 1.0 / std::sqrt(dims), WV_EUNSTABLE,
               "c_max dt/dx = " + std::to_string(cfl) + " exceeds the leapfrog limit 1/sqrt(dims)");
}

void prepare_model(wv_ctx* c, const float* cdev, const float* wavelet)
{
    check_speed(c, cdev);
    launch_square(cdev, c->m, c->N, c->st);
    launch_copy(c->c_last, cdev, c->N, c->st);
    if (wavelet)
        WV_HIP(hipMemcpyAsync(c->wavelet, wavelet, sizeof(float) * c->S * c->T, hipMemcpyDeviceToDevice, c->st));
}

bool is_ae(int mode) { return mode == WV_STORE_AE_BF16 || mode == WV_STORE_AE_FP8; }
bool is_time(int mode) { return mode == WV_STORE_AE_TIME; }
float* twin_buf(const wv_ctx* c, const TimeStore& T, int b) { return T.win + (long long)b * TWIN * c->S * c->N; }
int* texc_idx_slot(const wv_ctx* c, const TimeStore& T, int w, int s)
{
    return T.exc_idx + ((long long)w * c->S + s) * T.K;
}
float* texc_slot(const wv_ctx* c, const TimeStore& T, int w, int s)
{
    return T.exc + ((long long)w * c->S + s) * T.K * 2048;
}
TimeGrid ctx_time_grid(const wv_ctx* c) { return time_grid(c->g.nz, c->g.ny, c->g.nx, c->S); }
uint16_t* tlat_slot(const wv_ctx* c, const TimeStore& T, int w)
{
    return T.lat + (long long)w * c->TB * c->S * c->tlat_dim;
}
float* tmeta_slot(const wv_ctx* c, const TimeStore& T, int w) { return T.meta + (long long)w * c->TB * c->S * 2; }

// bytes of a time store with K exact vectors per window and source (its two
// window buffers are work space and not counted)
long long timestore_bytes(const wv_ctx* c, int K)
{
    const long long rows = (long long)c->nwin * c->TB * c->S;
    const long long kslots = (long long)c->nwin * c->S * K;
    return rows * (c->tlat_dim * 2 + 8) + kslots * (4 + 2048 * 4);
}

void alloc_timestore(wv_ctx* c, TimeStore& T, int K)
{
    const long long rows = (long long)c->nwin * c->TB * c->S;
    const long long kslots = (long long)c->nwin * c->S * K;
    T.lat = dev_alloc<uint16_t>(rows * c->tlat_dim);
    T.meta = dev_alloc<float>(rows * 2);
    T.K = K;
    if (K > 0) {
        T.exc_idx = dev_alloc<int>(kslots);
        T.exc = dev_alloc<float>(kslots * 2048);
    }
    T.win = dev_alloc<float>((size_t)2 * TWIN * c->S * c->N);
    T.buf_w[0] = T.buf_w[1] = -1;
    T.cur_w = -1;
}
int ae_fmt(int mode) { return mode == WV_STORE_AE_FP8 ? AE_LATENT_FP8 : AE_LATENT_BF16; }


uint8_t* lat_slot(wv_ctx* c, const LatStore& L, int idx, int s)
{
    return L.lat + ((long long)idx * c->S + s) * c->P * c->lat_bytes;
}
float* meta_slot(wv_ctx* c, const LatStore& L, int idx, int s)
{
    return L.meta ? L.meta + ((long long)idx * c->S + s) * c->P * 8 : nullptr;
}
uint16_t* meta16_slot(wv_ctx* c, const LatStore& L, int idx, int s)
{
    return L.meta16 ? L.meta16 + ((long long)idx * c->S + s) * c->P * 8 : nullptr;
}
int* rng_slot(wv_ctx* c, const LatStore& L, long long q) { return L.exc_rng + q * (c->nbd + 1); }
float* qs_slot(wv_ctx* c, const LatStore& L, int idx, int s)
{
    return L.qs ? L.qs + ((long long)idx * c->S + s) * c->P : nullptr;
}

// bytes of one latent store for the current mode and exception count
long long latstore_bytes(wv_ctx* c, int mode, int K)
{
    const long long slots = (long long)std::max(c->T - 1, 1) * c->S;
    const long long nbd = (c->P + DEC_BM - 1) / DEC_BM;
    return slots * (c->P * (c->lat_bytes + (c->m16 ? 16 : 32) + (mode == WV_STORE_AE_FP8 ? 4 : 0)) +
                    (long long)K * (512 * 4 + 4) +
                    (K > 0 ? (nbd + 1) * 4 : 0));
}

void alloc_latstore(wv_ctx* c, LatStore& L, int mode, int K)
{
    const long long slots = (long long)std::max(c->T - 1, 1) * c->S;
    L.lat = dev_alloc<uint8_t>(slots * c->P * c->lat_bytes);
    if (c->m16)
        L.meta16 = dev_alloc<uint16_t>(slots * c->P * 8);
    else
        L.meta = dev_alloc<float>(slots * c->P * 8);
    if (mode == WV_STORE_AE_FP8) L.qs = dev_alloc<float>(slots * c->P);
    if (K > 0) {
        L.exc_idx = dev_alloc<int>(slots * K);
        L.exc = dev_alloc<float>(slots * K * 512);
        L.exc_rng = dev_alloc<int>(slots * (c->nbd + 1));
    }
}

void wait_event(hipStream_t st, hipEvent_t ev);
hipStream_t side_stream(wv_ctx* c, int which);

// encode x_n of every source into the autoencoder store L on stream st, with the
// per-patch (min, max) partials mm of the step that wrote it when given (else the
// encode computes them)
void encode_state_into(wv_ctx* c, LatStore& L, int n, const float* state, hipStream_t st, const float* mm)
{
    const PatchGrid pg = patch_grid(c->g.nz, c->g.ny, c->g.nx);
    const int te = c->tm.begin(TM_ENCODE, st);
    for (int s = 0; s < c->S; ++s) {
        if (mm)
            ae_encode_state_mm(c->ae, pg, state + s * 4 * c->N, mm + (long long)s * c->P * c->H * 8, c->H,
                               ae_fmt(c->mode), lat_slot(c, L, n - 1, s), meta_slot(c, L, n - 1, s),
                               qs_slot(c, L, n - 1, s), st, meta16_slot(c, L, n - 1, s));
        else {
            WV_REQUIRE(!c->m16, WV_EINVAL, "16-bit metadata needs the step's (min, max) partials");
            ae_encode_state(c->ae, pg, state + s * 4 * c->N, ae_fmt(c->mode), lat_slot(c, L, n - 1, s),
                            meta_slot(c, L, n - 1, s), qs_slot(c, L, n - 1, s), st);
        }
    }
    c->tm.end(te, st);
}

// select and copy the exception patches of x_n (after its encode wrote the ranges)
void exceptions_into(wv_ctx* c, LatStore& L, int n, const float* state, hipStream_t st)
{
    if (c->K <= 0) return;
    const PatchGrid pg = patch_grid(c->g.nz, c->g.ny, c->g.nx);
    const int tx = c->tm.begin(TM_EXC_SELECT, st);
    for (int s = 0; s < c->S; ++s) {
        const long long q = (long long)(n - 1) * c->S + s;
        exceptions_store(pg, state + s * 4 * c->N, meta_slot(c, L, n - 1, s), c->K, L.exc_idx + q * c->K,
                         L.exc + q * c->K * 512, st, meta16_slot(c, L, n - 1, s));
        exceptions_ranges(pg, c->K, L.exc_idx + q * c->K, DEC_BM, rng_slot(c, L, q), st);
    }
    c->tm.end(tx, st);
}

// Window slot of level j (1..T-1) in store T, for the step about to write it.
// The buffer held window w - 2, whose compression must have read it first.
float* time_slot(wv_ctx* c, TimeStore& T, int j)
{
    const int t = (j - 1) % TWIN, w = (j - 1) / TWIN, b = w & 1;
    if (t == 0 && w >= 2) wait_event(c->st, T.ev_enc[b]);
    return twin_buf(c, T, b) + (long long)t * c->S * c->N;
}

// After the step that wrote level n into its slot: a full window (or the last,
// short one) is compressed on the store's side stream while the steps go on into
// the other buffer.
void time_store_level(wv_ctx* c, TimeStore& T, int n)
{
    if (n < 1 || n > c->T - 1) return;
    const int t = (n - 1) % TWIN, w = (n - 1) / TWIN, b = w & 1;
    if (t != TWIN - 1 && n != c->T - 1) return;
    float* buf = twin_buf(c, T, b);
    hipStream_t s1 = side_stream(c, T.side);
    WV_HIP(hipEventRecord(T.ev_fill[b], c->st));
    wait_event(s1, T.ev_fill[b]);
    const TimeGrid tg = ctx_time_grid(c);
    const int te = c->tm.begin(TM_ENCODE, s1);
    ae_time_encode(c->ae, tg, buf, t + 1, tlat_slot(c, T, w), tmeta_slot(c, T, w), s1);
    for (int s = 0; s < c->S && T.K > 0; ++s)
        time_exceptions_store(tg, buf, s, t + 1, tmeta_slot(c, T, w) + (long long)s * c->TB * 2, T.K,
                              texc_idx_slot(c, T, w, s), texc_slot(c, T, w, s), s1);
    c->tm.end(te, s1);
    WV_HIP(hipEventRecord(T.ev_enc[b], s1));
}

// store x_n (n = 1..T-1) of every source on the main stream (full storage), or
// into the autoencoder store L on stream st when given, with the per-patch
// (min, max) partials mm of the step that wrote it when given
// (else the encode computes them)
void store_state(wv_ctx* c, LatStore& L, int n, const float* state, hipStream_t st = nullptr,
                 const float* mm = nullptr)
{
    if (n < 1 || n > c->T - 1) return;
    if (!st) st = c->st;
    if (c->mode == WV_STORE_FULL) {
        for (int s = 0; s < c->S; ++s)
            WV_HIP(hipMemcpyAsync(c->ehist + ((long long)(n - 1) * c->S + s) * c->N, state + s * 4 * c->N,
                                  sizeof(float) * c->N, hipMemcpyDeviceToDevice, c->st));
    } else if (is_time(c->mode)) {
        (void)state;  // the forward step wrote e^n into its window slot
        time_store_level(c, c->ts, n);
    } else if (is_ae(c->mode)) {
        encode_state_into(c, L, n, state, st, mm);
        exceptions_into(c, L, n, state, st);
    }
}

// Make stream st wait for event ev, unless the host already sees it complete
// (then the wait packet, which costs the stream a few microseconds, is skipped).
void wait_event(hipStream_t st, hipEvent_t ev)
{
    const hipError_t q = hipEventQuery(ev);
    if (q == hipSuccess) return;
    if (q != hipErrorNotReady) WV_HIP(q);
    WV_HIP(hipStreamWaitEvent(st, ev, 0));
}

// 1: autoencoder stores and decodes run on the side streams, beside the stencil
// steps; 2: only the exception selection and copy do; 0: everything on the main
// stream in order. With several sources the stencil launch holds S times the
// work-groups and the side-stream kernels starve beside it (an 8-source 512^2 x 256
// decode ran 10x slower than alone), so such contexts use mode 2.
#ifndef WV_OVERLAP
#define WV_OVERLAP 1
#endif
hipStream_t side_stream(wv_ctx* c, int which)
{
    const int mode = (WV_OVERLAP == 1 && c->S > 1) ? 2 : WV_OVERLAP;
    if (which == 2) return mode == 1 ? c->side3 : c->st;
    if (which) return mode >= 1 ? c->side2 : c->st;
    return mode == 1 ? c->side : c->st;
}

// Autoencoder store of x_j (1 <= j <= T-1) written by the forward step just
// launched on the main stream, with its min/max partials in mm: encode on `side`,
// exception selection and copy on `side2`; ev_stored[j % 3] marks the end.
void store_state_async(wv_ctx* c, int j, const float* state, const float* mm)
{
    const PatchGrid pg = patch_grid(c->g.nz, c->g.ny, c->g.nx);
    const int b = j % 3;
    hipStream_t s1 = side_stream(c, 0), s2 = side_stream(c, 1);
    WV_HIP(hipEventRecord(c->ev_step[b], c->st));
    wait_event(s1, c->ev_step[b]);
    const int te = c->tm.begin(TM_ENCODE, s1);
    for (int s = 0; s < c->S; ++s)
        ae_encode_state_mm(c->ae, pg, state + s * 4 * c->N, mm + (long long)s * c->P * c->H * 8, c->H,
                           ae_fmt(c->mode), lat_slot(c, c->fs, j - 1, s), meta_slot(c, c->fs, j - 1, s),
                           qs_slot(c, c->fs, j - 1, s), s1, meta16_slot(c, c->fs, j - 1, s));
    c->tm.end(te, s1);
    if (c->K <= 0) {
        WV_HIP(hipEventRecord(c->ev_stored[b], s1));
        return;
    }
    WV_HIP(hipEventRecord(c->ev_enc[b], s1));
    wait_event(s2, c->ev_enc[b]);
    const int tx = c->tm.begin(TM_EXC_SELECT, s2);
    for (int s = 0; s < c->S; ++s) {
        const long long q = (long long)(j - 1) * c->S + s;
        exceptions_select(pg, meta_slot(c, c->fs, j - 1, s), c->K, c->fs.exc_idx + q * c->K, s2,
                          meta16_slot(c, c->fs, j - 1, s));
        exceptions_ranges(pg, c->K, c->fs.exc_idx + q * c->K, DEC_BM, rng_slot(c, c->fs, q), s2);
    }
    c->tm.end(tx, s2);
    const int tg = c->tm.begin(TM_EXC_GATHER, s2);
    for (int s = 0; s < c->S; ++s) {
        const long long q = (long long)(j - 1) * c->S + s;
        exceptions_gather(pg, state + s * 4 * c->N, c->K, c->fs.exc_idx + q * c->K, c->fs.exc + q * c->K * 512,
                          s2);
    }
    c->tm.end(tg, s2);
    WV_HIP(hipEventRecord(c->ev_stored[b], s2));
}

// make the main stream wait for everything queued on the side streams
void join_side(wv_ctx* c)
{
    for (hipStream_t st : {c->side, c->side2, c->side3}) {
        WV_HIP(hipEventRecord(c->ev_join, st));
        WV_HIP(hipStreamWaitEvent(c->st, c->ev_join, 0));
    }
}

void ensure_adj(wv_ctx* c)
{
    if (!c->adj[0]) {
        c->adj[0] = dev_alloc<float>(c->state_floats());
        c->adj[1] = dev_alloc<float>(c->state_floats());
        c->acc = dev_alloc<float>(2 * c->N * c->S);
        c->blk = dev_alloc<float>(c->N * c->S);
        c->ebuf = dev_alloc<float>(NEB * c->N * c->S);
    }
}

// e^n of every source from the FULL or AE store: pointer + per-source stride
float* ebuf_slot(wv_ctx* c, int b) { return c->ebuf + (long long)b * c->S * c->N; }

// decode the fields in mask of stored state n of every source from the AE store L
// into out (per-source stride `stride` floats; field f at + f N) on stream st, in
// launches of at most grid work-groups (0: one launch per field)
void decode_state(wv_ctx* c, const LatStore& L, int n, uint32_t mask, float* out, long long stride,
                  hipStream_t st, long long grid = 0)
{
    WV_REQUIRE(n >= 1 && n <= c->T - 1, WV_ESTATE, "stored state index out of range");
    const PatchGrid pg = patch_grid(c->g.nz, c->g.ny, c->g.nx);
    for (int s = 0; s < c->S; ++s) {
        // the exception patches of e are written with their exact values by the decode
        const long long q = (long long)(n - 1) * c->S + s;
        const ExcPatches ex{L.exc_idx + q * c->K, c->K, L.exc + q * c->K * 512,
                            c->K > 0 ? rng_slot(c, L, q) : nullptr};
        const int td = c->tm.begin(TM_DECODE, st);
        ae_decode_state(c->ae, pg, lat_slot(c, L, n - 1, s), meta_slot(c, L, n - 1, s), qs_slot(c, L, n - 1, s),
                        ae_fmt(c->mode), mask, out + s * stride, st, c->K > 0 ? &ex : nullptr,
                        meta16_slot(c, L, n - 1, s), grid);
        c->tm.end(td, st);
    }
}

// decode e^n of every source from the forward AE store into ebuf slot b on stream st
void decode_e(wv_ctx* c, int n, int b, hipStream_t st, long long grid = 0)
{
    decode_state(c, c->fs, n, 1u, ebuf_slot(c, b), c->N, st, grid);
}

// e^n of every source from the FULL or AE store (decoded on the main stream into
// ebuf slot 0): pointer + per-source stride
// queue the decompression of window w into buffer b on `side`, after the main
// stream's reads of b enqueued so far
void time_issue(wv_ctx* c, TimeStore& T, int w, int b)
{
    hipStream_t s1 = side_stream(c, T.side);
    WV_HIP(hipEventRecord(T.ev_free[b], c->st));
    wait_event(s1, T.ev_free[b]);
    const int nvalid = std::min(TWIN, c->T - 1 - w * TWIN);
    const TimeGrid tg = ctx_time_grid(c);
    const int td = c->tm.begin(TM_DECODE, s1);
    ae_time_decode(c->ae, tg, tlat_slot(c, T, w), tmeta_slot(c, T, w), nvalid, twin_buf(c, T, b), s1);
    for (int s = 0; s < c->S && T.K > 0; ++s)
        time_exceptions_restore(tg, twin_buf(c, T, b), s, nvalid, T.K, texc_idx_slot(c, T, w, s),
                                texc_slot(c, T, w, s), s1);
    c->tm.end(td, s1);
    WV_HIP(hipEventRecord(T.ev_ready[b], s1));
    T.buf_w[b] = w;
}

// Level n of the time-compressed store T: its window is decompressed whole; at the
// first read of a window the next one in the direction of travel (dir = -1 reverse
// time, +1 forward) is queued into the other buffer
const float* time_e(wv_ctx* c, TimeStore& T, int n, int dir)
{
    const int w = (n - 1) / TWIN;
    int b = T.buf_w[0] == w ? 0 : (T.buf_w[1] == w ? 1 : -1);
    if (b < 0) {
        b = T.buf_w[0] == T.cur_w && T.cur_w >= 0 ? 1 : 0;
        time_issue(c, T, w, b);
    }
    if (T.cur_w != w) {
        wait_event(c->st, T.ev_ready[b]);
        T.cur_w = w;
        const int wn = w + dir;
        if (wn >= 0 && wn < c->nwin && T.buf_w[0] != wn && T.buf_w[1] != wn) time_issue(c, T, wn, 1 - b);
    }
    return twin_buf(c, T, b) + (long long)((n - 1) % TWIN) * c->S * c->N;
}

const float* load_e(wv_ctx* c, int n, long long* stride, int dir = -1)
{
    WV_REQUIRE(n >= 1 && n <= c->T - 1, WV_ESTATE, "stored state index out of range");
    *stride = c->N;
    if (c->mode == WV_STORE_FULL) return c->ehist + (long long)(n - 1) * c->S * c->N;
    if (is_time(c->mode)) return time_e(c, c->ts, n, dir);
    ensure_adj(c);  // owns the decode target ebuf
    decode_e(c, n, 0, c->st);
    return ebuf_slot(c, 0);
}

// Decode pipeline of the sweeps that read the AE store (adjoint, incremental
// forward): e^n is decoded on `side` into slot n % NEB up to NEB - 1 steps before
// the main stream's step reads it, in launches of at most `grid` work-groups (pipe_start;
// 0: one launch). pipe_start marks all slots free; pipe_issue
// queues the decode of e^n once the slot's last reader is done; pipe_take makes
// the main stream wait for it; pipe_release marks the slot read.
void pipe_start(wv_ctx* c, long long grid = 0)
{
    ensure_adj(c);
    c->pipe_grid = grid;
    for (int b = 0; b < NEB; ++b) WV_HIP(hipEventRecord(c->ev_free[b], c->st));
}
void pipe_issue(wv_ctx* c, int n, int b)
{
    hipStream_t s1 = side_stream(c, 0);
    wait_event(s1, c->ev_free[b]);
    decode_e(c, n, b, s1, c->pipe_grid);
    WV_HIP(hipEventRecord(c->ev_ready[b], s1));
}
const float* pipe_take(wv_ctx* c, int b)
{
    wait_event(c->st, c->ev_ready[b]);
    return ebuf_slot(c, b);
}
void pipe_release(wv_ctx* c, int b) { WV_HIP(hipEventRecord(c->ev_free[b], c->st)); }

float* other_work(wv_ctx* c, const float* cur) { return cur == c->work[0] ? c->work[1] : c->work[0]; }

// Accuracy guard: GUARD_CHECKS stored states spread evenly over the forward solve
// (every guard_every-th) and the last one are decoded as the reverse solves would
// read them (exception patches exact) and compared with the true e, while the true
// state is still in its buffer; the worst relative L2 error decides.
int guard_every(const wv_ctx* c) { return std::max(1, (c->T - 1 + GUARD_CHECKS - 1) / GUARD_CHECKS); }

// check slot of stored state j, or -1 when j is not checked
int guard_slot(const wv_ctx* c, int j)
{
    if (!is_ae(c->mode) || c->guard_tol <= 0.0 || !c->gres || j < 1 || j > c->T - 1) return -1;
    const int every = guard_every(c);
    if (j % every == 0 && j / every <= GUARD_CHECKS) return j / every - 1;
    return j == c->T - 1 ? GUARD_CHECKS : -1;
}

// queue the check of stored state j, whose true state is x: on the store's side
// stream after the store (rotation slot b; ev_stored[b] then also covers the check,
// so the buffer is not reused before it), or on the main stream (b < 0)
void guard_check(wv_ctx* c, int j, const float* x, int b)
{
    const int slot = guard_slot(c, j);
    if (slot < 0) return;
    hipStream_t st = c->st;
    if (b >= 0) {
        st = side_stream(c, 0);
        wait_event(st, c->ev_stored[b]);
    }
    decode_state(c, c->fs, j, 1u, c->gbuf, c->N, st);
    for (int s = 0; s < c->S; ++s)
        launch_err_norms(c->gbuf + s * c->N, x + s * 4 * c->N, c->N, c->gpart, c->nblk_red,
                         c->gres + 2 * ((long long)slot * c->S + s), st);
    if (b >= 0) WV_HIP(hipEventRecord(c->ev_stored[b], st));
}

// after the forward sweep (its side work joined): per source, the largest error norm
// of a checked state relative to the largest e norm among the checked states (an
// early state holds little of the wavefield, so its own norm would magnify the
// decoder's floor-level noise); the worst over sources decides
void run_guard(wv_ctx* c)
{
    c->degraded = false;
    c->guard_err = -1.0;
    if (!is_ae(c->mode) || c->guard_tol <= 0.0 || !c->gres || c->T < 2) return;
    std::vector<double> h(2 * (size_t)(GUARD_CHECKS + 1) * c->S, 0.0);
    WV_HIP(hipMemcpyAsync(h.data(), c->gres, sizeof(double) * h.size(), hipMemcpyDeviceToHost, c->st));
    WV_HIP(hipStreamSynchronize(c->st));
    double worst = 0.0;
    for (int s = 0; s < c->S; ++s) {
        double emax = 0.0, nmax = 0.0;
        for (int j = 1; j <= c->T - 1; ++j) {
            const int slot = guard_slot(c, j);
            if (slot < 0) continue;
            const double e2 = h[2 * ((size_t)slot * c->S + s)], n2 = h[2 * ((size_t)slot * c->S + s) + 1];
            emax = std::isnan(e2) || std::isnan(emax) ? NAN : std::max(emax, e2);
            nmax = std::max(nmax, n2);
        }
        const double r = nmax > 0.0 ? std::sqrt(emax / nmax) : std::sqrt(emax);
        worst = std::isnan(r) || std::isnan(worst) ? NAN : std::max(worst, r);
    }
    c->guard_err = worst;
    c->degraded = !(worst <= c->guard_tol);
}

// Forward sweep over T steps from the zero state. Records traces, fills the FULL/AE
// store, writes checkpoint snapshots (snap[n] = slot of x_n or 0), captures.
// Returns the buffer holding x_{T-1}; *last receives the one holding x_T.
float* forward_sweep(wv_ctx* c, float* traces, const std::vector<int>* snap, float* capture, int every,
                     float** last, const std::vector<int>* ecap_idx = nullptr, float* ecap = nullptr)
{
    c->delta_ok = false;  // incremental states belong to the previous forward history
    if (is_time(c->mode)) {
        // the window buffers are refilled: nothing queued on `side` may still use them
        join_side(c);
        c->ts.buf_w[0] = c->ts.buf_w[1] = -1;
        c->ts.cur_w = -1;
        c->tdelta_ok = false;
    }
    // autoencoder stores run beside the steps (x_j in work[j % 3])
    const bool ae = is_ae(c->mode) && c->mmpart && c->has_y;
    if (ae && !c->work[2]) c->work[2] = dev_alloc<float>(c->state_floats());
    launch_fill(c->work[0], c->state_floats(), 0.f, c->st);
    float* cur = c->work[0];
    float* prev = cur;
    const int ncap = (capture && every > 0) ? (c->T - 1) / every : 0;
    const long long mm_stride = (long long)c->S * c->P * c->H * 8;
    for (int n = 0; n < c->T; ++n) {
        const int j = n + 1;  // this step writes x_j
        const bool store = j <= c->T - 1;
        float* out;
        if (ae) {
            out = c->work[j % 3];
            // the buffer and min/max slot held x_{j-3}: its store must be done
            if (j - 3 >= 1 && j - 3 <= c->T - 1) wait_event(c->st, c->ev_stored[j % 3]);
        } else {
            out = (snap && (*snap)[j] > 0) ? c->slot_ptr((*snap)[j]) : other_work(c, cur);
        }
        float* mm = (ae && store) ? c->mmpart + (j % 3) * mm_stride : nullptr;
        // time compression: the step writes e^j straight into its window slot; the
        // buffer held window w - 2, whose compression must have read it
        float* ew = is_time(c->mode) && store ? time_slot(c, c->ts, j) : nullptr;
        fwd_step(c, cur, out, n, traces, mm, ew);
        if (store) {
            if (ae)
                store_state_async(c, j, out, mm);
            else
                store_state(c, c->fs, j, out);
            guard_check(c, j, out, ae ? j % 3 : -1);
        }
        if (ncap > 0 && j % every == 0 && j / every <= ncap)
            WV_HIP(hipMemcpyAsync(capture + (long long)(j / every - 1) * c->state_floats(), out,
                                  sizeof(float) * c->state_floats(), hipMemcpyDeviceToDevice, c->st));
        if (ecap_idx && (*ecap_idx)[j] >= 0)
            for (int s = 0; s < c->S; ++s)
                launch_copy(ecap + ((long long)(*ecap_idx)[j] * c->S + s) * c->N, out + s * 4 * c->N, c->N, c->st);
        prev = cur;
        cur = out;
    }
    if (ae) join_side(c);
    c->last_fwd_steps = c->T;
    if (last) *last = cur;
    return prev;
}

// Reverse sweep. e^k comes from the FULL/AE store, or (checkpointing) from the
// action list starting at `first` with x_{T-1} in `xtm1`.
void reverse_sweep(wv_ctx* c, const float* resid, const std::vector<RevAction>* acts, size_t first,
                   float* xtm1)
{
    ensure_adj(c);
    c->ts.cur_w = -1;
    launch_fill(c->adj[0], c->state_floats(), 0.f, c->st);
    launch_fill(c->acc, 2 * c->N * c->S, 0.f, c->st);
    float* ain = c->adj[0];
    float* aout = c->adj[1];
    long long done = 0;  // adjoint steps of this sweep so far
    auto adjoint_k = [&](int k, const float* ek, long long stride) {
        adj_step(c, ain, aout, k, resid, ek, stride, acc_phase(done++, k));
        std::swap(ain, aout);
    };
    if (!acts && is_ae(c->mode)) {
        // e^{k-2} is decoded beside the adjoint steps k and k - 1, in launches of at most
        // REV_DEC_GRID work-groups
        pipe_start(c, REV_DEC_GRID);
        for (int n = c->T - 1; n >= std::max(1, c->T - NEB + 1); --n) pipe_issue(c, n, n % NEB);
        for (int k = c->T - 1; k >= 1; --k) {
            if (k - NEB + 1 >= 1) pipe_issue(c, k - NEB + 1, (k - NEB + 1) % NEB);
            adjoint_k(k, pipe_take(c, k % NEB), c->N);
            pipe_release(c, k % NEB);
        }
        return;
    }
    if (!acts) {
        for (int k = c->T - 1; k >= 1; --k) {
            long long stride;
            const float* e = load_e(c, k, &stride);
            adjoint_k(k, e, stride);
        }
        return;
    }
    float* cur = xtm1;
    long long extra = 0;
    for (size_t q = first; q < acts->size(); ++q) {
        const RevAction& A = (*acts)[q];
        if (A.kind == 3) {
            if (A.a >= 1) adjoint_k(A.a, cur, 4 * c->N);
        } else if (A.kind == 2) {
            if (A.b == 0) {
                launch_fill(c->work[0], c->state_floats(), 0.f, c->st);
                cur = c->work[0];
            } else {
                cur = c->slot_ptr(A.b);
            }
        } else if (A.kind == 0) {
            const bool to_slot = q + 1 < acts->size() && (*acts)[q + 1].kind == 1;
            for (int t = 0; t < A.b; ++t) {
                float* out = (to_slot && t == A.b - 1) ? c->slot_ptr((*acts)[q + 1].b) : other_work(c, cur);
                fwd_step(c, cur, out, A.a + t, nullptr);
                cur = out;
            }
            extra += A.b;
        }
    }
    c->last_fwd_steps += extra;
}

void finish_grad(wv_ctx* c, const float* cdev, float* g)
{
    launch_grad_finish(cdev, c->acc, c->N, c->S, -2.0 * c->g.dt / c->g.dx, g, c->st);
}

// gradient with checkpointing regardless of the store mode (also the fallback)
double gradient_checkpoint(wv_ctx* c, const float* cdev, const float* d_obs, double sigma, float* g,
                           int nslots)
{
    if (!c->slots || c->nslots != nslots) alloc_slots(c, nslots);
    long long fsteps = 0;
    const auto acts = revolve_schedule(c->T, c->nslots, &fsteps);
    size_t first = 0;
    const auto snap = sweep_snapshots(acts, c->T, &first);
    float* last = nullptr;
    const int saved = c->mode;
    c->mode = WV_STORE_CHECKPOINT;
    float* xtm1 = forward_sweep(c, c->traces, &snap, nullptr, 0, &last);
    c->mode = saved;
    const long long n = (long long)c->S * c->T * c->R;
    launch_misfit(c->traces, d_obs, c->resid, n, c->g.dt / (sigma * sigma), c->g.dt / (2 * sigma * sigma),
                  c->partial, c->nblk_red, c->dscal, c->st);
    double J;
    WV_HIP(hipMemcpyAsync(&J, c->dscal, sizeof(double), hipMemcpyDeviceToHost, c->st));
    reverse_sweep(c, c->resid, &acts, first, xtm1);
    finish_grad(c, cdev, g);
    WV_HIP(hipStreamSynchronize(c->st));
    return J;
}

// Side streams shared by every context on a device: one set of three per process
// and device, created by the first wv_create on the device and kept until the
// process ends. With a context's main stream they make four streams, so under HIP's
// default of four hardware queues per process each of them has a queue of its own
// however many contexts exist (per-context side streams gave a stream-to-queue
// mapping that depended on how many contexts had been created before). Work of
// different contexts on a shared side stream runs in order; every sweep ends with
// its main stream waiting for the side streams, so contexts used one after the
// other never wait for each other's side work.
constexpr int SIDE_MAX_DEVICES = 64;
std::mutex g_side_mu;
hipStream_t g_side[SIDE_MAX_DEVICES][3] = {};

void shared_side(wv_ctx* c)
{
    int dev = -1;
    WV_HIP(hipGetDevice(&dev));
    WV_REQUIRE(dev >= 0 && dev < SIDE_MAX_DEVICES, WV_EDEVICE, "device ordinal beyond the side-stream table");
    std::lock_guard<std::mutex> lock(g_side_mu);
    if (!g_side[dev][0]) {
        // all three or none: a failed creation leaves the table empty for the next context
        hipStream_t made[3] = {};
        for (int q = 0; q < 3; ++q) {
            const hipError_t e = hipStreamCreateWithFlags(&made[q], hipStreamNonBlocking);
            if (e != hipSuccess) {
                for (int r = 0; r < q; ++r) (void)hipStreamDestroy(made[r]);
                WV_HIP(e);
            }
        }
        for (int q = 0; q < 3; ++q) g_side[dev][q] = made[q];
    }
    c->side = g_side[dev][0];
    c->side2 = g_side[dev][1];
    c->side3 = g_side[dev][2];
}

}  // namespace

// ====================================================================================
extern "C" {

int wv_create(const wv_grid* grid, const int32_t* h_src, const int32_t* h_rec, void* stream, wv_ctx** out)
{
    return guarded([&]() -> int {
        WV_REQUIRE(grid && out, WV_EINVAL, "null argument");
        const wv_grid g = *grid;
        WV_REQUIRE(g.nz >= 2 && g.ny >= 1 && g.nx >= 2, WV_EINVAL, "grid too small");
        WV_REQUIRE((long long)g.ny * g.nx < (1LL << 30), WV_EINVAL, "a (y, x) plane must hold fewer than 2^30 cells");
        WV_REQUIRE(g.dx > 0 && g.dt > 0 && g.nt >= 1, WV_EINVAL, "dx, dt must be > 0 and nt >= 1");
        WV_REQUIRE(g.sponge >= 0 && g.nsrc >= 1 && g.nrec >= 0, WV_EINVAL, "bad sponge/nsrc/nrec");
        WV_REQUIRE(g.sponge == 0 || g.c_ref > 0, WV_EINVAL, "c_ref must be > 0 with an absorbing layer");
        WV_REQUIRE(h_src && (g.nrec == 0 || h_rec), WV_EINVAL, "null source/receiver list");
        std::unique_ptr<wv_ctx> c(new wv_ctx());
        c->g = g;
        c->has_y = g.ny > 1;
        c->N = (long long)g.nz * g.ny * g.nx;
        c->S = g.nsrc;
        c->T = g.nt;
        c->R = g.nrec;
        c->st = (hipStream_t)stream;
        std::vector<int> src(h_src, h_src + 3 * g.nsrc), rec;
        if (g.nrec) rec.assign(h_rec, h_rec + 3 * g.nrec);
        auto check_pts = [&](const std::vector<int>& v, const char* what) {
            for (size_t q = 0; q < v.size(); q += 3) {
                WV_REQUIRE(v[q] >= 0 && v[q] < g.nz && v[q + 1] >= 0 && v[q + 1] < g.ny && v[q + 2] >= 0 &&
                               v[q + 2] < g.nx,
                           WV_EINVAL, std::string(what) + " index outside the grid");
            }
        };
        check_pts(src, "source");
        check_pts(rec, "receiver");
        build_tables(c.get());
        c->tl = make_tiling(g.nz, g.ny, g.nx, rec);
        c->src_kji = dev_alloc<int>(src.size());
        WV_HIP(hipMemcpy(c->src_kji, src.data(), sizeof(int) * src.size(), hipMemcpyHostToDevice));
        const float one = 1.0f;
        c->src_w = dev_alloc<float>(1);
        WV_HIP(hipMemcpy(c->src_w, &one, sizeof(float), hipMemcpyHostToDevice));
        c->m = dev_alloc<float>(c->N);
        c->c_last = dev_alloc<float>(c->N);
        c->wavelet = dev_alloc<float>((size_t)c->S * c->T);
        c->work[0] = dev_alloc<float>(c->state_floats());
        c->work[1] = dev_alloc<float>(c->state_floats());
        const size_t ntr = (size_t)c->S * c->T * std::max(c->R, 1);
        c->traces = dev_alloc<float>(ntr);
        c->resid = dev_alloc<float>(ntr);
        c->dtr = dev_alloc<float>(ntr);
        c->dresid = dev_alloc<float>(ntr);
        shared_side(c.get());
        for (int b = 0; b < 3; ++b) {
            WV_HIP(hipEventCreateWithFlags(&c->ev_step[b], SYNC_EVENT_FLAGS));
            WV_HIP(hipEventCreateWithFlags(&c->ev_enc[b], SYNC_EVENT_FLAGS));
            WV_HIP(hipEventCreateWithFlags(&c->ev_stored[b], SYNC_EVENT_FLAGS));
        }
        for (int b = 0; b < NEB; ++b) {
            WV_HIP(hipEventCreateWithFlags(&c->ev_ready[b], SYNC_EVENT_FLAGS));
            WV_HIP(hipEventCreateWithFlags(&c->ev_free[b], SYNC_EVENT_FLAGS));
        }
        WV_HIP(hipEventCreateWithFlags(&c->ev_join, SYNC_EVENT_FLAGS));
        for (int b = 0; b < 3; ++b)
            for (hipEvent_t* e : {&c->ev_dstep[b], &c->ev_denc[b], &c->ev_dstored[b]})
                WV_HIP(hipEventCreateWithFlags(e, SYNC_EVENT_FLAGS));
        c->tds.side = 1;
        for (TimeStore* T : {&c->ts, &c->tds})
            for (int b = 0; b < 2; ++b)
                for (hipEvent_t* e : {&T->ev_fill[b], &T->ev_enc[b], &T->ev_ready[b], &T->ev_free[b]})
                    WV_HIP(hipEventCreateWithFlags(e, SYNC_EVENT_FLAGS));
        c->partial = dev_alloc<double>(3 * (size_t)c->nblk_red);
        c->dscal = dev_alloc<double>(8);
        c->dflag = dev_alloc<int>(1);
        *out = c.release();
        return WV_OK;
    });
}

int wv_destroy(wv_ctx* c)
{
    if (!c) return WV_OK;
    (void)hipStreamSynchronize(c->st);
    if (c->side) (void)hipStreamSynchronize(c->side);
    if (c->side2) (void)hipStreamSynchronize(c->side2);
    if (c->side3) (void)hipStreamSynchronize(c->side3);
    c->tm.destroy();
    free_store(c);
    free_tiling(c->tl);
    for (hipEvent_t e : {c->ev_step[0], c->ev_step[1], c->ev_step[2], c->ev_enc[0], c->ev_enc[1], c->ev_enc[2],
                         c->ev_stored[0], c->ev_stored[1], c->ev_stored[2], c->ev_join, c->ev_dstep[0],
                         c->ev_dstep[1], c->ev_dstep[2], c->ev_denc[0], c->ev_denc[1], c->ev_denc[2],
                         c->ev_dstored[0], c->ev_dstored[1], c->ev_dstored[2]})
        if (e) (void)hipEventDestroy(e);
    for (int b = 0; b < NEB; ++b) {
        if (c->ev_ready[b]) (void)hipEventDestroy(c->ev_ready[b]);
        if (c->ev_free[b]) (void)hipEventDestroy(c->ev_free[b]);
    }
    for (TimeStore* T : {&c->ts, &c->tds})
        for (int b = 0; b < 2; ++b)
            for (hipEvent_t e : {T->ev_fill[b], T->ev_enc[b], T->ev_ready[b], T->ev_free[b]})
                if (e) (void)hipEventDestroy(e);
    dev_free(c->tab);
    dev_free(c->src_kji);
    dev_free(c->src_w);
    for (float** p : {&c->m, &c->c_last, &c->wavelet, &c->work[0], &c->work[1], &c->adj[0], &c->adj[1],
                      &c->incb[0], &c->incb[1], &c->incb[2], &c->acc, &c->blk, &c->ebuf, &c->dm, &c->traces,
                      &c->resid, &c->dtr, &c->dresid, &c->adj2[0], &c->adj2[1], &c->dacc, &c->dblk, &c->qbuf, &c->dehist, &c->dbuf,
                      &c->prior_c0, &c->prior_w, &c->nvec, &c->pvec})
        dev_free(*p);
    dev_free(c->partial);
    dev_free(c->dscal);
    dev_free(c->dflag);
    delete c;
    return WV_OK;
}

namespace {
// the allocations and checks of one storage mode on a context whose store is free
void set_storage_mode(wv_ctx* c, int mode, int32_t n_checkpoints, ae_net* ae, int64_t mem_budget_bytes,
                      int fallback_policy, double guard_tol)
{
    c->mode = mode;
    c->budget = mem_budget_bytes;
    c->guard_tol = guard_tol;
    c->fallback = fallback_policy;
    c->ae = ae;
    c->nslots = n_checkpoints;
    c->degraded = false;
    c->have_grad = false;
    const int T = c->T;
    if (mode == WV_STORE_FULL) {
        const long long n = (long long)std::max(T - 1, 1) * c->S * c->N;
        WV_REQUIRE(c->budget <= 0 || n * 4 <= c->budget, WV_ENOMEM, "full history exceeds the memory budget");
        c->ehist = dev_alloc<float>(n);
        c->store_bytes = n * 4;
    } else if (mode == WV_STORE_CHECKPOINT) {
        alloc_slots(c, n_checkpoints);
        c->store_bytes = (int64_t)(n_checkpoints - 1) * c->state_floats() * 4;
    } else if (is_time(mode)) {
        WV_REQUIRE(ae, WV_EINVAL, "time compression needs an ae_net");
        WV_REQUIRE(ae_input_dim(ae) == TWIN * 64, WV_EINVAL, "time compression needs an input width of 2048");
        WV_REQUIRE(c->has_y && c->g.nz % 4 == 0 && c->g.ny % 4 == 0 && c->g.nx % 4 == 0, WV_ESHAPE,
                   "time compression needs a 3D grid divisible into 4^3 blocks");
        WV_REQUIRE(fallback_policy == WV_FALLBACK_NONE && guard_tol <= 0.0, WV_EINVAL,
                   "the accuracy guard and its fallback apply to the space modes");
        c->TB = ctx_time_grid(c).B;
        c->nwin = (std::max(T - 1, 1) + TWIN - 1) / TWIN;
        c->tlat_dim = ae_latent_dim(ae);
        const int K = (int)std::min<long long>(c->exc_req, c->TB);
        const long long bytes = timestore_bytes(c, K);
        WV_REQUIRE(c->budget <= 0 || bytes <= c->budget, WV_ENOMEM, "latent store exceeds the memory budget");
        alloc_timestore(c, c->ts, K);
        c->store_bytes = bytes;
    } else if (is_ae(mode)) {
        WV_REQUIRE(ae, WV_EINVAL, "autoencoder storage needs an ae_net");
        WV_REQUIRE(c->has_y && c->g.nz % 8 == 0 && c->g.ny % 8 == 0 && c->g.nx % 8 == 0, WV_ESHAPE,
                   "autoencoder storage needs a 3D grid divisible into 8^3 patches");
        const PatchGrid pg = patch_grid(c->g.nz, c->g.ny, c->g.nx);
        c->P = pg.P;
        c->lat_bytes = ae_latent_bytes_per_patch(ae, ae_fmt(mode));
        c->m16 = c->meta_req == 16;
        WV_REQUIRE(!c->m16 || (ae_input_dim(ae) == 2048 && ae_latent_dim(ae) == 32), WV_EINVAL,
                   "16-bit metadata needs the fused network shape (hidden 512, latent 32)");
        const int K = (int)std::min<long long>(c->exc_req, c->P);
        c->nbd = (int)((c->P + DEC_BM - 1) / DEC_BM);
        const long long bytes = latstore_bytes(c, mode, K);
        WV_REQUIRE(c->budget <= 0 || bytes <= c->budget, WV_ENOMEM, "latent store exceeds the memory budget");
        alloc_latstore(c, c->fs, mode, K);
        c->K = K;
        c->H = 8 / c->tl.by;
        c->mmpart = dev_alloc<float>((size_t)3 * c->S * c->P * c->H * 8);
        if (guard_tol > 0.0) {
            c->gbuf = dev_alloc<float>((size_t)c->S * c->N);
            c->gpart = dev_alloc<double>(3 * (size_t)c->nblk_red);
            c->gres = dev_alloc<double>(2 * (size_t)(GUARD_CHECKS + 1) * c->S);
        }
        c->store_bytes = bytes;
        if (fallback_policy == WV_FALLBACK_CHECKPOINT)
            WV_REQUIRE(n_checkpoints >= 1, WV_EINVAL, "fallback needs n_checkpoints >= 1");
    }
}
}  // namespace

int wv_set_storage(wv_ctx* c, int mode, int32_t n_checkpoints, ae_net* ae, int64_t mem_budget_bytes,
                   double guard_tol, int fallback_policy)
{
    return guarded([&]() -> int {
        WV_REQUIRE(c, WV_EINVAL, "null context");
        WV_REQUIRE(mode >= WV_STORE_NONE && mode <= WV_STORE_AE_TIME, WV_EINVAL, "unknown storage mode");
        WV_REQUIRE(fallback_policy == WV_FALLBACK_NONE || fallback_policy == WV_FALLBACK_CHECKPOINT, WV_EINVAL,
                   "unknown fallback policy");
        WV_HIP(hipStreamSynchronize(c->st));
        free_store(c);
        dev_free(c->slots);
        try {
            set_storage_mode(c, mode, n_checkpoints, ae, mem_budget_bytes, fallback_policy, guard_tol);
        } catch (...) {
            // a rejected mode leaves no partial store behind: the context stores nothing, so
            // the solves that need a history fail with WV_ESTATE until a mode is set
            free_store(c);
            c->mode = WV_STORE_NONE;
            c->ae = nullptr;
            throw;
        }
        return WV_OK;
    });
}

int wv_set_source_stencil(wv_ctx* c, int32_t radius, const float* h_weights)
{
    return guarded([&]() -> int {
        WV_REQUIRE(c && h_weights, WV_EINVAL, "null argument");
        WV_REQUIRE(radius >= 0 && radius <= 64, WV_EINVAL, "source radius must be in [0, 64]");
        const long long w = 2LL * radius + 1;
        const long long n = c->has_y ? w * w * w : w * w;
        for (long long q = 0; q < n; ++q)
            WV_REQUIRE(std::isfinite(h_weights[q]), WV_EINVAL, "source weights must be finite");
        WV_HIP(hipStreamSynchronize(c->st));
        // the new weights are in place before the old ones go, so a failed call keeps the
        // previous stencil whole
        float* wd = dev_alloc<float>(n);
        const hipError_t e = hipMemcpy(wd, h_weights, sizeof(float) * n, hipMemcpyHostToDevice);
        if (e != hipSuccess) dev_free(wd);
        WV_HIP(e);
        dev_free(c->src_w);
        c->src_w = wd;
        c->src_radius = radius;
        c->store_ok = false;
        c->have_grad = false;
        return WV_OK;
    });
}

int wv_set_ae_exceptions(wv_ctx* c, int32_t k_per_step)
{
    if (!c || k_per_step < 0) {
        set_error("bad argument");
        return WV_EINVAL;
    }
    c->exc_req = k_per_step;
    return WV_OK;
}

int wv_set_ae_metadata(wv_ctx* c, int32_t bits)
{
    if (!c || (bits != 32 && bits != 16)) {
        set_error("metadata bits must be 32 or 16");
        return WV_EINVAL;
    }
    c->meta_req = bits;
    return WV_OK;
}

int wv_set_delta_storage(wv_ctx* c, int32_t enable)
{
    return guarded([&]() -> int {
        WV_REQUIRE(c && (enable == 0 || enable == 1), WV_EINVAL, "bad argument");
        WV_HIP(hipStreamSynchronize(c->st));
        c->store_delta = enable == 1;
        if (!c->store_delta) {
            free_latstore(c->ds);
            free_timestore(c->tds);
            c->delta_bytes = 0;
            c->delta_ok = false;
            c->tdelta_ok = false;
        }
        return WV_OK;
    });
}

int wv_decode_delta(wv_ctx* c, int32_t n, uint32_t field_mask, float* state)
{
    return guarded([&]() -> int {
        WV_REQUIRE(c && state && field_mask != 0 && field_mask < 16, WV_EINVAL, "bad argument");
        WV_REQUIRE((is_ae(c->mode) && c->delta_ok) || (is_time(c->mode) && c->tdelta_ok), WV_ESTATE,
                   "no incremental states stored");
        if (is_time(c->mode)) {
            WV_REQUIRE(field_mask == 1u, WV_EINVAL, "the time store holds e only (field mask 1)");
            WV_REQUIRE(n >= 1 && n <= c->T - 1, WV_EINVAL, "level outside [1, T-1]");
            const float* de = time_e(c, c->tds, n, -1);
            for (int s = 0; s < c->S; ++s) launch_copy(state + (long long)s * 4 * c->N, de + s * c->N, c->N, c->st);
            return WV_OK;
        }
        decode_state(c, c->ds, n, field_mask, state, 4 * c->N, c->st);
        return WV_OK;
    });
}

int wv_storage_bytes(const wv_ctx* c, int64_t* h_bytes)
{
    if (!c || !h_bytes) {
        set_error("null argument");
        return WV_EINVAL;
    }
    *h_bytes = c->store_bytes + c->delta_bytes;
    return WV_OK;
}

namespace {

// forward solve filling the store of the current mode, with optional captures:
// whole states every `every` steps, and e of the levels marked in ecap_idx
void forward_solve(wv_ctx* c, const float* cdev, const float* wavelet, float* traces, float* final_state,
                   float* capture, int every, const std::vector<int>* ecap_idx, float* ecap);

}  // namespace

int wave_forward_e(wv_ctx* c, const float* cdev, const float* wavelet, const int32_t* h_steps, int32_t nsteps,
                   float* e_out)
{
    return guarded([&]() -> int {
        WV_REQUIRE(c && cdev && wavelet && nsteps >= 0 && (nsteps == 0 || (h_steps && e_out)), WV_EINVAL,
                   "null argument or negative count");
        std::vector<int> idx((size_t)c->T + 1, -1);
        for (int q = 0; q < nsteps; ++q) {
            const int n = h_steps[q];
            WV_REQUIRE(n >= 1 && n <= c->T, WV_EINVAL, "capture level outside [1, T]");
            WV_REQUIRE(idx[n] < 0, WV_EINVAL, "capture level listed twice");
            idx[n] = q;
        }
        forward_solve(c, cdev, wavelet, nullptr, nullptr, nullptr, 0, &idx, e_out);
        return WV_OK;
    });
}

int wv_load_e(wv_ctx* c, int32_t n, float* out)
{
    return guarded([&]() -> int {
        WV_REQUIRE(c && out, WV_EINVAL, "null argument");
        WV_REQUIRE(c->store_ok && (c->mode == WV_STORE_FULL || is_ae(c->mode) || is_time(c->mode)), WV_ESTATE,
                   "no stored forward history (full, autoencoder or time-compressed)");
        WV_REQUIRE(n >= 1 && n <= c->T - 1, WV_EINVAL, "level outside [1, T-1]");
        long long stride;
        const float* e = load_e(c, n, &stride);
        for (int s = 0; s < c->S; ++s) launch_copy(out + (long long)s * c->N, e + s * stride, c->N, c->st);
        WV_HIP(hipStreamSynchronize(c->st));
        return WV_OK;
    });
}

int wave_forward(wv_ctx* c, const float* cdev, const float* wavelet, float* traces, float* final_state,
                 float* capture, int32_t capture_every)
{
    return guarded([&]() -> int {
        WV_REQUIRE(c && cdev && wavelet, WV_EINVAL, "null argument");
        WV_REQUIRE(!capture || capture_every >= 1, WV_EINVAL, "capture_every must be >= 1");
        forward_solve(c, cdev, wavelet, traces, final_state, capture, capture_every, nullptr, nullptr);
        return WV_OK;
    });
}

namespace {

void forward_solve(wv_ctx* c, const float* cdev, const float* wavelet, float* traces, float* final_state,
               float* capture, int capture_every, const std::vector<int>* ecap_idx, float* ecap)
{
    prepare_model(c, cdev, wavelet);
    c->store_ok = false;
    c->have_grad = false;
    float* last = nullptr;
    float* xtm1;
    std::vector<RevAction> acts;
    if (c->mode == WV_STORE_CHECKPOINT) {
        long long fs = 0;
        acts = revolve_schedule(c->T, c->nslots, &fs);
        size_t first = 0;
        const auto snap = sweep_snapshots(acts, c->T, &first);
        xtm1 = forward_sweep(c, c->traces, &snap, capture, capture_every, &last, ecap_idx, ecap);
    } else {
        xtm1 = forward_sweep(c, c->traces, nullptr, capture, capture_every, &last, ecap_idx, ecap);
    }
    if (traces)
        WV_HIP(hipMemcpyAsync(traces, c->traces, sizeof(float) * c->S * c->T * c->R, hipMemcpyDeviceToDevice,
                              c->st));
    if (final_state)
        WV_HIP(hipMemcpyAsync(final_state, last, sizeof(float) * c->state_floats(), hipMemcpyDeviceToDevice,
                              c->st));
    run_guard(c);
    c->store_ok = c->mode != WV_STORE_NONE;
}

}  // namespace

int wave_adjoint(wv_ctx* c, const float* cdev, const float* residual, float* g)
{
    return guarded([&]() -> int {
        WV_REQUIRE(c && cdev && residual && g, WV_EINVAL, "null argument");
        WV_REQUIRE(c->store_ok, WV_ESTATE, "no forward history stored (call wave_forward first)");
        if (c->mode == WV_STORE_CHECKPOINT) {
            // the snapshots of the last sweep are intact; re-run the forward to place x_{T-1}
            long long fs = 0;
            const auto acts = revolve_schedule(c->T, c->nslots, &fs);
            size_t first = 0;
            const auto snap = sweep_snapshots(acts, c->T, &first);
            float* last = nullptr;
            float* xtm1 = forward_sweep(c, c->dtr, &snap, nullptr, 0, &last);
            reverse_sweep(c, residual, &acts, first, xtm1);
            c->store_ok = false;
        } else {
            reverse_sweep(c, residual, nullptr, 0, nullptr);
        }
        finish_grad(c, cdev, g);
        return WV_OK;
    });
}

int gradient(wv_ctx* c, const float* cdev, const float* wavelet, const float* d_obs, double sigma, float* g,
             double* h_misfit)
{
    return guarded([&]() -> int {
        WV_REQUIRE(c && cdev && wavelet && d_obs && g, WV_EINVAL, "null argument");
        WV_REQUIRE(sigma > 0 && std::isfinite(sigma), WV_EINVAL, "sigma must be positive");
        WV_REQUIRE(c->mode != WV_STORE_NONE, WV_ESTATE, "gradient needs a storage mode");
        c->sigma = sigma;
        int status = WV_OK;
        double J = 0.0;
        if (c->mode == WV_STORE_CHECKPOINT) {
            prepare_model(c, cdev, wavelet);
            J = gradient_checkpoint(c, cdev, d_obs, sigma, g, c->nslots);
            c->store_ok = false;
        } else {
            prepare_model(c, cdev, wavelet);
            float* last = nullptr;
            float* xtm1 = forward_sweep(c, c->traces, nullptr, nullptr, 0, &last);
            run_guard(c);
            c->store_ok = true;
            if (c->degraded && c->fallback == WV_FALLBACK_CHECKPOINT) {
                J = gradient_checkpoint(c, cdev, d_obs, sigma, g, std::max(c->nslots, 2));
                status = WV_OK_FALLBACK;
            } else {
                const long long n = (long long)c->S * c->T * c->R;
                launch_misfit(c->traces, d_obs, c->resid, n, c->g.dt / (sigma * sigma),
                              c->g.dt / (2 * sigma * sigma), c->partial, c->nblk_red, c->dscal, c->st);
                WV_HIP(hipMemcpyAsync(&J, c->dscal, sizeof(double), hipMemcpyDeviceToHost, c->st));
                reverse_sweep(c, c->resid, nullptr, 0, nullptr);
                finish_grad(c, cdev, g);
                WV_HIP(hipStreamSynchronize(c->st));
            }
        }
        c->have_grad = true;
        if (h_misfit) *h_misfit = J;
        return status;
    });
}

namespace {

// incremental forward into c->dtr; CHECKPOINT runs the companion forward and
// places snapshots for a following reverse sweep (returns x_{T-1} there).
// keep_de: the full-Newton product needs de^n later (FULL: de history; AE: the
// incremental latent store; time compression: the incremental time store)
float* inc_forward_sweep(wv_ctx* c, const float* cdev, const float* dc, const std::vector<int>* snap,
                         bool keep_de = false)
{
    ensure_inc(c);
    ensure_adj(c);
    c->ts.cur_w = -1;
    launch_dm(cdev, dc, c->dm, c->N, c->st);
    launch_fill(c->incb[0], c->state_floats(), 0.f, c->st);
    const bool pipe = !snap && is_ae(c->mode);
    const bool keep_full = keep_de && !snap && c->mode == WV_STORE_FULL;
    if (keep_full && !c->dehist) c->dehist = dev_alloc<float>((size_t)std::max(c->T - 1, 1) * c->S * c->N);
    // optional AE store of the incremental states dx_1 .. dx_{T-1} (same network and format)
    const bool keep_delta = pipe && (c->store_delta || keep_de);
    c->delta_ok = false;
    if (keep_delta && !c->ds.lat) {
        const long long bytes = latstore_bytes(c, c->mode, c->K);
        WV_REQUIRE(c->budget <= 0 || c->store_bytes + bytes <= c->budget, WV_ENOMEM,
                   "incremental latent store exceeds the memory budget");
        alloc_latstore(c, c->ds, c->mode, c->K);
        c->delta_bytes = bytes;
    }
    // time store of de^1 .. de^{T-1}: same network, block layout and exception count
    const bool keep_time = (keep_de || c->store_delta) && !snap && is_time(c->mode);
    c->tdelta_ok = false;
    if (keep_time) {
        if (!c->tds.lat) {
            const long long bytes = timestore_bytes(c, c->ts.K);
            WV_REQUIRE(c->budget <= 0 || c->store_bytes + bytes <= c->budget, WV_ENOMEM,
                       "incremental latent store exceeds the memory budget");
            alloc_timestore(c, c->tds, c->ts.K);
            c->delta_bytes = bytes;
        }
        // its window buffers are refilled: nothing queued on the side streams may still use them
        join_side(c);
        c->tds.buf_w[0] = c->tds.buf_w[1] = -1;
        c->tds.cur_w = -1;
    }
    // The incremental latent store runs beside the steps (and the decodes of e):
    // dx_j is encoded on `se` and its exception patches selected and copied on `sx`.
    // The states then rotate through three buffers, so the store of dx_j may take
    // until the step that overwrites it, two steps later.
    const hipStream_t se = side_stream(c, 2), sx = side_stream(c, 1);
    const bool dasync = keep_delta && (se != c->st || sx != c->st);
    if (dasync && !c->incb[2]) c->incb[2] = dev_alloc<float>(c->state_floats());
    // the step writing dx_j also writes its per-patch (min, max) partials into slot
    // j % 3 of the forward store's partial buffer, for the encode
    const bool dmm = keep_delta && c->mmpart && c->has_y;
    const long long mm_stride = (long long)c->S * c->P * c->H * 8;
    if (pipe) pipe_start(c);
    launch_fill(ebuf_slot(c, 0), c->N * c->S, 0.f, c->st);  // e^0 = 0
    float* din = c->incb[0];
    float* dout = c->incb[1];
    const bool ckpt = snap != nullptr;
    float* cur = nullptr;
    float* prev = nullptr;
    if (ckpt) {
        launch_fill(c->work[0], c->state_floats(), 0.f, c->st);
        cur = c->work[0];
    }
    for (int n = 0; n < c->T; ++n) {
        const float* en;
        long long stride;
        if (ckpt) {
            en = cur;
            stride = 4 * c->N;
        } else if (pipe) {
            // e^{n+2} is decoded beside the steps n and n + 1; slot n % NEB holds e^n
            if (n == 0)
                for (int q = 1; q < NEB - 1 && q <= c->T - 1; ++q) pipe_issue(c, q, q % NEB);
            if (n + NEB - 1 <= c->T - 1) pipe_issue(c, n + NEB - 1, (n + NEB - 1) % NEB);
            en = n == 0 ? ebuf_slot(c, 0) : pipe_take(c, n % NEB);
            stride = c->N;
        } else if (n == 0) {
            en = ebuf_slot(c, 0);  // e^0 = 0
            stride = c->N;
        } else {
            en = load_e(c, n, &stride, +1);
        }
        float* dew = keep_time && n + 1 <= c->T - 1 ? time_slot(c, c->tds, n + 1) : nullptr;
        if (dasync) {
            din = c->incb[n % 3];
            dout = c->incb[(n + 1) % 3];
            if (n >= 3) wait_event(c->st, c->ev_dstored[(n - 2) % 3]);  // dout held dx_{n-2}
        }
        float* dmmp = dmm && n + 1 <= c->T - 1 ? c->mmpart + ((n + 1) % 3) * mm_stride : nullptr;
        inc_step(c, din, dout, n, en, stride, c->dtr, dew, dmmp);
        if (pipe) pipe_release(c, n % NEB);
        std::swap(din, dout);
        if (keep_time) time_store_level(c, c->tds, n + 1);
        if (keep_delta && n + 1 <= c->T - 1) {
            const int j = n + 1, b = j % 3;
            if (dasync) {
                WV_HIP(hipEventRecord(c->ev_dstep[b], c->st));
                wait_event(se, c->ev_dstep[b]);
                encode_state_into(c, c->ds, j, din, se, dmmp);
                WV_HIP(hipEventRecord(c->ev_denc[b], se));
                wait_event(sx, c->ev_denc[b]);
                exceptions_into(c, c->ds, j, din, sx);
                WV_HIP(hipEventRecord(c->ev_dstored[b], sx));
            } else {
                store_state(c, c->ds, j, din, c->st, dmmp);
            }
        }
        if (keep_full && n + 1 <= c->T - 1)
            for (int s = 0; s < c->S; ++s)
                WV_HIP(hipMemcpyAsync(c->dehist + ((long long)n * c->S + s) * c->N, din + s * 4 * c->N,
                                      sizeof(float) * c->N, hipMemcpyDeviceToDevice, c->st));
        if (ckpt) {
            float* out = (*snap)[n + 1] > 0 ? c->slot_ptr((*snap)[n + 1]) : other_work(c, cur);
            fwd_step(c, cur, out, n, nullptr);
            prev = cur;
            cur = out;
        }
    }
    if (ckpt) c->last_fwd_steps = c->T;
    if (dasync) join_side(c);  // the reverse sweep decodes the incremental store on the main stream
    if (keep_delta) c->delta_ok = true;
    if (keep_time) c->tdelta_ok = true;
    return prev;
}

}  // namespace

int wave_inc_forward(wv_ctx* c, const float* cdev, const float* dc, float* dtraces)
{
    return guarded([&]() -> int {
        WV_REQUIRE(c && cdev && dc && dtraces, WV_EINVAL, "null argument");
        WV_REQUIRE(c->mode == WV_STORE_FULL || is_ae(c->mode) || is_time(c->mode) || c->mode == WV_STORE_CHECKPOINT,
                   WV_ESTATE, "incremental forward needs a storage mode");
        if (c->mode == WV_STORE_CHECKPOINT) {
            prepare_model(c, cdev, nullptr);
            std::vector<int> snap(c->T + 1, 0);
            inc_forward_sweep(c, cdev, dc, &snap);
        } else {
            WV_REQUIRE(c->store_ok, WV_ESTATE, "no forward history stored");
            inc_forward_sweep(c, cdev, dc, nullptr);
        }
        WV_HIP(hipMemcpyAsync(dtraces, c->dtr, sizeof(float) * c->S * c->T * c->R, hipMemcpyDeviceToDevice, c->st));
        return WV_OK;
    });
}

namespace {

// Reverse sweep of the full-Newton Hessian action (FULL, AE or time store): per step k,
// the mu step (residual of the last gradient) writes q and sums e^k q into acc;
// the dmu step (residual dt/sigma^2 dp) takes -dt dm q into eta and sums
// de^k q + e^k dq into dacc.
void reverse_sweep_newton(wv_ctx* c)
{
    ensure_adj(c);
    if (!c->adj2[0]) {
        c->adj2[0] = dev_alloc<float>(c->state_floats());
        c->adj2[1] = dev_alloc<float>(c->state_floats());
        c->dacc = dev_alloc<float>(2 * c->N * c->S);
        c->dblk = dev_alloc<float>(c->N * c->S);
        c->qbuf = dev_alloc<float>(c->N * c->S);
        c->dbuf = dev_alloc<float>(c->N * c->S);
    }
    for (float* p : {c->adj[0], c->adj2[0]}) launch_fill(p, c->state_floats(), 0.f, c->st);
    launch_fill(c->acc, 2 * c->N * c->S, 0.f, c->st);
    launch_fill(c->dacc, 2 * c->N * c->S, 0.f, c->st);
    float *ain = c->adj[0], *aout = c->adj[1], *din = c->adj2[0], *dout = c->adj2[1];
    c->ts.cur_w = -1;
    c->tds.cur_w = -1;
    long long done = 0;
    for (int k = c->T - 1; k >= 1; --k) {
        long long stride;
        const float* e = load_e(c, k, &stride);
        const float* de;
        if (c->mode == WV_STORE_FULL) {
            de = c->dehist + (long long)(k - 1) * c->S * c->N;
        } else if (is_time(c->mode)) {
            WV_REQUIRE(c->tdelta_ok, WV_ESTATE, "no incremental states stored");
            de = time_e(c, c->tds, k, -1);
        } else {
            decode_state(c, c->ds, k, 1u, c->dbuf, c->N, c->st);
            de = c->dbuf;
        }
        const int phase = acc_phase(done++, k);
        adj_step_x(c, MODE_ADJQ, ain, aout, k, c->resid, e, stride, phase, c->acc, c->blk);
        adj_step_x(c, MODE_ADJD, din, dout, k, c->dresid, e, stride, phase, c->dacc, c->dblk, de);
        std::swap(ain, aout);
        std::swap(din, dout);
    }
}

}  // namespace

int hessvec(wv_ctx* c, const float* cdev, const float* dc, float* Hdc, int gauss_newton)
{
    return guarded([&]() -> int {
        WV_REQUIRE(c && cdev && dc && Hdc, WV_EINVAL, "null argument");
        WV_REQUIRE(gauss_newton == 0 || gauss_newton == 1, WV_EINVAL, "gauss_newton must be 0 or 1");
        WV_REQUIRE(c->have_grad, WV_ESTATE, "hessvec needs a preceding gradient() call");
        // the stored history must belong to this c
        WV_HIP(hipMemsetAsync(c->dflag, 0, sizeof(int), c->st));
        launch_compare(cdev, c->c_last, c->N, c->dflag, c->st);
        int flag = 0;
        WV_HIP(hipMemcpyAsync(&flag, c->dflag, sizeof(int), hipMemcpyDeviceToHost, c->st));
        WV_HIP(hipStreamSynchronize(c->st));
        WV_REQUIRE(flag == 0, WV_ESTATE, "c differs from the c of the last gradient()");
        const double w = c->g.dt / (c->sigma * c->sigma);
        const long long ntr = (long long)c->S * c->T * c->R;
        int status = WV_OK;
        const bool use_ckpt = c->mode == WV_STORE_CHECKPOINT || (c->degraded && c->fallback == WV_FALLBACK_CHECKPOINT);
        if (!gauss_newton) {
            // full Newton: d/dc of the gradient along dc, -2 dt (dc acc + c dacc)
            WV_REQUIRE(!use_ckpt && (c->mode == WV_STORE_FULL || is_ae(c->mode) || is_time(c->mode)), WV_ESTATE,
                       "the full-Newton product needs a stored history (full, autoencoder or time)");
            WV_REQUIRE(c->store_ok, WV_ESTATE, "no forward history stored");
            inc_forward_sweep(c, cdev, dc, nullptr, true);
            launch_scale_weights(c->dtr, c->dresid, ntr, w, c->st);
            reverse_sweep_newton(c);
            launch_newton_finish(cdev, dc, c->acc, c->dacc, c->N, c->S, -2.0 * c->g.dt / c->g.dx, Hdc, c->st);
            WV_HIP(hipStreamSynchronize(c->st));
            return WV_OK;
        }
        if (use_ckpt) {
            if (!c->slots || c->nslots < 2) alloc_slots(c, std::max(c->nslots, 2));
            long long fs = 0;
            const auto acts = revolve_schedule(c->T, c->nslots, &fs);
            size_t first = 0;
            const auto snap = sweep_snapshots(acts, c->T, &first);
            float* xtm1 = inc_forward_sweep(c, cdev, dc, &snap);
            launch_scale_weights(c->dtr, c->dresid, ntr, w, c->st);
            reverse_sweep(c, c->dresid, &acts, first, xtm1);
            if (c->mode != WV_STORE_CHECKPOINT) status = WV_OK_FALLBACK;
            if (c->mode == WV_STORE_CHECKPOINT) c->store_ok = false;
        } else {
            WV_REQUIRE(c->store_ok, WV_ESTATE, "no forward history stored");
            inc_forward_sweep(c, cdev, dc, nullptr);
            launch_scale_weights(c->dtr, c->dresid, ntr, w, c->st);
            reverse_sweep(c, c->dresid, nullptr, 0, nullptr);
        }
        finish_grad(c, cdev, Hdc);
        WV_HIP(hipStreamSynchronize(c->st));
        return status;
    });
}

namespace {

double dot_host(wv_ctx* c, const float* a, const float* b)
{
    launch_dot(a, b, c->N, c->partial, c->nblk_red, c->dscal, c->st);
    double v = 0.0;
    WV_HIP(hipMemcpyAsync(&v, c->dscal, sizeof(double), hipMemcpyDeviceToHost, c->st));
    WV_HIP(hipStreamSynchronize(c->st));
    return v;
}

double cell_volume(const wv_ctx* c) { return c->has_y ? c->g.dx * c->g.dx * c->g.dx : c->g.dx * c->g.dx; }

// out = scale A u' (+ out), u' = u - u0 (u0 may be null)
void apply_prior(wv_ctx* c, const float* u, const float* u0, float* out, double scale, bool accumulate)
{
    const double h2 = c->g.dx * c->g.dx;
    launch_prior(u, u0, out, c->g.nz, c->g.ny, c->g.nx, c->prior_alpha, c->prior_theta[0] / h2,
                 c->prior_theta[1] / h2, c->prior_theta[2] / h2, scale, accumulate, c->st);
}

// R(c) = 1/2 dx^dims |A (c - c0)|^2 (when want_cost) and g += dx^dims A A (c - c0)
double prior_cost_grad(wv_ctx* c, const float* cdev, float* g, bool want_cost)
{
    if (c->prior_alpha == 0.0) return 0.0;
    apply_prior(c, cdev, c->prior_c0, c->prior_w, 1.0, false);
    const double R = want_cost ? 0.5 * cell_volume(c) * dot_host(c, c->prior_w, c->prior_w) : 0.0;
    if (g) apply_prior(c, c->prior_w, nullptr, g, cell_volume(c), true);
    return R;
}

void prior_hv(wv_ctx* c, const float* dc, float* Hdc)
{
    if (c->prior_alpha == 0.0) return;
    apply_prior(c, dc, nullptr, c->prior_w, 1.0, false);
    apply_prior(c, c->prior_w, nullptr, Hdc, cell_volume(c), true);
}

// conjugate gradients on A x = b from x = 0 (A symmetric positive definite) until
// |r| <= rtol |b| or maxit iterations, with the inner work vectors pvec[1..3];
// returns the iterations, *rel the final relative residual
int prior_solve(wv_ctx* c, const float* b, float* x, double rtol, int maxit, double* rel_out)
{
    const long long N = c->N;
    if (!c->pvec) c->pvec = dev_alloc<float>(4 * (size_t)N);
    float* r = c->pvec + N;
    float* d = c->pvec + 2 * N;
    float* Ad = c->pvec + 3 * N;
    launch_fill(x, N, 0.f, c->st);
    launch_copy(r, b, N, c->st);
    launch_copy(d, r, N, c->st);
    double rr = dot_host(c, r, r);
    const double bn = std::sqrt(rr);
    int it = 0;
    double rel = bn > 0.0 ? 1.0 : 0.0;
    while (rel > rtol && it < maxit) {
        apply_prior(c, d, nullptr, Ad, 1.0, false);
        const double a = rr / dot_host(c, d, Ad);
        launch_axpby(x, d, a, 1.0, N, c->st);
        launch_axpby(r, Ad, -a, 1.0, N, c->st);
        const double rr_new = dot_host(c, r, r);
        ++it;
        rel = std::sqrt(rr_new) / bn;
        launch_axpby(d, r, 1.0, rr_new / rr, N, c->st);
        rr = rr_new;
    }
    if (rel_out) *rel_out = rel;
    return it;
}

// z = (dx^dims A A)^-1 r, the prior covariance (two elliptic solves)
constexpr double PREC_RTOL = 1e-6;
constexpr int PREC_MAXIT = 1000;
void prior_covariance(wv_ctx* c, const float* r, float* z)
{
    if (!c->pvec) c->pvec = dev_alloc<float>(4 * (size_t)c->N);
    float* y = c->pvec;
    prior_solve(c, r, y, PREC_RTOL, PREC_MAXIT, nullptr);
    launch_axpby(y, y, 1.0 / cell_volume(c), 0.0, c->N, c->st);
    prior_solve(c, y, z, PREC_RTOL, PREC_MAXIT, nullptr);
}

// positive, finite and leapfrog-stable (the test of check_speed, without throwing)
bool speed_ok(wv_ctx* c, const float* cdev)
{
    launch_range(cdev, c->N, c->partial, c->nblk_red, c->dscal, c->st);
    double h[3];
    WV_HIP(hipMemcpyAsync(h, c->dscal, sizeof(h), hipMemcpyDeviceToHost, c->st));
    WV_HIP(hipStreamSynchronize(c->st));
    const double dims = c->has_y ? 3.0 : 2.0;
    return h[2] == 0.0 && h[0] > 0.0 && h[1] * c->g.dt / c->g.dx < 1.0 / std::sqrt(dims);
}

// a public entry point's failure, re-thrown inside a guarded call
void check_rc(int rc)
{
    if (rc < 0) throw Error{rc, wv_last_error()};
}

}  // namespace

int wv_set_prior(wv_ctx* c, double alpha, const double* h_theta, const float* c0)
{
    return guarded([&]() -> int {
        WV_REQUIRE(c, WV_EINVAL, "null context");
        WV_REQUIRE(std::isfinite(alpha) && alpha >= 0.0, WV_EINVAL, "alpha must be finite and >= 0");
        if (alpha == 0.0) {
            c->prior_alpha = 0.0;
            return WV_OK;
        }
        WV_REQUIRE(h_theta && c0, WV_EINVAL, "null argument");
        for (int a = 0; a < 3; ++a)
            WV_REQUIRE(std::isfinite(h_theta[a]) && h_theta[a] >= 0.0, WV_EINVAL, "theta must be finite and >= 0");
        if (!c->prior_c0) c->prior_c0 = dev_alloc<float>(c->N);
        if (!c->prior_w) c->prior_w = dev_alloc<float>(c->N);
        launch_copy(c->prior_c0, c0, c->N, c->st);
        WV_HIP(hipStreamSynchronize(c->st));
        c->prior_alpha = alpha;
        for (int a = 0; a < 3; ++a) c->prior_theta[a] = h_theta[a];
        return WV_OK;
    });
}

int wv_prior(wv_ctx* c, const float* cdev, float* g, double* h_cost)
{
    return guarded([&]() -> int {
        WV_REQUIRE(c && cdev, WV_EINVAL, "null argument");
        const double R = prior_cost_grad(c, cdev, g, h_cost != nullptr);
        if (h_cost) *h_cost = R;
        return WV_OK;
    });
}

int wv_prior_hessvec(wv_ctx* c, const float* dc, float* Hdc)
{
    return guarded([&]() -> int {
        WV_REQUIRE(c && dc && Hdc, WV_EINVAL, "null argument");
        prior_hv(c, dc, Hdc);
        return WV_OK;
    });
}

int wv_prior_sample(wv_ctx* c, const float* w, float* out, double rtol, int32_t maxit, int32_t* h_iters,
                    double* h_relres)
{
    return guarded([&]() -> int {
        WV_REQUIRE(c && w && out, WV_EINVAL, "null argument");
        WV_REQUIRE(c->prior_alpha > 0.0, WV_ESTATE, "no prior set (wv_set_prior with alpha > 0)");
        WV_REQUIRE(rtol > 0.0 && rtol < 1.0 && maxit >= 1, WV_EINVAL, "rtol in (0, 1) and maxit >= 1 required");
        const long long N = c->N;
        if (!c->nvec) c->nvec = dev_alloc<float>(8 * (size_t)N);
        float* b = c->nvec;
        float* x = c->nvec + N;
        launch_axpby(b, w, 1.0 / std::sqrt(cell_volume(c)), 0.0, N, c->st);
        double rel = 0.0;
        const int it = prior_solve(c, b, x, rtol, maxit, &rel);
        launch_lincomb(out, c->prior_c0, 1.0, x, N, c->st);
        WV_HIP(hipStreamSynchronize(c->st));
        if (h_iters) *h_iters = it;
        if (h_relres) *h_relres = rel;
        return WV_OK;
    });
}

int wv_newton_cg(wv_ctx* c, float* cvec, const float* wavelet, const float* d_obs, double sigma,
                 const wv_newton_cfg* cfg, wv_newton_rec* h_log, int32_t* h_iters, int32_t* h_reason)
{
    return guarded([&]() -> int {
        WV_REQUIRE(c && cvec && wavelet && d_obs && cfg && h_log, WV_EINVAL, "null argument");
        WV_REQUIRE(cfg->max_newton >= 0 && cfg->max_cg >= 1 && cfg->max_backtrack >= 0, WV_EINVAL,
                   "max_newton >= 0, max_cg >= 1 and max_backtrack >= 0 required");
        WV_REQUIRE(cfg->eta_max > 0.0 && cfg->eta_max < 1.0 && cfg->rel_tol >= 0.0 && cfg->c_armijo > 0.0 &&
                       cfg->c_armijo < 1.0,
                   WV_EINVAL, "eta_max and c_armijo must lie in (0, 1), rel_tol >= 0");
        WV_REQUIRE(cfg->gauss_newton == 0 || cfg->gauss_newton == 1, WV_EINVAL, "gauss_newton must be 0 or 1");
        WV_REQUIRE(cfg->precondition == 0 || cfg->precondition == 1, WV_EINVAL, "precondition must be 0 or 1");
        WV_REQUIRE(!cfg->precondition || c->prior_alpha > 0.0, WV_ESTATE,
                   "prior preconditioning needs a prior (wv_set_prior with alpha > 0)");
        WV_REQUIRE(c->mode != WV_STORE_NONE, WV_ESTATE, "Newton-CG needs a storage mode");
        const long long N = c->N;
        if (!c->nvec) c->nvec = dev_alloc<float>(8 * (size_t)N);
        float* g = c->nvec;
        float* gt = g + N;
        float* ct = g + 2 * N;
        float* p = g + 3 * N;
        float* r = g + 4 * N;
        float* d = g + 5 * N;
        float* Hd = g + 6 * N;
        // z = M r: the prior covariance, or r itself without preconditioning
        float* z = cfg->precondition ? g + 7 * N : r;
        auto record = [](double Jm, double R, double gn, int status) {
            wv_newton_rec q{};
            q.cost = Jm + R;
            q.misfit = Jm;
            q.prior = R;
            q.gnorm = gn;
            q.status = status;
            return q;
        };
        // the iterate: J, g and the stored history that the Hessian actions read
        double Jm = 0.0;
        int status = gradient(c, cvec, wavelet, d_obs, sigma, g, &Jm);
        check_rc(status);
        double R = prior_cost_grad(c, cvec, g, true);
        double J = Jm + R;
        const double g0 = std::sqrt(dot_host(c, g, g));
        h_log[0] = record(Jm, R, g0, status);
        int it = 0, reason = 0;
        for (; it < cfg->max_newton; ++it) {
            wv_newton_rec& rec = h_log[it];
            const double gn = rec.gnorm;
            if (gn <= cfg->rel_tol * g0) {
                reason = 1;
                break;
            }
            const double eta = std::min(cfg->eta_max, std::sqrt(gn / g0));
            // conjugate gradients on H p = -g from p = 0, preconditioned by M, the
            // forcing applied to the M-norm of the residual sqrt(r.Mr)
            launch_fill(p, N, 0.f, c->st);
            launch_axpby(r, g, -1.0, 0.0, N, c->st);
            if (cfg->precondition) prior_covariance(c, r, z);
            launch_copy(d, z, N, c->st);
            double rz = dot_host(c, r, z);
            const double r0 = std::sqrt(rz);
            int its = 0, neg = 0;
            double rel = 1.0;
            while (its < cfg->max_cg) {
                check_rc(hessvec(c, cvec, d, Hd, cfg->gauss_newton));
                prior_hv(c, d, Hd);
                const double dHd = dot_host(c, d, Hd);
                ++its;
                if (!(dHd > 0.0)) {
                    neg = 1;
                    if (its == 1) launch_copy(p, d, N, c->st);
                    rel = std::sqrt(rz) / r0;
                    break;
                }
                const double a = rz / dHd;
                launch_axpby(p, d, a, 1.0, N, c->st);
                launch_axpby(r, Hd, -a, 1.0, N, c->st);
                if (cfg->precondition) prior_covariance(c, r, z);
                const double rz_new = dot_host(c, r, z);
                rel = std::sqrt(rz_new) / r0;
                if (std::sqrt(rz_new) <= eta * r0) break;
                launch_axpby(d, z, 1.0, rz_new / rz, N, c->st);
                rz = rz_new;
            }
            const double gp = dot_host(c, g, p);
            // Armijo backtracking; every trial is a full gradient evaluation
            double a = 1.0, Jmt = 0.0, Rt = 0.0;
            int bt = 0, st_t = WV_OK;
            bool accepted = false;
            for (; bt <= cfg->max_backtrack; ++bt, a *= 0.5) {
                launch_lincomb(ct, cvec, a, p, N, c->st);
                if (!speed_ok(c, ct)) continue;
                st_t = gradient(c, ct, wavelet, d_obs, sigma, gt, &Jmt);
                check_rc(st_t);
                Rt = prior_cost_grad(c, ct, gt, true);
                if (Jmt + Rt <= J + cfg->c_armijo * a * gp) {
                    accepted = true;
                    break;
                }
            }
            rec.cg_iters = its;
            rec.neg_curv = neg;
            rec.cg_rel_res = rel;
            rec.backtracks = bt;
            if (!accepted) {
                reason = 2;
                break;
            }
            rec.step = a;
            launch_copy(cvec, ct, N, c->st);
            std::swap(g, gt);
            Jm = Jmt;
            R = Rt;
            J = Jm + R;
            h_log[it + 1] = record(Jm, R, std::sqrt(dot_host(c, g, g)), st_t);
        }
        WV_HIP(hipStreamSynchronize(c->st));
        if (h_iters) *h_iters = it;
        if (h_reason) *h_reason = reason;
        return WV_OK;
    });
}

int wv_revolve_schedule(int32_t nsteps, int32_t nslots, int32_t* h_actions, int64_t cap, int64_t* h_count,
                        int64_t* h_forward_steps)
{
    return guarded([&]() -> int {
        long long fs = 0;
        const auto acts = revolve_schedule(nsteps, nslots, &fs);
        if (h_count) *h_count = (int64_t)acts.size();
        if (h_forward_steps) *h_forward_steps = fs;
        if (h_actions)
            for (size_t q = 0; q < acts.size() && (int64_t)q < cap; ++q) {
                h_actions[3 * q] = acts[q].kind;
                h_actions[3 * q + 1] = acts[q].a;
                h_actions[3 * q + 2] = acts[q].b;
            }
        return WV_OK;
    });
}

// diagnostics used by tests and the benchmark
int wv_stats(const wv_ctx* c, int64_t* h_forward_steps, double* h_guard_err, int* h_degraded)
{
    if (!c) {
        set_error("null context");
        return WV_EINVAL;
    }
    if (h_forward_steps) *h_forward_steps = c->last_fwd_steps;
    if (h_guard_err) *h_guard_err = c->guard_err;
    if (h_degraded) *h_degraded = c->degraded ? 1 : 0;
    return WV_OK;
}

int wv_set_timing(wv_ctx* c, int32_t every)
{
    return guarded([&] {
        WV_REQUIRE(c, WV_EINVAL, "null context");
        WV_REQUIRE(every >= 0, WV_EINVAL, "every must be >= 0");
        c->tm.reset(every);
        return WV_OK;
    });
}

int wv_kernel_time(wv_ctx* c, int32_t cls, double* h_mean_us, int64_t* h_count)
{
    return guarded([&] {
        WV_REQUIRE(c, WV_EINVAL, "null context");
        WV_REQUIRE(cls >= 0 && cls < KernelTimer::NCLS, WV_EINVAL, "unknown kernel class");
        c->tm.collect();
        const long long n = c->tm.cnt[cls];
        if (h_mean_us) *h_mean_us = n > 0 ? 1e3 * c->tm.sum_ms[cls] / (double)n : 0.0;
        if (h_count) *h_count = n;
        return WV_OK;
    });
}

const char* wv_last_error(void) { return g_error.c_str(); }
const char* wv_version(void) { return "wavecomp 0.1 gfx950"; }

int wv_accumulation_block(void) { return WV_ACC_BLOCK; }

}  // extern "C"

// Staggered-grid leapfrog step kernels for gfx950: forward, fused adjoint with
// Kahan-compensated gradient accumulation, and incremental (linearised) forward.
//
// All three share one z-marching structure. A work-group owns a BX x BY tile of
// the (y, x) plane and a chunk of depth levels; per level it
//   1. builds the "potential" P on the plane tile plus a one-cell cross-shaped
//      ring in LDS (P = c^2 e forward, c^2 de + dm e^n incremental, S_e eta
//      adjoint), carrying the tile's own P of the next level in registers;
//   2. updates the face fields v_y, v_x from differences of P (the +1 faces just
//      outside the tile are recomputed by the edge threads), and v_z of the next
//      face from the register-carried column;
//   3. updates the cell field from the divergence of the new faces.
// Every cell is read and written once per step (plus L2-resident halos), so a
// step costs the algorithmic 36 B/cell forward, 56 B/cell adjoint.
//
// Forward (paper Sec. 2, Eq. (model), rho = 1):
//   v_a' = S_va (v_a + dt G_a(c^2 e) + dt b_a),   e' = S_e (e + dt D v').
// Adjoint (exact transpose of the forward step). With mu lagging eta by half a
// step, one launch maps (mu^{k+2}, eta^{k+1}) to (mu^{k+1}, eta^k):
//   mu_a' = S_va mu_a - dt G_a(S_e eta) + B^T r^{k+1},
//   q = D(S_v mu'),  eta' = S_e eta - dt c^2 q,  acc += e^k q.
// so dJ/d(c^2) = -dt sum_k e^k q^k (accumulated here without the 1/dx factor).
// The time sum is compensated (Kahan) per block of consecutive adjoint steps: the
// terms of a block are summed in a plain float32 partial (ACC_FIRST starts it,
// ACC_MID adds to it), and its last step (ACC_LAST) adds the partial plus its own
// term to the compensated pair; ACC_EACH adds every term to the pair directly.
// Incremental forward: the forward step with c^2 e replaced by c^2 de + dm e^n.
// Full-Newton Hessian action: the adjoint step of mu also writes its q (ADJQ); the
// incremental adjoint step of dmu (ADJD) subtracts dt dm q from eta' and accumulates
// de^k q + e^k dq, the derivative of e^k q along dc.

#include "wv_internal.h"

#ifndef WV_NT_STORE
#define WV_NT_STORE 1
#endif

namespace wv {

namespace {

constexpr int NF = 4;  // fields per state: e, v_z, v_y, v_x

// Read-only tables indexed by a work-group-uniform index (layer factors per
// level, receiver pointers) are read through the constant address space, so
// they become scalar loads. As plain global loads they would be vector loads
// whose wait also drains the column / plane prefetch of the next levels.
template <class T>
__device__ __forceinline__ T ldu(const T* p, long long idx)
{
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Wold-style-cast"
    return ((const __attribute__((address_space(4))) T*)p)[idx];
#pragma clang diagnostic pop
}

// Field access at a level base (uniform) plus a 32-bit byte offset within the
// plane, as raw buffer operations: the base stays in scalar registers, so the
// compiler cannot hoist per-lane 64-bit pointers (two VGPRs per field) out of
// the level loop. `bytes` bounds the offsets (one plane).
constexpr int BUF_DW3 = 0x00020000;  // raw 32-bit data format, no swizzle
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const float* base, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), (short)0, (int)bytes, BUF_DW3);
}
__device__ __forceinline__ float ld_plane(const float* base, unsigned bytes, unsigned off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(plane_rsrc(base, bytes), (int)off, 0, 0));
}
// aux 2: non-temporal (streamed output, not re-read by this launch)
__device__ __forceinline__ void st_plane_nt(float v, float* base, unsigned bytes, unsigned off)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), plane_rsrc(base, bytes), (int)off, 0, 2);
}
__device__ __forceinline__ void st_plane(float v, float* base, unsigned bytes, unsigned off)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), plane_rsrc(base, bytes), (int)off, 0, 0);
}

// Minimum waves per SIMD asked of the register allocator (occupancy of these
// latency-bound kernels), per variant.
#ifndef WV_WAVES_FWD_MM
#define WV_WAVES_FWD_MM 5
#endif
#ifndef WV_WAVES_ADJ
#define WV_WAVES_ADJ 5
#endif
#ifndef WV_WAVES_OTHER
#define WV_WAVES_OTHER 6
#endif
// prefetch distance in levels of the software pipeline
#ifndef WV_PF
#define WV_PF 1
#endif

// MM: also write the per-patch (min, max) partials of the new state (forward and
// incremental forward);
// ACC: the adjoint's gradient accumulation phase; EX: also write the new e to
// a.e_extra (forward and incremental forward: the time-compression window slot
// of this level)
template <int BX, int BY, int MODE, bool HAS_Y, bool MM, int ACC = ACC_EACH, bool EX = false>
__global__ void __launch_bounds__(BX* BY)
    __attribute__((amdgpu_waves_per_eu(MM ? WV_WAVES_FWD_MM : MODE == MODE_INC || MODE == MODE_FWD ? WV_WAVES_OTHER
                                                                                                  : WV_WAVES_ADJ)))
    wave_step_kernel(const StepArgs a)
{
    __shared__ float sP[BY + 2][BX + 2];
    __shared__ float sWy[HAS_Y ? BY + 1 : 1][BX];
    __shared__ float sWx[BY][BX + 1];
    __shared__ float sMM[MM ? BY : 1][BX / 8][8];  // per-row partial (min, max) of 8 patches
    __shared__ float sRec[BY * BX];                  // receiver exchange (levels with receivers)

    // ---- block -> (x tile, y tile, z chunk); spread so one XCD gets a contiguous range
    const int nblk = a.tiles_x * a.tiles_y * a.chunks_z;
    int b = blockIdx.x;
    if ((nblk & 7) == 0) b = (b & 7) * (nblk >> 3) + (b >> 3);
    const int txx = b % a.tiles_x;
    const int tyy = (b / a.tiles_x) % a.tiles_y;
    const int cz = b / (a.tiles_x * a.tiles_y);
    const int s = blockIdx.y;
    const int tile = tyy * a.tiles_x + txx;

    const int tid = threadIdx.x;
    const int tx = tid % BX, ty = tid / BX;
    const int i0 = txx * BX, j0 = tyy * BY;
    const int i = i0 + tx, j = j0 + ty;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const bool in_x = i < nx, in_y = j < ny;
    const bool inside = in_x && in_y;
    const int local = ty * BX + tx;
    const int k0 = cz * a.kc;
    const int k1 = min(nz, k0 + a.kc);
    const long long plane = (long long)ny * nx;
    const long long N = a.N;
    const long long cell = inside ? (long long)j * nx + i : 0;

    const float* __restrict__ inA = a.in + s * a.sstride;
    const float* __restrict__ inVz = inA + N;
    const float* __restrict__ inVy = inA + 2 * N;
    const float* __restrict__ inVx = inA + 3 * N;
    float* __restrict__ outA = a.out + s * a.sstride;
    float* __restrict__ outVz = outA + N;
    float* __restrict__ outVy = outA + 2 * N;
    float* __restrict__ outVx = outA + 3 * N;
    float* __restrict__ outE = EX ? a.e_extra + s * N : nullptr;
    const float* __restrict__ mm = a.m;
    const float* __restrict__ en = (MODE == MODE_INC) ? a.en + s * a.enstride : nullptr;
    constexpr bool ADJ = MODE == MODE_ADJ || MODE == MODE_ADJQ || MODE == MODE_ADJD;
    const float* __restrict__ ek = ADJ ? a.ek + s * a.ekstride : nullptr;
    float* __restrict__ acc = ADJ ? a.acc + s * 2 * N : nullptr;
    float* __restrict__ cmp = ADJ ? acc + N : nullptr;
    float* __restrict__ blk = ADJ ? a.blk + s * N : nullptr;
    float* __restrict__ qout = (MODE == MODE_ADJQ) ? a.qbuf + s * N : nullptr;   // q of this mu step
    const float* __restrict__ qin = (MODE == MODE_ADJD) ? a.qbuf + s * N : nullptr;
    const float* __restrict__ dek = (MODE == MODE_ADJD) ? a.dek + s * a.dekstride : nullptr;
    constexpr bool rd_pair = ADJ && (ACC == ACC_EACH || ACC == ACC_LAST);
    constexpr bool rd_blk = ADJ && (ACC == ACC_MID || ACC == ACC_LAST);

    // layer factors: S = wz * (wy * wx), the (y, x) product fixed per column
    const int jc = in_y ? j : 0, ic = in_x ? i : 0;
    const float wyx_c = a.wyc[jc] * a.wxc[ic];
    const float wyx_vy = a.wyf[jc] * a.wxc[ic];
    const float wyx_vx = a.wyc[jc] * a.wxf[ic];
    const int jh = j0 + BY, ih = i0 + BX;  // the +1 faces just outside the tile
    const bool halo_y = HAS_Y && ty == BY - 1 && in_x && jh < ny;
    const bool halo_x = tx == BX - 1 && in_y && ih < nx;
    const float wyx_vy_h = halo_y ? a.wyf[jh] * a.wxc[ic] : 0.f;
    const float wyx_vx_h = halo_x ? a.wyc[jc] * a.wxf[ih] : 0.f;

    // ring of P around the tile: rows j0-1, j0+BY (HAS_Y) and columns i0-1, i0+BX
    constexpr int NRING = HAS_Y ? 2 * BX + 2 * BY : 2;
    int rj = 0, ri = 0, rsy = 0, rsx = 0;
    bool ring = false, ring_in = false;
    if (tid < NRING) {
        ring = true;
        if (HAS_Y) {
            if (tid < BX) { rj = j0 - 1; ri = i0 + tid; rsy = 0; rsx = tid + 1; }
            else if (tid < 2 * BX) { rj = jh; ri = i0 + tid - BX; rsy = BY + 1; rsx = tid - BX + 1; }
            else if (tid < 2 * BX + BY) { rj = j0 + tid - 2 * BX; ri = i0 - 1; rsy = tid - 2 * BX + 1; rsx = 0; }
            else { rj = j0 + tid - 2 * BX - BY; ri = ih; rsy = tid - 2 * BX - BY + 1; rsx = BX + 1; }
        } else {
            rj = 0; ri = (tid == 0) ? i0 - 1 : ih; rsy = 1; rsx = (tid == 0) ? 0 : BX + 1;
        }
        ring_in = rj >= 0 && rj < ny && ri >= 0 && ri < nx;
    }
    const long long rcell = ring_in ? (long long)rj * nx + ri : 0;
    const float ring_wyx = ring_in ? a.wyc[rj] * a.wxc[ri] : 0.f;

    // receivers of this tile per level: rec_ent[lp[k] .. lp[k + 1])
    const int* lp = a.rec_ptr + (long long)tile * (nz + 1);
    // source of this wavefield: force density wavelet[s][n] * w[dk][dj][di] on the
    // v_z faces of a (2R+1)^dims box centred on its face
    int sk = 0, sj = 0, si = 0, R = 0;
    float bsrc = 0.f;
    if (MODE == MODE_FWD) {
        sk = a.src_kji[3 * s];
        sj = a.src_kji[3 * s + 1];
        si = a.src_kji[3 * s + 2];
        R = a.src_radius;
        bsrc = a.dt * a.wavelet[(long long)s * a.nt + a.step];
    }
    const int wdj = HAS_Y ? 2 * R + 1 : 1;
    const bool src_col = MODE == MODE_FWD && inside && abs(i - si) <= R && (HAS_Y ? abs(j - sj) <= R : true);
    const int src_col_off = src_col ? (HAS_Y ? (j - sj + R) : 0) * (2 * R + 1) + (i - si + R) : 0;
    const long long trow = ((long long)s * a.nt + a.tidx) * a.nrec;  // traces / residual row

    // extra term on the v_z face kk: dt b (forward source), B^T r (adjoint). The
    // adjoint gathers the residuals of the level's receivers into sRec: one thread
    // per run of entries on the same cell sums the run in receiver order. Called by
    // the whole work-group (the receiver test is uniform).
    auto face_inj = [&](int kk) -> float {
        float add = 0.f;
        if (MODE == MODE_FWD) {
            if (src_col && abs(kk - sk) <= R)
                add = bsrc * a.src_w[(kk - sk + R) * wdj * (2 * R + 1) + src_col_off];
        } else if (ADJ) {
            if (a.nrec > 0 && kk < nz) {
                const int q0 = ldu(lp, kk), q1 = ldu(lp, kk + 1);
                if (q1 > q0) {
                    sRec[local] = 0.f;
                    __syncthreads();
                    for (int q = q0 + tid; q < q1; q += BX * BY) {
                        const int4 e = a.rec_ent[q];
                        if (q > q0 && a.rec_ent[q - 1].y == e.y) continue;
                        float r = 0.f;
                        for (int u = q; u < q1; ++u) {
                            const int4 f = a.rec_ent[u];
                            if (f.y != e.y) break;
                            r += a.resid[trow + f.z];
                        }
                        sRec[e.y] = r;
                    }
                    __syncthreads();
                    add = sRec[local];
                }
            }
        }
        return add;
    };
    // new face value from old value V, difference dP and extra term
    auto face_new = [&](float S, float V, float dP, float add) -> float {
        if (ADJ) return S * V - a.dtdx * dP + add;
        return S * (V + a.dtdx * dP + add);
    };
    // what enters the divergence: v' (forward) or S_v mu' (adjoint)
    auto face_w = [&](float S, float Vn) -> float { return ADJ ? S * Vn : Vn; };

    // Software pipeline: the column data of level k+1+PF and the in-plane data of
    // level k+PF are loaded while level k is computed, into a ring of PF+1
    // register sets (no copies between levels). Every lane issues every load,
    // at a clamped in-grid address where its own operand does not exist (outside
    // lanes read cell 0, out-of-range levels the nearest level); such values are
    // never used, so the loads need no branches and the compiler can count the
    // outstanding ones instead of draining them.
    struct Col {  // own column at one level
        float A, m, Vz, dm, en;
    };
    struct Pln {  // in-plane operands of one level
        float Vy, Vx, Vyh, Vxh, rA, rm, rdm, ren, ek, acc, cmp, blk, dek, q;
    };
    // Addresses are a level base (uniform, scalar registers) plus a 32-bit byte
    // offset within the plane (a plane holds fewer than 2^30 cells).
    const unsigned o_c = (unsigned)cell * 4u;
    const unsigned o_r = (unsigned)rcell * 4u;
    const unsigned o_hy = halo_y ? (unsigned)(jh * nx + i) * 4u : o_c;
    const unsigned o_hx = halo_x ? (unsigned)(j * nx + ih) * 4u : o_c;
    const unsigned pb4 = (unsigned)plane * 4u;
    auto ld = [&](const float* f, long long lo, unsigned off) { return ld_plane(f + lo, pb4, off); };
    auto load_col = [&](int kk, Col& c) {
        const long long lo = (long long)min(max(kk, 0), nz - 1) * plane;
        c.A = ld(inA, lo, o_c);
        c.m = ld(mm, lo, o_c);
        c.Vz = ld(inVz, lo, o_c);
        if (MODE == MODE_INC) {
            c.dm = ld(a.dm, lo, o_c);
            c.en = ld(en, lo, o_c);
        }
        if (MODE == MODE_ADJD) c.dm = ld(a.dm, lo, o_c);
    };
    auto load_pln = [&](int kk, Pln& q) {
        const long long lo = (long long)kk * plane;
        if (HAS_Y) {
            q.Vy = ld(inVy, lo, o_c);
            q.Vyh = ld(inVy, lo, o_hy);
        }
        q.Vx = ld(inVx, lo, o_c);
        q.Vxh = ld(inVx, lo, o_hx);
        if (MODE == MODE_ADJD) {
            q.dek = ld(dek, lo, o_c);
            q.q = ld(qin, lo, o_c);
        }
        if (ADJ) {
            q.ek = ld(ek, lo, o_c);
            if (rd_pair) {
                q.acc = ld(acc, lo, o_c);
                q.cmp = ld(cmp, lo, o_c);
            }
            if (rd_blk) q.blk = ld(blk, lo, o_c);
        }
        q.rA = ld(inA, lo, o_r);
        if (!ADJ) q.rm = ld(mm, lo, o_r);
        if (MODE == MODE_INC) {
            q.rdm = ld(a.dm, lo, o_r);
            q.ren = ld(en, lo, o_r);
        }
    };
    auto P_col = [&](int kk, const Col& c) -> float {
        if (MODE == MODE_FWD) return c.m * c.A;
        if (MODE == MODE_INC) return c.m * c.A + c.dm * c.en;
        return (ldu(a.wzc, kk) * wyx_c) * c.A;
    };
    auto P_ring = [&](int kk, const Pln& q) -> float {
        if (!ring_in) return 0.f;
        if (MODE == MODE_FWD) return q.rm * q.rA;
        if (MODE == MODE_INC) return q.rm * q.rA + q.rdm * q.ren;
        return (ldu(a.wzc, kk) * ring_wyx) * q.rA;
    };

    // ---- prologue: P(k0), cell value, v_z'(k0); first pipeline stages.
    // Ring slot u holds column level k0+u (mod NB) and plane level k0+u (mod NB).
    constexpr int NB = WV_PF + 1;
    float P_cur = 0.f, A_cur = 0.f, m_cur = 0.f, dm_cur = 0.f, Vz_cur = 0.f, Wz_cur = 0.f;
    Col cb[NB];
    Pln pb[NB];
    {
        Col c0, cl;
        load_col(k0, c0);
        load_col(k0 - 1, cl);
#pragma unroll
        for (int u = 1; u <= WV_PF; ++u) load_col(min(k0 + u, k1), cb[u % NB]);
#pragma unroll
        for (int u = 0; u < WV_PF; ++u) load_pln(min(k0 + u, k1 - 1), pb[u]);
        A_cur = c0.A;
        m_cur = c0.m;
        if (MODE == MODE_ADJD) dm_cur = c0.dm;
        P_cur = inside ? P_col(k0, c0) : 0.f;
        const float P_lo = (inside && k0 > 0) ? P_col(k0 - 1, cl) : 0.f;
        const float add = face_inj(k0);
        const float S = ldu(a.wzf, k0) * wyx_c;
        Vz_cur = face_new(S, c0.Vz, P_cur - P_lo, add);
        Wz_cur = face_w(S, Vz_cur);
    }

    // running (min, max) of the 4 new fields over the current patch layer
    constexpr bool want_mm = MM && (MODE == MODE_FWD || MODE == MODE_INC) && HAS_Y;
    float mn0 = INFINITY, mn1 = INFINITY, mn2 = INFINITY, mn3 = INFINITY;
    float mx0 = -INFINITY, mx1 = -INFINITY, mx2 = -INFINITY, mx3 = -INFINITY;

    // one level k: reads cn (column level k+1) and pc (plane level k), loads
    // cnn (column level k+1+PF) and pn (plane level k+PF)
    auto level = [&](const int k, const Col& cn, Col& cnn, const Pln& pc, Pln& pn) {
        const long long lk = (long long)k * plane;
        const bool has_next = k + 1 < nz;
        // issue the loads of the next pipeline stages (levels past the chunk re-read
        // its last needed level rather than branching: column data up to k1, where
        // the last cell's upper face reads P and v_z; plane data up to k1 - 1). A
        // level past k1 belongs to the next chunk, which another work-group, often on
        // another XCD, reads much later, so fetching it here would cost HBM bytes.
        load_col(min(k + 1 + WV_PF, k1), cnn);
        load_pln(min(k + WV_PF, k1 - 1), pn);
        const float P_nx = (inside && has_next) ? P_col(k + 1, cn) : 0.f;
        const float Vz_nx_in = cn.Vz;
        const float Vy_in = pc.Vy, Vx_in = pc.Vx, Vy_h = pc.Vyh, Vx_h = pc.Vxh;
        const float e_k = pc.ek;
        float s_acc = rd_pair ? pc.acc : 0.f, s_cmp = rd_pair ? pc.cmp : 0.f;
        const float s_blk = rd_blk ? pc.blk : 0.f;
        const float Pr = P_ring(k, pc);

        sP[ty + 1][tx + 1] = P_cur;
        if (ring) sP[rsy][rsx] = Pr;
        __syncthreads();

        // ---- faces in the plane
        const float wzc = ldu(a.wzc, k);
        float Vy_new = 0.f, Vx_new = 0.f;
        if (HAS_Y) {
            const float S = wzc * wyx_vy;
            Vy_new = face_new(S, Vy_in, sP[ty + 1][tx + 1] - sP[ty][tx + 1], 0.f);
            sWy[ty][tx] = face_w(S, Vy_new);
            if (ty == BY - 1) {
                const float Sh = wzc * wyx_vy_h;
                const float Vh = face_new(Sh, Vy_h, sP[BY + 1][tx + 1] - sP[BY][tx + 1], 0.f);
                sWy[BY][tx] = face_w(Sh, Vh);
            }
        }
        {
            const float S = wzc * wyx_vx;
            Vx_new = face_new(S, Vx_in, sP[ty + 1][tx + 1] - sP[ty + 1][tx], 0.f);
            sWx[ty][tx] = face_w(S, Vx_new);
            if (tx == BX - 1) {
                const float Sh = wzc * wyx_vx_h;
                const float Vh = face_new(Sh, Vx_h, sP[ty + 1][BX + 1] - sP[ty + 1][BX], 0.f);
                sWx[ty][BX] = face_w(Sh, Vh);
            }
        }
        // ---- next z face of the own column
        float Vz_nx = 0.f, Wz_nx = 0.f;
        {
            const float add = face_inj(k + 1);
            if (has_next) {
                const float S = ldu(a.wzf, k + 1) * wyx_c;
                Vz_nx = face_new(S, Vz_nx_in, P_nx - P_cur, add);
                Wz_nx = face_w(S, Vz_nx);
            }
        }
        __syncthreads();

        // ---- cell update from the divergence of the new faces
        float dsum = Wz_nx - Wz_cur;
        if (HAS_Y) dsum += ((j + 1 < ny) ? sWy[ty + 1][tx] : 0.f) - sWy[ty][tx];
        dsum += ((i + 1 < nx) ? sWx[ty][tx + 1] : 0.f) - sWx[ty][tx];
        const float Se = wzc * wyx_c;
        float A_new;
        if (ADJ) {
            A_new = Se * A_cur - a.dtdx * m_cur * dsum;
            // the term of this step, plus the block's partial on its last step
            float term = e_k * dsum;
            if (MODE == MODE_ADJD) {
                // coupling to the mu step: eta' -= dt dm q; the sum takes de^k q + e^k dq
                A_new -= a.dtdx * dm_cur * pc.q;
                term += pc.dek * pc.q;
            }
            if (ACC == ACC_MID || ACC == ACC_LAST) term = s_blk + term;
            if (ACC == ACC_EACH || ACC == ACC_LAST) {
                // Kahan: s_acc += term
                const float y = term - s_cmp;
                const float t = s_acc + y;
                s_cmp = (t - s_acc) - y;
                s_acc = t;
            } else {
                s_acc = term;  // the block partial
            }
        } else {
            A_new = Se * (A_cur + a.dtdx * dsum);
        }
        if (inside) {
#if WV_NT_STORE
            st_plane_nt(A_new, outA + lk, pb4, o_c);
            st_plane_nt(Vz_cur, outVz + lk, pb4, o_c);
            if (HAS_Y) st_plane_nt(Vy_new, outVy + lk, pb4, o_c);
            st_plane_nt(Vx_new, outVx + lk, pb4, o_c);
            if (EX) st_plane_nt(A_new, outE + lk, pb4, o_c);
#else
            st_plane(A_new, outA + lk, pb4, o_c);
            st_plane(Vz_cur, outVz + lk, pb4, o_c);
            if (HAS_Y) st_plane(Vy_new, outVy + lk, pb4, o_c);
            st_plane(Vx_new, outVx + lk, pb4, o_c);
            if (EX) st_plane(A_new, outE + lk, pb4, o_c);
#endif
            if (ADJ) {
                if (ACC == ACC_EACH || ACC == ACC_LAST) {
                    st_plane(s_acc, acc + lk, pb4, o_c);
                    st_plane(s_cmp, cmp + lk, pb4, o_c);
                } else {
                    st_plane(s_acc, blk + lk, pb4, o_c);
                }
                if (MODE == MODE_ADJQ) st_plane(dsum, qout + lk, pb4, o_c);
            }
        }
        if constexpr (want_mm) {
            if (inside) {
                mn0 = fminf(mn0, A_new); mx0 = fmaxf(mx0, A_new);
                mn1 = fminf(mn1, Vz_cur); mx1 = fmaxf(mx1, Vz_cur);
                mn2 = fminf(mn2, Vy_new); mx2 = fmaxf(mx2, Vy_new);
                mn3 = fminf(mn3, Vx_new); mx3 = fmaxf(mx3, Vx_new);
            }
            if (((k + 1) & 7) == 0) {
                // reduce the 8 x-lanes of each patch, then the BY rows of the tile
#pragma unroll
                for (int o = 1; o < 8; o <<= 1) {
                    mn0 = fminf(mn0, __shfl_xor(mn0, o, 64)); mx0 = fmaxf(mx0, __shfl_xor(mx0, o, 64));
                    mn1 = fminf(mn1, __shfl_xor(mn1, o, 64)); mx1 = fmaxf(mx1, __shfl_xor(mx1, o, 64));
                    mn2 = fminf(mn2, __shfl_xor(mn2, o, 64)); mx2 = fmaxf(mx2, __shfl_xor(mx2, o, 64));
                    mn3 = fminf(mn3, __shfl_xor(mn3, o, 64)); mx3 = fmaxf(mx3, __shfl_xor(mx3, o, 64));
                }
                if ((tx & 7) == 0) {
                    float* d = sMM[ty][tx >> 3];
                    d[0] = mn0; d[1] = mx0; d[2] = mn1; d[3] = mx1;
                    d[4] = mn2; d[5] = mx2; d[6] = mn3; d[7] = mx3;
                }
                __syncthreads();
                if (tid < (BX / 8) * 8) {
                    const int q = tid >> 3, v = tid & 7;
                    float r = sMM[0][q][v];
#pragma unroll
                    for (int y = 1; y < BY; ++y) r = (v & 1) ? fmaxf(r, sMM[y][q][v]) : fminf(r, sMM[y][q][v]);
                    const int Px = nx >> 3, Py = ny >> 3;
                    const int px = txx * (BX / 8) + q, py = j0 >> 3, pz = k >> 3;
                    const int H = 8 / BY, h = (j0 & 7) / BY;
                    if (px < Px) {
                        const long long p = ((long long)pz * Py + py) * Px + px;
                        const long long P = (long long)(nz >> 3) * Py * Px;
                        a.mm_out[(((long long)s * P + p) * H + h) * 8 + v] = r;
                    }
                }
                mn0 = mn1 = mn2 = mn3 = INFINITY;
                mx0 = mx1 = mx2 = mx3 = -INFINITY;
            }
        }
        // traces: v_z of this level's new face at the receivers, through sRec
        if (!ADJ && a.nrec > 0) {
            const int q0 = ldu(lp, k), q1 = ldu(lp, k + 1);
            if (q1 > q0) {
                sRec[local] = Vz_cur;
                __syncthreads();
                for (int q = q0 + tid; q < q1; q += BX * BY) {
                    const int4 e = a.rec_ent[q];
                    a.traces[trow + e.z] = sRec[e.y];
                }
            }
        }
        P_cur = P_nx;
        A_cur = cn.A;
        m_cur = cn.m;
        if (MODE == MODE_ADJD) dm_cur = cn.dm;
        Vz_cur = Vz_nx;
        Wz_cur = Wz_nx;
    };
    // level k0+u uses column slot (u+1) % NB, plane slot u % NB, and refills the
    // slots of column k0+u (consumed one level earlier) and plane k0+u-1
    int kb = k0;
    for (; kb + NB <= k1; kb += NB) {
#pragma unroll
        for (int u = 0; u < NB; ++u)
            level(kb + u, cb[(u + 1) % NB], cb[u % NB], pb[u % NB], pb[(u + NB - 1) % NB]);
    }
#pragma unroll
    for (int u = 0; u < NB - 1; ++u)
        if (kb + u < k1) level(kb + u, cb[(u + 1) % NB], cb[u % NB], pb[u % NB], pb[(u + NB - 1) % NB]);
}

template <int BX, int BY, int MODE, bool HAS_Y>
void launch_adj(const StepArgs& a, dim3 grid, dim3 block, hipStream_t st)
{
    switch (a.acc_phase) {
    case ACC_FIRST: hipLaunchKernelGGL((wave_step_kernel<BX, BY, MODE, HAS_Y, false, ACC_FIRST>), grid, block, 0, st, a); break;
    case ACC_MID: hipLaunchKernelGGL((wave_step_kernel<BX, BY, MODE, HAS_Y, false, ACC_MID>), grid, block, 0, st, a); break;
    case ACC_LAST: hipLaunchKernelGGL((wave_step_kernel<BX, BY, MODE, HAS_Y, false, ACC_LAST>), grid, block, 0, st, a); break;
    default: hipLaunchKernelGGL((wave_step_kernel<BX, BY, MODE, HAS_Y, false, ACC_EACH>), grid, block, 0, st, a); break;
    }
}

template <int BX, int BY, bool HAS_Y>
void launch_mode(int mode, const StepArgs& a0, int nsrc, hipStream_t st)
{
    StepArgs a = a0;
    if (mode == MODE_ADJ || mode == MODE_ADJQ || mode == MODE_ADJD) {
        a.kc = a.kc_adj;
        a.chunks_z = a.chunks_adj;
    }
    if ((mode != MODE_FWD && mode != MODE_INC) || !HAS_Y) a.mm_out = nullptr;
    if (mode != MODE_FWD && mode != MODE_INC) a.e_extra = nullptr;
    dim3 grid(a.tiles_x * a.tiles_y * a.chunks_z, nsrc);
    dim3 block(BX * BY);
    switch (mode) {
    case MODE_FWD:
        if (HAS_Y && a.mm_out)
            hipLaunchKernelGGL((wave_step_kernel<BX, BY, MODE_FWD, HAS_Y, HAS_Y>), grid, block, 0, st, a);
        else if (a.e_extra)
            hipLaunchKernelGGL((wave_step_kernel<BX, BY, MODE_FWD, HAS_Y, false, ACC_EACH, true>), grid, block, 0,
                               st, a);
        else
            hipLaunchKernelGGL((wave_step_kernel<BX, BY, MODE_FWD, HAS_Y, false>), grid, block, 0, st, a);
        break;
    case MODE_ADJ: launch_adj<BX, BY, MODE_ADJ, HAS_Y>(a, grid, block, st); break;
    case MODE_ADJQ: launch_adj<BX, BY, MODE_ADJQ, HAS_Y>(a, grid, block, st); break;
    case MODE_ADJD: launch_adj<BX, BY, MODE_ADJD, HAS_Y>(a, grid, block, st); break;
    default:
        if (HAS_Y && a.mm_out)
            hipLaunchKernelGGL((wave_step_kernel<BX, BY, MODE_INC, HAS_Y, HAS_Y>), grid, block, 0, st, a);
        else if (a.e_extra)
            hipLaunchKernelGGL((wave_step_kernel<BX, BY, MODE_INC, HAS_Y, false, ACC_EACH, true>), grid, block, 0,
                               st, a);
        else
            hipLaunchKernelGGL((wave_step_kernel<BX, BY, MODE_INC, HAS_Y, false>), grid, block, 0, st, a);
        break;
    }
}

}  // namespace

#ifndef WV_TILE_BY
#define WV_TILE_BY 8
#endif
#ifndef WV_CHUNK_TARGET
#define WV_CHUNK_TARGET 2048
#endif
#ifndef WV_CHUNK_TARGET_ADJ
#define WV_CHUNK_TARGET_ADJ 8192
#endif
constexpr int TILE_BX = 64;
constexpr int TILE_BY = WV_TILE_BY;

void launch_step(int mode, bool has_y, const StepArgs& a, int nsrc, hipStream_t st)
{
    if (has_y)
        launch_mode<TILE_BX, TILE_BY, true>(mode, a, nsrc, st);
    else
        launch_mode<TILE_BX, 1, false>(mode, a, nsrc, st);
    WV_HIP(hipGetLastError());
}

Tiling make_tiling(int nz, int ny, int nx, const std::vector<int>& rec_kji)
{
    Tiling t;
    const bool has_y = ny > 1;
    t.bx = TILE_BX;
    t.by = has_y ? TILE_BY : 1;
    t.tiles_x = (nx + t.bx - 1) / t.bx;
    t.tiles_y = (ny + t.by - 1) / t.by;
    const int tiles = t.tiles_x * t.tiles_y;
    // enough work-groups to fill 256 CUs several times; chunks of a multiple of
    // 8 levels (patch layers) when the depth allows
    const ChunkPlan f = plan_chunks(nz, tiles, WV_CHUNK_TARGET), a = plan_chunks(nz, tiles, WV_CHUNK_TARGET_ADJ);
    t.kc = f.kc;
    t.chunks_z = f.chunks;
    t.kc_adj = a.kc;
    t.chunks_adj = a.chunks;
    // receivers bucketed by tile, then level, then local cell: one pointer per
    // (tile, level) so a work-group finds the receivers of a level in O(1)
    std::vector<int> ptr;
    std::vector<RecEnt> ent;
    bucket_receivers(nz, t.bx, t.by, t.tiles_x, t.tiles_y, rec_kji, ptr, ent);
    WV_HIP(hipMalloc(&t.rec_ptr, sizeof(int) * ptr.size()));
    WV_HIP(hipMemcpy(t.rec_ptr, ptr.data(), sizeof(int) * ptr.size(), hipMemcpyHostToDevice));
    WV_HIP(hipMalloc(&t.rec_ent, sizeof(int4) * std::max<size_t>(ent.size(), 1)));
    if (!ent.empty()) WV_HIP(hipMemcpy(t.rec_ent, ent.data(), sizeof(int4) * ent.size(), hipMemcpyHostToDevice));
    return t;
}

void free_tiling(Tiling& t)
{
    if (t.rec_ptr) (void)hipFree(t.rec_ptr);
    if (t.rec_ent) (void)hipFree(t.rec_ent);
    t.rec_ptr = nullptr;
    t.rec_ent = nullptr;
}

}  // namespace wv

// The deferred per-shift update of the shifted-COCG solver (the dominant kernel).
#include "device_common.h"

namespace scocg {

// ---------------------------------------------------------------------------------------
// Deferred per-shift update.  For every active pair and every step t < nact of the block
//   u_k <- r_t + b'_t u_k ;  x_k <- x_k + a'_t u_k
// x_k and u_k stay in registers across the block, so each is read and written once per
// block instead of once per iteration.  One thread per row; a workgroup covers 256 rows of
// one rhs and `G` shifts, NP pairs in flight per thread.  Every step runs for every pair:
// the coefficient table pads a pair's steps past its last one with a' = 0, b' = 1 and the
// residual history is zero past the block's last step, so those steps leave x_k (and u_k)
// as they are; the only branches left are uniform ones over whole pair groups.
// Coefficients are uniform across the workgroup (scalar loads).  x_k and u_k are streamed
// with nontemporal loads and stores: they are not reused before the next block.
// ---------------------------------------------------------------------------------------
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));

__device__ inline double2 ld_nt(const double2 *p)
{
    const d2v v = __builtin_nontemporal_load((const d2v *)p);
    return make_double2(v.x, v.y);
}
__device__ inline float2 ld_nt(const float2 *p)
{
    const f2v v = __builtin_nontemporal_load((const f2v *)p);
    return make_float2(v.x, v.y);
}
__device__ inline void st_nt(double2 *p, double2 v)
{
    const d2v w = {v.x, v.y};
    __builtin_nontemporal_store(w, (d2v *)p);
}
__device__ inline void st_nt(float2 *p, float2 v)
{
    const f2v w = {v.x, v.y};
    __builtin_nontemporal_store(w, (f2v *)p);
}

// Projection mode: TB steps for NP pairs held in registers, with or without the x_k update;
// pair cp[q]'s (a', b') table starts at coef + cp[q] * TB * 2.
template <int TB, typename V, int NP, bool WITH_X>
__device__ inline void apply_steps(const V *coef, const int64_t (&cp)[NP], const V (&r)[TB], V (&x)[NP], V (&u)[NP])
{
#pragma unroll
    for (int t = 0; t < TB; ++t) {
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const V *cf = coef + (cp[q] * TB + t) * 2;
            u[q] = cfma(cf[1], u[q], r[t]);
            if (WITH_X) x[q] = cfma(cf[0], u[q], x[q]);
        }
    }
}

template <int TB, typename V, int NP, bool PROJ>
__global__ void __launch_bounds__(WG) k_flush(const int32_t *__restrict__ blk, const double2 *__restrict__ ring,
                                              const V *__restrict__ coef, const int32_t *__restrict__ nact,
                                              V *__restrict__ X, V *__restrict__ P, double2 *__restrict__ Xproj,
                                              const int64_t *__restrict__ proj_row,
                                              const RhsDesc *__restrict__ desc, int64_t ntot, int64_t M, int G,
                                              int ngroups, const int32_t *__restrict__ wshift, int64_t Mst,
                                              int R, const int2 *__restrict__ items)
{
    // Row blocks run fastest in dispatch order, so the concurrently running workgroups of one
    // shift group stream long contiguous stretches of each pair's x and u.  (Dealing the shift
    // groups of one row block to one XCD instead, to reuse the residual history from L2, made
    // the launch slower: the x, u accesses then scatter over many DRAM pages.)  An uneven batch
    // passes its work list (rhs * ngroups + group, row block) in the same order.
    const int64_t y = items ? items[blockIdx.x].x : blockIdx.y;
    const int64_t j = y / ngroups;
    const int g = y % ngroups;
    const int64_t rb = items ? items[blockIdx.x].y : blockIdx.x;
    // this block's steps, ring slot of its first residual, first block (x, u start at 0)
    const int ns = blk[4 * j + 0];
    if (ns == 0) return;
    const int base = blk[4 * j + 1];
    const bool fresh = blk[4 * j + 2] != 0;
    const int64_t n = desc[j].n;
    const int64_t voff = desc[j].voff;
    const int64_t row = rb * WG + threadIdx.x;
    if (row >= n) return;
    // stored-direction slots k0 .. k1-1 of this workgroup; slot w holds shift kof(w) (a window
    // of seed candidates in projection mode, else shift w)
    const int64_t k0 = (int64_t)g * G;
    const int64_t k1 = min(k0 + G, Mst);
    auto kof = [&](int64_t w) -> int64_t { return (PROJ && wshift) ? (int64_t)wshift[j * Mst + w] : w; };
    // late in a solve most shift groups are frozen: skip them before reading the history
    bool group_active = false;
    for (int64_t k = k0; k < k1; ++k) group_active = group_active || nact[j * M + kof(k)] > 0;
    if (!group_active) return;
    V r[TB];
#pragma unroll
    for (int t = 0; t < TB; ++t) {
        if (t < ns) r[t] = to_v<V>(ring[(int64_t)((base + t) % R) * ntot + voff + row]);
        else r[t] = to_v<V>(cmk(0, 0));
    }
    X += M * voff;
    P += Mst * voff;
    const int64_t prow = PROJ ? proj_row[j] : -1;
    // projection mode needs x_k only in the workgroup that holds the kept row (uniform test)
    const int64_t row0 = rb * WG;
    const bool with_x = !PROJ || (prow >= row0 && prow < row0 + WG);
    for (int64_t k = k0; k < k1; k += NP) {
        V x[NP], u[NP];
        int na[NP];
        bool any = false;
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const int64_t pair = j * M + kof(k + q < k1 ? k + q : k);
            na[q] = (k + q < k1) ? nact[pair] : 0;
            any = any || na[q] > 0;
            x[q] = to_v<V>(cmk(0, 0));
            u[q] = x[q];
            if (na[q] > 0 && !fresh) {
                u[q] = ld_nt(P + (k + q) * n + row);
                if (PROJ) {
                    if (row == prow) x[q] = to_v<V>(Xproj[pair]);
                } else {
                    x[q] = ld_nt(X + (k + q) * n + row);
                }
            }
        }
        if (!any) continue;
        if constexpr (!PROJ) {
            // the same steps as apply_steps, written out: this form compiles to fewer
            // registers (121 against 147 VGPRs for FP64 and 24 steps: one more wave per SIMD)
#pragma unroll
            for (int t = 0; t < TB; ++t) {
#pragma unroll
                for (int q = 0; q < NP; ++q) {
                    // a slot past the group's end reuses the first pair's table (not stored)
                    const int64_t kq = (k + q < k1) ? k + q : k;
                    const V *cf = coef + ((j * M + kq) * TB + t) * 2;
                    u[q] = cfma(cf[1], u[q], r[t]);
                    x[q] = cfma(cf[0], u[q], x[q]);
                }
            }
        } else {
            // a slot past the group's end reuses the first pair's table (its result is not stored)
            int64_t cp[NP];
#pragma unroll
            for (int q = 0; q < NP; ++q) cp[q] = j * M + kof(k + q < k1 ? k + q : k);
            if (with_x) apply_steps<TB, V, NP, true>(coef, cp, r, x, u);
            else apply_steps<TB, V, NP, false>(coef, cp, r, x, u);
        }
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const int64_t pair = j * M + kof(k + q < k1 ? k + q : k);
            if (na[q] > 0) {
                st_nt(P + (k + q) * n + row, u[q]);
                if (PROJ) {
                    if (row == prow) Xproj[pair] = make_double2((double)x[q].x, (double)x[q].y);
                } else {
                    st_nt(X + (k + q) * n + row, x[q]);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------------------
// Long blocks (T >= 24).  The T residuals of a 64-row tile are staged once in LDS and shared
// by the FL_W waves of the workgroup; each wave takes runs of NPW active slots of the shift
// group (ranked from a ballot of the group's activity, so no loads steer the loop), keeps
// their x_k and u_k in registers (each history read serves all NPW) and fetches the next
// run's while it computes.  The coefficients
// are read with scalar loads in chunks of C steps: at each chunk boundary one wait covers
// the chunk's coefficients and residuals, then the next chunk's loads are issued and the
// chunk is computed while they are in flight.  (Left to itself the compiler waits for them
// two steps at a time, which exposes the L2 latency of every coefficient line; that, not
// register pressure, is what stops the register form above beyond T = 24.)  Every pair gets
// the steps of k_flush in the same order, so the results are the same bits.
// ---------------------------------------------------------------------------------------
constexpr int FL_W = 8;  // waves per workgroup of the long-block update

// s_waitcnt lgkmcnt(0) (gfx9 encoding, vmcnt and expcnt left at their maxima), fenced so
// that neither the compiler's code motion (empty asm with a memory clobber) nor the machine
// scheduler (scheduling barriers) moves loads or arithmetic across it
#define FLUSH_CHUNK_WAIT()                     \
    do {                                       \
        asm volatile("" ::: "memory");         \
        __builtin_amdgcn_sched_barrier(0);     \
        __builtin_amdgcn_s_waitcnt(0xC07F);    \
        __builtin_amdgcn_sched_barrier(0);     \
        asm volatile("" ::: "memory");         \
    } while (0)

// TB steps of NPW pairs: cf[q] is pair q's (a', b') table, lrow the thread's column of the
// LDS history (stride 64), shared by the pairs; WX = false leaves x alone (projection mode
// away from the kept row).  Each pair gets the steps in the order of k_flush.
template <int TB, int C, int NPW, typename V, bool WX>
__device__ inline void flush_pair_steps(const V *const (&cf)[NPW], const V *lrow, V (&x)[NPW], V (&u)[NPW])
{
    constexpr int NC = TB / C;
    V ca[2][NPW][C], cb[2][NPW][C], rr[2][C];
#pragma unroll
    for (int t = 0; t < C; ++t) {
#pragma unroll
        for (int q = 0; q < NPW; ++q) {
            if (WX) ca[0][q][t] = cf[q][2 * t];
            cb[0][q][t] = cf[q][2 * t + 1];
        }
        rr[0][t] = lrow[t * 64];
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        FLUSH_CHUNK_WAIT();
        if (c + 1 < NC) {
#pragma unroll
            for (int t = 0; t < C; ++t) {
                const int s = (c + 1) * C + t;
#pragma unroll
                for (int q = 0; q < NPW; ++q) {
                    if (WX) ca[(c + 1) & 1][q][t] = cf[q][2 * s];
                    cb[(c + 1) & 1][q][t] = cf[q][2 * s + 1];
                }
                rr[(c + 1) & 1][t] = lrow[s * 64];
            }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int t = 0; t < C; ++t) {
#pragma unroll
            for (int q = 0; q < NPW; ++q) {
                u[q] = cfma(cb[c & 1][q][t], u[q], rr[c & 1][t]);
                if (WX) x[q] = cfma(ca[c & 1][q][t], u[q], x[q]);
            }
        }
        // the chunk's arithmetic stays ahead of the next boundary
#pragma unroll
        for (int q = 0; q < NPW; ++q) asm volatile("" : "+v"(u[q].x), "+v"(u[q].y), "+v"(x[q].x), "+v"(x[q].y));
    }
}

template <int TB, int C, int NPW, typename V, bool PROJ>
__global__ void __launch_bounds__(64 * FL_W)
    k_flush_lds(const int32_t *__restrict__ blk, const double2 *__restrict__ ring, const V *__restrict__ coef,
                const int32_t *__restrict__ nact, V *__restrict__ X, V *__restrict__ P, double2 *__restrict__ Xproj,
                const int64_t *__restrict__ proj_row, const RhsDesc *__restrict__ desc, int64_t ntot, int64_t M, int G,
                int ngroups, const int32_t *__restrict__ wshift, int64_t Mst, int R, const int2 *__restrict__ items)
{
    static_assert(TB % C == 0, "the block length must be a whole number of chunks");
    const int64_t y = items ? items[blockIdx.x].x : blockIdx.y;
    const int64_t j = y / ngroups;
    const int g = y % ngroups;
    const int64_t tile = items ? items[blockIdx.x].y : blockIdx.x;
    const int ns = blk[4 * j + 0];
    if (ns == 0) return;
    const int base = blk[4 * j + 1];
    const bool fresh = blk[4 * j + 2] != 0;
    const int64_t n = desc[j].n;
    const int64_t voff = desc[j].voff;
    const int64_t row0 = tile * 64;
    if (row0 >= n) return;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    const int lane = threadIdx.x % 64;
    const int64_t row = row0 + lane;
    const bool valid = row < n;
    const int64_t rowc = valid ? row : n - 1;
    // slots k0 .. k1-1 (at most 64); slot s holds shift kof(s)
    const int64_t k0 = (int64_t)g * G;
    const int64_t k1 = min(k0 + G, Mst);
    auto kof = [&](int64_t s) -> int64_t { return (PROJ && wshift) ? (int64_t)wshift[j * Mst + s] : s; };
    const bool act = lane < k1 - k0 && nact[j * M + kof(k0 + lane)] > 0;
    const uint64_t mask = __ballot(act);
    if (mask == 0) return;  // frozen group: leave before reading the history
    __shared__ V lr[TB * 64];
    for (int t = w; t < TB; t += FL_W)
        lr[t * 64 + lane] = (t < ns && valid) ? to_v<V>(ring[(int64_t)((base + t) % R) * ntot + voff + row])
                                              : to_v<V>(cmk(0, 0));
    __syncthreads();
    // this wave's slots: runs of NPW consecutive active slots, every FL_W-th run, from run w
    uint64_t mine = 0;
    {
        int rank = 0;
        for (uint64_t m = mask; m; m &= m - 1, ++rank)
            if ((rank / NPW) % FL_W == w) mine |= m & (~m + 1);
    }
    if (mine == 0) return;
    if constexpr (!PROJ) X += M * voff;
    P += Mst * voff;
    const int64_t prow = PROJ ? proj_row[j] : -1;
    // projection mode needs x_k only in the workgroup that holds the kept row (uniform test)
    const bool with_x = !PROJ || (prow >= row0 && prow < row0 + 64);
    // an opaque base keeps the compiler from hoisting the history reads out of the pair loop
    int lo = lane;
    asm volatile("" : "+v"(lo));
    const V *lrow = lr + lo;
    // the next NPW slots of this wave; a missing one (-1) repeats the first, unstored
    auto take = [&](int64_t (&sl)[NPW]) {
#pragma unroll
        for (int q = 0; q < NPW; ++q) {
            sl[q] = -1;
            if (mine) {
                sl[q] = k0 + __builtin_ctzll(mine);
                mine &= mine - 1;
            }
        }
    };
    auto fetch = [&](const int64_t (&sl)[NPW], V (&x)[NPW], V (&u)[NPW]) {
#pragma unroll
        for (int q = 0; q < NPW; ++q) {
            const int64_t s = sl[q] >= 0 ? sl[q] : sl[0];
            x[q] = to_v<V>(cmk(0, 0));
            u[q] = x[q];
            if (fresh) continue;
            u[q] = ld_nt(P + s * n + rowc);
            if constexpr (PROJ) {
                if (row == prow) x[q] = to_v<V>(Xproj[j * M + kof(s)]);
            } else {
                x[q] = ld_nt(X + s * n + rowc);
            }
        }
    };
    int64_t sn[NPW];
    V xn[NPW], un[NPW];
    take(sn);
    fetch(sn, xn, un);
    while (true) {
        int64_t sl[NPW];
        V x[NPW], u[NPW];
        const V *cf[NPW];
#pragma unroll
        for (int q = 0; q < NPW; ++q) {
            sl[q] = sn[q];
            x[q] = xn[q];
            u[q] = un[q];
            cf[q] = coef + (j * M + kof(sl[q] >= 0 ? sl[q] : sl[0])) * TB * 2;
        }
        const bool more = mine != 0;
        if (more) {
            take(sn);
            fetch(sn, xn, un);
        }
        if (with_x) flush_pair_steps<TB, C, NPW, V, true>(cf, lrow, x, u);
        else flush_pair_steps<TB, C, NPW, V, false>(cf, lrow, x, u);
        if (valid) {
#pragma unroll
            for (int q = 0; q < NPW; ++q) {
                if (sl[q] < 0) continue;
                st_nt(P + sl[q] * n + row, u[q]);
                if constexpr (PROJ) {
                    if (row == prow) Xproj[j * M + kof(sl[q])] = make_double2((double)x[q].x, (double)x[q].y);
                } else {
                    st_nt(X + sl[q] * n + row, x[q]);
                }
            }
        }
        if (!more) break;
    }
}

// ---------------------------------------------------------------------------------------
// Expanded form on the FP64 matrix cores (full solutions, FP64 storage).  Per pair the block is
//   x_out = x_in + gamma u_in + sum_s c_s r_s,   u_out = delta u_in + sum_s d_s r_s
// with the weights c_s, d_s of k_pair_scalars: for a 64-row tile and a group of up to 64 shifts
// of one rhs that is the complex product [pairs x T] . [T x 64 rows] of the weights with the
// residual history, formed with v_mfma_f64_16x16x4f64 and Gauss's three real products
// (Re = C_r R_r - C_i R_i, Im = (C_r + C_i)(R_r + R_i) - C_r R_r - C_i R_i), so 12 instead of
// 16 flops per pair, row and step.  The MFMA lane layout on gfx950 (checked on the device):
// A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k, D[i][j] in lane j + 16 (i % 4), element
// i / 4.  Here i is a pair, j a row and k a step: a lane's four results are one row of four
// pairs, so each result row of 16 lanes is one pair's 16 consecutive rows (256 B).
// A workgroup: eight waves, the history of its 64 rows in LDS (as in k_flush_lds); the group's
// active shifts are compacted and wave w takes active slots 16 (w % 4) .. + 15 on rows
// 32 (w / 4) .. + 31 (two 16-row MFMA blocks).  Frozen slots cost nothing, and a pair's result
// depends only on its own weights and the history, not on which slot or batch it sits in.
// ---------------------------------------------------------------------------------------
typedef double v4d __attribute__((ext_vector_type(4)));

template <int TB>
__global__ void __launch_bounds__(64 * FL_W)
    k_flush_mfma(const int32_t *__restrict__ blk, const double2 *__restrict__ ring, const double *__restrict__ coefx,
                 const int32_t *__restrict__ nact, double2 *__restrict__ X, double2 *__restrict__ P,
                 const RhsDesc *__restrict__ desc, int64_t ntot, int64_t M, int G, int ngroups, int R,
                 int64_t KM, const int2 *__restrict__ items)
{
    static_assert(TB % 4 == 0 && FL_W == 8, "four steps per MFMA, eight waves");
    constexpr int KS = TB / 4;
    const int64_t y = items ? items[blockIdx.x].x : blockIdx.y;
    const int64_t j = y / ngroups;
    const int g = y % ngroups;
    const int64_t tile = items ? items[blockIdx.x].y : blockIdx.x;
    const int ns = blk[4 * j + 0];
    if (ns == 0) return;
    const int base = blk[4 * j + 1];
    const bool fresh = blk[4 * j + 2] != 0;
    const int64_t n = desc[j].n;
    const int64_t voff = desc[j].voff;
    const int64_t row0 = tile * 64;
    if (row0 >= n) return;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    const int lane = threadIdx.x % 64;
    const int64_t k0 = (int64_t)g * G;
    const int64_t k1 = min(k0 + G, M);
    const bool act = lane < k1 - k0 && nact[j * M + k0 + lane] > 0;
    const uint64_t mask = __ballot(act);
    if (mask == 0) return;  // frozen group: leave before reading the history
    const int nactive = __popcll(mask);
    __shared__ double2 lr[TB * 64];
    __shared__ int slot_of[64];
    const bool valid_row = row0 + lane < n;
    for (int t = w; t < TB; t += FL_W)
        lr[t * 64 + lane] = (t < ns && valid_row) ? ring[(int64_t)((base + t) % R) * ntot + voff + row0 + lane]
                                                  : cmk(0, 0);
    if (w == 0 && act) slot_of[__popcll(mask & ((1ull << lane) - 1ull))] = lane;
    __syncthreads();
    const int pg = w & 3, rh = w >> 2;
    if (16 * pg >= nactive) return;  // no active slots for this wave
    // A operands: lane -> active slot 16 pg + (lane % 16), step 4 kb + lane / 16
    const int ia = 16 * pg + (lane & 15);
    const bool va = ia < nactive;
    const double *cp = coefx + (j * M + k0 + slot_of[va ? ia : 0]);
    v4d acc[2][6];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int q = 0; q < 6; ++q) acc[rb][q] = (v4d){0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
    for (int kb = 0; kb < KS; ++kb) {
        const int st = 4 * kb + (lane >> 4);
        const double *c = cp + (int64_t)(st * 6) * KM;
        double a[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) a[q] = va ? c[q * KM] : 0.0;
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            const double2 r = lr[st * 64 + rh * 32 + rb * 16 + (lane & 15)];
            const double br = r.x, bi = r.y, bs = r.x + r.y;
            acc[rb][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], br, acc[rb][0], 0, 0, 0);
            acc[rb][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1], bi, acc[rb][1], 0, 0, 0);
            acc[rb][2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[2], bs, acc[rb][2], 0, 0, 0);
            acc[rb][3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[3], br, acc[rb][3], 0, 0, 0);
            acc[rb][4] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[4], bi, acc[rb][4], 0, 0, 0);
            acc[rb][5] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[5], bs, acc[rb][5], 0, 0, 0);
        }
    }
    X += M * voff;
    P += M * voff;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
        const int64_t row = row0 + rh * 32 + rb * 16 + (lane & 15);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = 16 * pg + (lane >> 4) + 4 * v;
            if (row >= n || i >= nactive) continue;
            const int64_t slot = k0 + slot_of[i];
            const double *gd = coefx + (int64_t)(6 * TB) * KM + (j * M + slot);
            double2 x = cmk(0, 0), u = cmk(0, 0);
            if (!fresh) {
                x = ld_nt(X + slot * n + row);
                u = ld_nt(P + slot * n + row);
            }
            const double t1 = acc[rb][0][v], t2 = acc[rb][1][v], t3 = acc[rb][2][v];
            const double e1 = acc[rb][3][v], e2 = acc[rb][4][v], e3 = acc[rb][5][v];
            const double2 gu = cmul(make_double2(gd[0], gd[KM]), u), du = cmul(make_double2(gd[2 * KM], gd[3 * KM]), u);
            const double2 xo = make_double2(x.x + gu.x + (t1 - t2), x.y + gu.y + (t3 - t1 - t2));
            const double2 uo = make_double2(du.x + (e1 - e2), du.y + (e3 - e1 - e2));
            st_nt(X + slot * n + row, xo);
            st_nt(P + slot * n + row, uo);
        }
    }
}

template <int TB>
static hipError_t flush_mfma(const SolveDev &s, hipStream_t st)
{
    const int G = s.shifts_per_wg;
    if (G < 1 || G > 64 || s.precision != 0 || !s.X || s.Xproj || s.wshift || s.Mst != s.M)
        return hipErrorInvalidConfiguration;
    const int ng = (int)((s.M + G - 1) / G);
    if (s.K * ng > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    const dim3 g = s.it_upd ? dim3((unsigned)s.n_it_upd) : dim3((unsigned)(s.nblk * (WG / 64)), (unsigned)(s.K * ng));
    hipLaunchKernelGGL((k_flush_mfma<TB>), g, dim3(64 * FL_W), 0, st, s.blk, s.ring, (const double *)s.coefx, s.nact,
                       (double2 *)s.X, (double2 *)s.P, s.desc, s.ntot, s.M, G, ng, s.R, s.K * s.M, s.it_upd);
    return hipGetLastError();
}

template <int TB, int C, int NPW, typename V>
static hipError_t flush_lds(const SolveDev &s, hipStream_t st)
{
    const int G = s.shifts_per_wg;
    if (G < 1 || G > 64) return hipErrorInvalidConfiguration;
    const int ng = (int)((s.Mst + G - 1) / G);
    if (s.K * ng > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    const dim3 g = s.it_upd ? dim3((unsigned)s.n_it_upd) : dim3((unsigned)(s.nblk * (WG / 64)), (unsigned)(s.K * ng));
    const V *coef = (const V *)s.coef;
    if (s.Xproj)
        hipLaunchKernelGGL((k_flush_lds<TB, C, NPW, V, true>), g, dim3(64 * FL_W), 0, st, s.blk, s.ring, coef, s.nact,
                           (V *)nullptr, (V *)s.P, s.Xproj, s.proj_row, s.desc, s.ntot, s.M, G, ng, s.wshift, s.Mst,
                           s.R, s.it_upd);
    else
        hipLaunchKernelGGL((k_flush_lds<TB, C, NPW, V, false>), g, dim3(64 * FL_W), 0, st, s.blk, s.ring, coef, s.nact,
                           (V *)s.X, (V *)s.P, (double2 *)nullptr, (const int64_t *)nullptr, s.desc, s.ntot, s.M, G, ng,
                           (const int32_t *)nullptr, s.M, s.R, s.it_upd);
    return hipGetLastError();
}

template <int TB, int C, int NPW>
static hipError_t flush_tb_lds(const SolveDev &s, hipStream_t st)
{
    if (s.precision == 0) return flush_lds<TB, C, NPW, double2>(s, st);
    return flush_lds<TB, C, NPW, float2>(s, st);
}

template <int TB, typename V, int NP>
static hipError_t flush_v(const SolveDev &s, hipStream_t st)
{
    const int G = s.shifts_per_wg;
    const int ng = (int)((s.Mst + G - 1) / G);
    if (s.K * ng > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    const dim3 g = s.it_upd ? dim3((unsigned)s.n_it_upd) : dim3((unsigned)s.nblk, (unsigned)(s.K * ng));
    const V *coef = (const V *)s.coef;
    if (s.Xproj)
        hipLaunchKernelGGL((k_flush<TB, V, NP, true>), g, dim3(WG), 0, st, s.blk, s.ring, coef, s.nact, (V *)nullptr,
                           (V *)s.P, s.Xproj, s.proj_row, s.desc, s.ntot, s.M, G, ng, s.wshift, s.Mst, s.R, s.it_upd);
    else
        hipLaunchKernelGGL((k_flush<TB, V, NP, false>), g, dim3(WG), 0, st, s.blk, s.ring, coef, s.nact, (V *)s.X,
                           (V *)s.P, (double2 *)nullptr, (const int64_t *)nullptr, s.desc, s.ntot, s.M, G, ng,
                           (const int32_t *)nullptr, s.M, s.R, s.it_upd);
    return hipGetLastError();
}

// Short blocks (T <= 16): the residual history in registers, pairs in flight per thread by
// its size (4 registers per step in FP64, 2 in FP32).
template <int TB>
static hipError_t flush_tb(const SolveDev &s, hipStream_t st)
{
    if (s.precision == 0) return flush_v<TB, double2, (TB <= 16 ? 2 : 1)>(s, st);
    return flush_v<TB, float2, (TB <= 16 ? 4 : 2)>(s, st);
}

hipError_t launch_flush(const SolveDev &s, hipStream_t st)
{
    if (s.expanded) {
        switch (s.TB) {
        case 24: return flush_mfma<24>(s, st);
        case 32: return flush_mfma<32>(s, st);
        case 40: return flush_mfma<40>(s, st);
        case 48: return flush_mfma<48>(s, st);
        default: return hipErrorInvalidValue;
        }
    }
    switch (s.TB) {
    case 1: return flush_tb<1>(s, st);
    case 2: return flush_tb<2>(s, st);
    case 4: return flush_tb<4>(s, st);
    case 8: return flush_tb<8>(s, st);
    case 16: return flush_tb<16>(s, st);
    // long blocks: chunks of C steps of NPW pairs, C * NPW * 8 scalar registers per
    // coefficient buffer (two buffers); two pairs per wave share each history read
    case 24: return flush_tb_lds<24, 3, 2>(s, st);
    case 32: return flush_tb_lds<32, 4, 1>(s, st);
    case 40: return flush_tb_lds<40, 5, 1>(s, st);
    case 48: return flush_tb_lds<48, 3, 2>(s, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace scocg

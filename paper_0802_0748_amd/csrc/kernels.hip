// HIP kernels of the shifted-COCG solver (gfx950, wave64): seed iteration, shift scalars,
// end-of-block decisions, residuals and observables.  The deferred per-shift update is in
// flush.hip.
//
// Data layout in HBM (n rows, K right-hand sides, M shifts; see RhsDesc for mixed sizes):
//   seed vectors r (ring of 2 TB + 1 slots), q : one contiguous vector per rhs; p likewise, or
//                                             two rhs interleaved (see p_index)
//   per-shift vectors x_k, u_k                                : pair-major, FP64 or FP32 complex
//   H : 64-row slices, each slice stored column-slot-major (slot k of the 64 rows is
//       contiguous), FP64 values
// All reductions are fixed-order: every workgroup writes a partial and one workgroup sums
// the partials in index order, so results do not depend on scheduling and a rhs gives the
// same bits whether it is solved alone or in a batch.
#include "device_common.h"
#include "hubbard_rows.h"

namespace scocg {

// ---------------------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------------------
// Tree sums over the NT threads of a workgroup (sh holds NT entries); the result is in
// every thread.  Level s adds entry t + s to entry t for t < s; the levels down to s = 64 go
// through LDS with a barrier each, the last six inside the first wave by lane shuffles (lane t
// adds lane t + s, the same additions in the same order, without a barrier per level).
template <int NT = WG>
__device__ inline double2 block_sum2(double2 v, double2 *sh)
{
    static_assert(NT >= 128, "the LDS levels end at s = 64");
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = NT / 2; s >= 64; s >>= 1) {
        if (t < s) sh[t] = cadd(sh[t], sh[t + s]);
        __syncthreads();
    }
    if (t < 64) {
        double2 x = sh[t];
        for (int s = 32; s > 0; s >>= 1) x = cadd(x, make_double2(__shfl_down(x.x, s, 64), __shfl_down(x.y, s, 64)));
        if (t == 0) sh[0] = x;
    }
    __syncthreads();
    const double2 r = sh[0];
    __syncthreads();
    return r;
}

template <int NT = WG>
__device__ inline double block_sum1(double v, double *sh)
{
    static_assert(NT >= 128, "the LDS levels end at s = 64");
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = NT / 2; s >= 64; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    if (t < 64) {
        double x = sh[t];
        for (int s = 32; s > 0; s >>= 1) x += __shfl_down(x, s, 64);
        if (t == 0) sh[0] = x;
    }
    __syncthreads();
    const double r = sh[0];
    __syncthreads();
    return r;
}

// block_sum2 and block_sum1 of two values at once: each has its own tree, the same additions
// in the same order as alone, with one set of barriers for both.
template <int NT = WG>
__device__ inline void block_sum21(double2 &v2, double &v1, double2 *sh2, double *sh1)
{
    static_assert(NT >= 128, "the LDS levels end at s = 64");
    const int t = threadIdx.x;
    sh2[t] = v2;
    sh1[t] = v1;
    __syncthreads();
    for (int s = NT / 2; s >= 64; s >>= 1) {
        if (t < s) {
            sh2[t] = cadd(sh2[t], sh2[t + s]);
            sh1[t] += sh1[t + s];
        }
        __syncthreads();
    }
    if (t < 64) {
        double2 x = sh2[t];
        double y = sh1[t];
        for (int s = 32; s > 0; s >>= 1) {
            x = cadd(x, make_double2(__shfl_down(x.x, s, 64), __shfl_down(x.y, s, 64)));
            y += __shfl_down(y, s, 64);
        }
        if (t == 0) {
            sh2[0] = x;
            sh1[0] = y;
        }
    }
    __syncthreads();
    v2 = sh2[0];
    v1 = sh1[0];
    __syncthreads();
}

// block_sum2 of two values at once (each its own tree, the same additions in the same order).
template <int NT = WG>
__device__ inline void block_sum22(double2 &va, double2 &vb, double2 *sha, double2 *shb)
{
    static_assert(NT >= 128, "the LDS levels end at s = 64");
    const int t = threadIdx.x;
    sha[t] = va;
    shb[t] = vb;
    __syncthreads();
    for (int s = NT / 2; s >= 64; s >>= 1) {
        if (t < s) {
            sha[t] = cadd(sha[t], sha[t + s]);
            shb[t] = cadd(shb[t], shb[t + s]);
        }
        __syncthreads();
    }
    if (t < 64) {
        double2 x = sha[t], y = shb[t];
        for (int s = 32; s > 0; s >>= 1) {
            x = cadd(x, make_double2(__shfl_down(x.x, s, 64), __shfl_down(x.y, s, 64)));
            y = cadd(y, make_double2(__shfl_down(y.x, s, 64), __shfl_down(y.y, s, 64)));
        }
        if (t == 0) {
            sha[0] = x;
            shb[0] = y;
        }
    }
    __syncthreads();
    va = sha[0];
    vb = shb[0];
    __syncthreads();
}

__device__ inline double load_coherent(const double *p)
{
    unsigned long long v = __hip_atomic_load((const unsigned long long *)p, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
    return __longlong_as_double((long long)v);
}

// Thread 0 has written this block's partials.  Returns true (in every thread) in the block
// that arrives last for counter slot j; that block then sees every partial.
__device__ inline bool arrive_last(uint32_t *cnt, int64_t j, uint32_t nblk)
{
    __shared__ int is_last;
    if (threadIdx.x == 0) {
        __threadfence();
        uint32_t prev = atomicAdd(&cnt[j], 1u);
        is_last = (prev == nblk - 1) ? 1 : 0;
    }
    __syncthreads();
    bool last = is_last != 0;
    if (last) __threadfence();
    return last;
}

// Fixed-order sum of nblk complex partials by NT threads (result in all threads): thread t
// adds partials t, t + NT, t + 2 NT, ... in order, then the threads' sums are added as a tree.  COHERENT: the partials were written by other workgroups of the same launch
// (read past the caches with atomic loads); otherwise by an earlier launch (plain loads, which
// the compiler can issue many at a time).
// With plain loads a thread fetches 32 of its partials at a time (the sum order is unchanged),
// so a row count with tens of thousands of partials is not bound by one load's latency each.
static constexpr int SUM_BATCH = 32;

template <bool COHERENT, int NT = WG>
__device__ inline double2 sum_partials2(const double2 *part, int64_t nblk, double2 *sh)
{
    double2 acc = cmk(0, 0);
    int64_t b = threadIdx.x;
    if (!COHERENT) {
        for (; b + (SUM_BATCH - 1) * NT < nblk; b += SUM_BATCH * NT) {
            double2 v[SUM_BATCH];
#pragma unroll
            for (int u = 0; u < SUM_BATCH; ++u) v[u] = part[b + u * NT];
#pragma unroll
            for (int u = 0; u < SUM_BATCH; ++u) acc = cadd(acc, v[u]);
        }
    }
    for (; b < nblk; b += NT) {
        if (COHERENT) {
            const double *pp = (const double *)(part + b);
            acc = cadd(acc, cmk(load_coherent(pp), load_coherent(pp + 1)));
        } else {
            acc = cadd(acc, part[b]);
        }
    }
    return block_sum2<NT>(acc, sh);
}

template <bool COHERENT, int NT = WG>
__device__ inline double sum_partials1(const double *part, int64_t nblk, double *sh)
{
    double acc = 0;
    int64_t b = threadIdx.x;
    if (!COHERENT) {
        for (; b + (SUM_BATCH - 1) * NT < nblk; b += SUM_BATCH * NT) {
            double v[SUM_BATCH];
#pragma unroll
            for (int u = 0; u < SUM_BATCH; ++u) v[u] = part[b + u * NT];
#pragma unroll
            for (int u = 0; u < SUM_BATCH; ++u) acc += v[u];
        }
    }
    for (; b < nblk; b += NT) acc += COHERENT ? load_coherent(part + b) : part[b];
    return block_sum1<NT>(acc, sh);
}

// sum_partials2 and sum_partials1 (plain loads) of two partial arrays at once: each thread adds
// its partials of each array in the same order as alone, then block_sum21.
template <int NT = WG>
__device__ inline void sum_partials21(const double2 *part2, const double *part1, int64_t nblk, double2 *sh2,
                                      double *sh1, double2 &out2, double &out1)
{
    double2 acc2 = cmk(0, 0);
    double acc1 = 0;
    int64_t b = threadIdx.x;
    for (; b + (SUM_BATCH - 1) * NT < nblk; b += SUM_BATCH * NT) {
        double2 v2[SUM_BATCH];
        double v1[SUM_BATCH];
#pragma unroll
        for (int u = 0; u < SUM_BATCH; ++u) {
            v2[u] = part2[b + u * NT];
            v1[u] = part1[b + u * NT];
        }
#pragma unroll
        for (int u = 0; u < SUM_BATCH; ++u) {
            acc2 = cadd(acc2, v2[u]);
            acc1 += v1[u];
        }
    }
    for (; b < nblk; b += NT) {
        acc2 = cadd(acc2, part2[b]);
        acc1 += part1[b];
    }
    block_sum21<NT>(acc2, acc1, sh2, sh1);
    out2 = acc2;
    out1 = acc1;
}

// The per-rhs reductions of the seed iteration (alpha, beta) run with WG threads, or with
// RWG_BIG threads for a right-hand side of at least RED_BIG_ROWS rows (a Hubbard sector of ten
// million rows leaves tens of thousands of partials).  The choice depends on the rhs's own
// row count only, so a right-hand side sums in the same order alone or in any batch.
static constexpr int RWG_BIG = 1024;

__device__ inline bool red_big(const RhsDesc &d) { return d.n >= RED_BIG_ROWS; }

// Partial sums of a right-hand side's seed reductions: one per 256-row block of its own rows
// (slots past them belong to larger right-hand sides of the batch and are not read).
__device__ inline int64_t nparts(const RhsDesc &d) { return (d.n + WG - 1) / WG; }

__device__ inline void reset_counter(uint32_t *cnt, int64_t j)
{
    if (threadIdx.x == 0) __hip_atomic_store(&cnt[j], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline bool seed_running(const SeedState &st, int TB)
{
    return st.status == SEED_RUNNING && st.step < TB;
}

__device__ inline double2 *ring_slot(const SolveDev &s, int slot, const RhsDesc &d)
{
    return s.ring + (int64_t)slot * s.ntot + d.voff;
}

// Seed directions.  With two right-hand sides per SpMV thread (rhs 2i and 2i+1 share one
// matrix, so voff_{2i+1} = voff_{2i} + n) the pair is interleaved element by element from
// voff_{2i} on: one gather of 32 bytes serves both.  Otherwise p_j is the plain vector at voff_j.
__device__ inline int64_t p_index(const SolveDev &s, int64_t j, const RhsDesc &d, int64_t row)
{
    if (s.spmv_rb == 2) return d.voff - (j & 1) * d.n + 2 * row + (j & 1);
    return d.voff + row;
}

// ---------------------------------------------------------------------------------------
// initialisation: r_0 = b, p = 0, rho = b.b, ||b||, seed state
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(WG) k_init(SolveDev s, const double2 *__restrict__ B,
                                             const int64_t *__restrict__ unit_idx,
                                             const int32_t *__restrict__ seed_idx, int32_t limit)
{
    __shared__ double2 sh2[WG];
    __shared__ double sh1[WG];
    const int64_t j = blockIdx.y;
    const RhsDesc d = s.desc[j];
    const int64_t row = (int64_t)blockIdx.x * WG + threadIdx.x;
    double2 b = cmk(0, 0);
    if (row < d.n) {
        if (B) b = B[d.voff + row];
        else b = cmk(row == unit_idx[j] ? 1.0 : 0.0, 0.0);
        ring_slot(s, 0, d)[row] = b;
        s.p[p_index(s, j, d, row)] = cmk(0, 0);
    }
    double2 bb = block_sum2(cmul(b, b), sh2);
    double nn = block_sum1(cabs2(b), sh1);
    if (threadIdx.x == 0) {
        s.part2[j * s.nblk + blockIdx.x] = bb;
        s.part1[j * s.nblk + blockIdx.x] = nn;
    }
    if (!arrive_last(s.cnt, j, (uint32_t)gridDim.x)) return;
    double2 rho = sum_partials2<true>(s.part2 + j * s.nblk, gridDim.x, sh2);
    double nb = sqrt(sum_partials1<true>(s.part1 + j * s.nblk, gridDim.x, sh1));
    if (threadIdx.x == 0) {
        SeedState st;
        int sd = seed_idx[j];
        st.zs = s.z[sd];
        st.alpha_prev = cmk(1, 0);
        st.beta_prev = cmk(0, 0);
        st.rho = rho;
        st.a0 = cmk(1, 0);
        st.b0 = cmk(0, 0);
        st.inv_pt = cmk(1, 0);
        st.inv_ppt = cmk(1, 0);
        st.nb = nb;
        st.rnorm = nb;
        st.seed = sd;
        st.iter = 0;
        st.step = 0;
        st.base = 0;
        st.status = nb > 0 ? SEED_RUNNING : SEED_STOPPED;
        st.sw_target = -1;
        st.n_active = nb > 0 ? (int32_t)s.M : 0;
        st.switches = 0;
        st.limit = limit;
        st.sw_age = 0;
        s.seed[j] = st;
    }
    reset_counter(s.cnt, j);
}

__global__ void __launch_bounds__(WG) k_init_pairs(SolveDev s)
{
    const int64_t pair = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (pair >= s.K * s.M) return;
    const int64_t j = pair / s.M;
    const bool live = s.seed[j].nb > 0;
    s.pi[pair] = cmk(1, 0);
    s.pi_prev[pair] = cmk(1, 0);
    s.beta_k[pair] = cmk(0, 0);
    s.res[pair] = live ? 1.0 : 0.0;
    s.iters[pair] = 0;
    s.pstatus[pair] = live ? PAIR_NOCONV : PAIR_OK;
    s.active[pair] = live ? 1 : 0;
    s.nact[pair] = 0;
    if (s.Xproj) s.Xproj[pair] = cmk(0, 0);
    if (s.Uproj) s.Uproj[pair] = cmk(0, 0);
}

// ---------------------------------------------------------------------------------------
// One seed iteration is five launches, none of which needs a grid-wide fence (kernel
// boundaries order them):
//   k_pupd    p_n = r_n + beta_{n-1} p_{n-1}                      (elementwise, in place)
//   k_spmv    q = (z_s 1 - H) p_n;  partial sums of p_n.q         (RB right-hand sides per thread)
//   k_alpha   alpha_n = rho_n / (p_n.q)                           (one workgroup per rhs)
//   k_rupd    r_{n+1} = r_n - alpha_n q;  partial sums of r.r and |r|^2
//   k_beta    rho_{n+1}, ||r_{n+1}||, beta_n, convergence of the seed (one workgroup per rhs)
// ---------------------------------------------------------------------------------------
// RB right-hand sides per thread: with RB = 2 the interleaved pair (j0, j0+1) is read and
// written as one 32-byte element.
template <int RB>
__global__ void __launch_bounds__(WG) k_pupd(SolveDev s)
{
    int64_t gq = blockIdx.y, rbq = blockIdx.x;
    if (s.it_grp) {
        const int2 it = s.it_grp[blockIdx.x];
        if (it.x < 0) return;  // filler of an XCD set
        gq = it.x;
        rbq = it.y;
    }
    const int64_t j0 = gq * RB;
    SeedState st[RB];
    bool run[RB];
    bool any = false;
#pragma unroll
    for (int b = 0; b < RB; ++b) {
        run[b] = j0 + b < s.K;
        if (run[b]) {
            st[b] = s.seed[j0 + b];
            run[b] = seed_running(st[b], s.TB);
        }
        any |= run[b];
    }
    if (!any) return;
    const RhsDesc d = s.desc[j0];
    const int64_t row = rbq * WG + threadIdx.x;
    if (s.wproj) {
        // vector projection: also the partials of s_n = w . r_n (bilinear), one per 256 rows
        __shared__ double2 sh2[WG];
        if (rbq * WG >= d.n) return;  // uniform: past this rhs's rows
        double2 wr[RB];
        if (row < d.n) {
            double2 *p = s.p + p_index(s, j0, d, row);
#pragma unroll
            for (int b = 0; b < RB; ++b) {
                wr[b] = cmk(0, 0);
                if (run[b]) {
                    const RhsDesc db = s.desc[j0 + b];
                    const double2 r = ring_slot(s, (st[b].base + st[b].step) % s.R, db)[row];
                    p[b] = cfma(st[b].beta_prev, p[b], r);
                    wr[b] = cmul(s.wproj[db.voff + row], r);
                }
            }
        } else {
#pragma unroll
            for (int b = 0; b < RB; ++b) wr[b] = cmk(0, 0);
        }
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            if (!run[b]) continue;  // uniform across the workgroup
            const double2 v = block_sum2(wr[b], sh2);
            if (threadIdx.x == 0) s.part3[(j0 + b) * s.nblk + rbq] = v;
        }
        return;
    }
    if (row >= d.n) return;
    double2 *p = s.p + p_index(s, j0, d, row);
    double2 pv[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b) pv[b] = p[b];
#pragma unroll
    for (int b = 0; b < RB; ++b) {
        if (run[b]) {
            const double2 r = ring_slot(s, (st[b].base + st[b].step) % s.R, s.desc[j0 + b])[row];
            pv[b] = cfma(st[b].beta_prev, pv[b], r);
        }
    }
#pragma unroll
    for (int b = 0; b < RB; ++b)
        if (run[b]) p[b] = pv[b];
}

// Workgroups are dealt to the 8 XCDs round-robin by linear index.  With at least 8 groups of
// right-hand sides every row block of one group is placed on the same XCD, so its vectors are
// fetched into one L2 only: the 1-D grid has nblk * 8 * ceil(G / 8) workgroups and linear index
// L runs group 8 * ((L / 8) / nblk) + L % 8, row block (L / 8) % nblk.  With fewer groups the
// row blocks of each group are spread over all XCDs (group L / nblk, row block L % nblk).
__device__ inline bool xcd_group_block(int64_t nblk, int64_t G, int64_t &g, int64_t &rb)
{
    const int64_t L = blockIdx.x;
    if (G < 8) {
        g = L / nblk;
        rb = L % nblk;
        return g < G;
    }
    const int64_t t = L >> 3;
    g = 8 * (t / nblk) + (L & 7);
    rb = t % nblk;
    return g < G;
}

// Matrix arrays reached through a descriptor are global memory; saying so lets the compiler
// use global (not flat) loads, which wait on the vector-memory counter only.
template <typename T>
__device__ inline const __attribute__((address_space(1))) T *gptr(const T *p)
{
    return (const __attribute__((address_space(1))) T *)p;
}


// Row `row` of H p for the matrix-free Hubbard operator, for RB right-hand sides whose p at
// row c is pv[RB * c + b].  The terms are added in the column order of the stored matrix
// (up-spin hops to lower configurations, then the down-spin row with the diagonal in its
// place, then up-spin hops to higher configurations), so the sums are those of the stored
// matrix's product.  Diagonal: U sum_i n_i,up n_i,dn + V sum_i n_i n_i+1 (periodic).
// Hop entries and their gathers are fetched HUB_CHUNK at a time, so a row does not wait on
// one table load and one gather per term.
static constexpr int HUB_CHUNK = 8;

template <int RB>
__device__ inline void hubbard_row(const HubbardOp *hp, int64_t row, const double2 *pv, double (&ax)[RB],
                                   double (&ay)[RB])
{
    const HubbardOp h = *hp;
    // rows are below 2^31 (checked at upload): 32-bit division
    const uint32_t dd32 = (uint32_t)h.Dd;
    const int64_t iu = (uint32_t)row / dd32;
    const int64_t id = row - iu * h.Dd;
    const auto *up_ptr = gptr(h.up_ptr);
    const auto *up_hop = gptr(h.up_hop);
    const auto *dn_ptr = gptr(h.dn_ptr);
    const auto *dn_hop = gptr(h.dn_hop);
    const int32_t u0 = up_ptr[iu], u1 = up_ptr[iu + 1];
    const int32_t d0 = dn_ptr[id], d1 = dn_ptr[id + 1];
    const uint32_t cu = gptr(h.up_conf)[iu], cd = gptr(h.dn_conf)[id];
    double2 pd[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b) pd[b] = pv[(int64_t)RB * row + b];
    const int on = __popc(cu & cd);
    const int inter = __popc(cu & ring_next(cu, h.L)) + __popc(cd & ring_next(cd, h.L)) +
                      __popc(cu & ring_next(cd, h.L)) + __popc(cd & ring_next(cu, h.L));
    const double diag = h.U * (double)on + h.V * (double)inter;
    auto hop_val = [&](uint32_t e) { return (e >> 31) ? h.t : -h.t; };
    auto add = [&](double v, const double2 (&pc)[RB]) {
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            ax[b] = fma(v, pc[b].x, ax[b]);
            ay[b] = fma(v, pc[b].y, ay[b]);
        }
    };
    // up-spin hops in order; `low` selects those to lower configurations (a < iu), which
    // come first in the sorted list, else the rest
    int32_t k = u0;
    auto up_terms = [&](bool low) {
        while (k < u1) {
            uint32_t e[HUB_CHUNK];
            bool ok[HUB_CHUNK];
            double2 pc[HUB_CHUNK][RB];
#pragma unroll
            for (int m = 0; m < HUB_CHUNK; ++m) {
                e[m] = (k + m < u1) ? up_hop[k + m] : 0xffffffffu;
                const int64_t a = e[m] & 0x7fffffffu;
                ok[m] = k + m < u1 && (!low || a < iu);
                if (ok[m]) {
#pragma unroll
                    for (int b = 0; b < RB; ++b) pc[m][b] = pv[(int64_t)RB * (a * h.Dd + id) + b];
                }
            }
            int used = 0;
#pragma unroll
            for (int m = 0; m < HUB_CHUNK; ++m) {
                if (ok[m] && used == m) {
                    add(hop_val(e[m]), pc[m]);
                    ++used;
                }
            }
            k += used;
            if (used < HUB_CHUNK) break;
        }
    };
    up_terms(true);
    // the down-spin row with the diagonal at its place (before the first hop to a higher index)
    bool diag_done = false;
    for (int32_t m0 = d0; m0 < d1; m0 += HUB_CHUNK) {
        uint32_t e[HUB_CHUNK];
        double2 pc[HUB_CHUNK][RB];
#pragma unroll
        for (int m = 0; m < HUB_CHUNK; ++m) {
            e[m] = (m0 + m < d1) ? dn_hop[m0 + m] : 0u;
            if (m0 + m < d1) {
                const int64_t bcol = e[m] & 0x7fffffffu;
#pragma unroll
                for (int b = 0; b < RB; ++b) pc[m][b] = pv[(int64_t)RB * (iu * h.Dd + bcol) + b];
            }
        }
#pragma unroll
        for (int m = 0; m < HUB_CHUNK; ++m) {
            if (m0 + m < d1) {
                if (!diag_done && (int64_t)(e[m] & 0x7fffffffu) > id) {
                    add(diag, pd);
                    diag_done = true;
                }
                add(hop_val(e[m]), pc[m]);
            }
        }
    }
    if (!diag_done) add(diag, pd);
    up_terms(false);
}

// LDS-tiled matrix-free Hubbard product: one workgroup per (up-spin configuration iu, rhs).
// The block p[iu, :] (the rows that share iu) is staged in LDS, so the down-spin hops read
// LDS; the up-spin hops of iu are the same for every row of the block and read contiguous
// stretches p[a, :].  Each row adds its terms in the stored matrix's column order (q equals
// the stored product bit for bit); the workgroup's partial of p.q goes to slot iu, and the
// slots past the last configuration are cleared.
static constexpr int HUB_WG = 1024;

__global__ void __launch_bounds__(HUB_WG) k_spmv_hub_lds(SolveDev s)
{
    __shared__ double2 pl[HUB_LDS_MAX];
    __shared__ double2 sh2[HUB_WG];
    const int64_t j = blockIdx.y;
    const SeedState st = s.seed[j];
    if (!seed_running(st, s.TB)) return;
    const RhsDesc d = s.desc[j];
    if (!d.hub) return;
    const HubbardOp h = *d.hub;
    const int64_t Dd = h.Dd;
    const int64_t Du = d.n / Dd;
    const int64_t iu = blockIdx.x;
    if (iu >= Du) return;
    // p of this rhs at row c is pv[RB * c] (RB = 2: interleaved with its partner)
    const int RB = s.spmv_rb;
    const double2 *pv = s.p + p_index(s, j, d, 0);
    const int64_t r0 = iu * Dd;
    for (int64_t c = threadIdx.x; c < Dd; c += HUB_WG) pl[c] = pv[(int64_t)RB * (r0 + c)];
    __syncthreads();
    const auto *up_ptr = gptr(h.up_ptr);
    const auto *up_hop = gptr(h.up_hop);
    const auto *dn_ptr = gptr(h.dn_ptr);
    const auto *dn_hop = gptr(h.dn_hop);
    const int32_t u0 = up_ptr[iu], u1 = up_ptr[iu + 1];
    // up-spin hops to lower configurations come first in the sorted list
    int32_t usplit = u0;
    while (usplit < u1 && (int64_t)(up_hop[usplit] & 0x7fffffffu) < iu) ++usplit;
    const uint32_t cu = gptr(h.up_conf)[iu];
    auto hop_val = [&](uint32_t e) { return (e >> 31) ? h.t : -h.t; };
    // Rows of this thread: id = threadIdx.x + i * HUB_WG.  The loops over hops run outside the
    // loop over rows, so the independent loads of a thread's rows are in flight together;
    // each row's own sum still takes its terms in column order.
    constexpr int RPT = (int)((HUB_LDS_MAX + HUB_WG - 1) / HUB_WG);
    double ax[RPT], ay[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        ax[i] = 0;
        ay[i] = 0;
    }
    auto up_range = [&](int32_t k0, int32_t k1) {
        for (int32_t k = k0; k < k1; ++k) {
            const uint32_t e = up_hop[k];  // the same hop for every row of the block
            const double v = hop_val(e);
            const double2 *pa = pv + (int64_t)RB * ((int64_t)(e & 0x7fffffffu) * Dd);
            double2 pc[RPT];
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                const int64_t id = threadIdx.x + (int64_t)i * HUB_WG;
                if (id < Dd) pc[i] = pa[(int64_t)RB * id];
            }
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                const int64_t id = threadIdx.x + (int64_t)i * HUB_WG;
                if (id < Dd) {
                    ax[i] = fma(v, pc[i].x, ax[i]);
                    ay[i] = fma(v, pc[i].y, ay[i]);
                }
            }
        }
    };
    up_range(u0, usplit);
    // the down-spin row of each row from LDS, with the diagonal at its place
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int64_t id = threadIdx.x + (int64_t)i * HUB_WG;
        if (id >= Dd) continue;
        const uint32_t cd = gptr(h.dn_conf)[id];
        const int on = __popc(cu & cd);
        const int inter = __popc(cu & ring_next(cu, h.L)) + __popc(cd & ring_next(cd, h.L)) +
                          __popc(cu & ring_next(cd, h.L)) + __popc(cd & ring_next(cu, h.L));
        const double diag = h.U * (double)on + h.V * (double)inter;
        const double2 pd = pl[id];
        bool diag_done = false;
        const int32_t d0 = dn_ptr[id], d1 = dn_ptr[id + 1];
        for (int32_t m0 = d0; m0 < d1; m0 += HUB_CHUNK) {
            uint32_t e[HUB_CHUNK];
#pragma unroll
            for (int m = 0; m < HUB_CHUNK; ++m) e[m] = (m0 + m < d1) ? dn_hop[m0 + m] : 0u;
#pragma unroll
            for (int m = 0; m < HUB_CHUNK; ++m) {
                if (m0 + m < d1) {
                    const int64_t b = e[m] & 0x7fffffffu;
                    if (!diag_done && b > id) {
                        ax[i] = fma(diag, pd.x, ax[i]);
                        ay[i] = fma(diag, pd.y, ay[i]);
                        diag_done = true;
                    }
                    const double2 pc = pl[b];
                    const double v = hop_val(e[m]);
                    ax[i] = fma(v, pc.x, ax[i]);
                    ay[i] = fma(v, pc.y, ay[i]);
                }
            }
        }
        if (!diag_done) {
            ax[i] = fma(diag, pd.x, ax[i]);
            ay[i] = fma(diag, pd.y, ay[i]);
        }
    }
    up_range(usplit, u1);
    double2 pq = cmk(0, 0);
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int64_t id = threadIdx.x + (int64_t)i * HUB_WG;
        if (id >= Dd) continue;
        const double2 pd = pl[id];
        const double2 qv = cfma(st.zs, pd, make_double2(-ax[i], -ay[i]));
        s.q[d.voff + r0 + id] = qv;
        pq = cadd(pq, cmul(pd, qv));
    }
    pq = block_sum2<HUB_WG>(pq, sh2);
    if (threadIdx.x == 0) {
        s.part2[j * s.nblk + iu] = pq;
        for (int64_t b = Du + iu; b < s.nblk; b += Du) s.part2[j * s.nblk + b] = cmk(0, 0);
    }
}

// Slots of a slice processed per batch: the column and value loads of SPMV_CHUNK slots are
// issued together, then their gathers, so each wave has many loads in flight.
static constexpr int SPMV_CHUNK = 8;
static constexpr int SPMV_TAIL = 4;

// q = (z_s 1 - H) p for RB right-hand sides that share one matrix (consecutive rhs j0 .. j0+RB-1):
// the column and value of each slot are loaded once and serve all RB gathers.  The products
// are summed in slot order in every configuration, so a rhs gets the same bits alone or in
// a batch.
// HUB: the instance for right-hand sides with a matrix-free Hubbard operator (a separate
// kernel, so the stored-matrix instance keeps its small register footprint); each instance
// leaves the other kind's right-hand sides alone.
template <int RB, bool HUB>
__global__ void __launch_bounds__(WG) k_spmv(SolveDev s)
{
    __shared__ double2 sh2[WG];
    __shared__ double2 sh2b[RB > 1 ? WG : 1];
    int64_t g, rb;
    if (s.it_grp) {
        const int2 it = s.it_grp[blockIdx.x];
        if (it.x < 0) return;  // filler of an XCD set
        g = it.x;
        rb = it.y;
    } else if (!xcd_group_block(s.nblk, (s.K + RB - 1) / RB, g, rb)) {
        return;
    }
    const int64_t j0 = g * RB;
    bool run[RB];
    SeedState st[RB];
    bool any = false;
#pragma unroll
    for (int b = 0; b < RB; ++b) {
        run[b] = j0 + b < s.K;
        if (run[b]) {
            st[b] = s.seed[j0 + b];
            run[b] = seed_running(st[b], s.TB);
        }
        any |= run[b];
    }
    if (!any) return;
    const RhsDesc d = s.desc[j0];
    if ((d.hub != nullptr) != HUB) return;
    if (rb * WG >= d.n) return;  // past this right-hand side's rows (its partials end before)
    const int lane = threadIdx.x & 63;
    // one 64-row slice per wave (wave-uniform, so its bookkeeping lives in scalar registers)
    const int64_t slice = rb * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t row = slice * 64 + lane;
    // p of rhs j0 + b at row c is pv[RB * c + b] (interleaved pair, or one plain vector); the
    // gathers of an idle partner (odd K, or a paused seed) read valid memory and are not used
    const double2 *pv = s.p + p_index(s, j0, d, 0);
    double ax[RB], ay[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b) {
        ax[b] = 0;
        ay[b] = 0;
    }
    if (HUB) {
        if (row < d.n) hubbard_row<RB>(d.hub, row, pv, ax, ay);
    } else if (slice < d.nslices) {
        const int64_t off = gptr(d.slice_ptr)[slice];
        const int w = gptr(d.slice_w)[slice];
        const auto *colp = gptr(d.ell_col) + off + lane;
        const auto *valp = gptr(d.ell_val) + off + lane;
        int k = 0;
        for (; k + SPMV_CHUNK <= w; k += SPMV_CHUNK) {
            int c[SPMV_CHUNK];
            double v[SPMV_CHUNK];
#pragma unroll
            for (int u = 0; u < SPMV_CHUNK; ++u) {
                c[u] = colp[(int64_t)(k + u) * 64];
                v[u] = valp[(int64_t)(k + u) * 64];
            }
            double2 pc[SPMV_CHUNK][RB];
#pragma unroll
            for (int u = 0; u < SPMV_CHUNK; ++u)
#pragma unroll
                for (int b = 0; b < RB; ++b) pc[u][b] = pv[(int64_t)RB * c[u] + b];
#pragma unroll
            for (int u = 0; u < SPMV_CHUNK; ++u)
#pragma unroll
                for (int b = 0; b < RB; ++b) {
                    ax[b] = fma(v[u], pc[u][b].x, ax[b]);
                    ay[b] = fma(v[u], pc[u][b].y, ay[b]);
                }
        }
        // the last w - k (< SPMV_CHUNK) slots, SPMV_TAIL at a time: their loads are also issued
        // together (the count is the same for the whole wave), then added in slot order
        for (; k < w; k += SPMV_TAIL) {
            const int rem = w - k;
            int c[SPMV_TAIL];
            double v[SPMV_TAIL];
#pragma unroll
            for (int u = 0; u < SPMV_TAIL; ++u) {
                c[u] = 0;
                v[u] = 0.0;
                if (u < rem) {
                    c[u] = colp[(int64_t)(k + u) * 64];
                    v[u] = valp[(int64_t)(k + u) * 64];
                }
            }
            double2 pc[SPMV_TAIL][RB];
#pragma unroll
            for (int u = 0; u < SPMV_TAIL; ++u)
#pragma unroll
                for (int b = 0; b < RB; ++b) pc[u][b] = u < rem ? pv[(int64_t)RB * c[u] + b] : cmk(0, 0);
#pragma unroll
            for (int u = 0; u < SPMV_TAIL; ++u)
                if (u < rem)
#pragma unroll
                    for (int b = 0; b < RB; ++b) {
                        ax[b] = fma(v[u], pc[u][b].x, ax[b]);
                        ay[b] = fma(v[u], pc[u][b].y, ay[b]);
                    }
        }
    }
    double2 pq[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b) {
        pq[b] = cmk(0, 0);
        if (run[b] && slice < d.nslices && row < d.n) {
            const double2 pr = pv[RB * row + b];
            const double2 qv = cfma(st[b].zs, pr, make_double2(-ax[b], -ay[b]));
            s.q[s.desc[j0 + b].voff + row] = qv;
            pq[b] = cmul(pr, qv);
        }
    }
    // run[] is uniform across the workgroup; both partials of a running pair share the barriers
    bool both = false;
    if constexpr (RB == 2) {
        both = run[0] && run[1];
        if (both) block_sum22(pq[0], pq[1], sh2, sh2b);
    }
    if (!both)
#pragma unroll
        for (int b = 0; b < RB; ++b)
            if (run[b]) pq[b] = block_sum2(pq[b], sh2);
    if (threadIdx.x == 0)
#pragma unroll
        for (int b = 0; b < RB; ++b)
            if (run[b]) s.part2[(j0 + b) * s.nblk + rb] = pq[b];
}

template <int NT>
__global__ void __launch_bounds__(NT) k_alpha(SolveDev s)
{
    __shared__ double2 sh2[NT];
    const int64_t j = blockIdx.x;
    const SeedState st = s.seed[j];
    if (!seed_running(st, s.TB)) return;
    if (red_big(s.desc[j]) != (NT == RWG_BIG)) return;
    const double2 tot = sum_partials2<false, NT>(s.part2 + j * s.nblk, nparts(s.desc[j]), sh2);
    if (s.wproj) {
        const double2 sn = sum_partials2<false, NT>(s.part3 + j * s.nblk, nparts(s.desc[j]), sh2);
        if (threadIdx.x == 0) s.shist[j * s.TB + st.step] = sn;
    }
    if (threadIdx.x == 0) {
        if (cis0(tot) || cis0(st.rho)) s.seed[j].status = SEED_BREAKDOWN;
        else s.ahist[j * s.TB + st.step] = cdiv(st.rho, tot);
    }
}

__global__ void __launch_bounds__(WG) k_rupd(SolveDev s)
{
    __shared__ double2 sh2[WG];
    __shared__ double sh1[WG];
    int64_t j = blockIdx.y, rb = blockIdx.x;
    if (s.it_rhs) {
        const int2 it = s.it_rhs[blockIdx.x];
        j = it.x;
        rb = it.y;
    }
    const SeedState st = s.seed[j];
    if (!seed_running(st, s.TB)) return;
    const RhsDesc d = s.desc[j];
    if (rb * WG >= d.n) return;  // past this right-hand side's rows
    const int64_t row = rb * WG + threadIdx.x;
    const int slot = (st.base + st.step) % s.R;
    const int nslot = (slot + 1) % s.R;
    const double2 a = s.ahist[j * s.TB + st.step];
    double2 rr = cmk(0, 0);
    double nn = 0;
    if (row < d.n) {
        const double2 r = ring_slot(s, slot, d)[row];
        const double2 q = s.q[d.voff + row];
        const double2 rn = cfma(make_double2(-a.x, -a.y), q, r);
        ring_slot(s, nslot, d)[row] = rn;
        rr = cmul(rn, rn);
        nn = cabs2(rn);
    }
    block_sum21(rr, nn, sh2, sh1);
    if (threadIdx.x == 0) {
        s.part2[j * s.nblk + rb] = rr;
        s.part1[j * s.nblk + rb] = nn;
    }
}

template <int NT>
__global__ void __launch_bounds__(NT) k_beta(SolveDev s)
{
    __shared__ double2 sh2[NT];
    __shared__ double sh1[NT];
    const int64_t j = blockIdx.x;
    const SeedState st = s.seed[j];
    if (!seed_running(st, s.TB)) return;
    if (red_big(s.desc[j]) != (NT == RWG_BIG)) return;
    const int64_t np = nparts(s.desc[j]);
    double2 rho_new;
    double rn2;
    sum_partials21<NT>(s.part2 + j * s.nblk, s.part1 + j * s.nblk, np, sh2, sh1, rho_new, rn2);
    const double rnorm = sqrt(rn2);
    if (threadIdx.x == 0) {
        const double2 a = s.ahist[j * s.TB + st.step];
        const double2 beta = cdiv(rho_new, st.rho);
        s.bhist[j * s.TB + st.step] = beta;
        s.rnhist[j * s.TB + st.step] = rnorm;
        SeedState *w = s.seed + j;
        w->alpha_prev = a;
        w->beta_prev = beta;
        w->rho = rho_new;
        w->rnorm = rnorm;
        const int32_t it = st.iter + 1;
        w->iter = it;
        w->step = st.step + 1;
        if (it >= st.limit) w->status = SEED_LIMIT;
        else if (!s.fixed && s.switching && rnorm / st.nb < s.tol) w->status = SEED_PAUSED;
    }
}

// ---------------------------------------------------------------------------------------
// shift scalars for the steps of the finished block (one thread per (rhs, shift) pair):
//   pi_{n+1} = (1 + alpha_n sigma) pi_n + (alpha_n beta_{n-1} / alpha_{n-1}) (pi_n - pi_{n-1})
//   alpha^k_n = (pi_n / pi_{n+1}) alpha_n,  beta^k_n = (pi_n / pi_{n+1})^2 beta_n
// Convergence of the pair: ||r_{n+1}|| / (|pi_{n+1}| ||b||) < tol.
//
// The vector update is carried out on the scaled direction u^k_n = pi_n p^k_n, for which
//   u^k_n = r_n + b'_n u^k_{n-1},   x^k_{n+1} = x^k_n + a'_n u^k_n,
//   a'_n = alpha^k_n / pi_n = alpha_n / pi_{n+1},
//   b'_n = beta^k_{n-1} pi_n / pi_{n-1} = beta_{n-1} pi_{n-1} / pi_n
// (two complex multiply-adds per step instead of three for p^k directly).  This thread
// writes (a'_n, b'_n) for every step of the block in which the pair is still active.
// ---------------------------------------------------------------------------------------
template <typename V>
__device__ inline unsigned long long pair_scalars_one(const SolveDev &s, int64_t pair, unsigned long long &flops)
{
    flops = 0ull;
    const int64_t j = pair / s.M, k = pair % s.M;
    const SeedState st = s.seed[j];
    const int ns = st.step;
    if (!s.active[pair] || ns == 0) {
        s.nact[pair] = 0;
        return 0ull;
    }
    const double2 sig = csub(s.z[s.zper ? j : k], st.zs);
    double2 ap = st.a0, bp = st.b0;
    double2 pi = s.pi[pair], pip = s.pi_prev[pair], bk = s.beta_k[pair];
    double res = s.res[pair];
    int act = 1, status = s.pstatus[pair], na = 0, iters = s.iters[pair];
    V *cf = (V *)s.coef + pair * (int64_t)s.TB * 2;
    for (int t = 0; t < ns; ++t) {
        const double2 a = s.ahist[j * s.TB + t];
        const double2 b = s.bhist[j * s.TB + t];
        const double2 c1 = cmul(cadd(cmk(1, 0), cmul(a, sig)), pi);
        const double2 c2 = cmul(cdiv(cmul(a, bp), ap), csub(pi, pip));
        const double2 pin = cadd(c1, c2);
        if (cis0(pin)) {
            status = PAIR_BREAKDOWN;
            act = 0;
            break;
        }
        const double2 ratio = cdiv(pi, pin);
        cf[2 * t + 0] = to_v<V>(cdiv(a, pin));
        cf[2 * t + 1] = to_v<V>(cmul(bp, cdiv(pip, pi)));
        bk = cmul(cmul(ratio, ratio), b);
        pip = pi;
        pi = pin;
        na = t + 1;
        iters = st.iter - ns + t + 1;
        res = s.rnhist[j * s.TB + t] / (sqrt(cabs2(pi)) * st.nb);
        ap = a;
        bp = b;
        if (!s.fixed && res < s.tol) {
            act = 0;
            status = PAIR_OK;
            break;
        }
    }
    s.pi[pair] = pi;
    s.pi_prev[pair] = pip;
    s.beta_k[pair] = bk;
    s.res[pair] = res;
    s.iters[pair] = iters;
    s.pstatus[pair] = status;
    s.active[pair] = act;
    s.nact[pair] = na;
    if (na == 0) return 0ull;
    if (s.wproj) {
        // vector projection: <w|x_k> and <w|u_k> of every pair follow the block's steps with
        // s_t = w . r_t in place of r_t (the update is linear); a stored direction still
        // gets its full u_k below, for a seed switch
        V x = to_v<V>(s.Xproj[pair]), u = to_v<V>(s.Uproj[pair]);
        for (int t = 0; t < na; ++t) {
            u = cfma(cf[2 * t + 1], u, to_v<V>(s.shist[j * s.TB + t]));
            x = cfma(cf[2 * t + 0], u, x);
        }
        s.Xproj[pair] = make_double2((double)x.x, (double)x.y);
        s.Uproj[pair] = make_double2((double)u.x, (double)u.y);
        if (s.wslot && s.wslot[pair] < 0) return 0ull;
    } else if (s.wslot && s.wslot[pair] < 0) {
        // no stored direction: carry x_k and u_k at the kept row only, with the same
        // arithmetic the deferred update applies to a stored direction
        const int64_t at = s.desc[j].voff + s.proj_row[j];
        V x = to_v<V>(s.Xproj[pair]), u = to_v<V>(s.Uproj[pair]);
        for (int t = 0; t < na; ++t) {
            const V r = to_v<V>(s.ring[(int64_t)((st.base + t) % s.R) * s.ntot + at]);
            u = cfma(cf[2 * t + 1], u, r);
            x = cfma(cf[2 * t + 0], u, x);
        }
        s.Xproj[pair] = make_double2((double)x.x, (double)x.y);
        s.Uproj[pair] = make_double2((double)u.x, (double)u.y);
        return 0ull;
    }
    // Steps past the pair's last one are padded with a' = 0, b' = 1, which leaves x_k
    // unchanged (and u_k too while the residual history is zero there), so the deferred
    // update runs every step without a per-pair branch.
    for (int t = na; t < s.TB; ++t) {
        cf[2 * t + 0] = to_v<V>(cmk(0, 0));
        cf[2 * t + 1] = to_v<V>(cmk(1, 0));
    }
    if (sizeof(V) == sizeof(double2) && s.expanded) {
        // The block's steps unrolled (u_in, x_in the values at the block's start):
        //   u_out = delta u_in + sum_s d_s r_s,   x_out = x_in + gamma u_in + sum_s c_s r_s,
        //   d_s = prod_{q=s+1}^{T-1} b'_q,  c_s = sum_{t>=s} a'_t prod_{q=s+1}^{t} b'_q,
        // by the backward recurrences c_s = a'_s + b'_{s+1} c_{s+1}, d_s = b'_{s+1} d_{s+1}
        // (c_{T-1} = a'_{T-1}, d_{T-1} = 1), gamma = b'_0 c_0, delta = b'_0 d_0.  Padded steps
        // (a' = 0, b' = 1) give c_s = 0, d_s = 1, as the step form does.
        // Layout [6 TB + 4][K M], pair fastest: the threads of a wave write consecutive pairs.
        const double2 *cfd = (const double2 *)cf;
        const int64_t KM = s.K * s.M;
        double *cx = s.coefx + pair;
        double2 c = cfd[2 * (s.TB - 1) + 0], d = cmk(1, 0);
        for (int t = s.TB - 1; t >= 0; --t) {
            if (t < s.TB - 1) {
                const double2 bn = cfd[2 * (t + 1) + 1];
                c = cadd(cfd[2 * t + 0], cmul(bn, c));
                d = cmul(bn, d);
            }
            double *e = cx + (int64_t)(6 * t) * KM;
            e[0 * KM] = c.x;
            e[1 * KM] = c.y;
            e[2 * KM] = c.x + c.y;
            e[3 * KM] = d.x;
            e[4 * KM] = d.y;
            e[5 * KM] = d.x + d.y;
        }
        const double2 b0 = cfd[1];
        const double2 gam = cmul(b0, c), del = cmul(b0, d);
        double *e = cx + (int64_t)(6 * s.TB) * KM;
        e[0 * KM] = gam.x;
        e[1 * KM] = gam.y;
        e[2 * KM] = del.x;
        e[3 * KM] = del.y;
    }
    // algorithmic bytes of this pair's deferred update: u_k (and x_k unless projected)
    // written once, and read once unless this is the first block
    const unsigned long long esz = s.precision == 0 ? 16ull : 8ull;
    const unsigned long long nv = s.X ? 2ull : 1ull;
    const unsigned long long rw = (st.iter - ns == 0) ? 1ull : 2ull;
    // algorithmic flops: the pair's own steps (not the padding), two complex multiply-adds
    // (16 flops) per row and step, one (8) where only u_k is stored
    flops = (unsigned long long)na * 8ull * nv * (unsigned long long)s.desc[j].n;
    return nv * rw * esz * (unsigned long long)s.desc[j].n;
}

template <typename V>
__global__ void __launch_bounds__(WG) k_pair_scalars(SolveDev s)
{
    __shared__ unsigned long long shb[WG], shf[WG];
    __shared__ unsigned int shc[WG];
    const int64_t pair = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (pair < s.K * s.M && pair % s.M == 0) {
        // what the deferred update of this block needs, fixed before the block ends
        const int64_t j = pair / s.M;
        const SeedState st = s.seed[j];
        s.blk[4 * j + 0] = st.step;
        s.blk[4 * j + 1] = st.base;
        s.blk[4 * j + 2] = st.iter == st.step ? 1 : 0;
    }
    unsigned long long f = 0ull;
    const unsigned long long b = pair < s.K * s.M ? pair_scalars_one<V>(s, pair, f) : 0ull;
    shb[threadIdx.x] = b;
    shf[threadIdx.x] = b > 0 ? f : 0ull;
    shc[threadIdx.x] = b > 0 ? 1u : 0u;
    __syncthreads();
    for (int h = WG / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            shb[threadIdx.x] += shb[threadIdx.x + h];
            shf[threadIdx.x] += shf[threadIdx.x + h];
            shc[threadIdx.x] += shc[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && shc[0] > 0) {
        atomicAdd(&s.stats[0], shb[0]);
        atomicAdd(&s.stats[1], (unsigned long long)shc[0]);
        atomicAdd(&s.stats[2], shf[0]);
    }
}

// ---------------------------------------------------------------------------------------
// End of block, one workgroup per rhs: stop / switch decisions (Sec. 3.3 seed switching).
// The new seed t is the active shift with the largest residual (lowest index on ties);
// pi_k <- pi_k / pi_t, pi_{k,prev} <- pi_{k,prev} / pi_{t,prev}, alpha_prev <- alpha^t_n,
// beta_prev <- beta^t_n, z_s <- z_t.
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(WG) k_block_finalize(SolveDev s)
{
    __shared__ int sh_cnt[WG];
    __shared__ int sh_brk[WG];
    __shared__ double sh_res[WG];
    __shared__ int sh_idx[WG];
    __shared__ int dec_switch, dec_brk;
    const int64_t j = blockIdx.x;
    const SeedState st = s.seed[j];
    const int tid = threadIdx.x;
    int cnt = 0, brk = 0, bi = -1;
    double br = -1;
    for (int64_t k = tid; k < s.M; k += WG) {
        const int64_t pair = j * s.M + k;
        if (s.active[pair]) {
            cnt++;
            const double r = s.res[pair];
            // a switch needs the new seed's full direction
            if (r > br && (!s.wslot || s.wslot[pair] >= 0)) {
                br = r;
                bi = (int)k;
            }
        }
        if (s.pstatus[pair] == PAIR_BREAKDOWN) brk = 1;
    }
    sh_cnt[tid] = cnt;
    sh_brk[tid] = brk;
    sh_res[tid] = br;
    sh_idx[tid] = bi;
    __syncthreads();
    for (int h = WG / 2; h > 0; h >>= 1) {
        if (tid < h) {
            sh_cnt[tid] += sh_cnt[tid + h];
            sh_brk[tid] |= sh_brk[tid + h];
            const double r2 = sh_res[tid + h];
            const int i2 = sh_idx[tid + h];
            if (i2 >= 0 && (r2 > sh_res[tid] || (r2 == sh_res[tid] && (sh_idx[tid] < 0 || i2 < sh_idx[tid])))) {
                sh_res[tid] = r2;
                sh_idx[tid] = i2;
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        const int n_active = sh_cnt[0];
        SeedState w = st;
        int sw = -1, mb = 0;
        if (st.status == SEED_STOPPED) {
            // finished earlier
        } else if (n_active == 0) {
            w.status = SEED_STOPPED;  // every pair has its own final status
        } else if (st.status == SEED_BREAKDOWN || sh_brk[0]) {
            w.status = SEED_STOPPED;  // breakdown ends every pair still active
            mb = 1;
        } else if (st.status == SEED_PAUSED) {
            sw = sh_idx[0];
            if (sw < 0) {
                // no stored direction is left to switch to: iterating the converged seed further
                // would let rounding break the collinearity of the residuals, so the pairs still
                // active stop here, unconverged
                w.status = SEED_STOPPED;
                mb = 2;
            } else if (sw == st.seed) {
                w.status = SEED_RUNNING;
            } else {
                // the scalars switch now; the vectors once this block's update is done
                w.status = SEED_SWITCH;
                w.sw_age = 0;
            }
        } else if (st.status == SEED_SWITCH) {
            w.sw_age = 1;
        } else if (st.status == SEED_LIMIT) {
            w.status = SEED_STOPPED;
        }
        // the deferred update read the block's residual history once per row
        if (st.step > 0)
            atomicAdd(&s.stats[0], (unsigned long long)st.step * 16ull * (unsigned long long)s.desc[j].n);
        w.base = (st.base + st.step) % s.R;
        w.step = 0;
        w.n_active = n_active;
        w.a0 = st.alpha_prev;
        w.b0 = st.beta_prev;
        if (st.status != SEED_SWITCH) w.sw_target = -1;
        s.seed[j] = w;
        dec_switch = (sw >= 0 && sw != st.seed) ? sw : -1;
        dec_brk = mb;
    }
    __syncthreads();
    if (dec_brk) {
        // 1: breakdown ends every active pair; 2: they stop unconverged (status stays NOCONV)
        for (int64_t k = tid; k < s.M; k += WG) {
            const int64_t pair = j * s.M + k;
            if (s.active[pair]) {
                if (dec_brk == 1) s.pstatus[pair] = PAIR_BREAKDOWN;
                s.active[pair] = 0;
            }
        }
    }
    const int t = dec_switch;
    if (t < 0) return;
    const double2 pt = s.pi[j * s.M + t];
    const double2 ppt = s.pi_prev[j * s.M + t];
    __syncthreads();
    for (int64_t k = tid; k < s.M; k += WG) {
        const int64_t pair = j * s.M + k;
        s.pi[pair] = cdiv(s.pi[pair], pt);
        s.pi_prev[pair] = cdiv(s.pi_prev[pair], ppt);
    }
    if (tid == 0) {
        SeedState *w = s.seed + j;
        const double2 ap = cdiv(cmul(st.alpha_prev, ppt), pt);
        const double2 bp = s.beta_k[j * s.M + t];
        w->alpha_prev = ap;
        w->beta_prev = bp;
        w->a0 = ap;
        w->b0 = bp;
        w->zs = s.z[t];
        w->seed = t;
        w->inv_pt = cdiv(cmk(1, 0), pt);
        w->inv_ppt = cdiv(cmk(1, 0), ppt);
        w->sw_target = t;
        w->switches = st.switches + 1;
        if (st.switches < s.M) {
            s.swlog[2 * (j * s.M + st.switches) + 0] = st.iter;
            s.swlog[2 * (j * s.M + st.switches) + 1] = t;
        }
    }
}

// Vectors of a seed switch to shift t after step n: r <- r / pi_t(n+1); the stored scaled
// directions of the active pairs move to the new seed's scale, u_k <- u_k / pi_t(n); the new
// seed's direction is p <- p_t(n) = u_t / pi_t(n); rho <- r.r.
template <typename V>
__global__ void __launch_bounds__(WG) k_switch_vectors(SolveDev s)
{
    __shared__ double2 sh2[WG];
    const int64_t j = blockIdx.y;
    const SeedState st = s.seed[j];
    // switched one block end after the decision, when the update of the rhs's last block
    // (launched before that block end) has finished
    if (st.status != SEED_SWITCH || st.sw_age < 1) return;
    const RhsDesc d = s.desc[j];
    const int64_t row = (int64_t)blockIdx.x * WG + threadIdx.x;
    double2 rr = cmk(0, 0);
    if (row < d.n) {
        double2 *rp = ring_slot(s, st.base, d) + row;
        const double2 r = cmul(*rp, st.inv_pt);
        *rp = r;
        V *P = (V *)s.P + s.Mst * d.voff;
        const V sc = to_v<V>(st.inv_ppt);
        const V zero = to_v<V>(cmk(0, 0));
        for (int64_t w = 0; w < s.Mst; ++w) {
            const int64_t k = s.wshift ? s.wshift[j * s.Mst + w] : w;
            if (!s.active[j * s.M + k]) continue;
            V *up = P + w * d.n + row;
            const V u = cfma(sc, *up, zero);
            *up = u;
            if (k == st.sw_target) s.p[p_index(s, j, d, row)] = make_double2((double)u.x, (double)u.y);
        }
        rr = cmul(r, r);
    }
    if ((s.wslot || s.wproj) && blockIdx.x == 0) {
        // the same rescale for the pairs carried by scalars at the kept row (with a vector
        // projection: the projected u_k of every pair)
        const V sc = to_v<V>(st.inv_ppt);
        const V zero = to_v<V>(cmk(0, 0));
        for (int64_t k = threadIdx.x; k < s.M; k += WG) {
            const int64_t pair = j * s.M + k;
            if (!s.active[pair] || (!s.wproj && s.wslot[pair] >= 0)) continue;
            const V u = cfma(sc, to_v<V>(s.Uproj[pair]), zero);
            s.Uproj[pair] = make_double2((double)u.x, (double)u.y);
        }
    }
    rr = block_sum2(rr, sh2);
    if (threadIdx.x == 0) s.part2[j * s.nblk + blockIdx.x] = rr;
    if (!arrive_last(s.cnt, j, (uint32_t)gridDim.x)) return;
    const double2 rho = sum_partials2<true>(s.part2 + j * s.nblk, gridDim.x, sh2);
    if (threadIdx.x == 0) {
        s.seed[j].rho = rho;
        s.seed[j].sw_target = -1;
        s.seed[j].sw_age = 0;
        s.seed[j].status = SEED_RUNNING;
    }
    reset_counter(s.cnt, j);
}

// ---------------------------------------------------------------------------------------
// outputs
// ---------------------------------------------------------------------------------------
__global__ void k_zero(uint32_t *p, size_t nwords)
{
    const size_t i = (size_t)blockIdx.x * WG + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * WG;
    for (size_t k = i; k < nwords; k += stride) p[k] = 0u;
}

__global__ void k_upcast(const float2 *__restrict__ src, double2 *__restrict__ dst, size_t count)
{
    const size_t i = (size_t)blockIdx.x * WG + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * WG;
    for (size_t k = i; k < count; k += stride) dst[k] = make_double2((double)src[k].x, (double)src[k].y);
}

// Residual of pair p = (j, k): r = b_j - (z - H) x_p in FP64 (z = z_k, or z_j when each rhs has
// its own shift).  Writes the partial sums of |r|^2 per row block and, if rout is given, the
// residual vector itself (row c of rout, stride rstride, for the c-th listed pair).
// grid: (row blocks of the largest matrix, pairs).
__global__ void __launch_bounds__(WG) k_true_res_part(const RhsDesc *__restrict__ desc, int64_t M, int zper,
                                                      const double2 *__restrict__ z, const double2 *__restrict__ B,
                                                      const int64_t *__restrict__ unit_idx,
                                                      const double2 *__restrict__ X,
                                                      const int64_t *__restrict__ pair_list,
                                                      double2 *__restrict__ rout, int64_t rstride,
                                                      double *__restrict__ part, int64_t nblk, int64_t c0)
{
    __shared__ double sh1[WG];
    const int64_t c = c0 + blockIdx.y;
    const int64_t pair = pair_list ? pair_list[c] : c;
    const int64_t j = pair / M, k = pair % M;
    const RhsDesc d = desc[j];
    const double2 zk = z[zper ? j : k];
    const int lane = threadIdx.x & 63;
    const int64_t slice = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t row = slice * 64 + lane;
    const double2 *x = X + M * d.voff + k * d.n;
    double e = 0;
    if (slice < d.nslices) {
        double ax = 0, ay = 0;
        if (d.hub) {
            if (row < d.n) {
                double hx[1] = {0}, hy[1] = {0};
                hubbard_row<1>(d.hub, row, x, hx, hy);
                ax = hx[0];
                ay = hy[0];
            }
        } else {
            const int64_t off = d.slice_ptr[slice];
            const int w = d.slice_w[slice];
            for (int q = 0; q < w; ++q) {
                const int col = d.ell_col[off + (int64_t)q * 64 + lane];
                const double v = d.ell_val[off + (int64_t)q * 64 + lane];
                const double2 xc = x[col];
                ax = fma(v, xc.x, ax);
                ay = fma(v, xc.y, ay);
            }
        }
        if (row < d.n) {
            double2 b;
            if (B) b = B[d.voff + row];
            else b = cmk(row == unit_idx[j] ? 1.0 : 0.0, 0.0);
            // b - (z x - H x)
            const double2 zx = cfma(zk, x[row], make_double2(-ax, -ay));
            const double2 r = csub(b, zx);
            if (rout) rout[c * rstride + row] = r;
            e = cabs2(r);
        }
    }
    e = block_sum1(e, sh1);
    if (threadIdx.x == 0) part[c * nblk + blockIdx.x] = e;
}

// x_p <- x_p + d_c for the listed pairs (refinement of a single-matrix solve, rows n)
__global__ void k_add_correction(int64_t n, const int64_t *__restrict__ pair_list, const double2 *__restrict__ D,
                                 double2 *__restrict__ X)
{
    const int64_t c = blockIdx.y;
    const int64_t row = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (row >= n) return;
    const int64_t pair = pair_list[c];
    X[pair * n + row] = cadd(X[pair * n + row], D[c * n + row]);
}

__global__ void k_true_res_final(int64_t count, int64_t M, const int64_t *__restrict__ pair_list,
                                 const double *__restrict__ part, int64_t nblk, const double *__restrict__ bnorm,
                                 double *__restrict__ out)
{
    const int64_t c = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (c >= count) return;
    double acc = 0;
    for (int64_t b = 0; b < nblk; ++b) acc += part[c * nblk + b];
    const int64_t pair = pair_list ? pair_list[c] : c;
    const double nb = bnorm[pair / M];
    out[c] = nb > 0 ? sqrt(acc) / nb : sqrt(acc);
}

// G[k][c] = x_{c,k}[rows[c]] from full storage or from the projected values
__global__ void k_gather_diag(const RhsDesc *__restrict__ desc, int64_t K, int64_t M,
                              const double2 *__restrict__ X, const double2 *__restrict__ Xproj,
                              const int64_t *__restrict__ rows, double2 *__restrict__ G)
{
    const int64_t pair = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (pair >= K * M) return;
    const int64_t j = pair / M, k = pair % M;
    G[k * K + j] = Xproj ? Xproj[pair] : X[M * desc[j].voff + k * desc[j].n + rows[j]];
}

// Density matrix, band energy and energy gradient of one batch of columns.
//   rho[(a, b)] += Re sum_k w_k x_{j,k}[a]     for the stored entries (a, b) of column b = cols_of_rhs[j]
//   Epart[j] = Re sum_k w_k z_k x_{j,k}[b]
// Column b's entries are found through row b's (the pattern is symmetric): entry e = (b, a) of
// row b names a, and its mirror is the position of (a, b).  Each column's entries are its own,
// so the workgroups of a batch (distinct columns) never write the same entry.
__global__ void k_density_rho(int64_t n, int64_t K, int64_t M, const double2 *__restrict__ X,
                              const int64_t *__restrict__ cols_of_rhs, const int64_t *__restrict__ row_ptr,
                              const int32_t *__restrict__ col, const int32_t *__restrict__ mirror,
                              const double2 *__restrict__ w, const double2 *__restrict__ z, double *__restrict__ rho,
                              double *__restrict__ Epart)
{
    const int64_t j = blockIdx.x;
    const int64_t b = cols_of_rhs[j];
    const int64_t e0 = row_ptr[b], e1 = row_ptr[b + 1];
    for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        const int64_t a = col[e];
        double acc = 0;
        for (int64_t k = 0; k < M; ++k) {
            const double2 x = X[(j * M + k) * n + a];
            acc += w[k].x * x.x - w[k].y * x.y;
        }
        if (rho) rho[mirror[e]] += acc;
    }
    if (threadIdx.x == 0) {
        double acc = 0;
        for (int64_t k = 0; k < M; ++k) {
            const double2 x = X[(j * M + k) * n + b];
            const double2 wz = cmul(w[k], z[k]);
            acc += wz.x * x.x - wz.y * x.y;
        }
        Epart[j] = acc;
    }
}

__global__ void k_sum_into(const double *__restrict__ part, int64_t count, double *__restrict__ out)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double acc = 0;
        for (int64_t i = 0; i < count; ++i) acc += part[i];
        out[0] += acc;
    }
}

// Partial sums of the pair contraction Re sum_p c_p x_p[a] x_p[b] over the stored entries
// e = (a, b) (the energy gradient and the adjoint of G, which needs no second solve because
// z - H is complex symmetric).  Work item: one row a, one segment of at most MAXW of its
// entries, one chunk of pairs; grid (row tiles of 256, segments, chunks).  Each item writes
// part[chunk][e] for its entries; k_chunk_sum adds the chunks in order, so the result does not
// depend on scheduling.  Per pair the 256 rows of a tile read x_p[a] contiguously and gather
// x_p[b] from the same pair vector (L2-resident for the tile's neighbourhood).
template <int MAXW>
__global__ void __launch_bounds__(WG) k_pair_outer(int64_t n, int64_t npairs, int64_t pch,
                                                   const double2 *__restrict__ X, const double2 *__restrict__ c,
                                                   const int64_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ col, int64_t nnz,
                                                   double *__restrict__ part)
{
    const int64_t a = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (a >= n) return;
    const int64_t seg0 = row_ptr[a] + (int64_t)blockIdx.y * MAXW;
    const int w = (int)min((int64_t)MAXW, row_ptr[a + 1] - seg0);
    if (w <= 0) return;
    const int64_t p0 = (int64_t)blockIdx.z * pch;
    const int64_t p1 = min(npairs, p0 + pch);
    int cols[MAXW];
    double acc[MAXW];
#pragma unroll
    for (int i = 0; i < MAXW; ++i) {
        cols[i] = (i < w) ? col[seg0 + i] : 0;
        acc[i] = 0;
    }
    for (int64_t p = p0; p < p1; ++p) {
        const double2 *x = X + p * n;
        const double2 xa = cmul(c[p], x[a]);
#pragma unroll
        for (int i = 0; i < MAXW; ++i) {
            if (i < w) {
                const double2 xb = x[cols[i]];
                acc[i] += xa.x * xb.x - xa.y * xb.y;
            }
        }
    }
    double *out = part + (int64_t)blockIdx.z * nnz + seg0;
#pragma unroll
    for (int i = 0; i < MAXW; ++i)
        if (i < w) out[i] = acc[i];
}

// grad[e] += sum over chunks, in chunk order
__global__ void k_chunk_sum(int64_t nnz, int64_t nchunk, const double *__restrict__ part, double *__restrict__ grad)
{
    const int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (e >= nnz) return;
    double acc = 0;
    for (int64_t c = 0; c < nchunk; ++c) acc += part[c * nnz + e];
    grad[e] += acc;
}

// per-pair weights for the band-energy derivative: c_p = w_k z_k for pair p = (j, k)
__global__ void k_pair_weights_wz(int64_t K, int64_t M, const double2 *__restrict__ w, const double2 *__restrict__ z,
                                  double2 *__restrict__ c)
{
    const int64_t p = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (p >= K * M) return;
    const int64_t k = p % M;
    c[p] = cmul(w[k], z[k]);
}

// per-pair weights for backward through G: c_p = conj(g[k][j])
__global__ void k_pair_weights_conj(int64_t K, int64_t M, const double2 *__restrict__ g, double2 *__restrict__ c)
{
    const int64_t p = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (p >= K * M) return;
    const int64_t j = p / M, k = p % M;
    const double2 v = g[k * K + j];
    c[p] = make_double2(v.x, -v.y);
}

// ---------------------------------------------------------------------------------------
// set-up and reports computed on the device (used by the entry point that allocates nothing,
// so that no per-rhs or per-pair table has to be built on the host)
// ---------------------------------------------------------------------------------------
// desc[j] = proto with its vectors at j * proto.n; seeds[j] = seed; idx[j] copied as given
__global__ void k_fill_desc(RhsDesc proto, int64_t K, int32_t seed, RhsDesc *__restrict__ desc,
                            int32_t *__restrict__ seeds)
{
    const int64_t j = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (j >= K) return;
    RhsDesc d = proto;
    d.voff = j * proto.n;
    desc[j] = d;
    seeds[j] = seed;
}

// flag[0] = 1 when every right-hand side has stopped
__global__ void k_all_stopped(const SeedState *__restrict__ seed, int64_t K, int32_t *__restrict__ flag)
{
    __shared__ int sh[WG];
    int run = 0;
    for (int64_t j = threadIdx.x; j < K; j += WG) run |= seed[j].status != SEED_STOPPED ? 1 : 0;
    sh[threadIdx.x] = run;
    __syncthreads();
    for (int h = WG / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] |= sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) flag[0] = sh[0] ? 0 : 1;
}

// Per-pair reports in the C ABI's layout, the worst status (2 breakdown, 1 not converged) and,
// from the first workgroup, the seed iterations and switches summed over right-hand sides.
// worst and totals start at zero.
__global__ void k_pack_report(int64_t K, int64_t M, int fixed, const int32_t *__restrict__ iters,
                              const int32_t *__restrict__ pstatus, const double *__restrict__ res,
                              const SeedState *__restrict__ seed, PairReportDev *__restrict__ rep,
                              int32_t *__restrict__ worst, long long *__restrict__ totals)
{
    const int64_t pair = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (pair < K * M) {
        const int32_t stv = pstatus[pair];
        PairReportDev r;
        r.iters = iters[pair];
        r.status = (fixed && stv == PAIR_NOCONV) ? PAIR_OK : stv;
        r.res = res[pair];
        r.res_true = -1.0;
        rep[pair] = r;
        const int code = stv == PAIR_BREAKDOWN ? 2 : ((stv == PAIR_NOCONV && !fixed) ? 1 : 0);
        if (code) atomicMax(worst, code);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        long long it = 0, sw = 0;
        for (int64_t j = 0; j < K; ++j) {
            it += seed[j].iter;
            sw += seed[j].switches;
        }
        totals[0] = it;
        totals[1] = sw;
    }
}

hipError_t launch_fill_desc(const RhsDesc &proto, int64_t K, int32_t seed, RhsDesc *desc, int32_t *seeds,
                            hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_desc, dim3((unsigned)((K + WG - 1) / WG)), dim3(WG), 0, st, proto, K, seed, desc, seeds);
    return hipGetLastError();
}

hipError_t launch_all_stopped(const SeedState *seed, int64_t K, int32_t *flag, hipStream_t st)
{
    hipLaunchKernelGGL(k_all_stopped, dim3(1), dim3(WG), 0, st, seed, K, flag);
    return hipGetLastError();
}

hipError_t launch_pack_report(int64_t K, int64_t M, int fixed, const int32_t *iters, const int32_t *pstatus,
                              const double *res, const SeedState *seed, PairReportDev *rep, int32_t *worst,
                              long long *totals, hipStream_t st)
{
    const int64_t KM = K * M;
    hipLaunchKernelGGL(k_pack_report, dim3((unsigned)((KM + WG - 1) / WG)), dim3(WG), 0, st, K, M, fixed, iters,
                       pstatus, res, seed, rep, worst, totals);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------------------
static inline dim3 grid2(int64_t x, int64_t y) { return dim3((unsigned)x, (unsigned)y, 1); }

hipError_t launch_init(const SolveDev &s, const double2 *B, const int64_t *unit_idx,
                       const int32_t *seed_idx, int32_t limit, hipStream_t st)
{
    hipLaunchKernelGGL(k_init, grid2(s.nblk, s.K), dim3(WG), 0, st, s, B, unit_idx, seed_idx, limit);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t KM = s.K * s.M;
    hipLaunchKernelGGL(k_init_pairs, dim3((unsigned)((KM + WG - 1) / WG)), dim3(WG), 0, st, s);
    return hipGetLastError();
}

hipError_t launch_seed_iteration(const SolveDev &s, hipStream_t st)
{
    const int RB = s.spmv_rb;
    const int64_t G = (s.K + RB - 1) / RB;
    const dim3 gp = s.it_grp ? dim3((unsigned)s.n_it_grp) : grid2(s.nblk, G);
    if (RB == 2) hipLaunchKernelGGL(k_pupd<2>, gp, dim3(WG), 0, st, s);
    else hipLaunchKernelGGL(k_pupd<1>, gp, dim3(WG), 0, st, s);
    const int64_t nwg = s.it_grp ? s.n_it_grp : (G < 8 ? s.nblk * G : s.nblk * 8 * ((G + 7) / 8));
    if (s.has_sell) {
        if (RB == 2) hipLaunchKernelGGL((k_spmv<2, false>), dim3((unsigned)nwg), dim3(WG), 0, st, s);
        else hipLaunchKernelGGL((k_spmv<1, false>), dim3((unsigned)nwg), dim3(WG), 0, st, s);
    }
    if (s.has_hub) {
        if (s.hub_lds)
            hipLaunchKernelGGL(k_spmv_hub_lds, dim3((unsigned)s.hub_du_max, (unsigned)s.K), dim3(HUB_WG), 0, st, s);
        else if (RB == 2) hipLaunchKernelGGL((k_spmv<2, true>), dim3((unsigned)nwg), dim3(WG), 0, st, s);
        else hipLaunchKernelGGL((k_spmv<1, true>), dim3((unsigned)nwg), dim3(WG), 0, st, s);
    }
    if (s.has_red_small) hipLaunchKernelGGL(k_alpha<WG>, dim3((unsigned)s.K), dim3(WG), 0, st, s);
    if (s.has_red_big) hipLaunchKernelGGL(k_alpha<RWG_BIG>, dim3((unsigned)s.K), dim3(RWG_BIG), 0, st, s);
    hipLaunchKernelGGL(k_rupd, s.it_rhs ? dim3((unsigned)s.n_it_rhs) : grid2(s.nblk, s.K), dim3(WG), 0, st, s);
    if (s.has_red_small) hipLaunchKernelGGL(k_beta<WG>, dim3((unsigned)s.K), dim3(WG), 0, st, s);
    if (s.has_red_big) hipLaunchKernelGGL(k_beta<RWG_BIG>, dim3((unsigned)s.K), dim3(RWG_BIG), 0, st, s);
    return hipGetLastError();
}

hipError_t launch_pair_scalars(const SolveDev &s, hipStream_t st)
{
    const int64_t KM = s.K * s.M;
    const dim3 g((unsigned)((KM + WG - 1) / WG));
    if (s.precision == 0) hipLaunchKernelGGL(k_pair_scalars<double2>, g, dim3(WG), 0, st, s);
    else hipLaunchKernelGGL(k_pair_scalars<float2>, g, dim3(WG), 0, st, s);
    return hipGetLastError();
}

hipError_t launch_block_finalize(const SolveDev &s, hipStream_t st)
{
    hipLaunchKernelGGL(k_block_finalize, dim3((unsigned)s.K), dim3(WG), 0, st, s);
    return hipGetLastError();
}

hipError_t launch_switch_vectors(const SolveDev &s, hipStream_t st)
{
    if (s.precision == 0) hipLaunchKernelGGL(k_switch_vectors<double2>, grid2(s.nblk, s.K), dim3(WG), 0, st, s);
    else hipLaunchKernelGGL(k_switch_vectors<float2>, grid2(s.nblk, s.K), dim3(WG), 0, st, s);
    return hipGetLastError();
}

hipError_t launch_zero(void *ptr, size_t bytes, hipStream_t st)
{
    if (bytes == 0) return hipSuccess;
    if (bytes % 4 != 0) return hipErrorInvalidValue;
    const size_t words = bytes / 4;
    size_t blocks = (words + WG - 1) / WG;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(WG), 0, st, (uint32_t *)ptr, words);
    return hipGetLastError();
}

hipError_t launch_store_solution(const SolveDev &s, double2 *Xout, hipStream_t st)
{
    if (s.precision == 0) return hipSuccess;
    const size_t count = (size_t)(s.M * s.ntot);
    size_t blocks = (count + WG - 1) / WG;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_upcast, dim3((unsigned)blocks), dim3(WG), 0, st, (const float2 *)s.X, Xout, count);
    return hipGetLastError();
}

hipError_t launch_residual(const SolveDev &s, const double2 *B, const int64_t *unit_idx, const double2 *X64,
                           const int64_t *pair_list, int64_t count, const double *bnorm, double2 *rout,
                           double *part, double *out_res, hipStream_t st)
{
    const int64_t gx = s.nblk;
    const int64_t chunk = 32768;
    for (int64_t c0 = 0; c0 < count; c0 += chunk) {
        const int64_t nc = (count - c0) < chunk ? (count - c0) : chunk;
        hipLaunchKernelGGL(k_true_res_part, grid2(gx, nc), dim3(WG), 0, st, s.desc, s.M, s.zper, s.z, B, unit_idx,
                           X64, pair_list, rout, s.n, part, gx, c0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_true_res_final, dim3((unsigned)((count + WG - 1) / WG)), dim3(WG), 0, st, count, s.M, pair_list,
                       part, gx, bnorm, out_res);
    return hipGetLastError();
}

hipError_t launch_add_correction(int64_t n, const int64_t *pair_list, int64_t count, const double2 *D, double2 *X,
                                 hipStream_t st)
{
    const int64_t chunk = 32768;
    for (int64_t c0 = 0; c0 < count; c0 += chunk) {
        const int64_t nc = (count - c0) < chunk ? (count - c0) : chunk;
        hipLaunchKernelGGL(k_add_correction, grid2((n + WG - 1) / WG, nc), dim3(WG), 0, st, n, pair_list + c0,
                           D + c0 * n, X);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_gather_diag(const SolveDev &s, const int64_t *rows, double2 *G, hipStream_t st)
{
    const int64_t KM = s.K * s.M;
    hipLaunchKernelGGL(k_gather_diag, dim3((unsigned)((KM + WG - 1) / WG)), dim3(WG), 0, st, s.desc, s.K, s.M,
                       (const double2 *)s.X, s.Xproj, rows, G);
    return hipGetLastError();
}

// Observable kernels used by the host driver directly.
hipError_t launch_density_rho(int64_t n, int64_t K, int64_t M, const double2 *X, const int64_t *cols_of_rhs,
                              const int64_t *row_ptr, const int32_t *col, const int32_t *mirror, const double2 *w,
                              const double2 *z, double *rho, double *Epart, double *Eacc, hipStream_t st)
{
    hipLaunchKernelGGL(k_density_rho, dim3((unsigned)K), dim3(64), 0, st, n, K, M, X, cols_of_rhs, row_ptr, col,
                       mirror, w, z, rho, Epart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum_into, dim3(1), dim3(64), 0, st, Epart, K, Eacc);
    return hipGetLastError();
}

hipError_t launch_pair_weights(int mode, int64_t K, int64_t M, const double2 *w, const double2 *z,
                               const double2 *g, double2 *c, hipStream_t st)
{
    const int64_t KM = K * M;
    if (mode == 0) hipLaunchKernelGGL(k_pair_weights_wz, dim3((unsigned)((KM + WG - 1) / WG)), dim3(WG), 0, st, K, M, w, z, c);
    else hipLaunchKernelGGL(k_pair_weights_conj, dim3((unsigned)((KM + WG - 1) / WG)), dim3(WG), 0, st, K, M, g, c);
    return hipGetLastError();
}

// Segment width and count for the longest row: rows of up to 8 or 20 entries take one
// segment of that width, longer rows segments of 32.
static void pair_outer_shape(int max_row, int &maxw, int64_t &nseg)
{
    maxw = max_row <= 8 ? 8 : (max_row <= 20 ? 20 : 32);
    nseg = max_row <= 0 ? 1 : (max_row + maxw - 1) / maxw;
}

int64_t pair_outer_chunks(int64_t n, int64_t npairs, int max_row)
{
    int maxw;
    int64_t nseg;
    pair_outer_shape(max_row, maxw, nseg);
    const int64_t tiles = (n + WG - 1) / WG;
    // about 2048 workgroups fill the 256 compute units several times over
    int64_t nchunk = (2048 + tiles * nseg - 1) / (tiles * nseg);
    nchunk = nchunk < 1 ? 1 : nchunk;
    nchunk = nchunk > npairs ? npairs : nchunk;
    nchunk = nchunk > 65535 ? 65535 : nchunk;
    return nchunk < 1 ? 1 : nchunk;
}

hipError_t launch_pair_outer(int64_t n, int64_t npairs, const double2 *X, const double2 *c, const int64_t *row_ptr,
                             const int32_t *col, int64_t nnz, int max_row, int64_t nchunk, double *part, double *grad,
                             hipStream_t st)
{
    if (npairs <= 0 || nnz <= 0) return hipSuccess;
    int maxw;
    int64_t nseg;
    pair_outer_shape(max_row, maxw, nseg);
    if (nseg > 65535 || nchunk < 1 || nchunk > 65535) return hipErrorInvalidValue;
    const int64_t pch = (npairs + nchunk - 1) / nchunk;
    const dim3 g((unsigned)((n + WG - 1) / WG), (unsigned)nseg, (unsigned)nchunk);
    // every chunk writes every stored entry (each lies in exactly one segment of its row)
    if (maxw == 8)
        hipLaunchKernelGGL(k_pair_outer<8>, g, dim3(WG), 0, st, n, npairs, pch, X, c, row_ptr, col, nnz, part);
    else if (maxw == 20)
        hipLaunchKernelGGL(k_pair_outer<20>, g, dim3(WG), 0, st, n, npairs, pch, X, c, row_ptr, col, nnz, part);
    else
        hipLaunchKernelGGL(k_pair_outer<32>, g, dim3(WG), 0, st, n, npairs, pch, X, c, row_ptr, col, nnz, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_chunk_sum, dim3((unsigned)((nnz + WG - 1) / WG)), dim3(WG), 0, st, nnz, nchunk,
                       (const double *)part, grad);
    return hipGetLastError();
}

}  // namespace scocg

// The deferred per-shift update of the shifted-COCG solver (the dominant kernel).
#include "device_common.h"

namespace scocg {

// ---------------------------------------------------------------------------------------
// Deferred per-shift update.  For every active pair and every step t < nact of the block
//   u_k <- r_t + b'_t u_k ;  x_k <- x_k + a'_t u_k
// x_k and u_k stay in registers across the block, so each is read and written once per
// block instead of once per iteration.  One thread per row; a workgroup covers 256 rows of
// one rhs and `G` shifts, NP pairs in flight per thread.  Coefficients and step counts are
// uniform across the workgroup (scalar loads).  x_k and u_k are streamed with nontemporal
// loads and stores: they are not reused before the next block.
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

template <int TB, typename V, int NP, bool PROJ>
__global__ void __launch_bounds__(WG) k_flush(const SeedState *__restrict__ seed, const double2 *__restrict__ ring,
                                              const V *__restrict__ coef, const int32_t *__restrict__ nact,
                                              V *__restrict__ X, V *__restrict__ P, double2 *__restrict__ Xproj,
                                              const int64_t *__restrict__ proj_row,
                                              const RhsDesc *__restrict__ desc, int64_t ntot, int64_t M, int G,
                                              int ngroups)
{
    const int64_t j = blockIdx.y / ngroups;
    const int g = blockIdx.y % ngroups;
    const int ns = seed[j].step;
    if (ns == 0) return;
    const int base = seed[j].base;
    const bool fresh = seed[j].iter == ns;
    const int64_t n = desc[j].n;
    const int64_t voff = desc[j].voff;
    const int64_t row = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (row >= n) return;
    V r[TB];
#pragma unroll
    for (int t = 0; t < TB; ++t) {
        if (t < ns) r[t] = to_v<V>(ring[(int64_t)((base + t) % (TB + 1)) * ntot + voff + row]);
        else r[t] = to_v<V>(cmk(0, 0));
    }
    X += M * voff;
    P += M * voff;
    const int64_t k0 = (int64_t)g * G;
    const int64_t k1 = min(k0 + G, M);
    const int64_t prow = PROJ ? proj_row[j] : -1;
    for (int64_t k = k0; k < k1; k += NP) {
        V x[NP], u[NP];
        int na[NP];
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const int64_t pair = j * M + k + q;
            na[q] = (k + q < k1) ? nact[pair] : 0;
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
#pragma unroll
        for (int t = 0; t < TB; ++t) {
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                if (t < na[q]) {
                    const V *cf = coef + ((j * M + k + q) * TB + t) * 2;
                    u[q] = cfma(cf[1], u[q], r[t]);
                    x[q] = cfma(cf[0], u[q], x[q]);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const int64_t pair = j * M + k + q;
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

static inline dim3 flush_grid(int64_t x, int64_t y) { return dim3((unsigned)x, (unsigned)y, 1); }

template <int TB, typename V, int NP>
static hipError_t flush_v(const SolveDev &s, hipStream_t st)
{
    const int G = s.shifts_per_wg;
    const int ng = (int)((s.M + G - 1) / G);
    const dim3 g = flush_grid(s.nblk, s.K * ng);
    const V *coef = (const V *)s.coef;
    if (s.Xproj)
        hipLaunchKernelGGL((k_flush<TB, V, NP, true>), g, dim3(WG), 0, st, s.seed, s.ring, coef, s.nact, (V *)nullptr,
                           (V *)s.P, s.Xproj, s.proj_row, s.desc, s.ntot, s.M, G, ng);
    else
        hipLaunchKernelGGL((k_flush<TB, V, NP, false>), g, dim3(WG), 0, st, s.seed, s.ring, coef, s.nact, (V *)s.X,
                           (V *)s.P, (double2 *)nullptr, (const int64_t *)nullptr, s.desc, s.ntot, s.M, G, ng);
    return hipGetLastError();
}

template <int TB>
static hipError_t flush_tb(const SolveDev &s, hipStream_t st)
{
    if (s.precision == 0) return flush_v<TB, double2, 2>(s, st);
    return flush_v<TB, float2, 4>(s, st);
}

hipError_t launch_flush(const SolveDev &s, hipStream_t st)
{
    switch (s.TB) {
    case 1: return flush_tb<1>(s, st);
    case 2: return flush_tb<2>(s, st);
    case 4: return flush_tb<4>(s, st);
    case 8: return flush_tb<8>(s, st);
    case 16: return flush_tb<16>(s, st);
    case 32: return flush_tb<32>(s, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace scocg

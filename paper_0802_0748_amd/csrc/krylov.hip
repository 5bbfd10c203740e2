// Krylov-subspace diagonalization (Sec. 3.2, eq. Ham_in_KS) for many unit right-hand sides:
// the three-term recurrence builds each orthonormal basis {K_n} of K_nu(H, |j>), in which H
// is the tridiagonal T with diagonal a_n = <K_n|H|K_n> and off-diagonal b_{n+1} = <K_{n+1}|H|K_n>;
// the local Green's function is then G_jj(z) = [(z - T)^{-1}]_11, evaluated as the continued
// fraction of T.  Per step, for every unfinished right-hand side:
//   w = H K_n - b_n K_{n-1};  a_n = K_n . w;  w <- w - a_n K_n;  b_{n+1} = ||w||;
//   K_{n+1} = w / b_{n+1}  (applied on the fly by the next step as w * (1 / b_{n+1})).
// Start vectors are unit vectors, so every basis vector is real.  Sums are fixed-order
// (per 256-row tile, then the tiles in index order), so results do not depend on scheduling.
#include "device_common.h"
#include "krylov.h"

namespace scocg {

typedef double d4v __attribute__((ext_vector_type(4)));
static_assert(LZ_TILE == WG, "one 256-row tile per workgroup");

// Tree sums of LZ_RB values over the WG threads (result in thread 0).
__device__ inline void block_sum_rb(double (&v)[LZ_RB], double (*sh)[WG])
{
    const int t = threadIdx.x;
#pragma unroll
    for (int b = 0; b < LZ_RB; ++b) sh[b][t] = v[b];
    __syncthreads();
    for (int h = WG / 2; h > 0; h >>= 1) {
        if (t < h) {
#pragma unroll
            for (int b = 0; b < LZ_RB; ++b) sh[b][t] += sh[b][t + h];
        }
        __syncthreads();
    }
#pragma unroll
    for (int b = 0; b < LZ_RB; ++b) v[b] = sh[b][0];
}

// Fixed-order sum of a right-hand side's tile partials by one workgroup (result in thread 0):
// thread t adds partials t, t + WG, ... in order, then the threads' sums as a tree.
__device__ inline double sum_tiles(const double *part, int64_t nblk, double *sh)
{
    double acc = 0;
    int64_t b = threadIdx.x;
    for (; b + 7 * WG < nblk; b += 8 * WG) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = part[b + u * WG];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; b < nblk; b += WG) acc += part[b];
    const int t = threadIdx.x;
    sh[t] = acc;
    __syncthreads();
    for (int h = WG / 2; h > 0; h >>= 1) {
        if (t < h) sh[t] += sh[t + h];
        __syncthreads();
    }
    return sh[0];
}

// w = H K_n - b_n K_{n-1} and the partials of K_n . w; K_n (= the previous w times 1/b_n, or
// the unit vector at step 0) is written out for the step after.
__global__ void __launch_bounds__(WG) k_lz_matvec(LzDev s, int n)
{
    __shared__ double sh[LZ_RB][WG];
    const int64_t g = blockIdx.y;
    bool run[LZ_RB];
    double bprev[LZ_RB], rb[LZ_RB];
    int64_t jj[LZ_RB];
    bool any = false;
#pragma unroll
    for (int b = 0; b < LZ_RB; ++b) {
        const LzRhs st = s.st[g * LZ_RB + b];
        run[b] = !st.done;
        bprev[b] = run[b] ? st.bprev : 0.0;
        rb[b] = (run[b] && n > 0) ? 1.0 / st.bprev : 0.0;
        jj[b] = st.j;
        any = any || run[b];
    }
    if (!any) return;  // uniform over the workgroup
    const int q = n & 1;
    const int64_t base = g * s.n;
    const d4v *Wp = (const d4v *)(s.W[q ^ 1]) + base;
    const d4v *Vp = (const d4v *)(s.V[q ^ 1]) + base;
    d4v *Vn = (d4v *)(s.V[q]) + base;
    d4v *Wn = (d4v *)(s.W[q]) + base;
    const int64_t row = (int64_t)blockIdx.x * WG + threadIdx.x;
    double dot[LZ_RB] = {0, 0, 0, 0};
    if (row < s.n) {
        double acc[LZ_RB] = {0, 0, 0, 0};
        const int64_t slice = row >> 6;
        const int lane = (int)(row & 63);
        const int64_t off = s.slice_ptr[slice];
        const int w = s.slice_w[slice];
        const int32_t *colp = s.ell_col + off + lane;
        const double *valp = s.ell_val + off + lane;
        // slots in the stored order; column and value loads of LZ_CHUNK slots are issued
        // before their gathers
        constexpr int LZ_CHUNK = 4;
        auto slot = [&](int32_t c, double v) {
            double x[LZ_RB];
            if (n == 0) {
#pragma unroll
                for (int b = 0; b < LZ_RB; ++b) x[b] = (c == jj[b]) ? 1.0 : 0.0;
            } else {
                const d4v wc = Wp[c];
#pragma unroll
                for (int b = 0; b < LZ_RB; ++b) x[b] = wc[b] * rb[b];
            }
#pragma unroll
            for (int b = 0; b < LZ_RB; ++b) acc[b] = fma(v, x[b], acc[b]);
        };
        int k = 0;
        for (; k + LZ_CHUNK <= w; k += LZ_CHUNK) {
            int32_t c[LZ_CHUNK];
            double v[LZ_CHUNK];
#pragma unroll
            for (int u = 0; u < LZ_CHUNK; ++u) {
                c[u] = colp[(int64_t)(k + u) * 64];
                v[u] = valp[(int64_t)(k + u) * 64];
            }
#pragma unroll
            for (int u = 0; u < LZ_CHUNK; ++u) slot(c[u], v[u]);
        }
        for (; k < w; ++k) slot(colp[(int64_t)k * 64], valp[(int64_t)k * 64]);
        d4v vo, wo;
        if (n == 0) {
#pragma unroll
            for (int b = 0; b < LZ_RB; ++b) {
                vo[b] = (row == jj[b]) ? 1.0 : 0.0;
                wo[b] = acc[b];
            }
        } else {
            const d4v wr = Wp[row], vr = Vp[row];
#pragma unroll
            for (int b = 0; b < LZ_RB; ++b) {
                vo[b] = wr[b] * rb[b];
                wo[b] = fma(-bprev[b], vr[b], acc[b]);
            }
        }
        Vn[row] = vo;
        Wn[row] = wo;
#pragma unroll
        for (int b = 0; b < LZ_RB; ++b) dot[b] = vo[b] * wo[b];
    }
    block_sum_rb(dot, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int b = 0; b < LZ_RB; ++b)
            if (run[b]) s.part[(g * LZ_RB + b) * s.nblk + blockIdx.x] = dot[b];
    }
}

// a_n from the partials of K_n . w
__global__ void __launch_bounds__(WG) k_lz_alpha(LzDev s, int n)
{
    __shared__ double sh[WG];
    const int64_t j = blockIdx.x;
    if (s.st[j].done) return;
    const double a = sum_tiles(s.part + j * s.nblk, s.nblk, sh);
    if (threadIdx.x == 0) {
        s.st[j].a = a;
        s.ab[j * 2 * s.nu + n] = a;
    }
}

// w <- w - a_n K_n and the partials of ||w||^2
__global__ void __launch_bounds__(WG) k_lz_axpy(LzDev s, int n)
{
    __shared__ double sh[LZ_RB][WG];
    const int64_t g = blockIdx.y;
    bool run[LZ_RB];
    double a[LZ_RB];
    bool any = false;
#pragma unroll
    for (int b = 0; b < LZ_RB; ++b) {
        const LzRhs st = s.st[g * LZ_RB + b];
        run[b] = !st.done;
        a[b] = run[b] ? st.a : 0.0;
        any = any || run[b];
    }
    if (!any) return;
    const int q = n & 1;
    const int64_t base = g * s.n;
    const d4v *Vn = (const d4v *)(s.V[q]) + base;
    d4v *Wn = (d4v *)(s.W[q]) + base;
    const int64_t row = (int64_t)blockIdx.x * WG + threadIdx.x;
    double nn[LZ_RB] = {0, 0, 0, 0};
    if (row < s.n) {
        const d4v v = Vn[row];
        d4v w = Wn[row];
#pragma unroll
        for (int b = 0; b < LZ_RB; ++b) {
            w[b] = fma(-a[b], v[b], w[b]);
            nn[b] = w[b] * w[b];
        }
        Wn[row] = w;
    }
    block_sum_rb(nn, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int b = 0; b < LZ_RB; ++b)
            if (run[b]) s.part[(g * LZ_RB + b) * s.nblk + blockIdx.x] = nn[b];
    }
}

// b_{n+1} = ||w||, the end test, and the state for the next step
__global__ void __launch_bounds__(WG) k_lz_beta(LzDev s, int n)
{
    __shared__ double sh[WG];
    const int64_t j = blockIdx.x;
    const LzRhs st = s.st[j];
    if (st.done) return;
    const double b = sqrt(sum_tiles(s.part + j * s.nblk, s.nblk, sh));
    if (threadIdx.x == 0) {
        s.ab[j * 2 * s.nu + s.nu + n] = b;
        LzRhs *w = s.st + j;
        w->m = n + 1;
        if (n == s.nu - 1 || b <= LZ_STOP_REL * (fabs(st.a) + st.bprev)) w->done = 1;
        else w->bprev = b;
    }
}

// G[k][r] = [(z_k - T_r)^{-1}]_11 by the continued fraction of T_r, innermost level first
__global__ void __launch_bounds__(WG) k_lz_greens(LzDev s, const double2 *__restrict__ z, int64_t M, int64_t K,
                                                  double2 *__restrict__ G)
{
    const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (i >= M * K) return;
    const int64_t k = i / K, r = i % K;
    const int m = s.st[r].m;
    const double *a = s.ab + r * 2 * s.nu;
    const double *b = a + s.nu;
    const double2 zk = z[k];
    double2 g = cdiv(cmk(1, 0), cmk(zk.x - a[m - 1], zk.y));
    for (int t = m - 2; t >= 0; --t) {
        const double bb = b[t] * b[t];
        g = cdiv(cmk(1, 0), cmk(zk.x - a[t] - bb * g.x, zk.y - bb * g.y));
    }
    G[k * K + r] = g;
}

hipError_t launch_lanczos_step(const LzDev &s, int n, hipStream_t st)
{
    const int64_t groups = s.K / LZ_RB;
    if (s.nblk > 0x7fffffffLL || groups > 65535 || s.K > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    const dim3 gv((unsigned)s.nblk, (unsigned)groups);
    hipLaunchKernelGGL(k_lz_matvec, gv, dim3(WG), 0, st, s, n);
    hipLaunchKernelGGL(k_lz_alpha, dim3((unsigned)s.K), dim3(WG), 0, st, s, n);
    hipLaunchKernelGGL(k_lz_axpy, gv, dim3(WG), 0, st, s, n);
    hipLaunchKernelGGL(k_lz_beta, dim3((unsigned)s.K), dim3(WG), 0, st, s, n);
    return hipGetLastError();
}

hipError_t launch_lanczos_greens(const LzDev &s, const double2 *z, int64_t M, int64_t K_out, double2 *G,
                                 hipStream_t st)
{
    const int64_t total = M * K_out;
    if (total == 0) return hipSuccess;
    if ((total + WG - 1) / WG > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_lz_greens, dim3((unsigned)((total + WG - 1) / WG)), dim3(WG), 0, st, s, z, M, K_out, G);
    return hipGetLastError();
}

}  // namespace scocg

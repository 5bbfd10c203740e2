// Rows of the matrix-free extended Hubbard operator (device code shared by the seed kernels
// and the three-term recurrence).
#pragma once
#include "scocg_internal.h"

namespace scocg {

// Occupations of the right neighbours on a ring of L sites: bit i of the result is bit
// (i + 1) mod L of c.
__device__ inline uint32_t ring_next(uint32_t c, int L) { return ((c >> 1) | ((c & 1u) << (L - 1))) & ((1u << L) - 1u); }

// The terms of row `row` of a matrix-free Hubbard operator, f(column, value) in increasing
// column order, the order of the stored sector matrix's row: up-spin hops to lower
// configurations, the down-spin hops with the diagonal at its place, up-spin hops to higher
// configurations.  Diagonal: U sum_i n_i,up n_i,dn + V sum_i n_i n_i+1 (periodic).
template <typename F>
__device__ inline void hubbard_row_terms(const HubbardOp *hp, int64_t row, F &&f)
{
    const HubbardOp h = *hp;
    const int64_t iu = (int64_t)((uint64_t)row / (uint64_t)h.Dd);
    const int64_t id = row - iu * h.Dd;
    const int32_t u0 = h.up_ptr[iu], u1 = h.up_ptr[iu + 1];
    const int32_t d0 = h.dn_ptr[id], d1 = h.dn_ptr[id + 1];
    const uint32_t cu = h.up_conf[iu], cd = h.dn_conf[id];
    const int on = __popc(cu & cd);
    const int inter = __popc(cu & ring_next(cu, h.L)) + __popc(cd & ring_next(cd, h.L)) +
                      __popc(cu & ring_next(cd, h.L)) + __popc(cd & ring_next(cu, h.L));
    const double diag = h.U * (double)on + h.V * (double)inter;
    auto val = [&](uint32_t e) { return (e >> 31) ? h.t : -h.t; };
    int32_t k = u0;
    for (; k < u1; ++k) {
        const uint32_t e = h.up_hop[k];
        const int64_t a = e & 0x7fffffffu;
        if (a >= iu) break;
        f(a * h.Dd + id, val(e));
    }
    bool diag_done = false;
    for (int32_t m = d0; m < d1; ++m) {
        const uint32_t e = h.dn_hop[m];
        const int64_t b = e & 0x7fffffffu;
        if (!diag_done && b > id) {
            f(row, diag);
            diag_done = true;
        }
        f(iu * h.Dd + b, val(e));
    }
    if (!diag_done) f(row, diag);
    for (; k < u1; ++k) {
        const uint32_t e = h.up_hop[k];
        f((int64_t)(e & 0x7fffffffu) * h.Dd + id, val(e));
    }
}

}  // namespace scocg

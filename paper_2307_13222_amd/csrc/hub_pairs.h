// Diagonal of the Hubbard two-body terms for one configuration, term by
// term (HPhi update paper Sec. 5, Eq. ham_general): per site pair
// V n_i n_j - JH (n_i,up n_j,up + n_i,dn n_j,dn), n_i = n_i,up + n_i,dn.
// Used where the diagonal is needed once per call (trace, the LOBPCG
// preconditioner); the H*v kernel takes the same sum from per-row tables.
#pragma once

#include "internal.h"

namespace hphi {

__device__ __forceinline__ double hub_pair_diag(const HubPairDev *p, int np, uint32_t u, uint32_t d)
{
    double s = 0.0;
    for (int k = 0; k < np; ++k) {
        const int i = p[k].i, j = p[k].j;
        const int ui = (u >> i) & 1, uj = (u >> j) & 1, di = (d >> i) & 1, dj = (d >> j) & 1;
        s += p[k].v * (double)((ui + di) * (uj + dj)) - p[k].jh * (double)(ui * uj + di * dj);
    }
    return s;
}

} // namespace hphi

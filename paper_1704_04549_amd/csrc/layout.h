// Layout of the opaque preconditioner buffer (kp_precond_bytes / kp_setup).
//
// Sections, each element-major and 256-byte aligned:
//   sigma   [E][4]            double
//   factors [E][nf][n][n]     double  (2D rank r: nf = 2r; 3D: nf = 5)
//   status  [E]               int32
//   kinds   [E][32]           int8    (block kinds of T2 for the Sylvester sweep)
//   axis    [E]               int8    (3D: the axis of the rank-1 split, 0 = x)
//   t64     [E][ne]           double  apply tables, ne = (7 + n) n^2
//   t32     [E][ne]           float
//   thi     [E][ne]           bf16    high part of the split bf16 tables
//   tlo     [E][ne]           bf16    low part
//   t2      [E][ne]           float   thi + tlo as float
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "elem_ops.h"

namespace kp {

struct PcLayout {
    size_t sigma, factors, status, kinds, axis, t64, t32, thi, tlo, t2, total;
    long nf, ne;
};

inline size_t align256(size_t x) { return (x + 255) / 256 * 256; }

inline bool pc_layout(int dim, int n, int rank, int64_t E, PcLayout* L) {
    if (n < 2 || n > kMaxN || E < 0) return false;
    if (dim == 2) {
        if (rank < 1 || rank > 3) return false;
        L->nf = 2 * rank;
    } else if (dim == 3) {
        if (rank != 2) return false;
        L->nf = 5;
    } else {
        return false;
    }
    const size_t nn = (size_t)n * n;
    L->ne = tab_entries(n);
    size_t off = 0;
    L->sigma = off; off = align256(off + E * 4 * sizeof(double));
    L->factors = off; off = align256(off + E * L->nf * nn * sizeof(double));
    L->status = off; off = align256(off + E * sizeof(int32_t));
    L->kinds = off; off = align256(off + E * kMaxN);
    L->axis = off; off = align256(off + E);
    L->t64 = off; off = align256(off + E * L->ne * sizeof(double));
    L->t32 = off; off = align256(off + E * L->ne * sizeof(float));
    L->thi = off; off = align256(off + E * L->ne * sizeof(uint16_t));
    L->tlo = off; off = align256(off + E * L->ne * sizeof(uint16_t));
    L->t2 = off; off = align256(off + E * L->ne * sizeof(float));
    L->total = off;
    return true;
}

}  // namespace kp

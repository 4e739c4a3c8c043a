// Segment Storage Format (Sec. "Storage format of the sparse matrices") to
// and from the block CSR the library works on.  Host code: a format
// conversion for input and output, not part of the expansion.
//
// SSF describes the non-zero entries of an n x n matrix as nseg segments of
// consecutive entries in dense coordinates, keyg = (c_s, c_e, r_s, r_e) per
// segment (here an [nseg][4] array), with the values in one array and keyv
// giving where each segment starts in it (redundant: NULL means "one after
// the other").  Indices are 1-based; a segment runs in row-major order from
// (r_s, c_s) to (r_e, c_e), so it may continue over a row end.  Block (I, J)
// of edge b is stored when any entry inside it is; entries the segments do
// not give are zero.  Export writes one segment per maximal run of
// consecutive block columns in every scalar row.
#include <stdint.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "../../include/chess.h"

namespace {

struct Piece {
    int64_t r, c0, c1, v;  // scalar row, first and last column (0-based), value index of c0
};

// Splits the segments into row pieces (in order); CHESS_E_ARG for segments
// out of range, reversed, unsorted or overlapping, or values past nval.
int pieces_of(int64_t n, int64_t nseg, const int64_t *keyg, const int64_t *keyv, int64_t nval,
              std::vector<Piece> &out) {
    int64_t prev_end = -1, pos = 0;
    for (int64_t s = 0; s < nseg; ++s) {
        const int64_t cs = keyg[4 * s] - 1, ce = keyg[4 * s + 1] - 1, rs = keyg[4 * s + 2] - 1, re = keyg[4 * s + 3] - 1;
        if (cs < 0 || ce < 0 || rs < 0 || re < 0 || cs >= n || ce >= n || rs >= n || re >= n) return CHESS_E_ARG;
        const int64_t a = rs * n + cs, e = re * n + ce;
        if (e < a || a <= prev_end) return CHESS_E_ARG;
        prev_end = e;
        const int64_t start = keyv ? keyv[s] - 1 : pos;
        if (start < 0 || start + (e - a + 1) > nval) return CHESS_E_ARG;
        pos = start + (e - a + 1);
        for (int64_t r = rs; r <= re; ++r) {
            const int64_t c0 = r == rs ? cs : 0, c1 = r == re ? ce : n - 1;
            out.push_back(Piece{r, c0, c1, start + (r * n + c0 - a)});
        }
    }
    return CHESS_OK;
}

}  // namespace

extern "C" {

int chess_ssf_to_bcsr(int32_t b, int64_t n, int64_t nseg, const int64_t *keyg, const int64_t *keyv,
                      const double *val, int64_t nval, int64_t *row_ptr, int32_t *col_idx,
                      double *val_bcsr, int64_t capacity, int64_t *nnzb_out) {
    if (b < 1 || n < 0 || nseg < 0 || (nseg > 0 && !keyg) || !nnzb_out || n % b != 0) return CHESS_E_ARG;
    const int64_t nb = n / b;
    if (nb > INT32_MAX) return CHESS_E_ARG;
    std::vector<Piece> pc;
    pc.reserve((size_t)nseg);
    if (const int rc = pieces_of(n, nseg, keyg, keyv, nval, pc); rc != CHESS_OK) return rc;
    // block columns of each block row (pieces come in row order)
    std::vector<int64_t> rp((size_t)nb + 1, 0);
    std::vector<int32_t> ci;
    std::vector<int32_t> cols;
    size_t p = 0;
    for (int64_t I = 0; I < nb; ++I) {
        cols.clear();
        size_t q = p;
        while (q < pc.size() && pc[q].r < (I + 1) * b) {
            for (int64_t J = pc[q].c0 / b; J <= pc[q].c1 / b; ++J) cols.push_back((int32_t)J);
            ++q;
        }
        std::sort(cols.begin(), cols.end());
        cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
        ci.insert(ci.end(), cols.begin(), cols.end());
        rp[(size_t)I + 1] = (int64_t)ci.size();
        p = q;
    }
    *nnzb_out = (int64_t)ci.size();
    if (!row_ptr && !col_idx && !val_bcsr) return CHESS_OK;  // size query
    if (capacity < (int64_t)ci.size()) return CHESS_E_CAPACITY;
    if (row_ptr) std::copy(rp.begin(), rp.end(), row_ptr);
    if (col_idx) std::copy(ci.begin(), ci.end(), col_idx);
    if (val_bcsr) {
        if (!val) return CHESS_E_ARG;
        const size_t bb = (size_t)b * b;
        std::memset(val_bcsr, 0, sizeof(double) * bb * ci.size());
        for (const Piece &x : pc) {
            const int64_t I = x.r / b, i = x.r % b;
            const int32_t *row = ci.data() + rp[(size_t)I];
            const int64_t len = rp[(size_t)I + 1] - rp[(size_t)I];
            // the piece's block columns are consecutive and all present
            int64_t k = std::lower_bound(row, row + len, (int32_t)(x.c0 / b)) - row;
            for (int64_t c = x.c0; c <= x.c1; ++c) {
                const int32_t J = (int32_t)(c / b);
                while (row[k] < J) ++k;
                val_bcsr[((size_t)(rp[(size_t)I] + k)) * bb + (size_t)i * b + (size_t)(c % b)] = val[x.v + (c - x.c0)];
            }
        }
    }
    return CHESS_OK;
}

int chess_bcsr_to_ssf(int32_t b, int32_t nbrows, const int64_t *row_ptr, const int32_t *col_idx,
                      const double *val_bcsr, int64_t *keyg, int64_t *keyv, double *val, int64_t capacity,
                      int64_t *nseg_out, int64_t *nval_out) {
    if (b < 1 || nbrows < 0 || !row_ptr || !nseg_out || !nval_out) return CHESS_E_ARG;
    if (row_ptr[0] != 0) return CHESS_E_ARG;
    int64_t nseg = 0;
    for (int32_t I = 0; I < nbrows; ++I) {
        const int64_t q0 = row_ptr[I], q1 = row_ptr[I + 1];
        if (q1 < q0 || (q1 > q0 && !col_idx)) return CHESS_E_ARG;
        for (int64_t q = q0; q < q1; ++q) {
            if (col_idx[q] < 0 || col_idx[q] >= nbrows || (q > q0 && col_idx[q] <= col_idx[q - 1])) return CHESS_E_ARG;
            if (q == q0 || col_idx[q] != col_idx[q - 1] + 1) nseg += b;  // a new run in each of the b rows
        }
    }
    *nseg_out = nseg;
    *nval_out = row_ptr[nbrows] * (int64_t)b * b;
    if (!keyg && !keyv && !val) return CHESS_OK;  // size query
    if (capacity < nseg) return CHESS_E_CAPACITY;
    if (val && !val_bcsr) return CHESS_E_ARG;
    const size_t bb = (size_t)b * b;
    int64_t s = 0, pos = 0;
    for (int32_t I = 0; I < nbrows; ++I) {
        const int64_t q0 = row_ptr[I], q1 = row_ptr[I + 1];
        for (int i = 0; i < b; ++i) {
            const int64_t r = (int64_t)I * b + i;
            for (int64_t q = q0; q < q1;) {
                int64_t qe = q;
                while (qe + 1 < q1 && col_idx[qe + 1] == col_idx[qe] + 1) ++qe;
                if (keyg) {
                    keyg[4 * s] = (int64_t)col_idx[q] * b + 1;
                    keyg[4 * s + 1] = (int64_t)col_idx[qe] * b + b;
                    keyg[4 * s + 2] = r + 1;
                    keyg[4 * s + 3] = r + 1;
                }
                if (keyv) keyv[s] = pos + 1;
                for (int64_t k = q; k <= qe; ++k) {
                    if (val) std::memcpy(val + pos, val_bcsr + (size_t)k * bb + (size_t)i * b, sizeof(double) * b);
                    pos += b;
                }
                ++s;
                q = qe + 1;
            }
        }
    }
    return CHESS_OK;
}

}  // extern "C"

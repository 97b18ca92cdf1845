// Candidate search space of the GPU path: rung sizes, ID arithmetic, unit
// rules and the compacted set of operand features kept in HBM.
//
// The paper generates candidates iteratively from primary features and an
// operator library (Software Description) and prunes dimensionally invalid
// expressions early (Physics-Informed Constraints).  IDs are positions in
// the canonical list described in include/discover.h; the GPU computes them
// arithmetically from (rung, operator, operand indices).
#pragma once

#include "dsc_common.h"

namespace dsc {

enum : int {
    OP_EXP = 0, OP_LOG, OP_SQRT, OP_SQ, OP_INV,
    OP_ADD, OP_SUB, OP_MUL, OP_DIV, OP_RDIV,
    OP_NONE = 15
};

// Plain-old-data view passed to kernels by value.
struct SpaceDev {
    int32_t p, R;
    int32_t pool[4];          // partner rung of binary operators at rung r
    uint32_t ops[4];          // operator mask of rung r
    int64_t L[4];             // raw size of rung r
    int64_t off[5];           // first raw index of rung r (off[R+1] = |P_R|)
    int64_t npairs[4];        // pairs per binary block at rung r
    int64_t block[4][10];     // first ID of operator block o at rung r (-1: disabled)
};

// ID of a binary candidate (op o, operands i < j raw) at rung r.
__host__ __device__ inline int64_t pair_id(const SpaceDev& s, int r, int o, int64_t i, int64_t j) {
    int64_t local = (s.pool[r] == r - 1)
                        ? (choose2(j) - choose2(s.off[r - 1]) + i)
                        : ((j - s.off[r - 1]) * s.off[s.pool[r] + 1] + i);
    return s.block[r][o] + local;
}

__host__ __device__ inline int64_t unary_id(const SpaceDev& s, int r, int o, int64_t a) {
    return s.block[r][o] + (a - s.off[r - 1]);
}

// Decode an ID into (rung, op, a, b); a = unary operand or i, b = j or -1.
__host__ __device__ inline void decode_id(const SpaceDev& s, int64_t id, int& rung, int& op,
                                          int64_t& a, int64_t& b) {
    if (id < s.p) {
        rung = 0; op = OP_NONE; a = id; b = -1;
        return;
    }
    int r = 1;
    while (r < s.R && id >= s.off[r + 1]) r++;
    rung = r;
    for (int o = 9; o >= 0; o--) {
        if (s.block[r][o] < 0 || id < s.block[r][o]) continue;
        int64_t q = id - s.block[r][o];
        op = o;
        if (o < OP_ADD) {
            a = s.off[r - 1] + q; b = -1;
            return;
        }
        if (s.pool[r] == r - 1) {
            int64_t Q = q + choose2(s.off[r - 1]);
            int64_t j = (int64_t)((1.0 + sqrt(1.0 + 8.0 * (double)Q)) * 0.5);
            while (j > 1 && choose2(j) > Q) j--;
            while (choose2(j + 1) <= Q) j++;
            a = Q - choose2(j); b = j;
        } else {
            int64_t w = s.off[s.pool[r] + 1];
            a = q % w; b = s.off[r - 1] + q / w;
        }
        return;
    }
    op = OP_NONE; a = -1; b = -1;   // unreachable for valid IDs
}

// Score slots of one problem's candidates.  IDs below s3 are their own
// slots.  With an operator-limited rung 3 only the unit-legal pairs get
// rung-3 slots: mul / div / rdiv (OP_ADD + q, q >= 2) of record r (a
// unit-legal rung-2 feature of the rung-3 plan, padding included) and
// partner c (compact) has slot sblk[q] + r pe + c; add / sub (q < 2), legal
// only between equal unit vectors, have slot sblk[q] + (16 w + i) 16 + j for
// row i and column j of add/sub work item w.  The rung-3 slot space is then
// about the size of the unit-valid part of the rung instead of the raw one,
// and so are the fill, histogram and compaction passes over it.
struct SlotMap {
    int64_t s3 = 0;           // first rung-3 slot (= first rung-3 ID)
    int64_t n = 0;            // slots
    int64_t sblk[5] = {-1, -1, -1, -1, -1};   // ascending where enabled, -1 disabled
    int32_t pe = 1;           // partners
    const int2* grec = nullptr;       // records: k (-1 unary, -2 padding), l | op2 << 28
    const int2* as_grec = nullptr;    // add / sub records, work items (row tile,
    const int2* as_work = nullptr;    // column tile) and column tiles (partner
    const int32_t* as_cols = nullptr; // | kind << 16)
    const int64_t* mat_raw = nullptr; // compact -> raw operand index
};

// Rung-3 slot of (mul / div / rdiv operator o, record r, partner c).
__host__ __device__ inline int64_t slot3(const SlotMap& m, int o, int64_t r, int c) {
    return m.sblk[o - OP_ADD] + r * m.pe + c;
}
// Rung-3 slot of (add / sub operator o, work item w, row i, column j).
__host__ __device__ inline int64_t slot3as(const SlotMap& m, int o, int64_t w, int i, int j) {
    return m.sblk[o - OP_ADD] + ((w * 16 + i) << 4) + j;
}

// ID of a slot (-1 for a padding slot, which is never written).
__device__ inline int64_t slot_id(const SlotMap& m, const SpaceDev& s, int64_t slot) {
    if (slot < m.s3 || !m.grec) return slot;
    int q = 4;
    while (q > 0 && (m.sblk[q] < 0 || slot < m.sblk[q])) q--;
    const int64_t v = slot - m.sblk[q];
    int2 rc;
    int c;
    if (q < 2) {
        const int2 wk = m.as_work[v >> 8];
        rc = m.as_grec[(int64_t)wk.x * 16 + ((v >> 4) & 15)];
        const int32_t cd = m.as_cols[wk.y * 16 + (v & 15)];
        if (cd < 0 || (cd >> 16) != 0) return -1;
        c = cd & 0xFFFF;
    } else {
        const int64_t r = v / m.pe;
        c = (int)(v - r * m.pe);
        rc = m.grec[r];
    }
    const int k = rc.x, l = rc.y & 0x0FFFFFFF, op2 = (int)((unsigned)rc.y >> 28);
    if (k == -2) return -1;
    const int64_t j2 = k < 0 ? unary_id(s, 2, op2, m.mat_raw[l]) : pair_id(s, 2, op2, m.mat_raw[k], m.mat_raw[l]);
    return pair_id(s, 3, OP_ADD + q, m.mat_raw[c], j2);
}

// Host description of one search space plus the operand features that are
// materialised in HBM (all unit-legal features of rungs below the streamed
// rung; for rung 0 the primaries themselves).
struct Space {
    SpaceDev d{};
    int B = 0;
    int streamed = 0;                  // rung whose candidates are streamed (0: none)
    bool stream3 = false;              // rung 3 (operator-limited) streamed on top of rung 2
    int64_t n_unit_valid_r3 = 0;       // unit-valid candidates of rung 3
    int64_t M_raw = 0;                 // raw features below the streamed rung
    std::vector<int64_t> mat_raw;      // compact -> raw index (ascending)
    std::vector<int32_t> raw2c;        // raw -> compact or -1 (size M_raw)
    std::vector<int8_t> mat_op;        // per compact feature: operator (OP_NONE for primaries)
    std::vector<int32_t> mat_a, mat_b; // compact operand indices (-1 if none)
    std::vector<int32_t> mat_unit;     // compact x B exponents scaled by 2^R
    std::vector<int32_t> rung_start;   // compact start of each materialised rung, + end
    int64_t n_unit_valid = 0;          // over all of P_R
    int64_t n_unit_valid_streamed = 0;

    int64_t n_raw() const { return d.off[d.R + 1]; }
    int32_t Mc() const { return (int32_t)mat_raw.size(); }
};

// Build the space; `units` is host [p][B] (may be NULL when B = 0).
// The canonical layout of the raw space (rung sizes, offsets, operator
// blocks): the ID enumeration that build_space, discover_count and
// discover_decode share.
void space_layout(SpaceDev& d, int p, const discover_screen_params& prm);
void build_space(Space& sp, int p, const discover_screen_params& prm, int B,
                 const int32_t* units);

// Host-side unit rule (exponents scaled by 2^R); returns legality.
bool unit_rule(int op, int B, const int32_t* ua, const int32_t* ub, int32_t* out);

std::string expr_of(const SpaceDev& s, int64_t id);

}  // namespace dsc

// Operator-limited rung 3 (binary operators, partner from a materialised
// rung, second operand a rung-2 feature regenerated on the fly): the plan
// of its work lists and the launch of its screening kernels.
//
// The products mul / div / rdiv of a partner x with a rung-2 feature g have
// moments that are sums of products over samples:
//   S1 = sum x g,  S2 = sum x^2 g^2,  P_t = sum (x y_t) g      (mul)
// and the same with h = 1/g (div) or w = 1/x (rdiv).  For a block of 16
// rung-2 features and 16 partner columns these are 16 x 16 matrix products
// over samples, computed on the FP64 matrix cores; add / sub (same-unit
// pairs only when units are given) run on the vector units.
#pragma once

#include <algorithm>
#include <memory>
#include <vector>

#include "dsc_space.h"

namespace dsc {

struct R3Plan {
    // every unit-legal rung-2 feature, per operator (binary ones in windows
    // of 64 x 64 operands, for L2 reuse): x = k (compact operand,
    // -1 for a unary operator), y = l | op2 << 28
    int2* grec = nullptr;
    int64_t n_grec = 0;
    // partner columns, 16 per tile: partner | kind << 16 (kind 0 mul, 1 rdiv:
    // tiles against g; kind 2 div: tiles against 1/g), -1 for padding
    int32_t* coldesc = nullptr;
    int n_ctiles = 0, n_gct = 0;      // tiles; the first n_gct multiply g
    std::vector<int32_t> h_coldesc;
    // add / sub over same-unit pairs: the records whose unit vector some
    // partner shares, grouped by unit vector and operator (runs padded to
    // 16); per unit vector, column tiles of up to 15 such partners plus a
    // column of ones (column 15); one wave per (row tile, column tile)
    int2* as_grec = nullptr;
    int64_t n_as_grec = 0;
    int32_t* as_coldesc = nullptr;
    int n_as_ctiles = 0;
    int2* as_work = nullptr;
    int64_t n_as_work = 0;
    uint32_t ops = 0;                 // rung-3 binary operators (bit o - OP_ADD)
    int pe = 0;                       // partner pool size (compact 0..pe-1)
    std::vector<void*> allocs;
    ~R3Plan();
};

std::shared_ptr<R3Plan> build_r3_plan(const Space& sp, uint32_t r3_ops);

// Per-call buffers of one problem's rung-3 screen.
inline int r3_quads(int n) { return 4 * (int)((n + 15) / 16); }
inline int r3_chunks(int n) { return (int)((n + 31) / 32); }
// Error coefficient of the precision form's split-BF16 moments: the score
// of a rung-3 candidate moves by at most cm kappa through them
// (3 ((n + 50) 2^-24 + 3 2^-16)).
inline double r3_moment_err(int n) { return 3.0 * ((n + 50) * 5.9604644775390625e-8 + 3.0 * 1.52587890625e-5); }
// The main tiles' operands (FP64 layout, or the precision form's), then the
// add/sub tiles' (FP64 layout) at r3_as_offset bytes.
inline size_t r3_as_offset(const R3Plan& p, int TP, int n) {
    const size_t f64 = (size_t)p.n_ctiles * (TP + 2) * r3_quads(n) * 64 * 8;
    const size_t lp = (size_t)p.n_ctiles * r3_chunks(n) * 512 * (4 + TP * 2);
    return (std::max(f64, lp) + 255) & ~(size_t)255;
}
// The add/sub tiles' operands end with the targets in the same lane order
// (one 16-column block: column t = target t), at r3_asy_offset bytes.
inline size_t r3_asy_offset(const R3Plan& p, int TP, int n) {
    return r3_as_offset(p, TP, n) + (size_t)p.n_as_ctiles * (TP + 2) * r3_quads(n) * 64 * 8;
}
inline size_t r3_bmat_bytes(const R3Plan& p, int TP, int n) {
    return r3_asy_offset(p, TP, n) + (size_t)r3_quads(n) * 64 * 8;
}
inline size_t r3_pstat_bytes(const R3Plan& p, int TP) {
    return (size_t)std::max(p.pe, 1) * (2 + TP + 2) * 8;
}

struct R3Launch {
    const R3Plan* plan;
    int n, ldn, TP, T, mode;
    const double *Vf, *Rf, *Cf, *mu, *msq;
    const uint8_t* valid;
    const int64_t* mat_raw;
    const double *Yn, *ysum;
    const uint8_t* r2v;
    const double *r2m, *r2q;
    SpaceDev sd;
    SlotMap sm;                       // score slot of each candidate
    int64_t N;                        // slots per target
    double* scores;
    unsigned long long* nscored;
    int64_t* fix_ids;                 // slots of the candidates left to the fix-up
    unsigned long long* fix_cnt;
    int64_t fix_cap;
    int precision;                    // DISCOVER_BF16_GUARD: precision form of mul/div/rdiv
    double delta;                     // its error bound per unit sqrt(kappa)
    double* bmat;                     // r3_bmat_bytes
    double* pstat;                    // r3_pstat_bytes: max |x|, min |x| per partner,
                                      // then the add/sub partner sums
};

void launch_r3(discover_ctx* ctx, const R3Launch& a, hipStream_t st);

}  // namespace dsc

// Host construction of the candidate space: rung/operator block layout,
// unit legality of the operand features kept in HBM, and unit-valid counts
// of the streamed rung.
#include "dsc_space.h"

#include <cstdarg>
#include <unordered_map>

namespace dsc {

static thread_local char g_err[1024] = "no error";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

const char* get_error() { return g_err; }

bool unit_rule(int op, int B, const int32_t* ua, const int32_t* ub, int32_t* out) {
    switch (op) {
    case OP_EXP:
    case OP_LOG:   // transcendental functions need a dimensionless argument
        for (int k = 0; k < B; k++)
            if (ua[k]) return false;
        for (int k = 0; k < B; k++) out[k] = 0;
        return true;
    case OP_SQRT:
        for (int k = 0; k < B; k++)
            if (ua[k] & 1) return false;
        for (int k = 0; k < B; k++) out[k] = ua[k] / 2;
        return true;
    case OP_SQ:
        for (int k = 0; k < B; k++) out[k] = 2 * ua[k];
        return true;
    case OP_INV:
        for (int k = 0; k < B; k++) out[k] = -ua[k];
        return true;
    case OP_ADD:
    case OP_SUB:   // only like quantities can be added
        for (int k = 0; k < B; k++)
            if (ua[k] != ub[k]) return false;
        for (int k = 0; k < B; k++) out[k] = ua[k];
        return true;
    case OP_MUL:
        for (int k = 0; k < B; k++) out[k] = ua[k] + ub[k];
        return true;
    case OP_DIV:
        for (int k = 0; k < B; k++) out[k] = ua[k] - ub[k];
        return true;
    case OP_RDIV:
        for (int k = 0; k < B; k++) out[k] = ub[k] - ua[k];
        return true;
    }
    return false;
}

void space_layout(SpaceDev& d, int p, const discover_screen_params& prm) {
    std::memset(&d, 0, sizeof d);
    d.p = p;
    d.R = prm.rung;
    d.L[0] = p;
    d.off[0] = 0;
    d.off[1] = p;
    for (int o = 0; o < 10; o++) d.block[0][o] = -1;
    for (int r = 1; r <= d.R; r++) {
        uint32_t m = prm.rung_ops[r] ? prm.rung_ops[r] : prm.ops;
        d.ops[r] = m & DISCOVER_OPS_ALL;
        int pool = prm.rung_pool[r] < 0 ? r - 1 : prm.rung_pool[r];
        DSC_REQUIRE(pool <= r - 1, "rung_pool[%d] = %d must be below rung %d", r, pool, r);
        d.pool[r] = pool;
        d.npairs[r] = pool == r - 1 ? choose2(d.off[r]) - choose2(d.off[r - 1])
                                    : d.L[r - 1] * d.off[pool + 1];
        int64_t id = d.off[r];
        for (int o = 0; o < 10; o++) {
            if (!(d.ops[r] >> o & 1u)) {
                d.block[r][o] = -1;
                continue;
            }
            d.block[r][o] = id;
            id += o < OP_ADD ? d.L[r - 1] : d.npairs[r];
        }
        d.L[r] = id - d.off[r];
        d.off[r + 1] = id;
    }
    for (int r = d.R + 1; r < 4; r++)
        for (int o = 0; o < 10; o++) d.block[r][o] = -1;
}

void build_space(Space& sp, int p, const discover_screen_params& prm, int B,
                 const int32_t* units) {
    SpaceDev& d = sp.d;
    space_layout(d, p, prm);
    sp.B = B;

    // Rung 3 is supported as an operator-limited rung: binary operators whose
    // first operand comes from a materialised rung (partner pool <= 1); the
    // rung-2 operand is regenerated on the fly from two rung-1 features.
    sp.stream3 = d.R == 3;
    if (sp.stream3) {
        if (d.pool[3] > 1)
            DSC_FAIL(DISCOVER_E_UNSUPPORTED,
                     "rung 3 needs an operator-limited partner pool (rung_pool[3] <= 1)");
        for (int o = 0; o < OP_ADD; o++)
            if (d.block[3][o] >= 0)
                DSC_FAIL(DISCOVER_E_UNSUPPORTED, "unary operators at rung 3 are not supported");
    }
    sp.streamed = d.R >= 1 ? (sp.stream3 ? 2 : d.R) : 0;
    sp.M_raw = sp.streamed ? d.off[sp.streamed] : p;
    DSC_REQUIRE(sp.M_raw <= (int64_t)1 << 22,
                "operand features below the streamed rung (%lld) exceed the HBM plan",
                (long long)sp.M_raw);

    // Enumerate the operand features in canonical order with units.
    const int Bq = B > 0 ? B : 1;
    const int32_t Q = 1 << d.R;
    std::vector<int32_t> ru((size_t)sp.M_raw * Bq, 0);
    std::vector<uint8_t> legal(sp.M_raw, 0);
    std::vector<int8_t> rop(sp.M_raw, OP_NONE);
    std::vector<int64_t> ra(sp.M_raw, -1), rb(sp.M_raw, -1);
    for (int f = 0; f < p; f++) {
        legal[f] = 1;
        for (int k = 0; k < B; k++) ru[(size_t)f * Bq + k] = units ? units[f * B + k] * Q : 0;
    }
    int top = sp.streamed ? sp.streamed - 1 : 0;   // highest materialised rung
    for (int r = 1; r <= top; r++) {
        int64_t t = d.off[r];
        for (int o = 0; o < 10; o++) {
            if (d.block[r][o] < 0) continue;
            if (o < OP_ADD) {
                for (int64_t a = d.off[r - 1]; a < d.off[r]; a++, t++) {
                    rop[t] = (int8_t)o; ra[t] = a;
                    legal[t] = legal[a] && unit_rule(o, B, &ru[a * Bq], nullptr, &ru[t * Bq]);
                }
            } else {
                for (int64_t j = d.off[r - 1]; j < d.off[r]; j++) {
                    int64_t ilim = d.pool[r] == r - 1 ? j : d.off[d.pool[r] + 1];
                    for (int64_t i = 0; i < ilim; i++, t++) {
                        rop[t] = (int8_t)o; ra[t] = i; rb[t] = j;
                        legal[t] = legal[i] && legal[j] &&
                                   unit_rule(o, B, &ru[i * Bq], &ru[j * Bq], &ru[t * Bq]);
                    }
                }
            }
        }
    }
    // Compact the legal ones (order preserved).
    sp.raw2c.assign(sp.M_raw, -1);
    sp.mat_raw.clear();
    sp.rung_start.assign(top + 2, 0);
    for (int r = 0; r <= top; r++) {
        sp.rung_start[r] = (int32_t)sp.mat_raw.size();
        for (int64_t t = d.off[r]; t < d.off[r + 1] && t < sp.M_raw; t++)
            if (legal[t]) {
                sp.raw2c[t] = (int32_t)sp.mat_raw.size();
                sp.mat_raw.push_back(t);
            }
    }
    sp.rung_start[top + 1] = (int32_t)sp.mat_raw.size();
    const int32_t Mc = sp.Mc();
    sp.mat_op.resize(Mc);
    sp.mat_a.resize(Mc);
    sp.mat_b.resize(Mc);
    sp.mat_unit.assign((size_t)Mc * Bq, 0);
    for (int32_t c = 0; c < Mc; c++) {
        int64_t t = sp.mat_raw[c];
        sp.mat_op[c] = rop[t];
        sp.mat_a[c] = ra[t] >= 0 ? sp.raw2c[ra[t]] : -1;
        sp.mat_b[c] = rb[t] >= 0 ? sp.raw2c[rb[t]] : -1;
        for (int k = 0; k < B; k++) sp.mat_unit[(size_t)c * Bq + k] = ru[t * Bq + k];
    }

    // Unit-valid count of the streamed rung.
    sp.n_unit_valid = Mc;
    sp.n_unit_valid_streamed = 0;
    if (sp.streamed) {
        const int r = sp.streamed;
        const int32_t c0 = sp.rung_start[r - 1], c1 = sp.rung_start[r];
        int64_t cnt = 0;
        std::vector<int32_t> tmp(Bq);
        for (int o = 0; o < OP_ADD; o++) {
            if (d.block[r][o] < 0) continue;
            for (int32_t c = c0; c < c1; c++)
                cnt += unit_rule(o, B, &sp.mat_unit[(size_t)c * Bq], nullptr, tmp.data());
        }
        const bool has_mul[3] = {d.block[r][OP_MUL] >= 0, d.block[r][OP_DIV] >= 0,
                                 d.block[r][OP_RDIV] >= 0};
        const int nmul = has_mul[0] + has_mul[1] + has_mul[2];
        const int nadd = (d.block[r][OP_ADD] >= 0) + (d.block[r][OP_SUB] >= 0);
        std::unordered_map<std::string, int64_t> seen;
        auto key = [&](int32_t c) {
            return std::string((const char*)&sp.mat_unit[(size_t)c * Bq], sizeof(int32_t) * Bq);
        };
        if (d.pool[r] == r - 1) {
            int64_t below = 0;
            for (int32_t c = 0; c < c1; c++) {
                if (c >= c0) {
                    cnt += (int64_t)nmul * below;
                    auto it = seen.find(key(c));
                    cnt += (int64_t)nadd * (it == seen.end() ? 0 : it->second);
                }
                below++;
                seen[key(c)]++;
            }
        } else {
            const int32_t pe = sp.rung_start[d.pool[r] + 1];
            for (int32_t c = 0; c < pe; c++) seen[key(c)]++;
            for (int32_t c = c0; c < c1; c++) {
                cnt += (int64_t)nmul * pe;
                auto it = seen.find(key(c));
                cnt += (int64_t)nadd * (it == seen.end() ? 0 : it->second);
            }
        }
        sp.n_unit_valid_streamed = cnt;
        sp.n_unit_valid += cnt;
    }
    if (sp.stream3) {
        // unit-valid rung-3 candidates: for every unit-legal rung-2 feature,
        // the legal partners in the pool (any for mul/div/rdiv, same
        // exponents for add/sub)
        const int32_t pe = sp.rung_start[d.pool[3] + 1];
        std::unordered_map<std::string, int64_t> pu;
        auto ukey = [&](const int32_t* u) {
            return std::string((const char*)u, sizeof(int32_t) * Bq);
        };
        for (int32_t c = 0; c < pe; c++) pu[ukey(&sp.mat_unit[(size_t)c * Bq])]++;
        const int nmul = (d.block[3][OP_MUL] >= 0) + (d.block[3][OP_DIV] >= 0) + (d.block[3][OP_RDIV] >= 0);
        const int nadd = (d.block[3][OP_ADD] >= 0) + (d.block[3][OP_SUB] >= 0);
        const int32_t c0 = sp.rung_start[1], c1 = sp.rung_start[2];
        std::vector<int32_t> u2(Bq);
        int64_t cnt = 0;
        auto count_j2 = [&](const int32_t* u) {
            cnt += (int64_t)nmul * pe;
            if (nadd) {
                auto it = pu.find(ukey(u));
                if (it != pu.end()) cnt += (int64_t)nadd * it->second;
            }
        };
        for (int o = 0; o < OP_ADD; o++) {
            if (d.block[2][o] < 0) continue;
            for (int32_t c = c0; c < c1; c++)
                if (unit_rule(o, B, &sp.mat_unit[(size_t)c * Bq], nullptr, u2.data())) count_j2(u2.data());
        }
        for (int o = OP_ADD; o <= OP_RDIV; o++) {
            if (d.block[2][o] < 0) continue;
            for (int32_t l = c0; l < c1; l++)
                for (int32_t k = 0; k < l; k++)
                    if (unit_rule(o, B, &sp.mat_unit[(size_t)k * Bq], &sp.mat_unit[(size_t)l * Bq], u2.data()))
                        count_j2(u2.data());
        }
        sp.n_unit_valid_r3 = cnt;
        sp.n_unit_valid += cnt;
    }
}

std::string expr_of(const SpaceDev& s, int64_t id) {
    int rung, op;
    int64_t a, b;
    decode_id(s, id, rung, op, a, b);
    if (op == OP_NONE) return "x" + std::to_string(id);
    static const char* un[] = {"exp", "log", "sqrt", "sq", "inv"};
    if (op < OP_ADD) return std::string(un[op]) + "(" + expr_of(s, a) + ")";
    std::string A = expr_of(s, a), Bs = expr_of(s, b);
    switch (op) {
    case OP_ADD: return "(" + A + " + " + Bs + ")";
    case OP_SUB: return "(" + A + " - " + Bs + ")";
    case OP_MUL: return "(" + A + " * " + Bs + ")";
    case OP_DIV: return "(" + A + " / " + Bs + ")";
    default: return "(" + Bs + " / " + A + ")";
    }
}

}  // namespace dsc

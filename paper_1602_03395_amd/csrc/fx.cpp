// Host runtime and C ABI of the free-flight expansion library.
//
// A plan holds, per axis, the FP64-built phase tables of the prescription (FF)
// (section 5.2) rounded to the data precision, the radix plans of the in-LDS
// transforms, and a schedule: the ordered list of per-axis passes that
// evaluates (FF). With the active axes p_1 < ... < p_k (p_k the contiguous one):
//
//   paper schedule (all prod_j lam_j terms q of (FFpsi)):
//     E(p_k), ..., E(p_2)   forward transform + chirp + pruned inverse along an
//                           axis, one output slice per magnification index
//                           (the shared prefixes of the d-dimensional FFTs of
//                           all q-terms are computed once);
//     EA(p_1)               the same along the slowest axis with the
//                           twiddle-gather-accumulate of its index folded in;
//     A(p_2), ..., A(p_k)   twiddle f and n'' gather of the remaining axes,
//                           summing the slices of each magnification index.
//   Each B^(q) is formed (per line, in LDS or in the slice tensors) and every
//   term f^(q) B^(q)[n''] enters the sum; only the order of the additions and
//   the sharing of common per-axis factors differ from a term-by-term loop.
//
//   axis-factorised schedule: EA(p_k), ..., EA(p_1) -- d successive 1-D
//   expansions, sum_j lam_j terms (the operator is a tensor product over
//   axes because every factor of (FF) and the free dispersion factorise).
//
// Long flights are processed in blocks of the outermost magnification index,
// accumulating into the output, so the workspace stays bounded (the
// sequential accumulation of section 7.1).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "fx_internal.h"
#include "plan.h"

namespace fx {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

RadixPlan make_radix_plan(int n) {
    RadixPlan p;
    p.n = n;
    int m = n;
    auto push = [&](int r) { p.rad[p.nst++] = r; m /= r; };
    while (m % 8 == 0 && p.nst < kMaxStages) push(8);
    while (m % 4 == 0 && p.nst < kMaxStages) push(4);
    while (m % 2 == 0 && p.nst < kMaxStages) push(2);
    while (m % 3 == 0 && p.nst < kMaxStages) push(3);
    for (int f = 5; m > 1 && p.nst < kMaxStages; f += 2) {
        while (m % f == 0 && p.nst < kMaxStages) push(f);
        if ((int64_t)f * f > m && m > 1 && p.nst < kMaxStages) {
            push(m);
            break;
        }
    }
    return p;
}

int lds_limit_bytes() {
    static int cached = -1;
    if (cached < 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
            cached = v;
        else
            cached = 65536;
    }
    return cached;
}

}  // namespace fx

using namespace fx;

namespace {

int64_t gcd64(int64_t a, int64_t b) {
    while (b) {
        int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

int64_t modinv(int64_t a, int64_t m) {
    if (m == 1) return 0;
    int64_t g0 = m, g1 = a % m, x0 = 0, x1 = 1;
    while (g1) {
        int64_t qd = g0 / g1;
        int64_t t = g0 - qd * g1; g0 = g1; g1 = t;
        t = x0 - qd * x1; x0 = x1; x1 = t;
    }
    if (g0 != 1) return -1;
    return ((x0 % m) + m) % m;
}

}  // namespace

namespace fx {

size_t csize(const fx_plan* p) { return p->dbl ? 16 : 8; }

bool use_cfp(const fx_plan* p, Kind kind, const AxisDev& a) {
    return p->use_cfp && a.HT != nullptr && cfp_applicable(kind, p->dbl, a.M, a.g) &&
           (int64_t)(cfp_lds_bytes(p->dbl, a.M, a.g) + ((size_t)a.lam * (a.M / a.g) + 4 * (size_t)(a.M + a.g)) * (p->dbl ? 16 : 8)) <=
               lds_limit_bytes();
}

int choose_ts(const fx_plan* p, Kind kind, int M, int64_t A, int64_t S) {
    if (p->use_p2 && p2_applicable(kind, M) && (int64_t)p2_lds_bytes(kind, p->dbl, M) <= lds_limit_bytes())
        return p2_tile_lines(M);
    if (p->use_p2 && ct_applicable(kind, M) && (int64_t)ct_lds_bytes(kind, p->dbl, M) <= lds_limit_bytes())
        return ct_tile_lines(M);
    int ts = std::max(1, p->ts_target / std::max(1, M));
    ts = std::min(ts, std::max(1, kMaxTilePoints / M));
    if (S == 1) ts = (int)std::min<int64_t>(ts, A);
    else ts = (int)std::min<int64_t>(ts, S);
    ts = std::max(ts, 1);
    const int lim = lds_limit_bytes();
    while (ts > 1 && (int64_t)pass_lds_bytes(kind, p->dbl, ts, M) > lim) --ts;
    return ts;
}

// Builds the op list for one block: q ranges per padded axis [qb[p], qb[p]+qn[p]); slices0 leading slices.
int num_cus() {
    static int cached = -1;
    if (cached < 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            cached = v;
        else
            cached = 256;
    }
    return cached;
}

// Builds the op list for one block: q ranges per padded axis [qb[p], qb[p]+qn[p]); slices0 leading slices.
// A fused EA pass whose lines alone cannot fill the device is split into E (parallel over the
// magnification index as well) followed by A; likewise EAH into AH + EH.
std::vector<Op> build_ops(const fx_plan* p, const int qb[3], const int qn[3], int64_t slices0, bool adjoint) {
    std::vector<Op> ops;
    int64_t lens[3] = {p->len[0], p->len[1], p->len[2]};
    int64_t slices = slices0;
    auto geom = [&](Kind kind, int ax, int64_t qin) {
        PassGeom g;
        g.A = 1;
        g.S = 1;
        for (int i = 0; i < ax; ++i) g.A *= lens[i];
        for (int i = ax + 1; i < 3; ++i) g.S *= lens[i];
        g.Qin = qin;
        g.qb = qb[ax];
        g.qn = qn[ax];
        const bool reg_eh = kind == Kind::EH && p->use_cfp && p->ax[ax].HT != nullptr && qn[ax] <= 64 &&
                            ehr_applicable(p->ax[ax].M, p->ax[ax].g);
        g.eaw = kind == Kind::EA && p->use_cfp && p->use_eaw && p->ax[ax].HTx != nullptr &&
                eaw_applicable(p->dbl, p->ax[ax].M, p->ax[ax].g, qn[ax]);
        g.erw = kind == Kind::E && p->use_cfp && p->use_erw > 0 && p->ax[ax].HT != nullptr && g.S == 1 &&
                erw_applicable(p->dbl, p->ax[ax].M, p->ax[ax].g) && (p->ax[ax].P >= 32 || p->use_erw == 2);
        g.erg = !g.erw && (kind == Kind::E || kind == Kind::EA || kind == Kind::EH) && p->use_cfp &&
                p->use_erw > 0 && p->ax[ax].HT != nullptr && erg_applicable(p->dbl, p->ax[ax].M, p->ax[ax].g) &&
                (p->ax[ax].P >= 32 || p->use_erw == 2);
        if (g.erg) {
            // the term staging must fit the LDS (EA: every term's TA and Tf values; EH: every term's TA)
            const int64_t need = kind == Kind::EH
                                     ? (int64_t)ehg_lds_bytes(p->dbl, p->ax[ax].M, p->ax[ax].g, qn[ax], g.S != 1)
                                     : (int64_t)erg_lds_bytes(p->dbl, kind, p->ax[ax].M, p->ax[ax].g,
                                                              kind == Kind::EA ? qn[ax] : 1, qn[ax], g.S != 1);
            if (need > lds_limit_bytes()) g.erg = false;
        }
        g.eas = !g.eaw && !g.erg && kind == Kind::EA && p->use_cfp && p->ax[ax].HTx != nullptr &&
                (p->use_eas == 2 || (p->use_eas == 1 && p->ax[ax].P >= 8 && p->ax[ax].g <= 16)) &&
                eas_applicable(p->dbl, p->ax[ax].M, p->ax[ax].g, qn[ax]);
        const bool reg = !g.eas && !g.eaw && (g.erw || g.erg || use_cfp(p, kind, p->ax[ax]) || reg_eh);
        g.eh2 = kind == Kind::EH && !reg_eh && !g.erg && p->use_eh2 && eh2_applicable(p->ax[ax].M, p->ax[ax].P);
        g.TS = g.erw ? erw_tile_lines(p->ax[ax].P)
               : g.erg ? erg_tile_lines(p->ax[ax].M, p->ax[ax].g)
               : g.eaw ? eaw_tile_lines()
               : g.eas ? eas_tile_lines(p->ax[ax].g)
                     : reg_eh ? ehr_tile_lines(p->ax[ax].g)
                              : reg ? cfp_tile_lines(p->ax[ax].g) : choose_ts(p, kind, p->ax[ax].M, g.A, g.S);
        auto set_tiles = [&]() {
            if (g.S == 1) g.ntiles = (g.A + g.TS - 1) / g.TS;
            else g.ntiles = g.A * ((g.S + g.TS - 1) / g.TS);
        };
        set_tiles();
        if (!reg && (kind == Kind::EH || kind == Kind::EAH)) {
            // these sum every term inside the workgroup: fewer lines per tile when the tiles alone
            // would leave CUs idle
            while (g.TS > 1 && g.Qin * g.ntiles < 2 * (int64_t)num_cus()) {
                g.TS = (g.TS + 1) / 2;
                set_tiles();
            }
        }
        g.max_blocks = p->persist > 0 ? p->persist * num_cus() : 0;
        g.reg_a = (kind == Kind::A || kind == Kind::AH) && p->use_asr && asr_applicable(p->ax[ax].g, p->asr_max_g);
        if (reg && kind == Kind::EA) {
            g.qc = g.qn;  // the fused pass sums every magnification index inside the workgroup
        } else if (reg_eh || (g.erg && kind == Kind::EH)) {
            g.qc = g.qn;  // every term of an output line inside one workgroup
        } else if (reg) {
            // magnification indices per workgroup: as many as keep >= cfp_blocks workgroups
            const int64_t base = g.Qin * g.ntiles;
            const int64_t want = std::max<int64_t>(1, (int64_t)p->cfp_blocks);
            g.qc = (int)std::max<int64_t>(1, std::min<int64_t>(g.qn, (base * g.qn + want - 1) / want));
            if (g.erw)
                while (g.qc > 1 && (int64_t)erw_lds_bytes(p->dbl, p->ax[ax].P, g.qc) > lds_limit_bytes()) --g.qc;
            if (g.erg)
                while (g.qc > 1 && (int64_t)erg_lds_bytes(p->dbl, kind, p->ax[ax].M, p->ax[ax].g, g.qc, g.qn, g.S != 1) >
                                       lds_limit_bytes())
                    --g.qc;
        }
        return g;
    };
    auto vol = [&]() { return slices * lens[0] * lens[1] * lens[2]; };
    auto emit = [&](Kind kind, int ax, const PassGeom& g, int64_t in_e) {
        Op o{kind, ax, g, in_e, vol()};
        ops.push_back(o);
    };
    // forward E: axis full -> pruned, slices x qn
    auto do_E = [&](int ax) {
        const int64_t in_e = vol();
        PassGeom g = geom(Kind::E, ax, slices);
        lens[ax] = p->ax[ax].P;
        slices *= qn[ax];
        emit(Kind::E, ax, g, in_e);
    };
    // forward A: axis pruned -> full, slices / qn
    auto do_A = [&](int ax) {
        const int64_t in_e = vol();
        slices /= qn[ax];
        lens[ax] = p->ax[ax].M;
        emit(Kind::A, ax, geom(Kind::A, ax, slices), in_e);
    };
    auto do_AH = [&](int ax) {
        const int64_t in_e = vol();
        PassGeom g = geom(Kind::AH, ax, slices);
        lens[ax] = p->ax[ax].P;
        slices *= qn[ax];
        emit(Kind::AH, ax, g, in_e);
    };
    auto do_EH = [&](int ax) {
        const int64_t in_e = vol();
        slices /= qn[ax];
        lens[ax] = p->ax[ax].M;
        emit(Kind::EH, ax, geom(Kind::EH, ax, slices), in_e);
    };
    auto split = [&](Kind kind, int ax) {
        if (!p->allow_split || qn[ax] < 2) return false;
        PassGeom g = geom(kind, ax, slices);
        return g.Qin * g.ntiles < 2 * (int64_t)num_cus();
    };
    auto do_EA = [&](int ax) {
        // the structured EA kernel spreads the terms over the waves of a workgroup: never split
        if (!geom(Kind::EA, ax, slices).eas && split(Kind::EA, ax)) { do_E(ax); do_A(ax); return; }
        emit(Kind::EA, ax, geom(Kind::EA, ax, slices), vol());
    };
    // the adjoint of EA runs as AH + EH when both have register forms (each is cheaper than the
    // fused generic pass), or when the fused launch would be small
    auto reg_adjoint = [&](int ax) {
        const AxisDev& a = p->ax[ax];
        return p->use_asr && asr_applicable(a.g, p->asr_max_g) && p->use_cfp && a.HT != nullptr &&
               qn[ax] <= 64 && ehr_applicable(a.M, a.g);
    };
    auto do_EAH = [&](int ax) {
        // also split where EH has its compile-time power-of-two kernel (the fused generic pass
        // runs one transform chain per term and workgroup)
        const bool eh2 = p->use_eh2 && eh2_applicable(p->ax[ax].M, p->ax[ax].P);
        // the register adjoint E in the lanes-per-line layout, where the intermediate of the split
        // (every term's pruned lines) stays well inside 32-bit indexing
        const bool ehg = geom(Kind::EH, ax, slices / std::max(1, qn[ax])).erg &&
                         vol() / p->ax[ax].M * p->ax[ax].P * qn[ax] < kIndexLimit / 4;
        if (reg_adjoint(ax) || eh2 || ehg || split(Kind::EAH, ax)) { do_AH(ax); do_EH(ax); return; }
        emit(Kind::EAH, ax, geom(Kind::EAH, ax, slices), vol());
    };
    const int k = p->nact;
    if (k == 0) return ops;
    if (p->schedule == FX_SCHED_AXIS_FACTORISED) {
        if (!adjoint) {
            for (int i = k - 1; i >= 0; --i) do_EA(p->act[i]);
        } else {
            for (int i = 0; i < k; ++i) do_EAH(p->act[i]);
        }
        return ops;
    }
    if (!adjoint) {
        for (int i = k - 1; i >= 1; --i) do_E(p->act[i]);
        do_EA(p->act[0]);
        for (int i = 1; i < k; ++i) do_A(p->act[i]);
        // fuse the last two accumulate passes (axes u < v) into one 2-D structured accumulate
        const size_t n = ops.size();
        if (p->use_aa && n >= 2 && ops[n - 2].kind == Kind::A && ops[n - 1].kind == Kind::A) {
            const Op& ou = ops[n - 2];
            const Op& ov = ops[n - 1];
            const int u = ou.axis, v = ov.axis;
            const AxisDev& au = p->ax[u];
            const AxisDev& av = p->ax[v];
            AAGeom a;
            a.O = ov.g.Qin;
            a.qn_u = ou.g.qn;
            a.qb_u = ou.g.qb;
            a.qn_v = ov.g.qn;
            a.qb_v = ov.g.qb;
            // lengths of the other axes as the fused pass sees them (u and v excluded)
            a.X = ou.g.A;                               // axes before u
            a.Z = ov.g.S;                               // axes after v
            a.Y = u < v ? ou.g.S / ((int64_t)av.P * a.Z) : 0;  // axes between u and v
            a.tsg = aa_tile_groups(au.g, av.g);
            // the register form wherever it applies; the LDS form only when asked for (FX_AA=1)
            const bool reg = u < v && aar_applicable(au.g, av.g, au.P, av.P, a);
            const bool lds = u < v && p->use_aa == 2 && aa_applicable(p->dbl, au.g, av.g) &&
                             (int64_t)aa_lds_bytes(p->dbl, au.g, av.g) <= lds_limit_bytes();
            if (reg || lds) {
                Op f = ou;
                f.kind = Kind::AA;
                f.axis2 = v;
                f.out_elems = ov.out_elems;
                f.aa = a;
                ops.pop_back();
                ops.back() = f;
            }
        }
    } else {
        for (int i = k - 1; i >= 1; --i) do_AH(p->act[i]);
        do_EAH(p->act[0]);
        for (int i = 1; i < k; ++i) do_EH(p->act[i]);
        // the adjoint of the fused accumulate: the first two AH passes (axes v > u), register form
        if (p->use_aa && ops.size() >= 2 && ops[0].kind == Kind::AH && ops[1].kind == Kind::AH &&
            ops[1].axis < ops[0].axis) {
            const Op& ov = ops[0];
            const Op& ou = ops[1];
            const int u = ou.axis, v = ov.axis;
            AAGeom a;
            a.O = ov.g.Qin;
            a.qn_u = ou.g.qn;
            a.qb_u = ou.g.qb;
            a.qn_v = ov.g.qn;
            a.qb_v = ov.g.qb;
            a.X = ou.g.A;
            a.Z = ov.g.S;
            a.Y = ou.g.S / ((int64_t)p->ax[v].P * a.Z);
            a.tsg = 1;
            if (aar_applicable(p->ax[u].g, p->ax[v].g, p->ax[u].P, p->ax[v].P, a)) {
                Op f = ou;
                f.kind = Kind::AAH;
                f.axis = u;
                f.axis2 = v;
                f.in_elems = ov.in_elems;
                f.aa = a;
                ops.erase(ops.begin());
                ops[0] = f;
            }
        }
    }
    return ops;
}

int64_t max_intermediate(const std::vector<Op>& ops) {
    int64_t m = 0;
    for (size_t i = 0; i + 1 < ops.size(); ++i) m = std::max(m, ops[i].out_elems);
    return m;
}

fx_status validate(const fx_problem* pr) {
    if (!pr) { set_error("problem is NULL"); return FX_EINVAL; }
    if (pr->ndim < 1 || pr->ndim > 3) { set_error("ndim must be 1, 2 or 3"); return FX_EINVAL; }
    for (int j = 0; j < pr->ndim; ++j) {
        if (pr->shape[j] < 1) { set_error("shape[j] must be >= 1"); return FX_EINVAL; }
        if (!(std::isfinite(pr->dx[j]) && pr->dx[j] > 0)) { set_error("dx[j] must be finite and > 0"); return FX_EINVAL; }
        if (pr->lambda[j] < 1) { set_error("lambda[j] must be an integer >= 1"); return FX_EINVAL; }
        if (std::isinf(pr->a[j]) || std::isinf(pr->abar[j])) { set_error("offsets must be finite or NaN"); return FX_EINVAL; }
    }
    if (!(std::isfinite(pr->m_over_hbar) && pr->m_over_hbar > 0)) { set_error("m_over_hbar must be finite and > 0"); return FX_EINVAL; }
    if (!std::isfinite(pr->t_flight)) { set_error("t_flight must be finite"); return FX_EINVAL; }
    if (pr->precision != FX_PREC_C128 && pr->precision != FX_PREC_C64_PHASE64) { set_error("unknown precision"); return FX_EINVAL; }
    if (pr->schedule != FX_SCHED_PAPER && pr->schedule != FX_SCHED_AXIS_FACTORISED) { set_error("unknown schedule"); return FX_EINVAL; }
    int64_t tot = 1;
    for (int j = 0; j < pr->ndim; ++j) {
        if (pr->shape[j] > kMaxAxis) { set_error("axis longer than 4096 points is not supported by the in-LDS transforms"); return FX_EUNSUPPORTED; }
        if ((int64_t)pr->lambda[j] * pr->shape[j] > (int64_t(1) << 26)) { set_error("lambda*M above 2^26 per axis is not supported"); return FX_EUNSUPPORTED; }
        tot *= pr->shape[j];
    }
    if (tot >= (int64_t(1) << 31)) { set_error("2^31 or more lattice points per field"); return FX_EUNSUPPORTED; }
    return FX_OK;
}

template <typename T>
void to_prec(const std::vector<double>& src, std::vector<unsigned char>& dst, size_t off) {
    T* d = (T*)(dst.data() + off);
    for (size_t i = 0; i < src.size(); ++i) d[i] = (T)src[i];
}

void workspace_layout(const fx_plan* p, int64_t slices, int64_t* nb_out, int64_t* buf_out, size_t* need_out) {
    workspace_layout_for(p, slices, true, nb_out, buf_out, need_out);
}

void workspace_layout_for(const fx_plan* p, int64_t slices, bool with_adjoint, int64_t* nb_out, int64_t* buf_out,
                          size_t* need_out) {
    const int k = p->nact;
    int qb[3] = {0, 0, 0}, qn[3];
    for (int i = 0; i < 3; ++i) qn[i] = p->ax[i].lam;
    int64_t outer_lam = (k > 0) ? p->ax[p->act[k - 1]].lam : 1;
    int64_t nb = outer_lam;
    const size_t cs = csize(p);
    auto need = [&](int64_t nbv) {
        int qn2[3] = {qn[0], qn[1], qn[2]};
        if (k > 0 && p->schedule == FX_SCHED_PAPER) qn2[p->act[k - 1]] = (int)nbv;
        std::vector<Op> f = build_ops(p, qb, qn2, slices, false);
        if (!with_adjoint) return max_intermediate(f);
        std::vector<Op> h = build_ops(p, qb, qn2, slices, true);
        return std::max(max_intermediate(f), max_intermediate(h));
    };
    if (p->schedule == FX_SCHED_PAPER) {
        if (p->nb_fixed > 0) nb = std::min<int64_t>(p->nb_fixed, outer_lam);
        else
            while (nb > 1 && ((size_t)need(nb) * 2 * cs > p->budget || need(nb) >= kIndexLimit)) nb = (nb + 1) / 2;
    }
    *nb_out = std::max<int64_t>(1, nb);
    *buf_out = need(*nb_out);
    *need_out = (size_t)(2 * *buf_out + slices * p->M) * cs + 1024;
}

// The kernels decode tiles, groups and grid positions in 32-bit arithmetic: every pass tensor
// (input, intermediates, output) must stay below kIndexLimit elements. Checked here, before any
// launch, so that an oversized layout fails as a whole instead of after some passes ran.
static bool layout_indexes_in_32_bits(const fx_plan* p) {
    if (p->slices * p->M >= kIndexLimit) return false;
    return p->buf_elems < kIndexLimit;
}

fx_status plan_setup_workspace(fx_plan* p, int64_t slices) {
    p->slices = slices;
    workspace_layout(p, slices, &p->nb_outer, &p->buf_elems, &p->ws_need);
    p->index_ok = layout_indexes_in_32_bits(p);
    return FX_OK;
}

fx_status ensure_workspace(fx_plan* p) {
    if (!p->index_ok) {
        set_error("a pass tensor of this problem (times its batch) reaches 2^31 elements, beyond the "
                  "kernels' 32-bit tile and grid indexing");
        return FX_EUNSUPPORTED;
    }
    if (p->ws && p->ws_bytes >= p->ws_need) return FX_OK;
    if (p->ws && !p->ws_owned) {
        set_error("caller workspace smaller than this call needs (fx_plan_workspace_size, "
                  "fx_plan_pair_workspace_size for pairs)");
        return FX_ENOMEM;
    }
    if (p->ws_owned && p->ws) {
        (void)hipFree(p->ws);
        p->ws = nullptr;
    }
    void* w = nullptr;
    if (hipMalloc(&w, p->ws_need) != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipMalloc of workspace failed");
        return FX_ENOMEM;
    }
    p->ws = w;
    p->ws_bytes = p->ws_need;
    p->ws_owned = true;
    return FX_OK;
}

// Runs the op list of one block. src: input tensor, dst: final output; X/Y ping-pong.
fx_status run_ops(fx_plan* p, const std::vector<Op>& ops, const void* src, void* dst, int accumulate, void* rho,
                  hipStream_t st, int slot0) {
    char* base = (char*)p->ws;
    void* bufs[2] = {base, base + (size_t)p->buf_elems * csize(p)};
    const void* cur = src;
    for (size_t i = 0; i < ops.size(); ++i) {
        const bool last = (i + 1 == ops.size());
        void* out = last ? dst : bufs[i % 2];
        const Op& o = ops[i];
        hipEvent_t ea = nullptr, eb = nullptr;
        if (p->timing) {
            for (hipEvent_t* ev : {&ea, &eb}) {
                if (!p->pool.empty()) { *ev = p->pool.back(); p->pool.pop_back(); }
                else FX_TRY_HIP(hipEventCreate(ev));
            }
            FX_TRY_HIP(hipEventRecord(ea, st));
        }
        hipError_t e = (o.kind == Kind::AA)
                           ? launch_pass_aa(p->dbl, cur, out, p->ax[o.axis], p->ax[o.axis2], o.aa,
                                            last ? accumulate : 0, last ? rho : nullptr, st)
                       : (o.kind == Kind::AAH)
                           ? launch_pass_aah(p->dbl, cur, out, p->ax[o.axis], p->ax[o.axis2], o.aa,
                                             last ? accumulate : 0, st)
                           : launch_pass(o.kind, p->dbl, cur, out, p->ax[o.axis], o.g, last ? accumulate : 0,
                                         last ? rho : nullptr, st);
        if (p->timing) {
            FX_TRY_HIP(hipEventRecord(eb, st));
            p->pending.push_back({slot0 + (int)i, ea, eb});
        }
        if (e != hipSuccess) {
            set_error(std::string("kernel launch failed: ") + hipGetErrorString(e));
            return FX_EDEVICE;
        }
        cur = out;
    }
    return FX_OK;
}

// Sum over the q-box [qb, qb+qn) per padded axis, blocked along the outermost axis.
fx_status run_box(fx_plan* p, const int qb[3], const int qn[3], const void* src, void* dst, int accumulate,
                  void* rho, bool adjoint, hipStream_t st) {
    const int k = p->nact;
    const size_t cs = csize(p);
    const int64_t vol = p->slices * p->M;
    if (k == 0) {
        // every axis is a single point with lam = 1: Psibar = Psi
        if (accumulate) {
            set_error("accumulating an identity expansion is not supported");
            return FX_EUNSUPPORTED;
        }
        FX_TRY_HIP(hipMemcpyAsync(dst, src, (size_t)vol * cs, hipMemcpyDeviceToDevice, st));
        if (rho && launch_density(p->dbl, dst, rho, vol, st) != hipSuccess) return FX_EDEVICE;
        return FX_OK;
    }
    const int outer = p->act[k - 1];
    const int64_t step = (p->schedule == FX_SCHED_PAPER) ? p->nb_outer : qn[outer];
    for (int64_t c = qb[outer]; c < qb[outer] + qn[outer]; c += step) {
        int b2[3] = {qb[0], qb[1], qb[2]}, n2[3] = {qn[0], qn[1], qn[2]};
        b2[outer] = (int)c;
        n2[outer] = (int)std::min<int64_t>(step, qb[outer] + qn[outer] - c);
        const bool first = (c == qb[outer]);
        const bool lastc = (c + step >= qb[outer] + qn[outer]);
        std::vector<Op> ops = build_ops(p, b2, n2, p->slices, adjoint);
        fx_status s = run_ops(p, ops, src, dst, first ? accumulate : 1, lastc ? rho : nullptr, st,
                              adjoint ? FX_ADJOINT_SLOT0 : 0);
        if (s != FX_OK) return s;
    }
    return FX_OK;
}

fx_status check_ptr(const void* ptr, const char* what) {
    if (!ptr) {
        set_error(std::string(what) + " is NULL");
        return FX_EINVAL;
    }
    return FX_OK;
}

// Fields per chunk of a stacked call: the largest chunk (<= count) whose pass layout indexes in
// 32 bits and whose workspace fits the plan's budget, or the caller's workspace when one was set.
// Leaves the plan set up for that chunk.
int64_t stack_chunk(fx_plan* p, int64_t count, size_t extra_bytes_per_field) {
    const bool caller_ws = p->ws && !p->ws_owned;
    const size_t cap = caller_ws ? p->ws_bytes : p->budget;
    int64_t c = count;
    while (c > 1) {
        plan_setup_workspace(p, c);
        if (p->index_ok && p->ws_need + (size_t)c * extra_bytes_per_field <= cap) break;
        c = (c + 1) / 2;
    }
    plan_setup_workspace(p, c);
    return c;
}


fx_status check_disjoint(const void* a, size_t na, const char* an, const void* b, size_t nb, const char* bn) {
    if (!a || !b || na == 0 || nb == 0) return FX_OK;
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    if (a0 < b0 + nb && b0 < a0 + na) {
        set_error(std::string(an) + " and " + bn + " overlap; inputs and outputs must be disjoint");
        return FX_EINVAL;
    }
    return FX_OK;
}

}  // namespace fx

extern "C" {

fx_status fx_problem_init(fx_problem* p) {
    if (!p) return FX_EINVAL;
    std::memset(p, 0, sizeof(*p));
    p->ndim = 1;
    for (int j = 0; j < FX_MAX_DIM; ++j) {
        p->shape[j] = 1;
        p->dx[j] = 1.0;
        p->a[j] = NAN;
        p->abar[j] = NAN;
        p->lambda[j] = 1;
    }
    p->m_over_hbar = 1.0;
    p->t_flight = 0.0;
    p->precision = FX_PREC_C128;
    p->schedule = FX_SCHED_PAPER;
    return FX_OK;
}

namespace fx {

fx_status create_plan(const fx_problem* prob, const double* const* phase, fx_plan** out) {
    if (!out) { set_error("out is NULL"); return FX_EINVAL; }
    fx_status s = validate(prob);
    if (s != FX_OK) return s;
    if (const char* inj = std::getenv("FX_FAULT_INJECT_PLAN")) {
        if (inj[0] == '1') { set_error("plan creation failed by FX_FAULT_INJECT_PLAN"); return FX_ENOMEM; }
    }
    fx_plan* p = new (std::nothrow) fx_plan();
    if (!p) { set_error("host allocation failed"); return FX_ENOMEM; }
    p->prob = *prob;
    p->prob_in = *prob;
    p->dbl = (prob->precision == FX_PREC_C128);
    p->ndim = prob->ndim;
    p->schedule = prob->schedule;
    const int off = 3 - prob->ndim;
    std::vector<AxisTables> tabs(3);
    for (int pa = 0; pa < 3; ++pa) {
        AxisParams ap;
        if (pa >= off) {
            const int j = pa - off;
            ap.M = prob->shape[j];
            ap.lam = prob->lambda[j];
            ap.dx = prob->dx[j];
            const double L = (double)ap.M * ap.dx;
            ap.a = std::isnan(prob->a[j]) ? -0.5 * L : prob->a[j];
            ap.abar = std::isnan(prob->abar[j]) ? ap.a + (1.0 - (double)ap.lam) * L / 2.0 : prob->abar[j];
            p->prob.a[j] = ap.a;
            p->prob.abar[j] = ap.abar;
        }
        ap.t = prob->t_flight;
        ap.m_over_hbar = prob->m_over_hbar;
        if (phase && pa >= off) {
            ap.phase = phase[pa - off];
            p->spectrum[pa] = (ap.phase != nullptr);
        }
        p->par[pa] = ap;
        p->len[pa] = ap.M;
        AxisDev& ad = p->ax[pa];
        ad.M = (int)ap.M;
        ad.lam = ap.lam;
        ad.g = (int)gcd64(ap.lam, ap.M);
        ad.P = ad.M / ad.g;
        ad.lg = (int)((ap.lam / ad.g) % ad.P);
        ad.lg_inv = (int)modinv(ad.lg, ad.P);
        ad.scale = 1.0 / (double)ap.M;
        ad.fm = make_radix_plan(ad.M);
        ad.fp = make_radix_plan(ad.P);
        ad.fg = make_radix_plan(ad.g);
        ap.want_ht = (cfp_applicable(Kind::E, p->dbl, (int)ap.M, ad.g) || erw_applicable(p->dbl, (int)ap.M, ad.g) ||
                      erg_applicable(p->dbl, (int)ap.M, ad.g)) &&
                     ap.lam * ap.M * (int64_t)ad.g <= (int64_t(1) << 26);
        tabs[pa] = build_axis_tables(ap);
        p->par[pa].phase = nullptr;  // the caller's table is not kept
        if (!(ap.M == 1 && ap.lam == 1)) p->act[p->nact++] = pa;
    }
    p->M = p->len[0] * p->len[1] * p->len[2];
    p->Q = (int64_t)p->ax[0].lam * p->ax[1].lam * p->ax[2].lam;
    for (int i = 0; i < p->nact; ++i) {
        const int M = p->ax[p->act[i]].M;
        const size_t lds = pass_lds_bytes(Kind::EA, p->dbl, 1, M);
        if ((int64_t)lds > lds_limit_bytes()) {
            set_error("axis too long for the in-LDS transform at this precision");
            delete p;
            return FX_EUNSUPPORTED;
        }
    }
    // Upload all tables in one allocation: per axis TA | TB | Tf | tw | HT | HTx | HTl.
    const size_t cs = csize(p);
    size_t total = 0;
    size_t offs[3][7];
    for (int pa = 0; pa < 3; ++pa) {
        const size_t lm = (size_t)p->ax[pa].lam * p->ax[pa].M;
        const size_t sz[7] = {lm, lm, lm, (size_t)p->ax[pa].M, tabs[pa].HT.size() / 2, tabs[pa].HTx.size() / 2,
                              tabs[pa].HTl.size() / 2};
        for (int t = 0; t < 7; ++t) {
            offs[pa][t] = total;
            total += ((sz[t] * cs + 255) / 256) * 256;
        }
    }
    std::vector<unsigned char> host(total, 0);
    for (int pa = 0; pa < 3; ++pa) {
        const std::vector<double>* src[7] = {&tabs[pa].TA, &tabs[pa].TB, &tabs[pa].Tf, &tabs[pa].tw, &tabs[pa].HT,
                                             &tabs[pa].HTx, &tabs[pa].HTl};
        for (int t = 0; t < 7; ++t) {
            if (p->dbl) to_prec<double>(*src[t], host, offs[pa][t]);
            else to_prec<float>(*src[t], host, offs[pa][t]);
        }
    }
    if (hipMalloc(&p->dtab, total) != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipMalloc of tables failed (no device?)");
        delete p;
        return FX_EDEVICE;
    }
    p->dtab_bytes = total;
    if (hipMemcpy(p->dtab, host.data(), total, hipMemcpyHostToDevice) != hipSuccess) {
        set_error("table upload failed");
        (void)hipFree(p->dtab);
        delete p;
        return FX_EDEVICE;
    }
    for (int pa = 0; pa < 3; ++pa) {
        char* b = (char*)p->dtab;
        p->ax[pa].TA = b + offs[pa][0];
        p->ax[pa].TB = b + offs[pa][1];
        p->ax[pa].Tf = b + offs[pa][2];
        p->ax[pa].tw = b + offs[pa][3];
        p->ax[pa].HT = tabs[pa].HT.empty() ? nullptr : b + offs[pa][4];
        p->ax[pa].HTx = tabs[pa].HTx.empty() ? nullptr : b + offs[pa][5];
        p->ax[pa].HTl = tabs[pa].HTl.empty() ? nullptr : b + offs[pa][6];
    }
    size_t budget = (size_t)8 << 30;
    if (const char* e = std::getenv("FX_WORKSPACE_MB")) budget = (size_t)std::max(1L, std::atol(e)) << 20;
    size_t freeb = 0, totb = 0;
    if (hipMemGetInfo(&freeb, &totb) == hipSuccess && freeb / 4 < budget) budget = std::max<size_t>(freeb / 4, 1 << 20);
    p->budget = budget;
    if (const char* e = std::getenv("FX_TILE_POINTS")) p->ts_target = std::max(1, std::atoi(e));
    if (const char* e = std::getenv("FX_NO_SPLIT")) p->allow_split = (e[0] != '1');
    if (const char* e = std::getenv("FX_NO_P2")) p->use_p2 = (e[0] != '1');
    if (const char* e = std::getenv("FX_NO_CFP")) p->use_cfp = (e[0] != '1');
    if (const char* e = std::getenv("FX_NO_ASR")) p->use_asr = (e[0] != '1');
    if (const char* e = std::getenv("FX_AA")) p->use_aa = (e[0] == '1') ? 2 : 0;
    if (const char* e = std::getenv("FX_EAS")) p->use_eas = (e[0] == '1') ? 2 : 1;
    if (std::getenv("FX_NO_EAS")) p->use_eas = 0;
    if (std::getenv("FX_NO_EAW")) p->use_eaw = false;
    if (const char* e = std::getenv("FX_ERW")) p->use_erw = std::atoi(e);
    if (std::getenv("FX_NO_EH2")) p->use_eh2 = false;
    if (const char* e = std::getenv("FX_ASR_MAXG")) p->asr_max_g = std::max(1, std::atoi(e));
    p->cfp_blocks = 2 * num_cus();
    if (const char* e = std::getenv("FX_CFP_BLOCKS")) p->cfp_blocks = std::max(1, std::atoi(e));
    plan_setup_workspace(p, 1);
    *out = p;
    return FX_OK;
}

}  // namespace fx

fx_status fx_plan_create(const fx_problem* prob, fx_plan** out) { return create_plan(prob, nullptr, out); }

fx_status fx_plan_create_spectrum(const fx_problem* prob, const double* const* phase, fx_plan** out) {
    if (!phase) { set_error("phase is NULL"); return FX_EINVAL; }
    fx_status s = validate(prob);
    if (s != FX_OK) return s;
    {
        for (int j = 0; j < prob->ndim; ++j) {
            if (!phase[j]) continue;
            const int64_t n = (int64_t)prob->lambda[j] * prob->shape[j];
            for (int64_t i = 0; i < n; ++i) {
                if (!std::isfinite(phase[j][i])) {
                    set_error("phase table holds a non-finite value");
                    return FX_EINVAL;
                }
            }
        }
    }
    return create_plan(prob, phase, out);
}

fx_status fx_plan_destroy(fx_plan* p) {
    if (!p) return FX_OK;
    for (const auto& pe : p->pending) {
        (void)hipEventSynchronize(pe.b);
        p->pool.push_back(pe.a);
        p->pool.push_back(pe.b);
    }
    for (hipEvent_t e : p->pool) (void)hipEventDestroy(e);
    if (p->ws_owned && p->ws) (void)hipFree(p->ws);
    if (p->dtab) (void)hipFree(p->dtab);
    if (p->ff_tab) (void)hipFree(p->ff_tab);
    if (p->ff_buf) (void)hipFree(p->ff_buf);
    bf_release(p);
    delete p;
    return FX_OK;
}

fx_status fx_plan_num_terms(const fx_plan* p, int64_t* q) {
    if (!p || !q) { set_error("NULL argument"); return FX_EINVAL; }
    *q = p->Q;
    return FX_OK;
}

fx_status fx_plan_workspace_size(const fx_plan* p, size_t* bytes) {
    if (!p || !bytes) { set_error("NULL argument"); return FX_EINVAL; }
    int64_t nb = 0, buf = 0;
    workspace_layout(p, 1, &nb, &buf, bytes);
    return FX_OK;
}

fx_status fx_plan_set_workspace(fx_plan* p, void* dev_ptr, size_t bytes) {
    if (!p) { set_error("plan is NULL"); return FX_EINVAL; }
    if (dev_ptr == nullptr && bytes == 0) {
        if (!p->ws_owned) { p->ws = nullptr; p->ws_bytes = 0; }
        return FX_OK;
    }
    if (!dev_ptr) { set_error("workspace pointer is NULL"); return FX_EINVAL; }
    if (((uintptr_t)dev_ptr) % 256 != 0) { set_error("workspace must be 256-byte aligned"); return FX_EINVAL; }
    size_t need = 0;
    (void)fx_plan_workspace_size(p, &need);
    if (bytes < need) { set_error("workspace smaller than fx_plan_workspace_size()"); return FX_ENOMEM; }
    if (p->ws_owned && p->ws) (void)hipFree(p->ws);
    p->ws = dev_ptr;
    p->ws_bytes = bytes;
    p->ws_owned = false;
    return FX_OK;
}

fx_status fx_expand(fx_plan* p, const void* psi0, void* psi_out, void* rho_out, void* stream) {
    if (!p) { set_error("plan is NULL"); return FX_EINVAL; }
    fx_status s = check_ptr(psi0, "psi0");
    if (s != FX_OK) return s;
    if (!psi_out && !rho_out) { set_error("psi_out and rho_out are both NULL"); return FX_EINVAL; }
    const size_t cb = (size_t)p->M * csize(p), rb = cb / 2;
    if ((s = check_disjoint(psi0, cb, "psi0", psi_out, cb, "psi_out")) != FX_OK) return s;
    if ((s = check_disjoint(psi0, cb, "psi0", rho_out, rb, "rho_out")) != FX_OK) return s;
    if ((s = check_disjoint(psi_out, cb, "psi_out", rho_out, rb, "rho_out")) != FX_OK) return s;
    if (p->slices != 1) plan_setup_workspace(p, 1);
    if ((s = ensure_workspace(p)) != FX_OK) return s;
    void* dst = psi_out ? psi_out : (char*)p->ws + (size_t)2 * p->buf_elems * csize(p);
    int qb[3] = {0, 0, 0}, qn[3] = {p->ax[0].lam, p->ax[1].lam, p->ax[2].lam};
    return run_box(p, qb, qn, psi0, dst, 0, rho_out, false, (hipStream_t)stream);
}


fx_status fx_expand_many(fx_plan* p, int64_t count, const void* psi0, void* psi_out, void* rho_out, void* stream) {
    if (!p) { set_error("plan is NULL"); return FX_EINVAL; }
    if (count < 1) { set_error("count must be >= 1"); return FX_EINVAL; }
    fx_status s = check_ptr(psi0, "psi0");
    if (s != FX_OK) return s;
    if (!psi_out && !rho_out) { set_error("psi_out and rho_out are both NULL"); return FX_EINVAL; }
    const size_t cb = (size_t)p->M * csize(p), rb = cb / 2;
    if ((s = check_disjoint(psi0, count * cb, "psi0", psi_out, count * cb, "psi_out")) != FX_OK) return s;
    if ((s = check_disjoint(psi0, count * cb, "psi0", rho_out, count * rb, "rho_out")) != FX_OK) return s;
    if ((s = check_disjoint(psi_out, count * cb, "psi_out", rho_out, count * rb, "rho_out")) != FX_OK) return s;
    const int64_t chunk = stack_chunk(p, count, 0);
    if ((s = ensure_workspace(p)) != FX_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    int qb[3] = {0, 0, 0}, qn[3] = {p->ax[0].lam, p->ax[1].lam, p->ax[2].lam};
    for (int64_t f = 0; f < count; f += chunk) {
        const int64_t c = std::min(chunk, count - f);
        if (c != p->slices) plan_setup_workspace(p, c);  // the last, shorter chunk needs less
        const char* src = (const char*)psi0 + (size_t)f * cb;
        void* dst = psi_out ? (char*)psi_out + (size_t)f * cb : (char*)p->ws + (size_t)2 * p->buf_elems * csize(p);
        void* rho = rho_out ? (char*)rho_out + (size_t)f * rb : nullptr;
        if ((s = run_box(p, qb, qn, src, dst, 0, rho, false, st)) != FX_OK) return s;
    }
    return FX_OK;
}

fx_status fx_expand_range(fx_plan* p, const void* psi0, void* psi_acc, int64_t q_begin, int64_t q_end,
                          int accumulate, void* stream) {
    if (!p) { set_error("plan is NULL"); return FX_EINVAL; }
    fx_status s = check_ptr(psi0, "psi0");
    if (s != FX_OK) return s;
    if ((s = check_ptr(psi_acc, "psi_acc")) != FX_OK) return s;
    if (q_begin < 0 || q_end < q_begin || q_end > p->Q) { set_error("need 0 <= q_begin <= q_end <= terms"); return FX_EINVAL; }
    if (p->schedule != FX_SCHED_PAPER) { set_error("term ranges exist only for the paper schedule"); return FX_EUNSUPPORTED; }
    if ((s = check_disjoint(psi0, (size_t)p->M * csize(p), "psi0", psi_acc, (size_t)p->M * csize(p), "psi_acc")) != FX_OK)
        return s;
    if (p->slices != 1) plan_setup_workspace(p, 1);
    if ((s = ensure_workspace(p)) != FX_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    if (q_begin == q_end) {
        if (!accumulate) FX_TRY_HIP(hipMemsetAsync(psi_acc, 0, (size_t)p->M * csize(p), st));
        return FX_OK;
    }
    // Linear index: C order over the active axes from the contiguous (slowest-varying index) to axis 0.
    const int k = p->nact;
    if (k == 0) {
        const int zb[3] = {0, 0, 0}, on[3] = {1, 1, 1};
        return run_box(p, zb, on, psi0, psi_acc, accumulate, nullptr, false, st);
    }
    // levels: outermost first
    int lev[3];
    for (int i = 0; i < k; ++i) lev[i] = p->act[k - 1 - i];
    // Recursive decomposition of [qb, qe) into boxes.
    struct Box { int qb[3]; int qn[3]; };
    std::vector<Box> boxes;
    std::function<void(int, int64_t, int64_t, Box)> rec = [&](int level, int64_t b, int64_t e, Box pre) {
        if (b >= e) return;
        const int ax = lev[level];
        int64_t inner = 1;
        for (int i = level + 1; i < k; ++i) inner *= p->ax[lev[i]].lam;
        if (level == k - 1) {
            Box bx = pre;
            bx.qb[ax] = (int)b;
            bx.qn[ax] = (int)(e - b);
            boxes.push_back(bx);
            return;
        }
        int64_t hb = b / inner, he = e / inner;
        if (hb == he) {
            Box bx = pre;
            bx.qb[ax] = (int)hb;
            bx.qn[ax] = 1;
            rec(level + 1, b - hb * inner, e - hb * inner, bx);
            return;
        }
        if (b % inner) {
            Box bx = pre;
            bx.qb[ax] = (int)hb;
            bx.qn[ax] = 1;
            rec(level + 1, b - hb * inner, inner, bx);
            hb += 1;
        }
        if (he > hb) {
            Box bx = pre;
            bx.qb[ax] = (int)hb;
            bx.qn[ax] = (int)(he - hb);
            for (int i = level + 1; i < k; ++i) {
                bx.qb[lev[i]] = 0;
                bx.qn[lev[i]] = p->ax[lev[i]].lam;
            }
            boxes.push_back(bx);
        }
        if (e % inner) {
            Box bx = pre;
            bx.qb[ax] = (int)he;
            bx.qn[ax] = 1;
            rec(level + 1, 0, e - he * inner, bx);
        }
    };
    Box root;
    for (int i = 0; i < 3; ++i) { root.qb[i] = 0; root.qn[i] = 1; }
    rec(0, q_begin, q_end, root);
    for (size_t i = 0; i < boxes.size(); ++i) {
        s = run_box(p, boxes[i].qb, boxes[i].qn, psi0, psi_acc, (i == 0) ? accumulate : 1, nullptr, false, st);
        if (s != FX_OK) return s;
    }
    return FX_OK;
}

fx_status fx_density(fx_plan* p, const void* psi, void* rho, void* stream) {
    if (!p) { set_error("plan is NULL"); return FX_EINVAL; }
    fx_status s = check_ptr(psi, "psi");
    if (s != FX_OK) return s;
    if ((s = check_ptr(rho, "rho")) != FX_OK) return s;
    if ((s = check_disjoint(psi, (size_t)p->M * csize(p), "psi", rho, (size_t)p->M * csize(p) / 2, "rho")) != FX_OK)
        return s;
    if (launch_density(p->dbl, psi, rho, p->M, (hipStream_t)stream) != hipSuccess) {
        set_error("density launch failed");
        return FX_EDEVICE;
    }
    return FX_OK;
}

fx_status fx_column_density(fx_plan* p, const void* rho, int axis, void* image, void* stream) {
    if (!p) { set_error("plan is NULL"); return FX_EINVAL; }
    fx_status s = check_ptr(rho, "rho");
    if (s != FX_OK) return s;
    if ((s = check_ptr(image, "image")) != FX_OK) return s;
    if (axis < 0 || axis >= p->ndim) { set_error("axis out of range"); return FX_EINVAL; }
    const int pa = axis + (3 - p->ndim);
    int64_t A = 1, S = 1;
    for (int i = 0; i < pa; ++i) A *= p->len[i];
    for (int i = pa + 1; i < 3; ++i) S *= p->len[i];
    const double w = (double)p->par[pa].lam * p->par[pa].dx;
    const size_t rs = csize(p) / 2;
    if ((s = check_disjoint(rho, (size_t)p->M * rs, "rho", image, (size_t)(A * S) * rs, "image")) != FX_OK) return s;
    if (launch_column(p->dbl, rho, image, A, p->len[pa], S, w, (hipStream_t)stream) != hipSuccess) {
        set_error("column density launch failed");
        return FX_EDEVICE;
    }
    return FX_OK;
}

fx_status fx_expand_adjoint(fx_plan* p, const void* grad_out, void* grad_in, void* stream) {
    if (!p) { set_error("plan is NULL"); return FX_EINVAL; }
    fx_status s = check_ptr(grad_out, "grad_psi_out");
    if (s != FX_OK) return s;
    if ((s = check_ptr(grad_in, "grad_psi0")) != FX_OK) return s;
    if ((s = check_disjoint(grad_out, (size_t)p->M * csize(p), "grad_psi_out", grad_in, (size_t)p->M * csize(p),
                            "grad_psi0")) != FX_OK)
        return s;
    if (p->slices != 1) plan_setup_workspace(p, 1);
    if ((s = ensure_workspace(p)) != FX_OK) return s;
    int qb[3] = {0, 0, 0}, qn[3] = {p->ax[0].lam, p->ax[1].lam, p->ax[2].lam};
    return run_box(p, qb, qn, grad_out, grad_in, 0, nullptr, true, (hipStream_t)stream);
}

fx_status fx_plan_set_timing(fx_plan* p, int enable) {
    if (!p) { set_error("plan is NULL"); return FX_EINVAL; }
    p->timing = (enable != 0);
    return FX_OK;
}

fx_status fx_plan_pass_times(fx_plan* p, int32_t* n_passes, int64_t* launches, double* ms, int32_t max) {
    if (!p || !n_passes) { set_error("NULL argument"); return FX_EINVAL; }
    for (const auto& pe : p->pending) {
        FX_TRY_HIP(hipEventSynchronize(pe.b));
        float f = 0.f;
        FX_TRY_HIP(hipEventElapsedTime(&f, pe.a, pe.b));
        if ((int)p->t_ms.size() <= pe.op) {
            p->t_ms.resize(pe.op + 1, 0.0);
            p->t_launch.resize(pe.op + 1, 0);
        }
        p->t_ms[pe.op] += f;
        p->t_launch[pe.op] += 1;
        p->pool.push_back(pe.a);
        p->pool.push_back(pe.b);
    }
    p->pending.clear();
    const int n = (int)p->t_ms.size();
    *n_passes = n;
    for (int i = 0; i < n && i < max; ++i) {
        if (launches) launches[i] = p->t_launch[i];
        if (ms) ms[i] = p->t_ms[i];
    }
    p->t_ms.clear();
    p->t_launch.clear();
    return FX_OK;
}

namespace {

// The kernel family launch_pass / launch_pass_aa dispatch an op to (same order of tests).
const char* kernel_of(const fx_plan* p, const Op& o) {
    const AxisDev& ax = p->ax[o.axis];
    const PassGeom& g = o.g;
    switch (o.kind) {
        case Kind::AA: return aar_applicable(ax.g, p->ax[o.axis2].g, ax.P, p->ax[o.axis2].P, o.aa) ? "k_AAR" : "k_AA";
        case Kind::AAH: return "k_AAHR";
        default: break;
    }
    if (o.kind == Kind::E && g.erw) return "k_ERW";
    if ((o.kind == Kind::E || o.kind == Kind::EA) && g.erg) return "k_ERG";
    if (o.kind == Kind::EH && g.erg) return "k_EHG";
    if (o.kind == Kind::EA && g.eaw) return "k_EAW";
    if (o.kind == Kind::EA && g.eas) return "k_EAS";
    if (g.qc > 0 && o.kind == Kind::EH) return "k_EHR";
    if (o.kind == Kind::EH && g.eh2) return "k_EH2";
    if (g.qc > 0) return o.kind == Kind::E ? "k_ER" : "k_EAR";
    const bool a = o.kind == Kind::A, ah = o.kind == Kind::AH;
    if ((a || ah) && g.reg_a && g.Qin * g.A * (int64_t)ax.P * g.S * 8 < (int64_t(1) << 31))
        return ax.g <= 8 ? (a ? "k_ASR" : "k_AHR") : (a ? "k_ASK" : "k_AHK");
    if (p2_applicable(o.kind, ax.M) && g.TS == p2_tile_lines(ax.M)) return o.kind == Kind::E ? "k_E2" : "k_EA2";
    if (ct_applicable(o.kind, ax.M) && g.TS == ct_tile_lines(ax.M)) return o.kind == Kind::E ? "k_Ect" : "k_EAct";
    switch (o.kind) {
        case Kind::E: return "k_E";
        case Kind::EA: return "k_EA";
        case Kind::EH: return "k_EH";
        case Kind::EAH: return "k_EAH";
        case Kind::AH: return "k_AH";
        case Kind::A:
            return (ax.g >= 4 && g.Qin * g.A * (int64_t)ax.P * g.S < (int64_t(1) << 31)) ? "k_AS" : "k_A";
        default: return "?";
    }
}

}  // namespace

fx_status fx_plan_describe(const fx_plan* p, char* buf, size_t len) {
    if (!p || !buf || len == 0) { set_error("NULL argument"); return FX_EINVAL; }
    int qb[3] = {0, 0, 0}, qn[3] = {p->ax[0].lam, p->ax[1].lam, p->ax[2].lam};
    if (p->nact > 0 && p->schedule == FX_SCHED_PAPER) qn[p->act[p->nact - 1]] = (int)p->nb_outer;
    std::string s = "{\"schedule\":\"";
    s += (p->schedule == FX_SCHED_PAPER) ? "paper" : "axis_factorised";
    s += "\",\"precision\":\"";
    s += p->dbl ? "c128" : "c64_phase64";
    s += "\",\"terms\":" + std::to_string(p->Q) + ",\"outer_block\":" + std::to_string(p->nb_outer) +
         ",\"slices\":" + std::to_string(p->slices) + ",\"workspace_bytes\":" + std::to_string(p->ws_need) +
         ",\"spectrum\":[";
    for (int j = 0; j < p->ndim; ++j) {
        s += j ? "," : "";
        s += p->spectrum[3 - p->ndim + j] ? "\"table\"" : "\"free\"";
    }
    static const char* names[] = {"E", "A", "EA", "EH", "AH", "EAH", "AA", "AAH"};
    for (int adj = 0; adj < 2; ++adj) {
    std::vector<Op> ops = build_ops(p, qb, qn, p->slices, adj != 0);
    s += adj ? "],\"adjoint_passes\":[" : "],\"passes\":[";
    for (size_t i = 0; i < ops.size(); ++i) {
        const Op& o = ops[i];
        const AxisDev& a = p->ax[o.axis];
        char tmp[256];
        std::snprintf(tmp, sizeof(tmp),
                      "%s{\"kind\":\"%s\",\"axis\":%d,\"M\":%d,\"P\":%d,\"lam\":%d,\"qn\":%d,\"Qin\":%lld,"
                      "\"A\":%lld,\"S\":%lld,\"TS\":%d,\"reg\":%d",
                      i ? "," : "", names[(int)o.kind], o.axis - (3 - p->ndim), a.M, a.P, a.lam, o.g.qn,
                      (long long)o.g.Qin, (long long)o.g.A, (long long)o.g.S, o.g.TS,
                      (o.g.qc > 0 || o.g.reg_a || o.g.eas || o.g.eaw) ? 1 : 0);
        s += tmp;
        s += std::string(",\"kernel\":\"") + kernel_of(p, o) + "\"";
        if (o.g.eas || o.g.eaw || (o.g.erg && o.kind == Kind::EA)) s += ",\"eas\":1";
        if (o.g.eh2) s += ",\"eh2\":1";
        if (o.kind == Kind::AA || o.kind == Kind::AAH) {
            const AxisDev& b = p->ax[o.axis2];
            std::snprintf(tmp, sizeof(tmp),
                          ",\"axis2\":%d,\"M2\":%d,\"P2\":%d,\"lam2\":%d,\"qn2\":%d,\"O\":%lld,\"X\":%lld,"
                          "\"Y\":%lld,\"Z\":%lld,\"g\":%d,\"g2\":%d",
                          o.axis2 - (3 - p->ndim), b.M, b.P, b.lam, o.aa.qn_v, (long long)o.aa.O,
                          (long long)o.aa.X, (long long)o.aa.Y, (long long)o.aa.Z, a.g, b.g);
            s += tmp;
        }
        s += "}";
    }
    }
    s += "]}";
    std::snprintf(buf, len, "%s", s.c_str());
    return FX_OK;
}

fx_status fx_batch_create(const fx_problem* probs, int32_t n, fx_batch** out);
fx_status fx_batch_destroy(fx_batch* b);
fx_status fx_batch_run(fx_batch* b, const void* const* psi0, void* const* psi_out, void* const* rho_out, void* stream);

const char* fx_status_string(fx_status s) {
    switch (s) {
        case FX_OK: return "FX_OK";
        case FX_EINVAL: return "FX_EINVAL: invalid argument";
        case FX_ENOMEM: return "FX_ENOMEM: out of memory or workspace too small";
        case FX_EDEVICE: return "FX_EDEVICE: HIP runtime or kernel error";
        case FX_EUNSUPPORTED: return "FX_EUNSUPPORTED: outside what this library supports";
        default: break;
    }
    return "unknown fx_status";
}

const char* fx_last_error(void) { return g_err.c_str(); }

}  // extern "C"

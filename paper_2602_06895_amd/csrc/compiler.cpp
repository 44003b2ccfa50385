// Channel compiler (section 2.2 of arXiv:2602.06895): recursive
// decomposition of a diagram topology into invariants, 2->2 blocks and
// decays, with the s-channel bound recursion (section 2.2.7) and the
// t-channel order (section 2.2.8) resolved at construction time.
#include "compiler.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace msx {
namespace {

constexpr double kPi = 3.14159265358979323846;

enum { N_LEAF = 0, N_CLUSTER = 1, N_TNODE = 2 };
constexpr int kNoSlot = 1 << 20;

struct Node {
    int kind = N_LEAF;
    int particle = -1;
    int parent = -1;
    std::vector<int> kids;
    double m = 0.0, w = 0.0, nu = 0.0;
    bool rambo = false;  // FastRambo cluster mass
    bool has_order = false;
    double order = 0.0;
    int slot = kNoSlot;
    int inv = -1;  // invariant index once scheduled
};

// Linear form c + sum_{j in mask} sqrt(s_j).
struct Form {
    double c = 0.0;
    uint32_t mask = 0;
    Form& operator+=(const Form& o) {
        c += o.c;
        mask |= o.mask;  // each invariant appears at most once on a path
        return *this;
    }
};

struct Ctx {
    std::string err;
    bool fail(const std::string& m) {
        if (err.empty()) err = m;
        return false;
    }
};

bool num(const JValue* v, double& out) {
    if (!v || v->kind != JValue::NUM) return false;
    out = v->num;
    return true;
}

double num_or(const JValue& o, const char* key, double dflt) {
    const JValue* v = o.get(key);
    return (v && v->kind == JValue::NUM) ? v->num : dflt;
}

MapParams make_map(double m, double w, double nu, double reg_a) {
    MapParams p{};
    if (w > 0.0) {
        p.kind = MAP_BW;
        p.m2 = m * m;
        p.mw = m * w;
        return p;
    }
    p.m2 = (m == 0.0) ? -reg_a : m * m;
    if (nu == 0.0) {
        p.kind = MAP_FLAT;
    } else if (nu == 1.0) {
        p.kind = MAP_LOG;
    } else {
        p.kind = MAP_POW;
        p.e = 1.0 - nu;
        p.inv_e = 1.0 / p.e;
        double r = std::round(p.inv_e);
        // x - m^2 = b^(1/e): integer powers up to 8 are done by multiplication
        p.int_pow = (std::fabs(p.inv_e - r) < 1e-12 && r >= 2.0 && r <= 8.0) ? (int32_t)r : 0;
    }
    return p;
}

struct ChannelBuilder {
    Ctx& cx;
    const std::vector<double>& masses;
    double nu_default, reg_a;
    std::vector<Node> nodes;

    ChannelBuilder(Ctx& c, const std::vector<double>& ms, double nu, double a)
        : cx(c), masses(ms), nu_default(nu), reg_a(a) {}

    int add(const JValue& leg, int parent) {
        int idx = (int)nodes.size();
        nodes.emplace_back();
        nodes[idx].parent = parent;
        if (leg.kind == JValue::NUM) {
            if (!leg.is_int() || leg.num < 1 || leg.num > (double)masses.size()) {
                cx.fail("particle label out of range");
                return -1;
            }
            nodes[idx].kind = N_LEAF;
            nodes[idx].particle = (int)leg.num - 1;
            nodes[idx].m = masses[nodes[idx].particle];
            return idx;
        }
        if (leg.kind != JValue::OBJ) {
            cx.fail("a leg is a particle label or a cluster object");
            return -1;
        }
        const JValue* d = leg.get("d");
        if (!d || d->kind != JValue::ARR || (d->arr.size() != 2 && d->arr.size() != 3)) {
            cx.fail("a cluster needs \"d\": [child, child] or [child, child, child]");
            return -1;
        }
        nodes[idx].kind = N_CLUSTER;
        nodes[idx].m = num_or(leg, "m", 0.0);
        nodes[idx].w = num_or(leg, "w", 0.0);
        nodes[idx].nu = num_or(leg, "nu", nu_default);
        if (const JValue* rb = leg.get("rambo")) nodes[idx].rambo = rb->kind == JValue::BOOL && rb->b;
        if (nodes[idx].rambo && d->arr.size() != 2) {
            cx.fail("a FastRambo cluster decays into two children");
            return -1;
        }
        if (nodes[idx].m < 0.0 || nodes[idx].w < 0.0 || (nodes[idx].w > 0.0 && nodes[idx].m <= 0.0)) {
            cx.fail("cluster mass/width must be >= 0 (a width needs a mass)");
            return -1;
        }
        double o;
        if (num(leg.get("order"), o)) {
            nodes[idx].has_order = true;
            nodes[idx].order = o;
        }
        for (const JValue& kid : d->arr) {
            int k = add(kid, idx);
            if (k < 0) return -1;
            nodes[idx].kids.push_back(k);
        }
        return idx;
    }

    void particles(int j, std::vector<int>& out) const {
        if (nodes[j].kind == N_LEAF) {
            out.push_back(nodes[j].particle);
            return;
        }
        for (int k : nodes[j].kids) particles(k, out);
    }
    uint32_t pmask(int j) const {
        std::vector<int> ps;
        particles(j, ps);
        uint32_t m = 0;
        for (int p : ps) m |= 1u << p;
        return m;
    }
};

// Minimal-mass form of node j given the set of sampled nodes.
Form min_form(const std::vector<Node>& nodes, int j, const std::vector<char>& sampled) {
    const Node& n = nodes[j];
    Form f;
    if (n.kind == N_LEAF) {
        f.c = n.m;
        return f;
    }
    if (sampled[j]) {
        f.mask = 1u << n.inv;
        return f;
    }
    for (int k : n.kids) f += min_form(nodes, k, sampled);
    return f;
}

MassSrc mass_src(const Node& n) {
    MassSrc s{};
    if (n.kind == N_LEAF) {
        s.inv = -1;
        s.m = n.m;
    } else {
        s.inv = n.inv;
    }
    return s;
}

bool compile_channel(Ctx& cx, const JValue& cj, const std::vector<double>& masses, bool hadronic,
                     double s_lab, double shat_min, double nu, double reg_a, ChannelTab& t,
                     std::vector<std::pair<int, uint32_t>>& props, std::vector<double>& prop_m,
                     std::vector<double>& prop_w) {
    std::memset(&t, 0, sizeof t);
    const int n = (int)masses.size();
    ChannelBuilder b(cx, masses, nu, reg_a);
    std::vector<Node>& nodes = b.nodes;
    std::string t_order;
    bool tchain = false;
    if (const JValue* ch = cj.get("chili")) {
        // Chili (section 2.4): no tree; per particle but the last p_T, y and
        // phi, then the last one's rapidity: 3 n - 2 dimensions
        if (ch->kind != JValue::BOOL || !ch->b) return cx.fail("\"chili\" must be true");
        if (!hadronic) return cx.fail("a Chili channel needs hadronic beams (x1, x2 follow from the momenta)");
        if (n < 2) return cx.fail("a Chili channel needs at least two final-state particles");
        t.chili = 1;
        t.n_final = n;
        t.hadronic = 1;
        t.n_slots = 2 * (n - 1);
        // no invariants are sampled; counting n - 1 picks a register class
        // whose staging column (1 + invariants + slots rows) holds the
        // 3 n - 2 dimensions
        t.n_inv = n - 1;
        t.jac_const = std::pow(2.0 * kPi, 4.0 - 3.0 * n) / s_lab;
        for (int k = 0; k < n; ++k) {
            t.final_slot[k] = k;
            t.chili_m[k] = masses[k];
        }
        t.dims = 3 * n - 2;
        t.kinds = 64;
        // the sample kernel stages the uniforms in a column of at least
        // max(kMaxUniq + 1, 1 + n_inv + n_slots) rows
        if (t.dims > std::max(kMaxUniq + 1, 1 + t.n_inv + t.n_slots))
            return cx.fail("internal: Chili dimensions exceed the staging column");
        props.clear();
        prop_m.clear();
        prop_w.clear();
        return true;
    }
    if (const JValue* legs = cj.get("t_chain")) {
        if (legs->kind != JValue::ARR || legs->arr.size() < 2)
            return cx.fail("\"t_chain\" needs at least two legs");
        tchain = true;
        nodes.emplace_back();
        nodes[0].kind = N_TNODE;
        nodes[0].nu = nu;
        for (const JValue& leg : legs->arr) {
            int k = b.add(leg, 0);
            if (k < 0) return false;
            nodes[0].kids.push_back(k);
        }
        if (const JValue* to = cj.get("t_order")) {
            if (to->kind != JValue::STR) return cx.fail("\"t_order\" must be a string");
            t_order = to->str;
        }
        if (const JValue* stj = cj.get("st")) {
            if (stj->kind != JValue::BOOL) return cx.fail("\"st\" must be true or false");
            t.st = stj->b ? 1 : 0;
        }
        int kappa = (int)nodes[0].kids.size() - 1;
        if ((int)t_order.size() != kappa - 1) return cx.fail("\"t_order\" needs kappa-1 letters");
        for (char c : t_order)
            if (c != 'A' && c != 'B') return cx.fail("\"t_order\" letters are A or B");
    } else if (const JValue* s = cj.get("s")) {
        if (b.add(*s, -1) < 0) return false;
        if (nodes[0].kind != N_CLUSTER) return cx.fail("a pure s-channel root must be a cluster");
    } else {
        return cx.fail("a channel needs \"t_chain\", \"s\" or \"chili\"");
    }
    if (!cx.err.empty()) return false;
    // every particle exactly once
    {
        std::vector<int> seen(n, 0);
        for (const Node& nd : nodes)
            if (nd.kind == N_LEAF) seen[nd.particle]++;
        for (int c : seen)
            if (c != 1) return cx.fail("every final-state particle must appear exactly once");
    }

    // ---- slots: assigned with the operations below (block b: codes 2b, 2b+1;
    // decay d: codes -2-2d, -1-2d, i.e. from the top of the slot file)

    // ---- invariants: 0 = s-hat (root), then clusters in sampling order
    std::vector<int> s_order;
    for (size_t j = 1; j < nodes.size(); ++j)
        if (nodes[j].kind == N_CLUSTER) s_order.push_back((int)j);
    std::stable_sort(s_order.begin(), s_order.end(), [&](int a, int c) {
        if (nodes[a].has_order != nodes[c].has_order) return nodes[a].has_order;
        if (nodes[a].has_order && nodes[a].order != nodes[c].order) return nodes[a].order < nodes[c].order;
        return a < c;
    });
    int kappa = tchain ? (int)nodes[0].kids.size() - 1 : 0;
    int n_inv = 1 + (int)s_order.size() + std::max(kappa - 1, 0);
    if (n_inv > kMaxInv) return cx.fail("too many time-like invariants");
    nodes[0].inv = 0;

    t.n_final = n;
    t.hadronic = hadronic ? 1 : 0;
    t.n_slots = 2 * (n - 1);
    t.jac_const = std::pow(2.0 * kPi, 4.0 - 3.0 * n);

    // s-hat
    {
        InvSpec& iv = t.inv[0];
        iv.set = b.pmask(0);
        if (!hadronic) {
            iv.map.kind = MAP_FIXED;
            iv.xmin = iv.xmax = s_lab;
        } else {
            double m = 0.0, w = 0.0, nr = nu;
            if (!tchain) {
                m = nodes[0].m;
                w = nodes[0].w;
                nr = nodes[0].nu;
            }
            iv.map = make_map(m, w, nr, reg_a);
            double msum = 0.0;
            for (double mm : masses) msum += mm;
            double lo = shat_min;
            if (msum * msum > lo) lo = msum * msum;
            iv.xmin = lo;
            iv.xmax = s_lab;
            if (!(iv.xmax > iv.xmin)) return cx.fail("s-hat range is empty");
            const MapParams& p = iv.map;
            if (p.kind == MAP_POW) {
                iv.A = std::pow(iv.xmax - p.m2, p.e);
                iv.B = std::pow(iv.xmin - p.m2, p.e);
            } else if (p.kind == MAP_LOG) {
                iv.A = std::log(iv.xmax - p.m2);
                iv.B = std::log(iv.xmin - p.m2);
            } else if (p.kind == MAP_BW) {
                iv.A = std::atan((iv.xmax - p.m2) / p.mw);
                iv.B = std::atan((iv.xmin - p.m2) / p.mw);
            }
            if ((p.kind == MAP_POW || p.kind == MAP_LOG) && !(iv.xmin - p.m2 > 0.0))
                return cx.fail("s-hat lower bound must lie above the mapping pole");
        }
    }

    // cluster invariants with the min/max mass recursion
    std::vector<char> sampled(nodes.size(), 0);
    sampled[0] = 1;
    int next_inv = 1;
    for (int j : s_order) {
        InvSpec& iv = t.inv[next_inv];
        Form fmin;
        for (int k : nodes[j].kids) fmin += min_form(nodes, k, sampled);
        Form fsub;
        int v = j;
        while (!sampled[v]) {
            int par = nodes[v].parent;
            for (int sib : nodes[par].kids)
                if (sib != v) fsub += min_form(nodes, sib, sampled);
            v = par;
        }
        iv.map = make_map(nodes[j].m, nodes[j].w, nodes[j].nu, reg_a);
        if (nodes[j].rambo) {
            // FastRambo (section 2.2.9, table tab:rambo_fit): slopes c_k*
            static const double kRamboC[8] = {0.0, 2.0, 2.712001, 3.084521, 3.313073, 3.467512, 3.578833, 3.662872};
            std::vector<int> ps;
            b.particles(j, ps);
            const int k = (int)ps.size() - 1;
            if (k < 1 || k > 7) return cx.fail("a FastRambo cluster needs 2 to 8 particles");
            MapParams rp{};
            rp.kind = MAP_RAMBO;
            rp.int_pow = k;
            rp.e = 1.0 / k;
            rp.inv_e = k;
            rp.mw = kRamboC[k];
            iv.map = rp;
        }
        iv.set = b.pmask(j);
        iv.parent = nodes[v].inv;
        iv.min_const = fmin.c;
        iv.min_mask = fmin.mask;
        iv.max_const = fsub.c;
        iv.max_mask = fsub.mask;
        nodes[j].inv = next_inv++;
        sampled[j] = 1;
    }

    // t-channel generation order and its time-like invariants
    std::vector<int> sigma(kappa + 2, -1), from_a(kappa + 1, 0), tinv(kappa + 1, -1);
    if (tchain) {
        const std::vector<int>& legs = nodes[0].kids;
        int lo = 0, hi = kappa;
        for (int i = 1; i < kappa; ++i) {
            if (t_order[i - 1] == 'A') {
                sigma[i] = legs[lo++];
                from_a[i] = 1;
            } else {
                sigma[i] = legs[hi--];
            }
        }
        sigma[kappa] = legs[lo];
        sigma[kappa + 1] = legs[hi];
        auto leg_form = [&](int leg) {
            Form f;
            if (nodes[leg].kind == N_LEAF) f.c = nodes[leg].m;
            else f.mask = 1u << nodes[leg].inv;
            return f;
        };
        tinv[0] = 0;
        for (int i = 1; i < kappa; ++i) {
            InvSpec& iv = t.inv[next_inv];
            Form fmin, fsub = leg_form(sigma[i]);
            for (int j = i + 1; j <= kappa + 1; ++j) fmin += leg_form(sigma[j]);
            iv.set = 0;
            for (int j = i + 1; j <= kappa + 1; ++j) iv.set |= b.pmask(sigma[j]);
            iv.map = make_map(0.0, 0.0, nu, reg_a);
            iv.parent = tinv[i - 1];
            iv.min_const = fmin.c;
            iv.min_mask = fmin.mask;
            iv.max_const = fsub.c;
            iv.max_mask = fsub.mask;
            tinv[i] = next_inv++;
        }
        // 2->2 blocks
        for (int i = 1; i <= kappa; ++i) {
            BlockSpec& bs = t.blk[i - 1];
            bs.tmap = make_map(0.0, 0.0, nu, reg_a);
            bs.com = (i == 1) ? 1 : 0;
            bs.m0_inv = tinv[i - 1];
            MassSrc rem{};
            rem.inv = tinv[i];
            const uint32_t rest = i < kappa ? t.inv[tinv[i]].set : 0u;
            if (i == kappa) {
                bs.side = 2;
                bs.m1 = mass_src(nodes[sigma[kappa]]);
                bs.m2 = mass_src(nodes[sigma[kappa + 1]]);
                bs.set1 = b.pmask(sigma[kappa]);
                bs.set2 = b.pmask(sigma[kappa + 1]);
                nodes[sigma[kappa]].slot = 2 * (i - 1);
                nodes[sigma[kappa + 1]].slot = 2 * (i - 1) + 1;
            } else if (from_a[i]) {
                bs.side = 0;
                bs.m1 = mass_src(nodes[sigma[i]]);
                bs.m2 = rem;
                bs.set1 = b.pmask(sigma[i]);
                bs.set2 = rest;
                nodes[sigma[i]].slot = 2 * (i - 1);
            } else {
                bs.side = 1;
                bs.m1 = rem;
                bs.m2 = mass_src(nodes[sigma[i]]);
                bs.set1 = rest;
                bs.set2 = b.pmask(sigma[i]);
                nodes[sigma[i]].slot = 2 * (i - 1) + 1;
            }
        }
    }
    t.n_inv = next_inv;
    t.n_blocks = kappa;

    // (phi, theta) decays and 1 -> 3 decays, depth-first, parents first.  A
    // 1 -> 3 decay takes two entries: its third child goes to the first slot
    // of the second (decay d writes slot codes -2-2d, -1-2d), which keeps the
    // slot count at 2 (n - 1) and every slot index a constant in the kernel.
    int nd = 0, n3 = 0;
    for (size_t j = 0; j < nodes.size(); ++j) {
        if (nodes[j].kind != N_CLUSTER) continue;
        const bool three = nodes[j].kids.size() == 3;
        if (nd + (three ? 1 : 0) >= kMaxFinal) return cx.fail("too many decays");
        DecaySpec& ds = t.dec[nd];
        ds.parent_rest = (j == 0) ? 1 : 0;
        ds.parent_slot = (j == 0) ? 0 : nodes[j].slot;
        ds.parent_inv = nodes[j].inv;
        Node& k0 = nodes[nodes[j].kids[0]];
        Node& k1 = nodes[nodes[j].kids[1]];
        ds.m1 = mass_src(k0);
        ds.m2 = mass_src(k1);
        ds.parent_set = b.pmask((int)j);
        ds.set1 = b.pmask(nodes[j].kids[0]);
        ds.set2 = b.pmask(nodes[j].kids[1]);
        k0.slot = -2 - 2 * nd;
        k1.slot = -1 - 2 * nd;
        ds.kind = 0;
        if (three) {
            Node& k2 = nodes[nodes[j].kids[2]];
            ds.kind = 1;
            ds.m3 = mass_src(k2);
            ds.set3 = b.pmask(nodes[j].kids[2]);
            k2.slot = -4 - 2 * nd;
            DecaySpec& pad = t.dec[nd + 1];
            std::memset(&pad, 0, sizeof pad);
            pad.kind = 2;
            ++nd;
            ++n3;
        }
        ++nd;
    }
    t.n_decays = nd;
    if (t.n_blocks + t.n_decays != n - 1) return cx.fail("internal: operation count");
    for (size_t j = 0; j < nodes.size(); ++j) {
        if (nodes[j].kind != N_LEAF) continue;
        if (nodes[j].slot == kNoSlot) return cx.fail("internal: particle without a slot");
        t.final_slot[nodes[j].particle] = nodes[j].slot;
    }
    // map kinds used (bit values as in the kernels: 1 integer-root power law,
    // 2 general power law, 4 log, 8 flat, 16 Breit-Wigner, 32 FastRambo;
    // 64 marks a Chili channel, 128 a channel with 1 -> 3 decays)
    auto kind_bit = [](const MapParams& p) -> int32_t {
        switch (p.kind) {
            case MAP_POW: return p.int_pow ? 1 : 2;
            case MAP_LOG: return 4;
            case MAP_FLAT: return 8;
            case MAP_BW: return 16;
            case MAP_RAMBO: return 32;
            default: return 0;
        }
    };
    t.kinds = 0;
    for (int i = 0; i < t.n_inv; ++i) t.kinds |= kind_bit(t.inv[i].map);
    for (int i = 0; i < t.n_blocks; ++i) t.kinds |= kind_bit(t.blk[i].tmap);
    if (n3) t.kinds |= 128;
    if (t.st && t.n_blocks > 1) t.kinds |= 256;  // (s~, t) blocks (KIND_ST)
    // two per two-body decay, five per 1 -> 3 decay (which holds two entries)
    t.dims = (hadronic ? 2 : 0) + (int)s_order.size() + std::max(kappa - 1, 0) + 2 * kappa + 2 * (nd - 2 * n3) +
             5 * n3;
    if (t.dims > kMaxDims) return cx.fail("too many random dimensions");
    // the sample kernel's per-thread staging column has at least
    // max(kMaxUniq + 1, 1 + invariants + slots) rows
    if (t.dims > std::max(kMaxUniq + 1, 1 + t.n_inv + t.n_slots))
        return cx.fail("internal: dimension count exceeds the staging column");

    // propagators of the diagram (for the local channel weights)
    props.clear();
    prop_m.clear();
    prop_w.clear();
    if (tchain) {
        uint32_t acc = 0;
        for (int i = 0; i < kappa; ++i) {
            acc |= b.pmask(nodes[0].kids[i]);
            props.emplace_back(1, acc);
            prop_m.push_back(0.0);
            prop_w.push_back(0.0);
        }
    }
    for (size_t j = 0; j < nodes.size(); ++j) {
        if (nodes[j].kind != N_CLUSTER) continue;
        props.emplace_back(0, b.pmask((int)j));
        prop_m.push_back(nodes[j].m);
        prop_w.push_back(nodes[j].w);
    }
    return true;
}

int find_or_add_uniq(ProcessTab& pt, int tt, uint32_t set) {
    for (int u = 0; u < pt.n_uniq; ++u)
        if (pt.uniq_t[u] == tt && pt.uniq_set[u] == set) return u;
    if (pt.n_uniq >= kMaxUniq) return -1;
    int u = pt.n_uniq++;
    pt.uniq_t[u] = tt;
    pt.uniq_set[u] = set;
    pt.uniq_massive[u] = -1;  // alpha form not yet assigned
    pt.uniq_f[u] = -1;
    return u;
}

bool compile_process(Ctx& cx, const JValue& pj, Compiled& out) {
    if (pj.kind != JValue::OBJ) return cx.fail("a process is a JSON object");
    ProcessTab pt;
    std::memset(&pt, 0, sizeof pt);
    double sqrt_s;
    if (!num(pj.get("sqrt_s"), sqrt_s) || !(sqrt_s > 0.0)) return cx.fail("\"sqrt_s\" must be > 0");
    const JValue* ms = pj.get("masses");
    if (!ms || ms->kind != JValue::ARR || ms->arr.empty()) return cx.fail("\"masses\" must be a list");
    std::vector<double> masses;
    for (const JValue& m : ms->arr) {
        if (m.kind != JValue::NUM || !(m.num >= 0.0)) return cx.fail("masses must be >= 0");
        masses.push_back(m.num);
    }
    const int n = (int)masses.size();
    if (n < 2 || n > kMaxFinal) return cx.fail("between 2 and 8 final-state particles are supported");
    bool hadronic = true;
    if (const JValue* bm = pj.get("beams")) {
        if (bm->kind != JValue::STR || (bm->str != "hadronic" && bm->str != "fixed"))
            return cx.fail("\"beams\" is \"hadronic\" or \"fixed\"");
        hadronic = bm->str == "hadronic";
    }
    double nu = num_or(pj, "nu", 0.8);
    double reg_a = num_or(pj, "regulator", 1e-3);
    double shat_min = num_or(pj, "shat_min", 0.0);
    double nb = num_or(pj, "vegas_bins", 64.0);
    if (!(reg_a > 0.0)) return cx.fail("\"regulator\" must be > 0");
    if (nb != std::floor(nb) || nb < 1 || nb > kMaxBins) return cx.fail("\"vegas_bins\" must be in 1..128");
    double s_lab = sqrt_s * sqrt_s;
    double msum = 0.0;
    for (double m : masses) msum += m;
    if (!hadronic && msum >= sqrt_s) return cx.fail("final-state masses exceed sqrt_s");

    pt.n_final = n;
    pt.hadronic = hadronic ? 1 : 0;
    pt.s_lab = s_lab;
    pt.ang = -1;
    // integrand
    if (const JValue* ig = pj.get("integrand")) {
        if (ig->kind != JValue::OBJ) return cx.fail("\"integrand\" must be an object");
        if (const JValue* pdf = ig->get("pdf")) {
            if (pdf->kind != JValue::ARR || pdf->arr.size() != 2 || pdf->arr[0].kind != JValue::NUM ||
                pdf->arr[1].kind != JValue::NUM)
                return cx.fail("\"pdf\" is [a, b]");
            if (!hadronic) return cx.fail("\"pdf\" needs hadronic beams");
            pt.pdf = 1;
            pt.pdf_a = pdf->arr[0].num;
            pt.pdf_b = pdf->arr[1].num;
            if (pt.pdf_b == std::floor(pt.pdf_b) && pt.pdf_b >= 1.0 && pt.pdf_b <= 16.0) pt.pdf_b_int = (int32_t)pt.pdf_b;
        }
        double ptmin = num_or(*ig, "pt_min", 0.0);
        pt.pt_min2 = ptmin > 0.0 ? ptmin * ptmin : 0.0;
        if (const JValue* ang = ig->get("ang")) {
            if (!ang->is_int() || ang->num < 1 || ang->num > n) return cx.fail("\"ang\" is a particle label");
            if (hadronic) return cx.fail("\"ang\" needs fixed beams");
            pt.ang = (int)ang->num - 1;
        }
        if (const JValue* props = ig->get("props")) {
            if (props->kind != JValue::ARR) return cx.fail("\"props\" must be a list");
            for (const JValue& pr : props->arr) {
                if (pt.n_fprop >= kMaxFactors) return cx.fail("too many integrand factors");
                const JValue* parts = pr.get("particles");
                if (!parts || parts->kind != JValue::ARR || parts->arr.empty())
                    return cx.fail("an integrand factor needs \"particles\"");
                uint32_t set = 0;
                for (const JValue& q : parts->arr) {
                    if (!q.is_int() || q.num < 1 || q.num > n) return cx.fail("particle label out of range");
                    set |= 1u << ((int)q.num - 1);
                }
                const JValue* tt = pr.get("t");
                int is_t = (tt && tt->kind == JValue::BOOL && tt->b) ? 1 : 0;
                const JValue* bw = pr.get("bw");
                int is_bw = (bw && bw->kind == JValue::BOOL && bw->b) ? 1 : 0;
                int u = find_or_add_uniq(pt, is_t, set);
                if (u < 0) return cx.fail("too many distinct invariants");
                if (pt.uniq_f[u] >= 0) return cx.fail("two integrand factors on the same invariant");
                int f = pt.n_fprop++;
                pt.f_uniq[f] = u;
                pt.uniq_f[u] = f;
                pt.f_bw[f] = is_bw;
                double m = num_or(pr, "m", 0.0), w = num_or(pr, "w", 0.0), mu = num_or(pr, "mu", 0.0);
                pt.f_m2[f] = m * m;
                pt.f_mw[f] = m * w;
                pt.f_mu2[f] = mu * mu;
                if (is_bw && !(m * w > 0.0)) return cx.fail("a Breit-Wigner factor needs m, w > 0");
                if (!is_bw && !(mu > 0.0)) return cx.fail("a 1/(|q^2|+mu^2) factor needs mu > 0");
            }
        }
    }
    const JValue* chs = pj.get("channels");
    if (!chs || chs->kind != JValue::ARR || chs->arr.empty()) return cx.fail("\"channels\" must be a non-empty list");
    int nch = (int)chs->arr.size();
    bool use_alpha = pj.has("alpha_mu") && nch > 1;
    if (use_alpha) {
        double amu = num_or(pj, "alpha_mu", 0.0);
        if (!(amu > 0.0)) return cx.fail("\"alpha_mu\" must be > 0");
        if (nch > kMaxChanPerProc) return cx.fail("too many channels for local weights");
        pt.alpha_mu2 = amu * amu;
        pt.n_chan = nch;
    } else {
        pt.n_chan = 1;
    }
    int pidx = (int)out.procs.size();
    for (int c = 0; c < nch; ++c) {
        if ((int)out.chans.size() >= kMaxChannels) return cx.fail("too many channels");
        ChannelTab t;
        std::vector<std::pair<int, uint32_t>> props;
        std::vector<double> pm, pw;
        if (!compile_channel(cx, chs->arr[c], masses, hadronic, s_lab, shat_min, nu, reg_a, t, props, pm, pw))
            return false;
        t.process = pidx;
        t.alpha_index = use_alpha ? c : 0;
        if (t.chili) t.chili_ptmin2 = pt.pt_min2;
        if (use_alpha) {
            uint32_t mask = 0;
            for (size_t q = 0; q < props.size(); ++q) {
                int u = find_or_add_uniq(pt, props[q].first, props[q].second);
                if (u < 0) return cx.fail("too many distinct invariants");
                int massive = pm[q] > 0.0 ? 1 : 0;
                double m2 = pm[q] * pm[q], mw = pm[q] * pw[q];
                if (pt.uniq_massive[u] < 0) {
                    pt.uniq_massive[u] = massive;
                    pt.uniq_m2[u] = m2;
                    pt.uniq_mw[u] = mw;
                } else if (pt.uniq_massive[u] != massive || pt.uniq_m2[u] != m2 || pt.uniq_mw[u] != mw) {
                    return cx.fail("one invariant has different propagator masses in two channels");
                }
                mask |= 1u << u;
            }
            pt.chan_mask[c] = mask;
            if (t.chili) pt.chan_prior |= 1u << c;
        }
        ChannelMeta meta;
        meta.process = pidx;
        meta.dims = t.dims;
        meta.n_momenta = n + 2;
        meta.hadronic = hadronic ? 1 : 0;
        meta.nbins = (int)nb;
        out.chans.push_back(t);
        out.meta.push_back(meta);
    }
    // a channel without a diagram takes the constant local weight 1 / n;
    // the diagram channels share the rest (subtracted one share at a time,
    // as the weight evaluation order defines it)
    pt.prior_share = 1.0 / pt.n_chan;
    pt.tree_share = 1.0;
    for (int c = 0; c < pt.n_chan; ++c)
        if ((pt.chan_prior >> c) & 1) pt.tree_share -= 1.0 / pt.n_chan;
    for (int u = 0; u < pt.n_uniq; ++u) {
        UniqSpec& q = pt.uq[u];
        q.set = pt.uniq_set[u];
        q.t = pt.uniq_t[u];
        const int f = pt.uniq_f[u];
        q.fkind = f < 0 ? 0 : (pt.f_bw[f] ? 1 : 2);
        q.fa = f < 0 ? 0.0 : (pt.f_bw[f] ? pt.f_m2[f] : pt.f_mu2[f]);
        q.fb = f < 0 ? 0.0 : (pt.f_bw[f] ? pt.f_mw[f] * pt.f_mw[f] : 0.0);
        q.massive = pt.uniq_massive[u];
        q.am2 = pt.uniq_m2[u];
        q.amw2 = pt.uniq_mw[u] * pt.uniq_mw[u];
    }
    out.procs.push_back(pt);
    return true;
}

}  // namespace

bool compile_processes(const JValue& root, Compiled& out, std::string& err) {
    Ctx cx;
    out = Compiled();
    if (root.kind != JValue::OBJ) {
        err = "the description must be a JSON object";
        return false;
    }
    if (const JValue* ps = root.get("processes")) {
        if (ps->kind != JValue::ARR || ps->arr.empty() || ps->arr.size() > (size_t)kMaxProcesses) {
            err = "\"processes\" must be a list of 1..8 processes";
            return false;
        }
        for (const JValue& p : ps->arr)
            if (!compile_process(cx, p, out)) {
                err = cx.err;
                return false;
            }
    } else if (!compile_process(cx, root, out)) {
        err = cx.err;
        return false;
    }
    return true;
}

}  // namespace msx

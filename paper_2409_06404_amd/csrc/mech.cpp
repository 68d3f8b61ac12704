// Mechanism loader: parse the "crf-mech 1" text, validate it, derive the
// device tables and upload them in one allocation.
//
// The paper's solver takes its chemistry as a mechanism "in Cantera format"
// and turns it into platform code (Section 2); here the mechanism becomes a set
// of plain tables that table-driven kernels read.

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>

#include "crf_internal.h"

namespace crf {

namespace {

struct Lines {
    std::vector<std::string> v;
    size_t pos = 0;
    bool next(std::istringstream &ss) {
        if (pos >= v.size()) return false;
        ss.clear();
        ss.str(v[pos++]);
        return true;
    }
};

bool read_lines(const char *path, Lines &out) {
    std::ifstream f(path);
    if (!f) return false;
    std::string line;
    while (std::getline(f, line)) {
        size_t a = line.find_first_not_of(" \t\r");
        if (a == std::string::npos || line[a] == '#') continue;
        size_t b = line.find_last_not_of(" \t\r");
        out.v.push_back(line.substr(a, b - a + 1));
    }
    return true;
}

bool parse_pair(const std::string &tok, int &k, double &v) {
    size_t c = tok.find(':');
    if (c == std::string::npos) return false;
    char *end = nullptr;
    long kk = std::strtol(tok.c_str(), &end, 10);
    if (end != tok.c_str() + c) return false;
    const char *vs = tok.c_str() + c + 1;
    double vv = std::strtod(vs, &end);
    if (end == vs || *end != '\0') return false;
    k = (int)kk;
    v = vv;
    return true;
}

crf_status perr(int line, const std::string &what) {
    return fail(CRF_E_PARSE, "mechanism line " + std::to_string(line) + ": " + what);
}

}  // namespace

crf_status parse_mechanism(const char *path, HostMech &h) {
    Lines L;
    if (!path || !read_lines(path, L)) return fail(CRF_E_PARSE, std::string("cannot read mechanism file ") + (path ? path : "(null)"));
    std::istringstream ss;
    std::string kw;
    auto lineno = [&]() { return (int)L.pos; };
    if (!L.next(ss) || !(ss >> kw) || kw != "crf-mech") return perr(lineno(), "expected 'crf-mech 1' header");
    int ver = 0;
    if (!(ss >> ver) || ver != 1) return perr(lineno(), "unsupported format version");
    // header keys
    int ne = -1;
    while (L.next(ss)) {
        if (!(ss >> kw)) return perr(lineno(), "empty line");
        if (kw == "gas-constant") { if (!(ss >> h.R)) return perr(lineno(), "bad gas-constant"); }
        else if (kw == "standard-pressure") { if (!(ss >> h.p0)) return perr(lineno(), "bad standard-pressure"); }
        else if (kw == "elements") { if (!(ss >> ne) || ne <= 0 || ne > 64) return perr(lineno(), "bad element count"); break; }
        else return perr(lineno(), "unexpected keyword '" + kw + "'");
    }
    if (ne < 0) return perr(lineno(), "missing elements section");
    if (!(h.R > 0) || !(h.p0 > 0)) return fail(CRF_E_MECH, "gas-constant and standard-pressure must be given and positive");
    for (int e = 0; e < ne; ++e) {
        std::string sym; double w;
        if (!L.next(ss) || !(ss >> sym >> w)) return perr(lineno(), "bad element line");
        if (!(w > 0)) return fail(CRF_E_MECH, "element " + sym + ": atomic weight must be positive");
        h.elements.push_back(sym); h.aw.push_back(w);
    }
    int ns = 0;
    if (!L.next(ss) || !(ss >> kw >> ns) || kw != "species" || ns <= 0 || ns > 4096) return perr(lineno(), "bad species header");
    h.names.resize(ns); h.comp.assign((size_t)ns * ne, 0); h.W.assign(ns, 0.0);
    h.nasa.assign((size_t)ns * 16, 0.0);
    for (int k = 0; k < ns; ++k) {
        if (!L.next(ss) || !(ss >> h.names[k])) return perr(lineno(), "bad species line");
        double W = 0;
        for (int e = 0; e < ne; ++e) {
            int c;
            if (!(ss >> c) || c < 0) return perr(lineno(), "bad element count of species " + h.names[k]);
            h.comp[(size_t)k * ne + e] = c;
            W += c * h.aw[e];
        }
        if (!(W > 0)) return fail(CRF_E_MECH, "species " + h.names[k] + " has no atoms");
        h.W[k] = W;
        double tl, tm, th;
        if (!(ss >> tl >> tm >> th)) return perr(lineno(), "bad temperature ranges of species " + h.names[k]);
        if (!(tl < tm && tm < th)) return fail(CRF_E_MECH, "species " + h.names[k] + ": need T_lo < T_mid < T_hi");
        double *nz = &h.nasa[(size_t)k * 16];
        nz[0] = tm;
        for (int j = 0; j < 14; ++j)
            if (!(ss >> nz[1 + j])) return perr(lineno(), "need 14 NASA coefficients for species " + h.names[k]);
    }
    int nr = 0;
    if (!L.next(ss) || !(ss >> kw >> nr) || kw != "reactions" || nr < 0 || nr > (1 << 20)) return perr(lineno(), "bad reactions header");
    h.lnA.resize(nr); h.b.resize(nr); h.theta.resize(nr); h.info.resize(nr); h.dnu_sum.resize(nr); h.ri.resize(nr);
    for (int i = 0; i < nr; ++i) {
        int ln = (int)L.pos + 1;
        if (!L.next(ss)) return perr(ln, "missing reaction");
        std::string kind;
        if (!(ss >> kw >> kind) || kw != "reaction") return perr(ln, "expected 'reaction <kind>'");
        int kc;
        if (kind == "elementary") kc = RXN_ELEMENTARY;
        else if (kind == "threebody") kc = RXN_THREEBODY;
        else if (kind == "troe") kc = RXN_TROE;
        else return fail(CRF_E_UNSUPPORTED, "reaction " + std::to_string(i) + ": unsupported kind '" + kind + "'");
        RxnInts r; for (int s = 0; s < 8; ++s) r.v[s] = -1;
        int info = kc;
        std::vector<long> el(ne, 0);
        int dsum = 0;
        for (int side = 0; side < 2; ++side) {
            int cnt;
            if (!(ss >> kw >> cnt) || kw != (side == 0 ? "reactants" : "products")) return perr(ln, "expected reactants/products");
            if (cnt <= 0 || cnt > MAX_SIDE) return fail(CRF_E_UNSUPPORTED, "reaction " + std::to_string(i) + ": 1-3 distinct species per side supported");
            int order = 0;
            for (int c = 0; c < cnt; ++c) {
                std::string tok; int k; double v;
                if (!(ss >> tok) || !parse_pair(tok, k, v)) return perr(ln, "bad species:coefficient token");
                if (k < 0 || k >= ns) return fail(CRF_E_MECH, "reaction " + std::to_string(i) + ": species index out of range");
                int nu = (int)v;
                if ((double)nu != v || nu < 1 || nu > 3) return fail(CRF_E_UNSUPPORTED, "reaction " + std::to_string(i) + ": integer coefficients 1..3 only");
                int slot = side * MAX_SIDE + c;
                for (int s = side * MAX_SIDE; s < slot; ++s)
                    if (r.v[s] == k) return fail(CRF_E_MECH, "reaction " + std::to_string(i) + ": species repeated on one side");
                r.v[slot] = k;
                info |= nu << (6 + 2 * slot);
                order += nu;
                for (int e = 0; e < ne; ++e) el[e] += (side == 0 ? -1 : 1) * (long)nu * h.comp[(size_t)k * ne + e];
                dsum += side == 0 ? -nu : nu;
            }
            if (order > 3) return fail(CRF_E_UNSUPPORTED, "reaction " + std::to_string(i) + ": total order above 3 on one side");
            info |= cnt << (side == 0 ? 2 : 4);
        }
        for (int a = 0; a < MAX_SIDE; ++a)
            for (int c = MAX_SIDE; c < SLOTS; ++c)
                if (r.v[a] >= 0 && r.v[a] == r.v[c]) return fail(CRF_E_UNSUPPORTED, "reaction " + std::to_string(i) + ": species on both sides");
        for (int e = 0; e < ne; ++e)
            if (el[e] != 0) return fail(CRF_E_MECH, "reaction " + std::to_string(i) + ": element " + h.elements[e] + " not balanced");
        if (!(ss >> kw >> h.lnA[i] >> h.b[i] >> h.theta[i]) || kw != "arrhenius") return perr(ln, "bad arrhenius block");
        if (!std::isfinite(h.lnA[i]) || !std::isfinite(h.b[i]) || !std::isfinite(h.theta[i])) return fail(CRF_E_MECH, "reaction " + std::to_string(i) + ": non-finite Arrhenius parameters");
        int neff;
        if (!(ss >> kw >> neff) || kw != "efficiencies" || neff < 0 || neff > 255) return perr(ln, "bad efficiencies block");
        if (neff > 0 && kc == RXN_ELEMENTARY) return fail(CRF_E_MECH, "reaction " + std::to_string(i) + ": efficiencies on an elementary reaction");
        r.v[6] = (int)h.eff_sp.size();
        int ntroe_idx = 0;
        for (int c = 0; c < neff; ++c) {
            std::string tok; int k; double v;
            if (!(ss >> tok) || !parse_pair(tok, k, v)) return perr(ln, "bad efficiency token");
            if (k < 0 || k >= ns) return fail(CRF_E_MECH, "reaction " + std::to_string(i) + ": efficiency species out of range");
            if (!(v >= 0) || !std::isfinite(v)) return fail(CRF_E_MECH, "reaction " + std::to_string(i) + ": efficiencies must be finite and >= 0");
            h.eff_sp.push_back(k);
            h.eff_m1.push_back(v - 1.0);
        }
        if (kc == RXN_TROE) {
            double t[7];
            if (!(ss >> kw) || kw != "troe") return perr(ln, "troe reaction without troe block");
            for (int j = 0; j < 7; ++j) if (!(ss >> t[j])) return perr(ln, "troe block needs 7 numbers");
            if (!(t[4] > 0) || !(t[5] > 0) || !(t[6] >= 0) || !std::isfinite(t[3]))
                return fail(CRF_E_MECH, "reaction " + std::to_string(i) + ": Troe needs T*** > 0, T* > 0, T** >= 0");
            ntroe_idx = (int)(h.troe.size() / 8);
            double rec[8] = {t[0], t[1], t[2], t[3], 1.0 / t[4], 1.0 / t[5], t[6], 0.0};
            h.troe.insert(h.troe.end(), rec, rec + 8);
        }
        std::string extra;
        if (ss >> extra) return perr(ln, "trailing token '" + extra + "'");
        r.v[7] = neff | (ntroe_idx << 8);
        h.ri[i] = r;
        h.info[i] = info;
        h.dnu_sum[i] = dsum;
    }
    // Group reactions by kind (elementary, three-body, falloff): a wavefront evaluates 64
    // consecutive reactions at once, so grouping keeps the falloff branch in as few
    // wavefront rounds as possible.  Production rates do not depend on reaction order.
    {
        std::vector<int> order(nr);
        for (int i = 0; i < nr; ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return info_kind(h.info[a]) < info_kind(h.info[b]); });
        auto perm = [&](auto &v) { auto c = v; for (int i = 0; i < nr; ++i) v[i] = c[order[i]]; };
        perm(h.lnA); perm(h.b); perm(h.theta); perm(h.info); perm(h.dnu_sum); perm(h.ri);
    }
    // transport
    if (!L.next(ss) || !(ss >> kw) || kw != "transport") return perr(lineno(), "missing transport section");
    h.mu_fit.assign((size_t)ns * 4, NAN); h.lam_fit.assign((size_t)ns * 4, NAN);
    h.dif_full.assign((size_t)ns * ns * 4, 0.0); h.dif_seen.assign((size_t)ns * ns, 0);
    std::vector<char> mu_seen(ns, 0), lam_seen(ns, 0);
    bool ended = false;
    while (L.next(ss)) {
        if (!(ss >> kw)) return perr(lineno(), "empty line");
        if (kw == "end") { ended = true; break; }
        double c[4];
        if (kw == "viscosity" || kw == "conductivity") {
            int k;
            if (!(ss >> k >> c[0] >> c[1] >> c[2] >> c[3]) || k < 0 || k >= ns) return perr(lineno(), "bad " + kw + " line");
            double *dst = kw == "viscosity" ? &h.mu_fit[(size_t)k * 4] : &h.lam_fit[(size_t)k * 4];
            for (int j = 0; j < 4; ++j) dst[j] = c[j];
            (kw == "viscosity" ? mu_seen : lam_seen)[k] = 1;
        } else if (kw == "diffusion") {
            int j, k;
            if (!(ss >> j >> k >> c[0] >> c[1] >> c[2] >> c[3]) || j < 0 || k < 0 || j >= ns || k >= ns || j == k)
                return perr(lineno(), "bad diffusion line");
            for (int q = 0; q < 4; ++q) {
                h.dif_full[((size_t)j * ns + k) * 4 + q] = c[q];
                h.dif_full[((size_t)k * ns + j) * 4 + q] = c[q];
            }
            h.dif_seen[(size_t)j * ns + k] = h.dif_seen[(size_t)k * ns + j] = 1;
        } else {
            return perr(lineno(), "unexpected transport keyword '" + kw + "'");
        }
    }
    if (!ended) return perr(lineno(), "missing 'end'");
    for (int k = 0; k < ns; ++k) {
        if (!mu_seen[k] || !lam_seen[k]) return fail(CRF_E_MECH, "species " + h.names[k] + ": missing viscosity or conductivity fit");
        for (int j = 0; j < ns; ++j)
            if (j != k && !h.dif_seen[(size_t)j * ns + k])
                return fail(CRF_E_MECH, "missing diffusion fit for pair " + std::to_string(std::min(j, k)) + "," + std::to_string(std::max(j, k)));
    }
    return CRF_OK;
}
// ---------------------------------------------------------------------------- Jacobian plan
// The segmented Jacobian kernel evaluates one reaction per thread and stores, per
// point, the reaction's derivative data in LDS:
//   d values  (index x < nd): dq_i/dC of molecule slot s of reaction i (mass-action
//             part; a species with coefficient nu fills nu slots), then
//             dq_i/d[M] (eps - 1) for every third-body efficiency exception;
//             stored at byte 8 (1 + x) and, negated, at byte 8 (1 + nd + x); byte 0
//             holds 0.0 (the no-op record);
//   quad      (RDq + 32 i): dq_i/dT at fixed C, q_i, dq_i/d[M], sum_j C_j dq_i/dC_j;
//             entry nr is zero.
// The accumulator matrix A (species rows k, stride sr) is then plain sums of these:
//   A[k][0..3] = sum_i dnu_ki quad_i                     ("quad" targets)
//   A[k][5+j]  = sum_i dnu_ki (dq_i/dC_j + exception terms)  ("d" targets)
// Each target is summed by one lane, in rounds that every lane of a wavefront runs in
// lockstep: a quad round reads JS_LQ records per lane (32 r | dnu as a signed 3-bit
// field), a d round JS_LD records (LDS byte offsets of the signed copy; |dnu| = 2, 3
// repeat the record).  A target longer than one round continues in the same lane in
// the next round of its kind; the lane's target word (bits 0-14 A index, bit 15 =
// store and reset after this round) is the first 16-bit field of the round.  Targets
// are packed into shelves of 64 lanes x R rounds (first fit, longest first) and the
// shelves are dealt to the wavefronts, costliest first, onto the least-loaded one.
namespace {

struct GatherTarget {
    int aidx;
    std::vector<unsigned> recs;
};

struct Shelf {
    int R = 0;
    std::vector<std::vector<int>> lane;   // targets of each lane, in order
    std::vector<int> load;                // rounds used by each lane
};

std::vector<Shelf> pack_shelves(const std::vector<GatherTarget> &tg, int L) {
    std::vector<int> order(tg.size());
    for (size_t t = 0; t < tg.size(); ++t) order[t] = (int)t;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return tg[a].recs.size() > tg[b].recs.size(); });
    std::vector<Shelf> sh;
    for (int t : order) {
        const int u = ((int)tg[t].recs.size() + L - 1) / L;
        bool placed = false;
        for (auto &s : sh) {
            for (int l = 0; l < 64 && !placed; ++l)
                if (s.load[l] + u <= s.R) {
                    s.lane[l].push_back(t);
                    s.load[l] += u;
                    placed = true;
                }
            if (placed) break;
        }
        if (!placed) {
            Shelf s;
            s.R = u;
            s.lane.assign(64, {});
            s.load.assign(64, 0);
            s.lane[0].push_back(t);
            s.load[0] = u;
            sh.push_back(std::move(s));
        }
    }
    return sh;
}

// Writes the rounds of `shelves` (all of one kind, L records per round) for one
// wavefront into `out` starting at word `base`; `words` = 32-bit words per lane and round.
void emit_rounds(const std::vector<GatherTarget> &tg, const std::vector<const Shelf *> &shelves, int L,
                 int words, unsigned trash_word, unsigned zero_rec, std::vector<unsigned> &out, size_t base) {
    size_t round = 0;
    for (const Shelf *s : shelves) {
        for (int l = 0; l < 64; ++l) {
            std::vector<unsigned> f;   // 16-bit fields of this lane, round after round
            for (int t : s->lane[l]) {
                const auto &g = tg[t];
                const int u = ((int)g.recs.size() + L - 1) / L;
                for (int part = 0; part < u; ++part) {
                    f.push_back((unsigned)g.aidx | (part == u - 1 ? 0x8000u : 0u));
                    for (int j = 0; j < L; ++j) {
                        const size_t x = (size_t)part * L + j;
                        f.push_back(x < g.recs.size() ? g.recs[x] : zero_rec);
                    }
                }
            }
            while ((int)(f.size() / (1 + L)) < s->R) {
                f.push_back(trash_word);
                for (int j = 0; j < L; ++j) f.push_back(zero_rec);
            }
            for (int r = 0; r < s->R; ++r)
                for (int x = 0; x <= L; ++x) {
                    // field x of round r: word x / 2 (low or high half); quad rounds split
                    // their 8 words into two uint4 halves laid out [half][lane][4]
                    const int w = x / 2;
                    const size_t idx = words == 8 ? base + (round + r) * 512 + (w / 4) * 256 + (size_t)l * 4 + (w % 4)
                                                  : base + (round + r) * 128 + (size_t)l * 2 + w;
                    out[idx] |= (f[(size_t)r * (1 + L) + x] & 0xffffu) << (16 * (x & 1));
                }
        }
        round += s->R;
    }
}

}  // namespace

void build_jac_plan(HostMech &h) {
    h.jp_ok = 0;
    h.jp_thr.clear();
    h.jp_recs.clear();
    h.jp_prog.clear();
    const int ns = h.ns(), nr = h.nr();
    auto no = [&](const std::string &why) {
        h.jp_ok = 0;
        h.jp_why = why;
        h.jp_thr.clear();
        h.jp_recs.clear();
        h.jp_prog.clear();
    };
    if (ns < 1 || nr < 1) return no("empty mechanism");
    if (ns > 64) return no("more than 64 species (the state phase is one species per lane)");
    if (nr > JS_THREADS) return no("more reactions than threads per workgroup");
    // threads: non-Troe reactions first; Troe reactions from the next wavefront boundary
    // (the falloff branch then runs on as few wavefronts as possible)
    int n_non = 0, n_tr = 0;
    for (int i = 0; i < nr; ++i) (info_kind(h.info[i]) == RXN_TROE ? n_tr : n_non)++;
    int tstart = (n_non + 63) / 64 * 64;
    if (tstart + n_tr > JS_THREADS) tstart = n_non;
    std::vector<int> thr_of(nr);
    {
        int a = 0, b = tstart;
        for (int i = 0; i < nr; ++i) thr_of[i] = info_kind(h.info[i]) == RXN_TROE ? b++ : a++;
    }
    // molecule slots and positions of the d values
    std::vector<std::array<int, SLOTS>> mol(nr);
    std::vector<int> dpos(nr), xpos(nr), nfm(nr), nrm(nr);
    int nd = 0;
    for (int i = 0; i < nr; ++i) {
        const int info = h.info[i];
        const RxnInts &ri = h.ri[i];
        mol[i].fill(-1);
        int nf = 0, np = 0;
        for (int s = 0; s < info_nreac(info); ++s)
            for (int c = 0; c < info_nu(info, s); ++c) {
                if (nf == MAX_SIDE) return no("a reaction with more than 3 reactant molecules");
                mol[i][nf++] = ri.v[s];
            }
        for (int s = 0; s < info_nprod(info); ++s)
            for (int c = 0; c < info_nu(info, MAX_SIDE + s); ++c) {
                if (np == MAX_SIDE) return no("a reaction with more than 3 product molecules");
                mol[i][MAX_SIDE + np++] = ri.v[MAX_SIDE + s];
            }
        nfm[i] = nf;
        nrm[i] = np;
        dpos[i] = nd;
        nd += nf + np;
    }
    for (int i = 0; i < nr; ++i) {
        xpos[i] = nd;
        nd += h.ri[i].v[7] & 255;
    }
    if (8 * (1 + 2 * nd) > 0xffff) return no("too many derivative values for 16-bit records");
    const int sr = (ns + 5 + 3) / 4 * 4;
    const int a_trash = ns * sr;
    if (a_trash + 4 > 0x7fff) return no("accumulator matrix too large for 15-bit targets");
    h.jp_nd = nd;
    h.jp_sr = sr;
    // per-thread constants
    h.jp_thr.assign(JS_THREADS, JsThr{-1, 0, 0, 0, 0, 0, -1, 0});
    for (int i = 0; i < nr; ++i) {
        JsThr &c = h.jp_thr[thr_of[i]];
        const int info = h.info[i];
        auto sp = [&](int s) { return (unsigned)(mol[i][s] < 0 ? ns : mol[i][s]); };
        c.r = i;
        c.sp03 = (int)(sp(0) | sp(1) << 8 | sp(2) << 16 | sp(3) << 24);
        c.sp45 = (int)(sp(4) | sp(5) << 8 | (unsigned)nfm[i] << 16 | (unsigned)nrm[i] << 19 |
                       (unsigned)info_kind(info) << 22);
        c.dpos = dpos[i];
        c.xpos = xpos[i] | (h.ri[i].v[7] & 255) << 16;
        c.exc0 = h.ri[i].v[6];
        c.troe = info_kind(info) == RXN_TROE ? (h.ri[i].v[7] >> 8) : -1;
        c.dnu = h.dnu_sum[i];
    }
    // gather targets
    std::vector<std::vector<unsigned>> qrec(ns);
    std::map<int, std::vector<unsigned>> drec;
    for (int i = 0; i < nr; ++i) {
        std::map<int, int> dn;
        for (int s = 0; s < SLOTS; ++s)
            if (mol[i][s] >= 0) dn[mol[i][s]] += s < MAX_SIDE ? -1 : 1;
        const int n_exc = h.ri[i].v[7] & 255;
        for (const auto &kv : dn) {
            const int k = kv.first, v = kv.second;
            if (v == 0) continue;
            qrec[k].push_back(32u * (unsigned)i | ((unsigned)v & 7u));
            const int reps = v < 0 ? -v : v;
            const int neg = v < 0 ? nd : 0;
            for (int s = 0; s < SLOTS; ++s) {
                if (mol[i][s] < 0) continue;
                const int x = dpos[i] + (s < MAX_SIDE ? s : nfm[i] + s - MAX_SIDE);
                for (int c = 0; c < reps; ++c) drec[k * sr + 5 + mol[i][s]].push_back(8u * (unsigned)(1 + neg + x));
            }
            for (int e = 0; e < n_exc; ++e) {
                const int j = h.eff_sp[h.ri[i].v[6] + e];
                for (int c = 0; c < reps; ++c) drec[k * sr + 5 + j].push_back(8u * (unsigned)(1 + neg + xpos[i] + e));
            }
        }
    }
    std::vector<GatherTarget> tq, td;
    for (int k = 0; k < ns; ++k)
        if (!qrec[k].empty()) tq.push_back({k * sr, qrec[k]});
    for (auto &kv : drec) td.push_back({kv.first, kv.second});
    const std::vector<Shelf> sq = pack_shelves(tq, JS_LQ), sd = pack_shelves(td, JS_LD);
    // deal shelves to wavefronts (cost ~ VALU per round of each kind)
    constexpr int CQ = 9 * JS_LQ + 14, CD = 3 * JS_LD + 6;
    struct Item { int cost, kind, idx; };
    std::vector<Item> items;
    for (size_t s = 0; s < sq.size(); ++s) items.push_back({sq[s].R * CQ, 0, (int)s});
    for (size_t s = 0; s < sd.size(); ++s) items.push_back({sd[s].R * CD, 1, (int)s});
    std::stable_sort(items.begin(), items.end(), [](const Item &a, const Item &b) { return a.cost > b.cost; });
    std::vector<int> wload(JS_WAVES, 0);
    std::vector<std::vector<const Shelf *>> wq(JS_WAVES), wd(JS_WAVES);
    for (const Item &it : items) {
        int w = 0;
        for (int u = 1; u < JS_WAVES; ++u)
            if (wload[u] < wload[w]) w = u;
        wload[w] += it.cost;
        (it.kind == 0 ? wq[w] : wd[w]).push_back(it.kind == 0 ? &sq[it.idx] : &sd[it.idx]);
    }
    // emit
    h.jp_prog.assign(4 * JS_WAVES, 0);
    size_t words = 0;
    std::vector<size_t> qoff(JS_WAVES), doff(JS_WAVES);
    for (int w = 0; w < JS_WAVES; ++w) {
        int nq = 0, ndr = 0;
        for (const Shelf *s : wq[w]) nq += s->R;
        for (const Shelf *s : wd[w]) ndr += s->R;
        qoff[w] = words;
        words += (size_t)nq * 512;
        doff[w] = words;
        words += (size_t)ndr * 128;
        h.jp_prog[4 * w + 0] = nq;
        h.jp_prog[4 * w + 1] = ndr;
        h.jp_prog[4 * w + 2] = (int)qoff[w];
        h.jp_prog[4 * w + 3] = (int)doff[w];
    }
    h.jp_recs.assign(words ? words : 4, 0u);
    for (int w = 0; w < JS_WAVES; ++w) {
        emit_rounds(tq, wq[w], JS_LQ, 8, (unsigned)a_trash | 0x8000u, 32u * (unsigned)nr, h.jp_recs, qoff[w]);
        emit_rounds(td, wd[w], JS_LD, 2, (unsigned)a_trash | 0x8000u, 0u, h.jp_recs, doff[w]);
    }
    // self-check: replay the rounds and compare every target's records with the stoichiometry
    {
        std::map<int, std::vector<unsigned>> got_q, got_d;
        auto field = [&](size_t round_base, int words_pl, int l, int x) {
            const int w = x / 2;
            const size_t idx = words_pl == 8 ? round_base + (w / 4) * 256 + (size_t)l * 4 + (w % 4)
                                             : round_base + (size_t)l * 2 + w;
            return (h.jp_recs[idx] >> (16 * (x & 1))) & 0xffffu;
        };
        const unsigned q_lim = 32u * (unsigned)(nr + 1), d_lim = 8u * (unsigned)(1 + 2 * nd);
        for (int w = 0; w < JS_WAVES; ++w)
            for (int kind = 0; kind < 2; ++kind) {
                const int L = kind == 0 ? JS_LQ : JS_LD, wpl = kind == 0 ? 8 : 2;
                const int nrnd = h.jp_prog[4 * w + kind];
                const size_t base = kind == 0 ? qoff[w] : doff[w];
                for (int l = 0; l < 64; ++l) {
                    std::vector<unsigned> cur;
                    for (int r = 0; r < nrnd; ++r) {
                        const size_t rb = base + (size_t)r * (wpl == 8 ? 512 : 128);
                        const unsigned tw = field(rb, wpl, l, 0);
                        for (int x = 1; x <= L; ++x) {
                            const unsigned rec = field(rb, wpl, l, x);
                            if (kind == 0 ? (rec & 0xffe0u) >= q_lim : (rec >= d_lim || (rec & 7u) != 0))
                                return no("plan self-check: record out of range");
                            const bool zero = kind == 0 ? (rec & 7u) == 0 : rec == 0;
                            if (!zero) cur.push_back(rec);
                        }
                        if (tw & 0x8000u) {
                            const int a = (int)(tw & 0x7fffu);
                            if (a + (kind == 0 ? 4 : 1) > a_trash + 4) return no("plan self-check: target out of range");
                            if (kind == 0 && (a % 4) != 0) return no("plan self-check: misaligned quad target");
                            if (a != a_trash) {
                                auto &dst = kind == 0 ? got_q : got_d;
                                if (dst.count(a)) return no("plan self-check: target written twice");
                                dst[a] = cur;
                            } else if (!cur.empty()) {
                                return no("plan self-check: records on the trash target");
                            }
                            cur.clear();
                        }
                    }
                    if (!cur.empty()) return no("plan self-check: unterminated target");
                }
            }
        auto same = [](std::vector<unsigned> a, std::vector<unsigned> b) {
            std::sort(a.begin(), a.end());
            std::sort(b.begin(), b.end());
            return a == b;
        };
        if (got_q.size() != tq.size() || got_d.size() != td.size()) return no("plan self-check: target count");
        for (const auto &g : tq)
            if (!got_q.count(g.aidx) || !same(got_q[g.aidx], g.recs)) return no("plan self-check: quad records");
        for (const auto &g : td)
            if (!got_d.count(g.aidx) || !same(got_d[g.aidx], g.recs)) return no("plan self-check: d records");
    }
    // LDS layout (bytes; A is sized for double accumulators in both precisions)
    auto up16 = [](int b) { return (b + 15) / 16 * 16; };
    int off = up16(8 * (1 + 2 * nd));
    h.jp_off_rdq = off;  off += up16(32 * (nr + 1));
    h.jp_off_a = off;    off += up16(8 * (ns * sr + 4));
    h.jp_off_sp = off;   off += up16(32 * (ns + 1));
    h.jp_off_row = off;  off += up16(16 * ns);
    h.jp_off_p = off;    off += up16(8 * JS_PWAVES * sr);
    h.jp_off_sc = off;   off += up16(8 * 16);
    h.jp_lds = off;
    if (off > JS_MAX_LDS) return no("LDS footprint " + std::to_string(off) + " B above the limit");
    h.jp_ok = 1;
    h.jp_why.clear();
}

// ---------------------------------------------------------------------------- upload
namespace {

struct Packer {
    std::vector<unsigned char> buf;
    size_t add(const void *src, size_t bytes) {
        size_t off = (buf.size() + 255) & ~size_t(255);
        buf.resize(off + bytes);
        if (bytes) std::memcpy(buf.data() + off, src, bytes);
        return off;
    }
    template <class T> size_t add(const std::vector<T> &v) { return add(v.data(), v.size() * sizeof(T)); }
};

}  // namespace

crf_status upload_mechanism(crf_mech *mm, int device) {
    const HostMech &h = mm->host;
    const int ns = h.ns(), nr = h.nr();
    // derived species tables
    std::vector<double> invW(ns), w4(ns), iw4(ns), wc((size_t)ns * ns);
    for (int k = 0; k < ns; ++k) {
        invW[k] = 1.0 / h.W[k];
        w4[k] = std::pow(h.W[k], 0.25);
        iw4[k] = 1.0 / w4[k];
    }
    for (int j = 0; j < ns; ++j)
        for (int k = 0; k < ns; ++k)
            wc[(size_t)j * ns + k] = 1.0 / std::sqrt(8.0 * (1.0 + h.W[k] / h.W[j]));
    std::vector<double> dif;
    std::vector<int> pjk;
    for (int j = 0; j < ns; ++j)
        for (int k = j + 1; k < ns; ++k) {
            for (int q = 0; q < 4; ++q) dif.push_back(h.dif_full[((size_t)j * ns + k) * 4 + q]);
            pjk.push_back(j | (k << 16));
        }
    Packer P;
    size_t oW = P.add(h.W), oInvW = P.add(invW), oNasa = P.add(h.nasa), oMu = P.add(h.mu_fit),
           oLam = P.add(h.lam_fit), oW4 = P.add(w4), oIw4 = P.add(iw4), oWc = P.add(wc), oDif = P.add(dif),
           oPjk = P.add(pjk), oLnA = P.add(h.lnA), oB = P.add(h.b), oTh = P.add(h.theta), oInfo = P.add(h.info),
           oDs = P.add(h.dnu_sum), oRi = P.add(h.ri), oTroe = P.add(h.troe), oEs = P.add(h.eff_sp),
           oEm = P.add(h.eff_m1), oJt = P.add(h.jp_thr), oJr = P.add(h.jp_recs), oJp = P.add(h.jp_prog);
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) return fail(CRF_E_DEVICE, "hipGetDevice failed (no HIP device?)");
    if (hipSetDevice(device) != hipSuccess) return fail(CRF_E_DEVICE, "hipSetDevice(" + std::to_string(device) + ") failed");
    void *d = nullptr;
    if (hipMalloc(&d, P.buf.size() ? P.buf.size() : 256) != hipSuccess) { hipSetDevice(prev); return fail(CRF_E_NOMEM, "hipMalloc of mechanism tables failed"); }
    if (hipMemcpy(d, P.buf.data(), P.buf.size(), hipMemcpyHostToDevice) != hipSuccess) {
        hipFree(d); hipSetDevice(prev);
        return fail(CRF_E_DEVICE, "hipMemcpy of mechanism tables failed");
    }
    hipSetDevice(prev);
    auto at = [&](size_t off) { return (const void *)((const unsigned char *)d + off); };
    DevMech &m = mm->dev;
    m.ns = ns; m.nr = nr; m.n_troe = (int)(h.troe.size() / 8); m.n_exc = (int)h.eff_sp.size();
    m.n_pairs = (int)pjk.size(); m.R = h.R; m.p0 = h.p0;
    m.W = (const double *)at(oW); m.invW = (const double *)at(oInvW); m.nasa = (const double *)at(oNasa);
    m.mu_fit = (const double *)at(oMu); m.lam_fit = (const double *)at(oLam); m.w4 = (const double *)at(oW4);
    m.iw4 = (const double *)at(oIw4); m.wilke_c = (const double *)at(oWc); m.dif_fit = (const double *)at(oDif);
    m.pair_jk = (const int *)at(oPjk); m.lnA = (const double *)at(oLnA); m.b = (const double *)at(oB);
    m.theta = (const double *)at(oTh); m.info = (const int *)at(oInfo); m.dnu_sum = (const int *)at(oDs);
    m.ri = (const RxnInts *)at(oRi); m.troe = (const double *)at(oTroe); m.eff_sp = (const int *)at(oEs);
    m.eff_m1 = (const double *)at(oEm);
    m.jp_thr = (const int *)at(oJt); m.jp_recs = (const unsigned *)at(oJr); m.jp_prog = (const int *)at(oJp);
    m.jp_ok = h.jp_ok; m.jp_nd = h.jp_nd; m.jp_sr = h.jp_sr; m.jp_lds = h.jp_lds;
    m.jp_off_rdq = h.jp_off_rdq; m.jp_off_a = h.jp_off_a; m.jp_off_sp = h.jp_off_sp;
    m.jp_off_row = h.jp_off_row; m.jp_off_p = h.jp_off_p; m.jp_off_sc = h.jp_off_sc;
    mm->dev_buf = d;
    mm->device = device;
    return CRF_OK;
}

}  // namespace crf

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
#include <functional>
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
    if (!L.next(ss) || !(ss >> kw >> ns) || kw != "species" || ns <= 0) return perr(lineno(), "bad species header");
    if (ns > MAX_SPECIES)
        return fail(CRF_E_UNSUPPORTED, std::to_string(ns) + " species; at most " + std::to_string(MAX_SPECIES) +
                                           " are supported (per-point species arrays live in LDS)");
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
        RxnVar var{0, 0, 0, 0};
        if (kind == "elementary") kc = RXN_ELEMENTARY;
        else if (kind == "threebody") kc = RXN_THREEBODY;
        else if (kind == "troe") kc = RXN_TROE;
        else if (kind == "lindemann") { kc = RXN_TROE; var.flags |= VAR_LINDEMANN; }
        else if (kind == "sri") { kc = RXN_TROE; var.flags |= VAR_SRI; }
        else if (kind == "plog") { kc = RXN_ELEMENTARY; var.flags |= VAR_PLOG; }
        else if (kind == "chebyshev") { kc = RXN_ELEMENTARY; var.flags |= VAR_CHEB; }
        else return fail(CRF_E_UNSUPPORTED, "reaction " + std::to_string(i) + ": unsupported kind '" + kind + "'");
        const std::string rn = "reaction " + std::to_string(i);
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
        auto finite_all = [](const double *v, int n) {
            for (int j = 0; j < n; ++j) if (!std::isfinite(v[j])) return false;
            return true;
        };
        if (kc == RXN_TROE && !(var.flags & (VAR_LINDEMANN | VAR_SRI))) {
            double t[7];
            if (!(ss >> kw) || kw != "troe") return perr(ln, "troe reaction without troe block");
            for (int j = 0; j < 7; ++j) if (!(ss >> t[j])) return perr(ln, "troe block needs 7 numbers");
            if (!(t[4] > 0) || !(t[5] > 0) || !(t[6] >= 0) || !std::isfinite(t[3]))
                return fail(CRF_E_MECH, rn + ": Troe needs T*** > 0, T* > 0, T** >= 0");
            ntroe_idx = (int)(h.troe.size() / 8);
            double rec[8] = {t[0], t[1], t[2], t[3], 1.0 / t[4], 1.0 / t[5], t[6], 0.0};
            h.troe.insert(h.troe.end(), rec, rec + 8);
        } else if (var.flags & VAR_LINDEMANN) {
            double t[3];
            if (!(ss >> kw) || kw != "falloff") return perr(ln, "lindemann reaction without falloff block");
            for (int j = 0; j < 3; ++j) if (!(ss >> t[j])) return perr(ln, "falloff block needs 3 numbers");
            if (!finite_all(t, 3)) return fail(CRF_E_MECH, rn + ": non-finite falloff parameters");
            ntroe_idx = (int)(h.troe.size() / 8);
            double rec[8] = {t[0], t[1], t[2], 0, 0, 0, 0, 0};
            h.troe.insert(h.troe.end(), rec, rec + 8);
        } else if (var.flags & VAR_SRI) {
            double t[8];
            if (!(ss >> kw) || kw != "sri") return perr(ln, "sri reaction without sri block");
            for (int j = 0; j < 8; ++j) if (!(ss >> t[j])) return perr(ln, "sri block needs 8 numbers");
            if (!finite_all(t, 8) || !(t[3] >= 0) || !(t[5] > 0) || !(t[6] > 0))
                return fail(CRF_E_MECH, rn + ": SRI needs a >= 0, c > 0, d > 0");
            ntroe_idx = (int)(h.troe.size() / 8);
            h.troe.insert(h.troe.end(), t, t + 8);
        } else if (var.flags & VAR_PLOG) {
            int np_;
            if (!(ss >> kw >> np_) || kw != "plog" || np_ < 1 || np_ > 64) return perr(ln, "bad plog block");
            var.rate_off = (int)h.vtab.size();
            h.vtab.push_back(np_);
            double lastp = 0.0;
            for (int j = 0; j < np_; ++j) {
                double e[4];
                for (int q = 0; q < 4; ++q) if (!(ss >> e[q])) return perr(ln, "plog entry needs 4 numbers");
                if (!finite_all(e, 4) || !(e[0] > lastp)) return fail(CRF_E_MECH, rn + ": PLOG pressures must be positive and ascending");
                lastp = e[0];
                const double rec[4] = {std::log(e[0]), e[1], e[2], e[3]};
                h.vtab.insert(h.vtab.end(), rec, rec + 4);
            }
        } else if (var.flags & VAR_CHEB) {
            double r4[4];
            int nT, nP;
            if (!(ss >> kw) || kw != "chebyshev") return perr(ln, "bad chebyshev block");
            for (int q = 0; q < 4; ++q) if (!(ss >> r4[q])) return perr(ln, "chebyshev block needs Tmin Tmax Pmin Pmax");
            if (!(ss >> nT >> nP) || nT < 1 || nP < 1 || nT > 16 || nP > 16) return perr(ln, "chebyshev needs 1..16 x 1..16 coefficients");
            if (!finite_all(r4, 4) || !(0 < r4[0] && r4[0] < r4[1]) || !(0 < r4[2] && r4[2] < r4[3]))
                return fail(CRF_E_MECH, rn + ": Chebyshev needs 0 < Tmin < Tmax and 0 < Pmin < Pmax");
            var.rate_off = (int)h.vtab.size();
            const double head[6] = {(double)nT, (double)nP, 1.0 / r4[0], 1.0 / r4[1], std::log10(r4[2]), std::log10(r4[3])};
            h.vtab.insert(h.vtab.end(), head, head + 6);
            for (int q = 0; q < nT * nP; ++q) {
                double a;
                if (!(ss >> a) || !std::isfinite(a)) return perr(ln, "bad chebyshev coefficient");
                h.vtab.push_back(a);
            }
        }
        // optional modifiers
        std::string extra;
        while (ss >> extra) {
            if (extra == "reverse") {
                double t[3];
                for (int j = 0; j < 3; ++j) if (!(ss >> t[j])) return perr(ln, "reverse block needs 3 numbers");
                if (!finite_all(t, 3)) return fail(CRF_E_MECH, rn + ": non-finite reverse parameters");
                if (kc == RXN_TROE) return fail(CRF_E_UNSUPPORTED, rn + ": explicit reverse rates of falloff reactions are not supported");
                if (var.flags & (VAR_REVERSE | VAR_IRREV)) return fail(CRF_E_MECH, rn + ": more than one reverse specification");
                var.flags |= VAR_REVERSE;
                var.rev_off = (int)h.vtab.size();
                h.vtab.insert(h.vtab.end(), t, t + 3);
            } else if (extra == "irreversible") {
                if (var.flags & (VAR_REVERSE | VAR_IRREV)) return fail(CRF_E_MECH, rn + ": more than one reverse specification");
                var.flags |= VAR_IRREV;
            } else if (extra == "orders") {
                int no;
                if (!(ss >> no) || no < 1 || no > MAX_SIDE) return perr(ln, "bad orders block");
                if (var.flags & VAR_ORDERS) return fail(CRF_E_MECH, rn + ": orders given twice");
                double ord[MAX_SIDE];
                for (int sl = 0; sl < MAX_SIDE; ++sl) ord[sl] = r.v[sl] >= 0 ? (double)info_nu(info, sl) : 0.0;
                for (int j = 0; j < no; ++j) {
                    std::string tok; int k; double v;
                    if (!(ss >> tok) || !parse_pair(tok, k, v)) return perr(ln, "bad order token");
                    int sl = -1;
                    for (int q = 0; q < MAX_SIDE; ++q) if (r.v[q] == k) sl = q;
                    if (sl < 0) return fail(CRF_E_UNSUPPORTED, rn + ": orders are supported for reactant species only");
                    if (!(v > 0) || !std::isfinite(v)) return fail(CRF_E_MECH, rn + ": orders must be positive and finite");
                    ord[sl] = v;
                }
                var.flags |= VAR_ORDERS;
                var.ord_off = (int)h.vtab.size();
                h.vtab.insert(h.vtab.end(), ord, ord + MAX_SIDE);
            } else {
                return perr(ln, "trailing token '" + extra + "'");
            }
        }
        if (var.flags != 0) ++h.n_var;
        h.var.push_back(var);
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
        perm(h.lnA); perm(h.b); perm(h.theta); perm(h.info); perm(h.dnu_sum); perm(h.ri); perm(h.var);
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
// point, the reaction's derivative data in LDS as FP64 "d values" (index x, byte 8 x):
//   x = 0                  0.0 (the no-op record)
//   x = 1 + dpos_i + s     dq_i/dC of molecule slot s of reaction i (mass-action part;
//                          a species with coefficient nu fills nu slots)
//   x = 1 + xpos_i + e     dq_i/d[M] (eps - 1) for efficiency exception e of reaction i
//   x = qb + 4 i + c       c = 0: dq_i/dT at fixed C, 1: q_i, 2: dq_i/d[M],
//                          3: sum_j C_j dq_i/dC_j  (qb a multiple of 4: aligned quads)
//   x = pb + p             partial sums of the gather
// The accumulator matrix A (species rows k, stride sr, FP64) is plain sums of these:
//   A[k][c]     = sum_i dnu_ki value(qb + 4 i + c),  c = 0..3
//   A[k][5 + j] = sum_i dnu_ki (dq_i/dC_j + exception terms)
// Every target entry becomes a small reduction tree of tasks; a task is one lane of one
// round: it adds at most JS_LD records (byte offset of a value | dnu or +1 as a signed
// 3-bit field) and stores the sum to its destination word (the first 16-bit field of the
// lane's round: the LDS index of the destination in 8-byte units).  A target's tasks run
// on one wavefront.  The kernel reads a round's values during the round before, so a task
// that reads a partial runs at least two rounds after the task that stores it; within
// that rule the tasks are list-scheduled (longest remaining chain first, at most 64 per
// round), so levels of different trees share rounds.  Trees are dealt to the wavefronts
// to balance their tasks; within a round, tasks are placed on lanes (and their records
// ordered) so that the lanes of each 16- and 32-lane group address different LDS banks
// where possible.
namespace {

struct PlanTask {
    bool partial;                 // destination is a partial slot (else the final entry)
    int dest;                     // partial index or A entry
    std::vector<unsigned> recs;
    int level;
};

struct PlanTree {
    int final_dest;
    std::vector<unsigned> leaves; // the target's leaf records (for the self-check)
    std::vector<PlanTask> tasks;
    int depth;
};

// Splits `recs` into tasks of at most L records; full chunks become partial sums,
// leftovers are carried to the next level with the new partial records.  Partials are
// symbolic here (PARTIAL_REC | id); LDS slots are assigned once the rounds are known.
constexpr unsigned PARTIAL_REC = 0x80000000u;

void build_tree(PlanTree &t, std::vector<unsigned> recs, int L, int &n_partial) {
    int level = 0;
    while ((int)recs.size() > L) {
        std::vector<unsigned> next;
        const size_t full = recs.size() / L * L;
        for (size_t c = 0; c < full; c += L) {
            const int p = n_partial++;
            t.tasks.push_back({true, p, std::vector<unsigned>(recs.begin() + c, recs.begin() + c + L), level});
            next.push_back(PARTIAL_REC | (unsigned)p);
        }
        for (size_t c = full; c < recs.size(); ++c) next.push_back(recs[c]);
        recs = std::move(next);
        ++level;
    }
    t.tasks.push_back({false, t.final_dest, recs, level});
    t.depth = level + 1;
}

int coef_of(unsigned rec) { return ((int)(rec & 7u) ^ 4) - 4; }

}  // namespace

template <class T> static std::vector<T> cat(std::vector<T> a, const std::vector<T> &b) {
    a.insert(a.end(), b.begin(), b.end());
    return a;
}

// Order and orientation of the pairs of one round of the transport pair schedule.  Any
// order gives the same sums (a round adds into each species once).  The tile kernel with W
// wavefronts puts W consecutive pairs of a round into one 16-lane part of an LDS instruction,
// and row j of the wavefront's points starts at bank slot j mod W (tt_rs), so W consecutive
// pairs whose first members are distinct mod W, and whose second members are too, touch
// every bank once.  Each group of W pairs is filled greedily (a pair and orientation adding
// no repeated residue on either side, else the fewest), restarted from other positions
// (a fixed pseudo-random sequence) until a group without repeats is found or 32 attempts
// are made; a group is then sorted by its first members' residues.
static std::vector<std::pair<int, int>> order_round_pairs(std::vector<std::pair<int, int>> rest, int W) {
    std::vector<std::pair<int, int>> out;
    unsigned long long seed = 0x9e3779b97f4a7c15ull;
    auto rnd = [&]() {
        seed ^= seed << 13;
        seed ^= seed >> 7;
        seed ^= seed << 17;
        return seed;
    };
    while (!rest.empty()) {
        const int g = std::min<int>(W, (int)rest.size());
        std::vector<int> bidx;
        std::vector<std::pair<int, int>> bgrp;
        int best_cost = 1 << 30;
        for (int attempt = 0; attempt < 32 && best_cost > 0; ++attempt) {
            const size_t s0 = attempt == 0 ? 0 : (size_t)(rnd() % rest.size());
            std::vector<char> used(rest.size(), 0);
            std::vector<int> idx;
            std::vector<std::pair<int, int>> grp;
            unsigned lmask = 0, rmask = 0;
            int cost = 0;
            for (int t = 0; t < g; ++t) {
                int bi = -1, bf = 0, bc = 3;
                for (size_t u = 0; u < rest.size() && bc > 0; ++u) {
                    const size_t i = (s0 + u) % rest.size();
                    if (used[i]) continue;
                    for (int f = 0; f < 2; ++f) {
                        const int a = f ? rest[i].second : rest[i].first, b = f ? rest[i].first : rest[i].second;
                        const int c = (int)((lmask >> (a % W)) & 1u) + (int)((rmask >> (b % W)) & 1u);
                        if (c < bc) {
                            bc = c;
                            bi = (int)i;
                            bf = f;
                            if (c == 0) break;
                        }
                    }
                }
                if (bi < 0) break;   // not reached: g never exceeds the pairs left
                used[bi] = 1;
                const int a = bf ? rest[bi].second : rest[bi].first, b = bf ? rest[bi].first : rest[bi].second;
                lmask |= 1u << (a % W);
                rmask |= 1u << (b % W);
                cost += bc;
                idx.push_back(bi);
                grp.emplace_back(a, b);
            }
            if ((int)idx.size() == g && cost < best_cost) {
                best_cost = cost;
                bidx = idx;
                bgrp = grp;
            }
        }
        std::stable_sort(bgrp.begin(), bgrp.end(), [W](const std::pair<int, int> &x, const std::pair<int, int> &y) {
            return x.first % W < y.first % W;
        });
        out.insert(out.end(), bgrp.begin(), bgrp.end());
        std::sort(bidx.begin(), bidx.end());
        for (int t = g - 1; t >= 0; --t) rest.erase(rest.begin() + bidx[t]);
    }
    return out;
}

void build_jac_plan(HostMech &h) {
    h.jp_ok = 0;
    h.jp_thr.clear();
    h.jp_recs.clear();
    h.jp_prog.clear();
    h.jp_mrx.clear();
    const int ns = h.ns(), nr = h.nr();
    auto no = [&](const std::string &why) {
        h.jp_ok = 0;
        h.jp_why = why;
        h.jp_thr.clear();
        h.jp_recs.clear();
        h.jp_prog.clear();
        h.jp_mrx.clear();
    };
    if (ns < 1 || nr < 1) return no("empty mechanism");
    for (int i = 0; i < nr; ++i)   // the rate phase forms products of whole molecules
        if (h.var[i].flags & VAR_ORDERS) return no("reactions with non-integer forward orders");
    if (ns > 64) return no("more than 64 species (the state phase is one species per lane)");
    if (nr > JS_THREADS) return no("more reactions than threads per workgroup");
    {   // emission: column pairs x row phases over JS_EWAVES wavefronts, at most JS_EROWS rows each
        const int n1 = ns + 1, npair = (n1 + 1) / 2, rphase = JS_EWAVES * 64 / npair;
        if (rphase < 1 || (n1 + rphase - 1) / rphase > JS_EROWS) return no("Jacobian rows per emitting thread");
    }
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
    const int qb = (1 + nd + 3) / 4 * 4;          // first quad value (a multiple of 4: 16-byte quads in FP32)
    const int pb = qb + 4 * nr;                   // first partial
    const int sr = (ns + 5 + 1) / 2 * 2;
    h.jp_nd = nd;
    h.jp_qb = qb;
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
        c.troe = info_kind(info) == RXN_TROE ? (h.ri[i].v[7] >> 8) & 0xffff : 0xffff;
        c.dnu = h.dnu_sum[i];
    }
    // [M] slots, formed with the state: falloff reactions first (only they need ln [M]);
    // reactions with the same efficiency exceptions share a slot
    std::map<std::vector<std::pair<int, double>>, int> mslot_of;
    for (int pass = 0; pass < 2; ++pass)
        for (int i = 0; i < nr; ++i) {
            const int kind = info_kind(h.info[i]);
            if (kind == RXN_ELEMENTARY || (kind == RXN_TROE) != (pass == 0)) continue;
            std::vector<std::pair<int, double>> key;
            for (int e = 0; e < (h.ri[i].v[7] & 255); ++e)
                key.emplace_back(h.eff_sp[h.ri[i].v[6] + e], h.eff_m1[h.ri[i].v[6] + e]);
            auto it = mslot_of.find(key);
            int slot;
            if (it != mslot_of.end()) {
                slot = it->second;
            } else {
                slot = (int)h.jp_mrx.size() / 2;
                mslot_of.emplace(key, slot);
                h.jp_mrx.push_back(h.ri[i].v[6]);
                h.jp_mrx.push_back(h.ri[i].v[7] & 255);
            }
            h.jp_thr[thr_of[i]].troe |= slot << 16;
        }
    for (int i = 0; i < nr; ++i)
        if (info_kind(h.info[i]) == RXN_ELEMENTARY) h.jp_thr[thr_of[i]].troe |= 0xffff << 16;
    // gather targets (leaf records) keyed by A entry
    std::map<int, std::vector<unsigned>> drec;
    for (int i = 0; i < nr; ++i) {
        std::map<int, int> dn;
        for (int s = 0; s < SLOTS; ++s)
            if (mol[i][s] >= 0) dn[mol[i][s]] += s < MAX_SIDE ? -1 : 1;
        const int n_exc = h.ri[i].v[7] & 255;
        const bool third = info_kind(h.info[i]) != RXN_ELEMENTARY;
        for (const auto &kv : dn) {
            const int k = kv.first, v = kv.second;
            if (v == 0) continue;
            const unsigned cf = (unsigned)v & 7u;
            for (int c = 0; c < 4; ++c)
                if (c != 2 || third) drec[k * sr + c].push_back(8u * (unsigned)(qb + 4 * i + c) | cf);
            for (int s = 0; s < SLOTS; ++s) {
                if (mol[i][s] < 0) continue;
                const int x = dpos[i] + (s < MAX_SIDE ? s : nfm[i] + s - MAX_SIDE);
                drec[k * sr + 5 + mol[i][s]].push_back(8u * (unsigned)(1 + x) | cf);
            }
            for (int e = 0; e < n_exc; ++e) {
                const int j = h.eff_sp[h.ri[i].v[6] + e];
                drec[k * sr + 5 + j].push_back(8u * (unsigned)(1 + xpos[i] + e) | cf);
            }
        }
    }
    // reduction trees
    std::vector<PlanTree> trees;
    int nsym = 0;   // symbolic partials
    for (auto &kv : drec) {
        PlanTree t{kv.first, kv.second, {}, 0};
        build_tree(t, kv.second, JS_LD, nsym);
        trees.push_back(std::move(t));
    }
    // deal the trees to the wavefronts: estimated rounds = the larger of ceil(tasks / 64)
    // and the longest chain (2 depth - 1 rounds); the makespan first, then the fewest
    // tasks, then the smallest increase
    constexpr int MAXLV = 8;
    std::vector<std::array<int, MAXLV>> cnt(JS_WAVES);
    for (auto &c : cnt) c.fill(0);
    auto rounds_of = [&](const std::array<int, MAXLV> &lv) {
        int n = 0, deep = 0;
        for (int l = 0; l < MAXLV; ++l)
            if (lv[l]) {
                n += lv[l];
                deep = l + 1;
            }
        return std::max((n + 63) / 64, 2 * deep - 1);
    };
    std::vector<int> order(trees.size());
    for (size_t t = 0; t < trees.size(); ++t) order[t] = (int)t;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if (trees[a].depth != trees[b].depth) return trees[a].depth > trees[b].depth;
        return trees[a].tasks.size() > trees[b].tasks.size();
    });
    std::vector<int> wave_of(trees.size(), -1), wtasks(JS_WAVES, 0), wrounds(JS_WAVES, 0);
    for (int t : order) {
        const PlanTree &tr = trees[t];
        if (tr.depth > MAXLV) return no("reduction tree too deep");
        const int span = *std::max_element(wrounds.begin(), wrounds.end());
        int best = -1, best_span = 0, best_inc = 0;
        for (int w = 0; w < JS_WAVES; ++w) {
            auto lv = cnt[w];
            for (const auto &tk : tr.tasks) lv[tk.level]++;
            const int rd = rounds_of(lv);
            if (rd > JS_DMAX) continue;
            const int nspan = std::max(span, rd), inc = rd - wrounds[w];
            if (best < 0 || nspan < best_span || (nspan == best_span && wtasks[w] < wtasks[best]) ||
                (nspan == best_span && wtasks[w] == wtasks[best] && inc < best_inc)) {
                best = w;
                best_span = nspan;
                best_inc = inc;
            }
        }
        if (best < 0) return no("gather rounds exceed the per-wavefront register budget");
        wave_of[t] = best;
        for (const auto &tk : tr.tasks) cnt[best][tk.level]++;
        wtasks[best] += (int)tr.tasks.size();
        wrounds[best] = rounds_of(cnt[best]);
    }
    // rounds per wavefront by list scheduling: a task is ready two rounds after the last
    // store of a partial it reads; the ready tasks with the longest remaining chain go
    // first, at most 64 per round; the rounds are padded to JS_DMAX
    struct Slot { int tree, task; };
    std::vector<std::vector<std::vector<Slot>>> rounds(JS_WAVES);
    {
        std::vector<int> producer_round(nsym, -1);
        for (int w = 0; w < JS_WAVES; ++w) {
            std::vector<Slot> todo;
            for (size_t t = 0; t < trees.size(); ++t)
                if (wave_of[t] == w)
                    for (size_t q = 0; q < trees[t].tasks.size(); ++q) todo.push_back({(int)t, (int)q});
            auto height = [&](const Slot &sl) { return trees[sl.tree].depth - 1 - trees[sl.tree].tasks[sl.task].level; };
            std::stable_sort(todo.begin(), todo.end(), [&](const Slot &a, const Slot &b) { return height(a) > height(b); });
            std::vector<char> done(todo.size(), 0);
            size_t left = todo.size();
            for (int r = 0; left > 0; ++r) {
                if (r >= JS_DMAX) return no("gather rounds exceed the per-wavefront register budget");
                rounds[w].emplace_back();
                for (size_t x = 0; x < todo.size() && rounds[w][r].size() < 64; ++x) {
                    if (done[x]) continue;
                    const PlanTask &tk = trees[todo[x].tree].tasks[todo[x].task];
                    bool ready = true;
                    for (unsigned rec : tk.recs)
                        if (rec & PARTIAL_REC) {
                            const int pr = producer_round[rec & ~PARTIAL_REC];
                            ready = ready && pr >= 0 && pr <= r - 2;
                        }
                    if (!ready) continue;
                    rounds[w][r].push_back(todo[x]);
                    done[x] = 1;
                    --left;
                }
                for (const Slot &sl : rounds[w][r]) {
                    const PlanTask &tk = trees[sl.tree].tasks[sl.task];
                    if (tk.partial) producer_round[tk.dest] = r;
                }
            }
            wrounds[w] = (int)rounds[w].size();
            rounds[w].resize(JS_DMAX);
        }
    }
    // LDS slots of the partials, per wavefront with reuse: a partial lives from the round
    // that stores it to the round that reads it (whose loads are issued in the round
    // before); a slot is reused only from that reading round on
    std::vector<int> slot_of(nsym, -1), wround(nsym, -1), rround(nsym, -1), pwave(nsym, -1);
    for (int w = 0; w < JS_WAVES; ++w)
        for (int r = 0; r < JS_DMAX; ++r)
            for (const Slot &sl : rounds[w][r]) {
                const PlanTask &tk = trees[sl.tree].tasks[sl.task];
                if (tk.partial) {
                    wround[tk.dest] = r;
                    pwave[tk.dest] = w;
                }
                for (unsigned rec : tk.recs)
                    if (rec & PARTIAL_REC) rround[rec & ~PARTIAL_REC] = r;
            }
    int npd = 0;
    for (int w = 0; w < JS_WAVES; ++w) {
        std::vector<int> free_slots;
        std::vector<std::vector<int>> release(JS_DMAX + 1);
        for (int r = 0; r < JS_DMAX; ++r) {
            for (int slot : release[r]) free_slots.push_back(slot);
            for (const Slot &sl : rounds[w][r]) {
                const PlanTask &tk = trees[sl.tree].tasks[sl.task];
                if (!tk.partial) continue;
                const int p = tk.dest;
                if (rround[p] <= r || pwave[p] != w) return no("plan: partial read before it is written");
                int slot;
                if (!free_slots.empty()) {
                    slot = free_slots.back();
                    free_slots.pop_back();
                } else {
                    slot = npd++;
                }
                slot_of[p] = slot;
                release[rround[p]].push_back(slot);
            }
        }
    }
    auto resolve = [&](unsigned rec) -> unsigned {
        return (rec & PARTIAL_REC) ? 8u * (unsigned)(pb + slot_of[rec & ~PARTIAL_REC]) | 1u : rec;
    };
    if (8 * (pb + npd) > 0xfff8) return no("too many derivative values for 16-bit records");
    // LDS layout (bytes)
    auto up = [](int b, int a) { return (b + a - 1) / a * a; };
    const int n_troe = (int)(h.troe.size() / 8);
    int off = up(8 * (pb + npd), 32);
    h.jp_off_a = off;    off = up(off + 8 * (ns * sr + 4), 16);
    h.jp_off_sp = off;   off = up(off + 2 * 32 * (ns + 1), 16);
    h.jp_off_row = off;  off = up(off + 16 * ns, 16);
    h.jp_off_p = off;    off = up(off + 8 * JS_PWAVES * sr, 16);
    h.jp_off_sc = off;   off = up(off + 8 * 32, 16);
    h.jp_off_tp = off;   off = up(off + 8 * JS_TP * n_troe, 16);
    h.jp_off_tq = off;   off = up(off + 8 * JS_TQ * n_troe, 16);
    h.jp_off_ns = off;   off = up(off + 8 * 16 * ns, 16);
    h.jp_off_iw = off;   off = up(off + 8 * ns, 16);
    h.jp_off_ex = off;   off = up(off + 12 * (int)h.eff_sp.size(), 16);
    h.jp_nm = (int)h.jp_mrx.size() / 2;
    h.jp_off_mx = off;   off = up(off + 8 * h.jp_nm, 16);
    h.jp_off_mq = off;   off = up(off + 16 * h.jp_nm, 16);
    h.jp_lds = off;
    if (off > JS_MAX_LDS) return no("LDS footprint " + std::to_string(off) + " B above the limit");
    const int a_trash = ns * sr;
    const unsigned trash = (unsigned)(h.jp_off_a / 8 + a_trash);
    if (trash > 0xffff) return no("accumulator matrix beyond 16-bit destination words");
    auto dest_word = [&](const PlanTask &tk) -> unsigned {
        return tk.partial ? (unsigned)(pb + slot_of[tk.dest]) : (unsigned)(h.jp_off_a / 8 + tk.dest);
    };

    h.jp_prog.assign(8 * JS_WAVES, 0);
    h.jp_rmax = 0;
    for (int w = 0; w < JS_WAVES; ++w) {
        h.jp_prog[8 * w + 0] = wrounds[w];
        h.jp_rmax = std::max(h.jp_rmax, wrounds[w]);
        h.jp_prog[8 * w + 1] = w * JS_DMAX * 128;   // first 32-bit word of the wavefront's rounds
    }
    constexpr int L = JS_LD, WPL = 2, RSZ = 64 * WPL;
    h.jp_recs.assign((size_t)JS_WAVES * JS_DMAX * RSZ, 0u);
    for (int w = 0; w < JS_WAVES; ++w)
        for (int r = 0; r < JS_DMAX; ++r) {
            // lanes and record order of this round's tasks, chosen so that in every LDS
            // instruction of the round (one per record field, and the store) the lanes of
            // each 16- and 32-lane group address different banks where possible
            std::vector<std::array<unsigned, 1 + L>> lane_f(64);
            std::array<std::array<std::array<std::array<int, 32>, 4>, 2>, 1 + L> cnt_b{};
            auto key_of = [&](int x, unsigned v) { return (x == 0 ? 8u * v : (v & 0xfff8u)) / 8u; };
            auto cost_of = [&](int l, const std::array<unsigned, 1 + L> &f) {
                int c = 0;
                for (int x = 0; x <= L; ++x) {
                    if (x > 0 && (f[x] & 7u) == 0) continue;   // no-op records read one broadcast address
                    const unsigned a = key_of(x, f[x]);
                    c += cnt_b[x][0][l / 16][a % 16] + cnt_b[x][1][l / 32][a % 32];
                }
                return c;
            };
            std::vector<bool> used(64, false);
            for (const Slot &sl : rounds[w][r]) {
                const PlanTask &tk = trees[sl.tree].tasks[sl.task];
                std::array<unsigned, 1 + L> f;
                f.fill(0u);
                f[0] = dest_word(tk);
                for (size_t x = 0; x < tk.recs.size(); ++x) f[1 + x] = resolve(tk.recs[x]);
                std::array<int, L> idx;
                for (int x = 0; x < L; ++x) idx[x] = x;
                int best_l = -1, best_c = 0;
                std::array<unsigned, 1 + L> best_f = f, g = f;
                do {
                    for (int x = 0; x < L; ++x) g[1 + x] = f[1 + idx[x]];
                    for (int l = 0; l < 64; ++l) {
                        if (used[l]) continue;
                        const int c = cost_of(l, g);
                        if (best_l < 0 || c < best_c) {
                            best_l = l;
                            best_c = c;
                            best_f = g;
                        }
                    }
                } while (std::next_permutation(idx.begin(), idx.end()));
                used[best_l] = true;
                lane_f[best_l] = best_f;
                for (int x = 0; x <= L; ++x) {
                    if (x > 0 && (best_f[x] & 7u) == 0) continue;
                    const unsigned a = key_of(x, best_f[x]);
                    cnt_b[x][0][best_l / 16][a % 16]++;
                    cnt_b[x][1][best_l / 32][a % 32]++;
                }
            }
            for (int l = 0; l < 64; ++l) {
                if (!used[l]) {
                    lane_f[l].fill(0u);
                    lane_f[l][0] = trash;
                }
                for (int x = 0; x <= L; ++x)
                    h.jp_recs[(size_t)w * JS_DMAX * RSZ + (size_t)r * RSZ + (size_t)l * WPL + x / 2] |=
                        (lane_f[l][x] & 0xffffu) << (16 * (x & 1));
            }
        }
    // self-check: replay the rounds symbolically (LDS word -> leaf records with their
    // coefficients) in the kernel's order: the loads of round r are issued before the
    // store of round r - 1, so they see the stores of rounds <= r - 2; compare every final
    // entry with its target's leaves
    {
        std::map<unsigned, std::map<unsigned, int>> fin;
        const unsigned leaf_lim = 8u * (unsigned)pb;
        for (int w = 0; w < JS_WAVES; ++w) {
            std::map<unsigned, std::map<unsigned, int>> val;           // partial slots of this wavefront
            std::vector<std::pair<unsigned, std::map<unsigned, int>>> pending;   // stores of round r - 1
            for (int r = 0; r <= JS_DMAX; ++r) {
                std::vector<std::pair<unsigned, std::map<unsigned, int>>> stores;
                if (r < JS_DMAX)
                    for (int l = 0; l < 64; ++l) {
                        auto field = [&](int x) {
                            return (h.jp_recs[(size_t)w * JS_DMAX * RSZ + (size_t)r * RSZ + (size_t)l * WPL + x / 2] >>
                                    (16 * (x & 1))) & 0xffffu;
                        };
                        std::map<unsigned, int> v;
                        for (int x = 1; x <= L; ++x) {
                            const unsigned rec = field(x), addr = rec & 0xfff8u;
                            const int coef = coef_of(rec);
                            if (coef == 0) continue;
                            if (addr == 0) return no("plan self-check: record on the zero entry");
                            if (addr < leaf_lim) {
                                v[addr] += coef;
                            } else {
                                auto it = val.find(addr);
                                if (it == val.end()) return no("plan self-check: partial read before written");
                                for (const auto &lv : it->second) v[lv.first] += coef * lv.second;
                            }
                        }
                        stores.push_back({8u * field(0), v});
                    }
                for (auto &st : pending) {   // round r - 1's stores land after round r's loads
                    if (st.first == 8u * trash) {
                        for (const auto &lv : st.second)
                            if (lv.second) return no("plan self-check: records on the trash target");
                        continue;
                    }
                    if (st.first >= (unsigned)h.jp_off_a) {
                        if (fin.count(st.first)) return no("plan self-check: final entry written twice");
                        fin[st.first] = st.second;
                    } else {
                        if (st.first < leaf_lim) return no("plan self-check: bad partial destination");
                        val[st.first] = st.second;
                    }
                }
                pending = std::move(stores);
            }
        }
        for (const auto &tr : trees) {
            std::map<unsigned, int> want;
            for (unsigned rec : tr.leaves) want[rec & 0xfff8u] += coef_of(rec);
            for (auto it = want.begin(); it != want.end();) it = it->second == 0 ? want.erase(it) : std::next(it);
            auto it = fin.find((unsigned)(h.jp_off_a + 8 * tr.final_dest));
            if (it == fin.end()) return no("plan self-check: target never written");
            std::map<unsigned, int> got = it->second;
            for (auto g = got.begin(); g != got.end();) g = g->second == 0 ? got.erase(g) : std::next(g);
            if (got != want) return no("plan self-check: target sum differs from the stoichiometry");
        }
        if (fin.size() != trees.size()) return no("plan self-check: stray final entries");
    }
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
    // round-robin schedule of the species pairs (circle method): round r pairs the
    // positions of a circle of n2 (even) entries, fixed entry 0, the others rotated
    const int n2 = ns + (ns & 1), tr_slots = n2 / 2, tr_rounds = n2 - 1;
    // pair order of the FP64 tables (tr_jk, tr_off FP64 part, tr_fit: the FP64 tile and the
    // species-per-lane kernel) and of the mixed ones (tr_off mixed part, tr_fit32), each for
    // its precision's tile width; byte offsets of the pair's rows fit 16 bits while the tile fits
    const int tw64 = tile_transport_waves(ns + 1, false), tw32 = tile_transport_waves(ns + 1, true);
    const int wa = tw64 ? tw64 : 4, wb = tw32 ? tw32 : 4;
    std::vector<int> tr_jk;
    std::vector<double> tr_fit;
    std::vector<float> tr_fit32;
    std::vector<unsigned> tr_off64, tr_off32;
    auto fit = [&](int j, int k, int c) {
        const int lo = std::min(j, k), hi = std::max(j, k);
        return hi < ns ? h.dif_full[((size_t)lo * ns + hi) * 4 + c] : 0.0;
    };
    for (int r = 0; r < tr_rounds; ++r) {
        std::vector<int> circ(n2);
        circ[0] = 0;
        for (int q = 1; q < n2; ++q) circ[q] = 1 + (q - 1 + r) % (n2 - 1);
        std::vector<std::pair<int, int>> pr;
        for (int q = 0; q < tr_slots; ++q) pr.emplace_back(circ[q], circ[n2 - 1 - q]);
        const auto oa = order_round_pairs(pr, wa);
        const auto ob = wb == wa ? oa : order_round_pairs(pr, wb);
        for (const auto &jk : oa) {
            const int j = jk.first, k = jk.second;
            tr_jk.push_back(j | k << 16);
            const unsigned rs = 8u * tt_rs(wa);
            tr_off64.push_back(rs * j | (rs * k) << 16);
            for (int c = 0; c < 4; ++c) tr_fit.push_back(fit(j, k, c));
        }
        for (const auto &jk : ob) {
            const int j = jk.first, k = jk.second;
            const unsigned rs = 8u * tt_rs(wb);
            tr_off32.push_back(rs * j | (rs * k) << 16);
            for (int c = 0; c < 4; ++c) tr_fit32.push_back((float)fit(j, k, c));
        }
    }
    // the lane-per-reaction kernels take 64 reactions at a time, and a wavefront pays for a
    // branch once if any of its lanes takes it: falloff reactions first, then third-body
    // ones, so that the longest branches run in as few groups of 64 as possible
    std::vector<int> rxn_order;
    for (int kind : {RXN_TROE, RXN_THREEBODY, RXN_ELEMENTARY})
        for (int rate : {(int)VAR_CHEB, (int)VAR_PLOG, 0})      // then the tabulated rate forms together
            for (int i = 0; i < nr; ++i)
                if (info_kind(h.info[i]) == kind && (h.var[i].flags & VAR_RATE_MASK) == rate) rxn_order.push_back(i);
    std::vector<double> vtab = h.vtab;
    if (vtab.empty()) vtab.push_back(0.0);
    Packer P;
    size_t oW = P.add(h.W), oInvW = P.add(invW), oNasa = P.add(h.nasa), oMu = P.add(h.mu_fit),
           oLam = P.add(h.lam_fit), oW4 = P.add(w4), oIw4 = P.add(iw4), oWc = P.add(wc),
           oLnA = P.add(h.lnA), oB = P.add(h.b), oTh = P.add(h.theta), oInfo = P.add(h.info),
           oDs = P.add(h.dnu_sum), oRi = P.add(h.ri), oTroe = P.add(h.troe), oEs = P.add(h.eff_sp),
           oEm = P.add(h.eff_m1), oJt = P.add(h.jp_thr), oJr = P.add(h.jp_recs), oJp = P.add(h.jp_prog), oJm = P.add(h.jp_mrx),
           oTj = P.add(tr_jk), oTo = P.add(cat(tr_off64, tr_off32)), oTf = P.add(tr_fit), oTf32 = P.add(tr_fit32), oRo = P.add(rxn_order), oVar = P.add(h.var),
           oVt = P.add(vtab);
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
    m.R = h.R; m.p0 = h.p0;
    m.W = (const double *)at(oW); m.invW = (const double *)at(oInvW); m.nasa = (const double *)at(oNasa);
    m.mu_fit = (const double *)at(oMu); m.lam_fit = (const double *)at(oLam); m.w4 = (const double *)at(oW4);
    m.iw4 = (const double *)at(oIw4); m.wilke_c = (const double *)at(oWc);
    m.tr_jk = (const int *)at(oTj); m.tr_off = (const unsigned *)at(oTo); m.tr_fit = (const double *)at(oTf); m.tr_fit32 = (const float *)at(oTf32);
    m.tr_rounds = tr_rounds; m.tr_slots = tr_slots;
    m.lnA = (const double *)at(oLnA); m.b = (const double *)at(oB);
    m.theta = (const double *)at(oTh); m.info = (const int *)at(oInfo); m.rxn_order = (const int *)at(oRo); m.dnu_sum = (const int *)at(oDs);
    m.ri = (const RxnInts *)at(oRi); m.troe = (const double *)at(oTroe); m.eff_sp = (const int *)at(oEs);
    m.eff_m1 = (const double *)at(oEm);
    m.var = (const RxnVar *)at(oVar); m.vtab = (const double *)at(oVt); m.n_var = h.n_var;
    m.jp_thr = (const int *)at(oJt); m.jp_recs = (const unsigned *)at(oJr); m.jp_prog = (const int *)at(oJp);
    m.jp_mrx = (const int *)at(oJm); m.jp_nm = h.jp_nm; m.jp_off_mx = h.jp_off_mx; m.jp_off_mq = h.jp_off_mq;
    m.jp_qb = h.jp_qb;
    m.jp_ok = h.jp_ok; m.jp_nd = h.jp_nd; m.jp_sr = h.jp_sr; m.jp_lds = h.jp_lds; m.jp_rmax = h.jp_rmax;
    m.jp_off_a = h.jp_off_a; m.jp_off_sp = h.jp_off_sp;
    m.jp_off_row = h.jp_off_row; m.jp_off_p = h.jp_off_p; m.jp_off_sc = h.jp_off_sc;
    m.jp_off_tp = h.jp_off_tp; m.jp_off_ex = h.jp_off_ex; m.jp_off_tq = h.jp_off_tq;
    m.jp_off_ns = h.jp_off_ns; m.jp_off_iw = h.jp_off_iw;
    mm->dev_buf = d;
    mm->device = device;
    return CRF_OK;
}

}  // namespace crf

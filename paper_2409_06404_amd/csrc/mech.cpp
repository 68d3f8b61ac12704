// Mechanism loader: parse the "crf-mech 1" text, validate it, derive the
// device tables and upload them in one allocation.
//
// The paper's solver takes its chemistry as a mechanism "in Cantera format"
// and turns it into platform code (Section 2); here the mechanism becomes a set
// of plain tables that table-driven kernels read.

#include <algorithm>
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

// ---------------------------------------------------------------------------- Jacobian schedule
// The register-schedule Jacobian kernel first stores, per point, every reaction's
// derivative data in LDS ("reaction data", RD):
//   RD[dofs[i] + r]   dq_i/dC of the r-th used slot of reaction i (mass-action part)
//   RD[rd_exc + x]    dq_i/d[M] (eps_x - 1) for efficiency exception x of reaction i
//   RD[rd_t + i]      dq_i/dT at fixed concentrations
//   RD[rd_q + i]      q_i
//   RD[rd_mf + i]     dq_i/d[M]
//   RD[rd_sig + i]    sum_j C_j dq_i/dC_j
// and then assembles the accumulator matrix A[(1 + k) * sr + c] (species rows) as
// plain sums over these values:
//   c < Ns   : sum_i dnu_ki (dq_i/dC_c mass-action + exception terms)
//   c = Ns   : sum_i dnu_ki dq_i/dT        c = Ns + 1 : sum_i dnu_ki q_i (= w_k)
//   c = Ns+2 : sum_i dnu_ki dq_i/d[M]     (the efficiency-1 part of every column)
//   c = Ns+3 : sum_i dnu_ki sum_j C_j dq_i/dC_j  (= sum_j J_C[k][j] C_j)
// Every entry is computed by exactly one thread (no atomics): contributions are
// grouped by target entry and the entries are dealt to `threads` threads, longest
// first, onto the least-loaded thread; each thread's stream is padded to the common
// length with no-op records.  A record is one 32-bit word, kept in registers:
//   bits 0-12 src, bits 13-15 coef + 4 (coef = dnu_ki in -3..3), bit 16 closes an
//   entry, bits 17-31 target.
// When the mechanism does not fit these fields or the length limit, js_len = 0 and
// the Jacobian falls back to the row-block kernel.
void build_jac_schedule(HostMech &h, int threads) {
    const int ns = h.ns(), nr = h.nr();
    h.dofs.assign(nr, 0);
    int nd = 0;
    for (int i = 0; i < nr; ++i) {
        h.dofs[i] = nd;
        nd += info_nreac(h.info[i]) + info_nprod(h.info[i]);
    }
    h.rd_exc = nd;
    h.rd_t = nd + (int)h.eff_sp.size();
    h.rd_q = h.rd_t + nr;
    h.rd_mf = h.rd_q + nr;
    h.rd_sig = h.rd_mf + nr;
    h.rd_size = h.rd_sig + nr;
    h.js_sr = (ns + 4) | 1;
    h.js_len = 0;
    h.jsched.clear();
    if (h.rd_size > (1 << 13) || (ns + 1) * h.js_sr > (1 << 15) || ns > JAC_MAX_SPECIES ||
        nr > JAC_RXN_PER_THREAD * threads)
        return;
    std::map<int, std::vector<std::pair<int, int>>> by_target;   // target -> (src, coef)
    for (int i = 0; i < nr; ++i) {
        const int info = h.info[i];
        const int nre = info_nreac(info), npr = info_nprod(info);
        const RxnInts &r = h.ri[i];
        int used[SLOTS], nused = 0;
        for (int s = 0; s < SLOTS; ++s)
            if (s < MAX_SIDE ? s < nre : (s - MAX_SIDE) < npr) used[nused++] = s;
        for (int ua = 0; ua < nused; ++ua) {
            const int a = used[ua];
            const int k = r.v[a];
            const int dn = (a < MAX_SIDE ? -1 : 1) * info_nu(info, a);
            const int row = (1 + k) * h.js_sr;
            by_target[row + ns].push_back({h.rd_t + i, dn});
            by_target[row + ns + 1].push_back({h.rd_q + i, dn});
            if (info_kind(info) != RXN_ELEMENTARY) by_target[row + ns + 2].push_back({h.rd_mf + i, dn});
            by_target[row + ns + 3].push_back({h.rd_sig + i, dn});
            for (int ub = 0; ub < nused; ++ub) by_target[row + r.v[used[ub]]].push_back({h.dofs[i] + ub, dn});
            const int n_exc = r.v[7] & 255;
            for (int e = 0; e < n_exc; ++e)
                by_target[row + h.eff_sp[r.v[6] + e]].push_back({h.rd_exc + r.v[6] + e, dn});
        }
    }
    // longest-processing-time assignment of entries to threads
    std::vector<std::pair<int, int>> order;   // (count, target)
    for (auto &kv : by_target) order.push_back({(int)kv.second.size(), kv.first});
    std::sort(order.begin(), order.end(),
              [](auto &x, auto &y) { return x.first > y.first || (x.first == y.first && x.second < y.second); });
    std::vector<std::vector<unsigned>> stream(threads);
    std::vector<int> load(threads, 0);
    for (auto &ct : order) {
        int t = 0;
        for (int u = 1; u < threads; ++u)
            if (load[u] < load[t]) t = u;
        const auto &lst = by_target[ct.second];
        for (size_t c = 0; c < lst.size(); ++c) {
            const bool last = c + 1 == lst.size();
            stream[t].push_back((unsigned)lst[c].first | ((unsigned)(lst[c].second + 4) << 13) |
                                (last ? (1u << 16) | ((unsigned)ct.second << 17) : 0u));
        }
        load[t] += (int)lst.size();
    }
    int len = 0;
    for (int t = 0; t < threads; ++t) len = std::max(len, load[t]);
    if (len > JAC_SCHED_MAX) return;
    h.js_len = len;
    h.jsched.assign((size_t)len * threads, 4u << 13);      // padding: src 0, coef 0
    for (int t = 0; t < threads; ++t)
        for (int it = 0; it < load[t]; ++it) h.jsched[(size_t)it * threads + t] = stream[t][it];
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
    build_jac_schedule(mm->host, JAC_THREADS);
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
           oEm = P.add(h.eff_m1), oDofs = P.add(h.dofs), oJs = P.add(h.jsched);
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
    m.dofs = (const int *)at(oDofs); m.jsched = (const unsigned *)at(oJs);
    m.js_len = h.js_len; m.js_threads = JAC_THREADS; m.rd_size = h.rd_size; m.rd_exc = h.rd_exc;
    m.rd_t = h.rd_t; m.rd_q = h.rd_q; m.rd_mf = h.rd_mf; m.rd_sig = h.rd_sig; m.js_sr = h.js_sr;
    mm->dev_buf = d;
    mm->device = device;
    return CRF_OK;
}

}  // namespace crf

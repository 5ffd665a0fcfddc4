// C-ABI of libpccp: model building and validation, compilation of the model
// to packed per-kind propagator tables (§2: constraints to propagators; §3:
// names erased to store indices), device upload, launch configuration and
// result read-back.  The device work itself is in pccp_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cctype>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/pccp.h"
#include "pccp_launch.h"
#include "pccp_types.h"

using namespace pccp;

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;

static int32_t fail(int32_t code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

#define HIPCHK(call)                                                                    \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(PCCP_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

int32_t pccp::internal_fail(int32_t code, const std::string &msg) { return fail(code, msg); }

extern "C" const char *pccp_last_error(void) { return g_last_error.c_str(); }
extern "C" const char *pccp_version(void) { return "pccp 0.1 (gfx950)"; }

// ------------------------------------------------------------------ model
struct pccp_model {
    std::vector<int32_t> lb, ub;
    std::vector<int32_t> row_ptr{0}, coef, var, rhs;
    std::vector<int32_t> reif;  // 4 per item: b, si, sj, d
    std::vector<int32_t> dec;
    int32_t objective = -1;
    // guarded commands: 4 per command (x, side, k, div); guards (y, side, c)
    // and terms (a, y) by CSR pointers
    std::vector<int32_t> cmd, cmd_gptr{0}, guard, cmd_tptr{0}, cterm;
};

extern "C" int32_t pccp_model_create(pccp_model **out)
{
    if (!out) return fail(PCCP_E_INVALID_ARG, "pccp_model_create: out is NULL");
    *out = new (std::nothrow) pccp_model();
    return *out ? PCCP_OK : fail(PCCP_E_NOMEM, "pccp_model_create: out of memory");
}

extern "C" int32_t pccp_model_destroy(pccp_model *m)
{
    delete m;
    return PCCP_OK;
}

extern "C" int32_t pccp_model_add_vars(pccp_model *m, int32_t n, const int32_t *lb,
                                       const int32_t *ub, int32_t *first_id)
{
    if (!m || n < 0 || (n > 0 && (!lb || !ub)))
        return fail(PCCP_E_INVALID_ARG, "pccp_model_add_vars: bad arguments");
    if ((int64_t)m->lb.size() + n > kMaxVars)
        return fail(PCCP_E_UNSUPPORTED, "pccp_model_add_vars: more than 65535 variables");
    if (first_id) *first_id = (int32_t)m->lb.size();
    m->lb.insert(m->lb.end(), lb, lb + n);
    m->ub.insert(m->ub.end(), ub, ub + n);
    return PCCP_OK;
}

extern "C" int32_t pccp_model_add_linear_le(pccp_model *m, int32_t nterms, const int32_t *coef,
                                            const int32_t *var, int32_t rhs)
{
    if (!m || nterms < 1 || !coef || !var)
        return fail(PCCP_E_INVALID_ARG, "pccp_model_add_linear_le: bad arguments");
    m->coef.insert(m->coef.end(), coef, coef + nterms);
    m->var.insert(m->var.end(), var, var + nterms);
    m->rhs.push_back(rhs);
    m->row_ptr.push_back((int32_t)m->coef.size());
    return PCCP_OK;
}

extern "C" int32_t pccp_model_add_reified_overlap(pccp_model *m, int32_t b, int32_t si,
                                                  int32_t sj, int32_t d)
{
    if (!m) return fail(PCCP_E_INVALID_ARG, "pccp_model_add_reified_overlap: model is NULL");
    m->reif.insert(m->reif.end(), {b, si, sj, d});
    return PCCP_OK;
}

extern "C" int32_t pccp_model_add_guarded(pccp_model *m, int32_t x, int32_t side, int32_t k,
                                          int32_t div, int32_t nguards, const int32_t *gvar,
                                          const int32_t *gside, const int32_t *gc, int32_t nterms,
                                          const int32_t *coef, const int32_t *var)
{
    if (!m || nguards < 0 || nterms < 0 || (nguards > 0 && (!gvar || !gside || !gc)) ||
        (nterms > 0 && (!coef || !var)))
        return fail(PCCP_E_INVALID_ARG, "pccp_model_add_guarded: bad arguments");
    m->cmd.insert(m->cmd.end(), {x, side, k, div});
    for (int32_t g = 0; g < nguards; ++g) m->guard.insert(m->guard.end(), {gvar[g], gside[g], gc[g]});
    m->cmd_gptr.push_back((int32_t)(m->guard.size() / 3));
    for (int32_t t = 0; t < nterms; ++t) m->cterm.insert(m->cterm.end(), {coef[t], var[t]});
    m->cmd_tptr.push_back((int32_t)(m->cterm.size() / 2));
    return PCCP_OK;
}

extern "C" int32_t pccp_model_set_decision_vars(pccp_model *m, int32_t n, const int32_t *vars)
{
    if (!m || n < 0 || (n > 0 && !vars))
        return fail(PCCP_E_INVALID_ARG, "pccp_model_set_decision_vars: bad arguments");
    m->dec.assign(vars, vars + n);
    return PCCP_OK;
}

extern "C" int32_t pccp_model_set_objective(pccp_model *m, int32_t v)
{
    if (!m || v < -1) return fail(PCCP_E_INVALID_ARG, "pccp_model_set_objective: bad arguments");
    m->objective = v;
    return PCCP_OK;
}

extern "C" int32_t pccp_model_info(const pccp_model *m, int32_t *nvars, int32_t *nlinear,
                                   int32_t *nterms, int32_t *nreified, int32_t *ndecision)
{
    if (!m) return fail(PCCP_E_INVALID_ARG, "pccp_model_info: model is NULL");
    if (nvars) *nvars = (int32_t)m->lb.size();
    if (nlinear) *nlinear = (int32_t)m->rhs.size();
    if (nterms) *nterms = (int32_t)m->coef.size();
    if (nreified) *nreified = (int32_t)(m->reif.size() / 4);
    if (ndecision) *ndecision = (int32_t)m->dec.size();
    return PCCP_OK;
}

// ------------------------------------------------------------------ model files
// Format (little-endian): the line "PCCP-MODEL 1", one line of JSON with
// the top-level integer fields nvars, nrows, nterms, nreif, ndec and
// objective, and optionally ncmd, nguards, ncterms (absent = 0; other
// fields, e.g. a generator's parameters, are ignored), then the int32
// arrays lb[nvars], ub[nvars], row_ptr[nrows + 1], coef[nterms],
// var[nterms], rhs[nrows], reif[4 nreif] (b, si, sj, d), dec[ndec], and
// when ncmd > 0: cmd[4 ncmd] (x, side, k, div), cmd_gptr[ncmd + 1],
// guard[3 nguards] (y, side, c), cmd_tptr[ncmd + 1], cterm[2 ncterms]
// (a, y).
static const char kModelMagic[] = "PCCP-MODEL 1\n";

// value of the top-level integer field `key` of a one-line JSON object
static bool json_top_int(const std::string &h, const char *key, int64_t &out)
{
    int depth = 0;
    bool in_str = false;
    size_t kstart = 0;
    for (size_t i = 0; i < h.size(); ++i) {
        const char ch = h[i];
        if (in_str) {
            if (ch == '\\') { ++i; continue; }
            if (ch != '"') continue;
            in_str = false;
            if (depth != 1 || h.compare(kstart, i - kstart, key) != 0 || strlen(key) != i - kstart)
                continue;
            size_t j = i + 1;
            while (j < h.size() && isspace((unsigned char)h[j])) ++j;
            if (j >= h.size() || h[j] != ':') continue;
            ++j;
            while (j < h.size() && isspace((unsigned char)h[j])) ++j;
            char *end = nullptr;
            const long long v = strtoll(h.c_str() + j, &end, 10);
            if (end == h.c_str() + j) return false;
            out = v;
            return true;
        }
        if (ch == '"') { in_str = true; kstart = i + 1; }
        else if (ch == '{' || ch == '[') ++depth;
        else if (ch == '}' || ch == ']') --depth;
    }
    return false;
}

extern "C" int32_t pccp_model_save_file(const pccp_model *m, const char *path)
{
    if (!m || !path) return fail(PCCP_E_INVALID_ARG, "pccp_model_save_file: bad arguments");
    FILE *f = fopen(path, "wb");
    if (!f) return fail(PCCP_E_INVALID_ARG, std::string("pccp_model_save_file: cannot open ") + path);
    char hdr[320];
    const size_t ncmd = m->cmd.size() / 4;
    snprintf(hdr, sizeof(hdr),
             "{\"nvars\": %zu, \"nrows\": %zu, \"nterms\": %zu, \"nreif\": %zu, \"ndec\": %zu, "
             "\"objective\": %d, \"ncmd\": %zu, \"nguards\": %zu, \"ncterms\": %zu}\n",
             m->lb.size(), m->rhs.size(), m->coef.size(), m->reif.size() / 4, m->dec.size(),
             (int)m->objective, ncmd, m->guard.size() / 3, m->cterm.size() / 2);
    bool ok = fputs(kModelMagic, f) >= 0 && fputs(hdr, f) >= 0;
    auto put = [&](const std::vector<int32_t> &v) {
        if (ok && !v.empty()) ok = fwrite(v.data(), 4, v.size(), f) == v.size();
    };
    put(m->lb); put(m->ub); put(m->row_ptr); put(m->coef); put(m->var); put(m->rhs);
    put(m->reif); put(m->dec);
    if (ncmd > 0) {
        put(m->cmd); put(m->cmd_gptr); put(m->guard); put(m->cmd_tptr); put(m->cterm);
    }
    ok = (fclose(f) == 0) && ok;
    return ok ? PCCP_OK : fail(PCCP_E_INVALID_ARG, std::string("pccp_model_save_file: write failed: ") + path);
}

extern "C" int32_t pccp_model_load_file(const char *path, pccp_model **out)
{
    if (!path || !out) return fail(PCCP_E_INVALID_ARG, "pccp_model_load_file: bad arguments");
    *out = nullptr;
    FILE *f = fopen(path, "rb");
    if (!f) return fail(PCCP_E_INVALID_ARG, std::string("pccp_model_load_file: cannot open ") + path);
    auto line = [&](std::string &l) {
        l.clear();
        int ch;
        while ((ch = fgetc(f)) != EOF && ch != '\n') {
            l.push_back((char)ch);
            if (l.size() > (1u << 26)) return false;
        }
        return ch == '\n';
    };
    std::string magic, hdr;
    int64_t V = -1, R = -1, T = -1, Q = -1, D = -1, obj = -2, NC = 0, NG = 0, NT = 0;
    // an optional field: absent is 0, present must be an integer
    auto opt_int = [&](const char *key, int64_t &out) {
        if (hdr.find(std::string("\"") + key + "\"") == std::string::npos) { out = 0; return true; }
        return json_top_int(hdr, key, out);
    };
    if (!line(magic) || magic + "\n" != kModelMagic || !line(hdr) ||
        !json_top_int(hdr, "nvars", V) || !json_top_int(hdr, "nrows", R) ||
        !json_top_int(hdr, "nterms", T) || !json_top_int(hdr, "nreif", Q) ||
        !json_top_int(hdr, "ndec", D) || !json_top_int(hdr, "objective", obj) || V < 0 ||
        V > kMaxVars || R < 0 || T < 0 || Q < 0 || D < 0 || obj < -1 || obj >= V ||
        R > INT32_MAX - 1 || T > INT32_MAX || Q > INT32_MAX / 4 ||
        !opt_int("ncmd", NC) || !opt_int("nguards", NG) || !opt_int("ncterms", NT) ||
        NC < 0 || NG < 0 || NT < 0 || NC > INT32_MAX / 4 - 1 || NG > INT32_MAX / 3 ||
        NT > INT32_MAX / 2 || (NC == 0 && (NG > 0 || NT > 0))) {
        fclose(f);
        return fail(PCCP_E_MODEL, std::string("pccp_model_load_file: bad header in ") + path);
    }
    pccp_model *m = new (std::nothrow) pccp_model();
    if (!m) { fclose(f); return fail(PCCP_E_NOMEM, "pccp_model_load_file: out of memory"); }
    bool ok = true;
    auto get = [&](std::vector<int32_t> &v, int64_t n) {
        if (!ok) return;
        try { v.assign((size_t)n, 0); } catch (...) { ok = false; return; }
        if (n > 0) ok = fread(v.data(), 4, (size_t)n, f) == (size_t)n;
    };
    get(m->lb, V); get(m->ub, V); get(m->row_ptr, R + 1); get(m->coef, T); get(m->var, T);
    get(m->rhs, R); get(m->reif, 4 * Q); get(m->dec, D);
    if (NC > 0) {
        get(m->cmd, 4 * NC); get(m->cmd_gptr, NC + 1); get(m->guard, 3 * NG);
        get(m->cmd_tptr, NC + 1); get(m->cterm, 2 * NT);
    }
    const bool at_end = ok && fgetc(f) == EOF;
    fclose(f);
    if (ok && at_end) {
        // the row pointer must run from 0 to nterms without decreasing, with
        // at least one term per row (as pccp_model_add_linear_le builds it)
        ok = m->row_ptr[0] == 0 && m->row_ptr[R] == T;
        for (int64_t r = 0; ok && r < R; ++r) ok = m->row_ptr[r + 1] > m->row_ptr[r];
        // the command pointers run from 0 to their counts without decreasing
        if (ok && NC > 0) {
            ok = m->cmd_gptr[0] == 0 && m->cmd_gptr[NC] == NG && m->cmd_tptr[0] == 0 &&
                 m->cmd_tptr[NC] == NT;
            for (int64_t q = 0; ok && q < NC; ++q)
                ok = m->cmd_gptr[q + 1] >= m->cmd_gptr[q] && m->cmd_tptr[q + 1] >= m->cmd_tptr[q];
        }
    }
    if (!ok || !at_end) {
        delete m;
        return fail(PCCP_E_MODEL, std::string("pccp_model_load_file: truncated or inconsistent arrays in ") + path);
    }
    m->objective = (int32_t)obj;
    *out = m;
    return PCCP_OK;
}

// ------------------------------------------------------------------ compiled model
// Packed tables (see pccp_types.h): difference rows, reified items, other
// rows with their terms, decision variables.
struct Compiled {
    int32_t nvars = 0, ndec = 0, objective = -1;
    int32_t nI = 0;                   // variables stored as pairs; the rest are Booleans
    std::vector<int32_t> lb0, ub0, dec;   // in store numbering
    std::vector<int32_t> vorig, vnew;     // store index <-> the model's index
    std::vector<int32_t> lb0_model, ub0_model;  // the initial box in the model's numbering
    std::vector<int2> diff, reif;
    std::vector<int4> rows;
    std::vector<uint32_t> terms;
    // Boolean knapsack rows: {rhs, len} and terms at a fixed stride of
    // bgroup * bchunks slots per row (unused slots 0)
    std::vector<int2> brows;
    std::vector<uint32_t> bterms;
    int32_t bgroup = 4, bchunks = 1, nbterms = 0;
    // guarded commands (see pccp_types.h, kind 5)
    std::vector<int4> cmds;
    std::vector<uint32_t> ccnt;
    std::vector<int2> cent;
    // learned-branching tables (see pccp_types.h)
    std::vector<float> fstat;
    std::vector<int32_t> fr_ptr, fb_ptr, fb;
    std::vector<int2> fr;
    // propagators reading each variable (see DevModel::adj)
    std::vector<int32_t> adj_ptr;
    std::vector<uint32_t> adj;
};

// Which propagators read which bound of which variable: a propagator has to
// run again only after a bound it reads was tightened.  Difference row
// x - y <= c reads lb(x) and ub(y); a reified item reads both bounds of b,
// si and sj; a linear row reads lb of its positive terms and ub of its
// negative ones (the tell on a term does not depend on that term's own
// bound); a Boolean row reads lb of its terms.  Entries of one variable are
// grouped by kind.
static void compile_adjacency(Compiled &c)
{
    const int32_t V = c.nvars;
    std::vector<std::vector<uint32_t>> a(V);
    auto add = [&](int32_t x, uint32_t idx, uint32_t kind, uint32_t reads) {
        a[x].push_back(idx | (kind << 16) | reads);
    };
    for (size_t i = 0; i < c.diff.size(); ++i) {
        const uint32_t w = (uint32_t)c.diff[i].x;
        add((int32_t)(w & 0xffff), (uint32_t)i, 0, kAdjLb);
        add((int32_t)(w >> 16), (uint32_t)i, 0, kAdjUb);
    }
    for (size_t i = 0; i < c.reif.size(); ++i) {
        const uint32_t w0 = (uint32_t)c.reif[i].x, w1 = (uint32_t)c.reif[i].y;
        add((int32_t)(w0 & 0xffff), (uint32_t)i, 1, kAdjLb | kAdjUb);
        if ((w0 >> 16) != (w0 & 0xffff)) add((int32_t)(w0 >> 16), (uint32_t)i, 1, kAdjLb | kAdjUb);
        if ((w1 & 0xffff) != (w0 >> 16) && (w1 & 0xffff) != (w0 & 0xffff))
            add((int32_t)(w1 & 0xffff), (uint32_t)i, 1, kAdjLb | kAdjUb);
    }
    for (size_t i = 0; i < c.rows.size(); ++i)
        for (int32_t t = c.rows[i].x; t < c.rows[i].x + c.rows[i].y; ++t) {
            const int32_t coef = (int32_t)c.terms[t] >> 16;
            add((int32_t)(c.terms[t] & 0xffff), (uint32_t)i, 2, coef > 0 ? kAdjLb : kAdjUb);
        }
    const size_t SL = (size_t)c.bgroup * c.bchunks;
    for (size_t i = 0; i < c.brows.size(); ++i)
        for (int32_t t = 0; t < c.brows[i].y; ++t)
            add((int32_t)(c.bterms[SL * i + t] & 0xffff), (uint32_t)i, 3, kAdjLb);
    // a guarded command reads the bound each guard tests and the bound each
    // term of f is read through (a variable read twice is listed twice)
    for (size_t q = 0; q < c.cmds.size(); ++q) {
        const int ng = (int)(c.ccnt[q] & 0xffffu), nt = (int)(c.ccnt[q] >> 16), e0 = c.cmds[q].w;
        for (int u = 0; u < ng + nt; ++u) {
            const uint32_t w = (uint32_t)c.cent[e0 + u].x;
            add((int32_t)(w & 0xffff), (uint32_t)q, 4, ((w >> 16) & 1u) ? kAdjUb : kAdjLb);
        }
    }
    c.adj_ptr.assign(V + 1, 0);
    c.adj.clear();
    for (int32_t x = 0; x < V; ++x) {
        c.adj.insert(c.adj.end(), a[x].begin(), a[x].end());
        c.adj_ptr[x + 1] = (int32_t)c.adj.size();
    }
}

// Static part of the branching features of every decision variable q
// (x = dec[q], H = max(1, ub0 - lb0)): 1/H, the share of the largest
// variable degree (rows + reified items containing the variable), the
// static load (mean over the reified items with si = x of d * w(b) / H,
// w(b) = sum of a / c over rows a*b + ... <= c with a > 0, c > 0), 1/N;
// and the tables the dynamic features read: rows x - y <= c leaving x,
// and the b of the items with si = x.
static void compile_features(const pccp_model *m, Compiled &c)
{
    const int32_t V = c.nvars, D = c.ndec;
    std::vector<double> deg(V, 0.0), w(V, 0.0);
    const int32_t R = (int32_t)m->rhs.size();
    for (int32_t r = 0; r < R; ++r)
        for (int32_t t = m->row_ptr[r]; t < m->row_ptr[r + 1]; ++t) {
            deg[m->var[t]] += 1.0;
            if (m->coef[t] > 0 && m->rhs[r] > 0) w[m->var[t]] += (double)m->coef[t] / m->rhs[r];
        }
    const size_t Q = m->reif.size() / 4;
    for (size_t q = 0; q < Q; ++q)
        for (int k = 0; k < 3; ++k) deg[m->reif[4 * q + k]] += 1.0;
    double maxdeg = 1.0;
    for (double d : deg) maxdeg = std::max(maxdeg, d);
    // rows x - y <= c by their +1 variable, items by si
    std::vector<std::vector<int2>> out_rows(V);
    for (int32_t r = 0; r < R; ++r) {
        const int32_t a0 = m->row_ptr[r];
        if (m->row_ptr[r + 1] - a0 != 2) continue;
        if (m->coef[a0] == 1 && m->coef[a0 + 1] == -1)
            out_rows[m->var[a0]].push_back(make_int2(m->var[a0 + 1], m->rhs[r]));
        else if (m->coef[a0] == -1 && m->coef[a0 + 1] == 1)
            out_rows[m->var[a0 + 1]].push_back(make_int2(m->var[a0], m->rhs[r]));
    }
    std::vector<std::vector<int32_t>> items_b(V);
    std::vector<double> load(V, 0.0);
    for (size_t q = 0; q < Q; ++q) {
        const int32_t *it = &m->reif[4 * q];
        items_b[it[1]].push_back(it[0]);
        load[it[1]] += (double)it[3] * w[it[0]];
    }
    c.fstat.assign(8 * (size_t)D, 0.f);
    c.fr_ptr.assign(D + 1, 0);
    c.fb_ptr.assign(D + 1, 0);
    for (int32_t q = 0; q < D; ++q) {
        const int32_t x = c.dec[q];
        const double H = std::max(1.0, (double)c.ub0[x] - (double)c.lb0[x]);
        const double N = std::max<double>(1.0, (double)items_b[x].size());
        float lo_bits;
        const int32_t lo = c.lb0[x];
        memcpy(&lo_bits, &lo, 4);
        c.fstat[8 * q + 0] = lo_bits;
        c.fstat[8 * q + 1] = (float)(1.0 / H);
        c.fstat[8 * q + 2] = (float)(deg[x] / maxdeg);
        c.fstat[8 * q + 3] = (float)(load[x] / N / H);
        c.fstat[8 * q + 4] = (float)(1.0 / N);
        c.fr.insert(c.fr.end(), out_rows[x].begin(), out_rows[x].end());
        c.fb.insert(c.fb.end(), items_b[x].begin(), items_b[x].end());
        c.fr_ptr[q + 1] = (int32_t)c.fr.size();
        c.fb_ptr[q + 1] = (int32_t)c.fb.size();
    }
}

// The store keeps the variables whose initial domain is not inside [0, 1]
// as int32 pairs and the others (Booleans) as one byte each, pairs first:
// a copy of the model renumbered in that order (each group in the model's
// order).  An index out of range is kept out of range, so that the checks
// below still refuse it.
static void renumber(const pccp_model *m, pccp_model &r, Compiled &c)
{
    const int32_t V = (int32_t)m->lb.size();
    c.vorig.clear();
    for (int pass = 0; pass < 2; ++pass)
        for (int32_t x = 0; x < V; ++x) {
            const bool isb = m->lb[x] >= 0 && m->ub[x] <= 1;
            if (isb == (pass == 1)) c.vorig.push_back(x);
        }
    c.nI = 0;
    for (int32_t x = 0; x < V; ++x) c.nI += !(m->lb[x] >= 0 && m->ub[x] <= 1);
    c.vnew.assign(V, 0);
    for (int32_t i = 0; i < V; ++i) c.vnew[c.vorig[i]] = i;
    auto map = [&](int32_t x) { return x >= 0 && x < V ? c.vnew[x] : x; };
    r = *m;
    c.lb0_model = m->lb;
    c.ub0_model = m->ub;
    for (int32_t i = 0; i < V; ++i) {
        r.lb[i] = m->lb[c.vorig[i]];
        r.ub[i] = m->ub[c.vorig[i]];
    }
    for (int32_t &x : r.var) x = map(x);
    for (size_t q = 0; q < r.reif.size() / 4; ++q)
        for (int k = 0; k < 3; ++k) r.reif[4 * q + k] = map(r.reif[4 * q + k]);
    for (int32_t &x : r.dec) x = map(x);
    r.objective = map(r.objective);
    for (size_t q = 0; q < r.cmd.size() / 4; ++q) r.cmd[4 * q] = map(r.cmd[4 * q]);
    for (size_t g = 0; g < r.guard.size() / 3; ++g) r.guard[3 * g] = map(r.guard[3 * g]);
    for (size_t t = 0; t < r.cterm.size() / 2; ++t) r.cterm[2 * t + 1] = map(r.cterm[2 * t + 1]);
}

static int32_t compile_renumbered(const pccp_model *m, Compiled &c);

static int32_t compile_model(const pccp_model *m0, Compiled &c)
{
    if ((int64_t)m0->lb.size() > kMaxVars) return fail(PCCP_E_UNSUPPORTED, "more than 65535 variables");
    pccp_model r;
    renumber(m0, r, c);
    return compile_renumbered(&r, c);
}

static int32_t compile_renumbered(const pccp_model *m, Compiled &c)
{
    const int64_t LIM = (int64_t)1 << 30;
    const int32_t V = (int32_t)m->lb.size();
    if (V > kMaxVars) return fail(PCCP_E_UNSUPPORTED, "more than 65535 variables");
    c.nvars = V;
    c.lb0 = m->lb;
    c.ub0 = m->ub;
    int64_t maxabs = 0;
    std::vector<int64_t> mag(V);
    for (int32_t v = 0; v < V; ++v) {
        mag[v] = std::max(std::llabs((int64_t)m->lb[v]), std::llabs((int64_t)m->ub[v]));
        maxabs = std::max(maxabs, mag[v]);
    }
    if (maxabs >= LIM) return fail(PCCP_E_OVERFLOW, "a variable bound is beyond 2^30 in magnitude");
    if (m->objective < -1 || m->objective >= V)
        return fail(PCCP_E_MODEL, "objective variable out of range");
    c.objective = m->objective;
    {
        std::vector<char> isdec(V, 0);
        for (int32_t x : m->dec) {
            if (x < 0 || x >= V) return fail(PCCP_E_MODEL, "decision variable out of range");
            if (isdec[x]) return fail(PCCP_E_MODEL, "decision variable listed twice");
            isdec[x] = 1;
        }
    }
    c.dec = m->dec;
    c.ndec = (int32_t)m->dec.size();
    const int32_t R = (int32_t)m->rhs.size();
    std::vector<char> seen(V, 0);
    for (int32_t r = 0; r < R; ++r) {
        const int32_t a0 = m->row_ptr[r], a1 = m->row_ptr[r + 1];
        int64_t tot = std::llabs((int64_t)m->rhs[r]);
        for (int32_t t = a0; t < a1; ++t) {
            const int32_t x = m->var[t], a = m->coef[t];
            if (x < 0 || x >= V) return fail(PCCP_E_MODEL, "row " + std::to_string(r) + ": variable out of range");
            if (a == 0) return fail(PCCP_E_MODEL, "row " + std::to_string(r) + ": zero coefficient");
            if (seen[x]) return fail(PCCP_E_MODEL, "row " + std::to_string(r) + ": variable repeated");
            seen[x] = 1;
            tot += std::llabs((int64_t)a) * mag[x];
        }
        for (int32_t t = a0; t < a1; ++t) seen[m->var[t]] = 0;
        if (tot >= LIM) return fail(PCCP_E_OVERFLOW, "row " + std::to_string(r) + ": sum |a|*|bound| + |c| >= 2^30");
        const bool is_diff = (a1 - a0 == 2) &&
                             ((m->coef[a0] == 1 && m->coef[a0 + 1] == -1) ||
                              (m->coef[a0] == -1 && m->coef[a0 + 1] == 1));
        bool is_bool = !is_diff && a1 > a0;
        for (int32_t t = a0; t < a1 && is_bool; ++t)
            is_bool = m->coef[t] > 0 && m->lb[m->var[t]] >= 0 && m->ub[m->var[t]] <= 1;
        if (is_diff) {
            const int32_t x = m->coef[a0] == 1 ? m->var[a0] : m->var[a0 + 1];
            const int32_t y = m->coef[a0] == 1 ? m->var[a0 + 1] : m->var[a0];
            c.diff.push_back(make_int2((int32_t)((uint32_t)x | ((uint32_t)y << 16)), m->rhs[r]));
        } else if (is_bool) {
            // laid out below, once the longest row is known
            c.brows.push_back(make_int2(m->rhs[r], r));
        } else {
            c.rows.push_back(make_int4((int32_t)c.terms.size(), a1 - a0, m->rhs[r], 0));
            for (int32_t t = a0; t < a1; ++t) {
                const int32_t a = m->coef[t];
                if (a < -32768 || a > 32767)
                    return fail(PCCP_E_UNSUPPORTED, "row " + std::to_string(r) + ": coefficient outside int16");
                c.terms.push_back((uint32_t)m->var[t] | ((uint32_t)(uint16_t)(int16_t)a << 16));
            }
        }
    }
    // Boolean rows: the smallest group (4, 8, 16 lanes) that covers the
    // longest row in at most 4 terms per lane, else 16 lanes
    {
        int lmax = 1;
        for (const int2 &b : c.brows) {
            const int32_t r = b.y;
            lmax = std::max(lmax, m->row_ptr[r + 1] - m->row_ptr[r]);
        }
        c.bgroup = 16;
        for (int g : {4, 8, 16})
            if ((lmax + g - 1) / g <= 4) { c.bgroup = g; break; }
        c.bchunks = (lmax + c.bgroup - 1) / c.bgroup;
        const size_t SL = (size_t)c.bgroup * c.bchunks;
        c.bterms.assign(SL * c.brows.size(), 0u);
        c.nbterms = 0;
        for (size_t i = 0; i < c.brows.size(); ++i) {
            const int32_t r = c.brows[i].y, a0 = m->row_ptr[r], a1 = m->row_ptr[r + 1];
            for (int32_t t = a0; t < a1; ++t) {
                const int32_t a = m->coef[t];
                if (a > 32767)
                    return fail(PCCP_E_UNSUPPORTED, "row " + std::to_string(r) + ": coefficient outside int16");
                c.bterms[SL * i + (t - a0)] = (uint32_t)m->var[t] | ((uint32_t)a << 16);
            }
            c.brows[i].y = a1 - a0;
            c.nbterms += a1 - a0;
        }
    }
    const size_t Q = m->reif.size() / 4;
    for (size_t q = 0; q < Q; ++q) {
        const int32_t *it = &m->reif[4 * q];
        for (int k = 0; k < 3; ++k)
            if (it[k] < 0 || it[k] >= V)
                return fail(PCCP_E_MODEL, "reified item " + std::to_string(q) + ": variable out of range");
        if (it[3] < -32768 || it[3] > 32767)
            return fail(PCCP_E_UNSUPPORTED, "reified item " + std::to_string(q) + ": d outside int16");
        if (2 * maxabs + std::llabs((int64_t)it[3]) + 1 >= LIM)
            return fail(PCCP_E_OVERFLOW, "reified item " + std::to_string(q) + ": bounds + d beyond 2^30");
        c.reif.push_back(make_int2((int32_t)((uint32_t)it[0] | ((uint32_t)it[1] << 16)),
                                   (int32_t)((uint32_t)it[2] | ((uint32_t)(uint16_t)(int16_t)it[3] << 16))));
    }
    // guarded commands: the targets, guards and terms in range, div >= 1, and
    // |k| + sum |a| * |bound| < 2^30 so that f fits in int32
    const size_t NCMD = m->cmd.size() / 4;
    if (m->cmd_gptr.size() != NCMD + 1 || m->cmd_tptr.size() != NCMD + 1)
        return fail(PCCP_E_MODEL, "guarded commands: inconsistent pointers");
    for (size_t q = 0; q < NCMD; ++q) {
        const int32_t *cm = &m->cmd[4 * q];
        const std::string tag = "guarded command " + std::to_string(q);
        if (cm[0] < 0 || cm[0] >= V) return fail(PCCP_E_MODEL, tag + ": target out of range");
        if (cm[1] != 0 && cm[1] != 1) return fail(PCCP_E_MODEL, tag + ": side must be 0 or 1");
        if (cm[3] < 1) return fail(PCCP_E_MODEL, tag + ": div must be >= 1");
        const int32_t g0 = m->cmd_gptr[q], g1 = m->cmd_gptr[q + 1];
        const int32_t t0 = m->cmd_tptr[q], t1 = m->cmd_tptr[q + 1];
        if (g0 < 0 || g1 < g0 || (size_t)g1 * 3 > m->guard.size() || t0 < 0 || t1 < t0 ||
            (size_t)t1 * 2 > m->cterm.size())
            return fail(PCCP_E_MODEL, tag + ": inconsistent pointers");
        if (g1 - g0 > 65535 || t1 - t0 > 65535)
            return fail(PCCP_E_UNSUPPORTED, tag + ": more than 65535 guards or terms");
        int64_t tot = std::llabs((int64_t)cm[2]);
        c.cmds.push_back(make_int4((int32_t)((uint32_t)cm[0] | ((uint32_t)cm[1] << 16)), cm[2], cm[3],
                                   (int32_t)c.cent.size()));
        c.ccnt.push_back((uint32_t)(g1 - g0) | ((uint32_t)(t1 - t0) << 16));
        for (int32_t g = g0; g < g1; ++g) {
            const int32_t *gd = &m->guard[3 * (size_t)g];
            if (gd[0] < 0 || gd[0] >= V) return fail(PCCP_E_MODEL, tag + ": guard variable out of range");
            if (gd[1] != 0 && gd[1] != 1) return fail(PCCP_E_MODEL, tag + ": guard side must be 0 or 1");
            c.cent.push_back(make_int2((int32_t)((uint32_t)gd[0] | ((uint32_t)gd[1] << 16)), gd[2]));
        }
        for (int32_t t = t0; t < t1; ++t) {
            const int32_t a = m->cterm[2 * (size_t)t], y = m->cterm[2 * (size_t)t + 1];
            if (y < 0 || y >= V) return fail(PCCP_E_MODEL, tag + ": term variable out of range");
            if (a == 0) return fail(PCCP_E_MODEL, tag + ": zero coefficient");
            tot += std::llabs((int64_t)a) * mag[y];
            if (tot >= LIM) return fail(PCCP_E_OVERFLOW, tag + ": |k| + sum |a|*|bound| >= 2^30");
            // the bound that keeps f monotone: lb for a > 0 in a lower-bound
            // tell, ub for a < 0; the opposite in an upper-bound tell
            const bool reads_ub = cm[1] == 0 ? a < 0 : a > 0;
            c.cent.push_back(make_int2((int32_t)((uint32_t)y | ((uint32_t)reads_ub << 16)), a));
        }
        if (tot >= LIM) return fail(PCCP_E_OVERFLOW, tag + ": |k| >= 2^30");
    }
    if (c.cent.size() > (size_t)INT32_MAX)
        return fail(PCCP_E_UNSUPPORTED, "guarded commands: too many guards and terms");
    compile_features(m, c);
    // adjacency entries hold 16-bit indices
    if (c.diff.size() <= 65536 && c.reif.size() <= 65536 && c.rows.size() <= 65536 &&
        c.brows.size() <= 65536 && c.cmds.size() <= 65536)
        compile_adjacency(c);
    else
        c.adj_ptr.assign(c.nvars + 1, 0);
    return PCCP_OK;
}

// ------------------------------------------------------------------ device buffers
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    int32_t ensure(size_t need)
    {
        if (need <= bytes) return PCCP_OK;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        hipError_t e = hipMalloc(&p, need);
        if (e != hipSuccess) {
            p = nullptr;
            return fail(PCCP_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        }
        bytes = need;
        return PCCP_OK;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <typename T> T *as() const { return reinterpret_cast<T *>(p); }
};

// search workspace (grow-only), and the graph of the last launch
struct Workspace {
    DevBuf models, inst, globals, qseq, qdata, roots, best, trail, gstack;
    hipGraphExec_t graph = nullptr;
    std::vector<char> graph_key;
    void release()
    {
        models.release(); inst.release(); globals.release(); qseq.release();
        qdata.release(); roots.release(); best.release(); trail.release(); gstack.release();
        if (graph) (void)hipGraphExecDestroy(graph);
        graph = nullptr;
        graph_key.clear();
    }
};

struct pccp_solver {
    int device = 0;
    hipStream_t stream = nullptr;
    pccp_config cfg{};
    Compiled c;
    size_t desc_bytes = 0;
    DevBuf tables;      // the packed tables
    DevBuf dmodel;      // DevModel on the device
    DevModel hmodel{};  // same, host copy (device pointers)
    DevBuf box;         // pccp_propagate staging
    std::vector<int32_t> dom_lb, dom_ub;
    bool have_domains = false;
    Workspace ws;
    DevBuf sols;
    int64_t sol_count = 0;
    int64_t sol_kept = 0;
    std::vector<int32_t> best_vals;
    int32_t best = INT32_MAX;
    pccp_stats stats{};
    bool have_stats = false;
    int branching = PCCP_BRANCH_FIRST_FAIL;
    const void *mlp = nullptr;
    int num_cus = 0, wall_khz = 0;
    size_t lds_max = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

static void fill_defaults(pccp_config &cfg)
{
    if (cfg.wg_size <= 0) cfg.wg_size = 256;
    if (cfg.max_depth <= 0) cfg.max_depth = 1024;
    if (cfg.sol_cap < 0) cfg.sol_cap = 0;
}

static int32_t check_cfg(const pccp_config &cfg)
{
    if (cfg.wg_size % 64 != 0 || cfg.wg_size > kMaxWg)
        return fail(PCCP_E_INVALID_ARG, "wg_size must be a multiple of 64 and <= 1024");
    if (cfg.launch < 0 || cfg.launch > 1)
        return fail(PCCP_E_INVALID_ARG, "launch must be 0 (graph) or 1 (plain)");
    if (cfg.num_wgs < 0 || cfg.queue_cap < 0 || cfg.desc_lds < 0 || cfg.desc_lds > 2 ||
        cfg.root_lds < 0 || cfg.root_lds > 2 || cfg.max_depth > (1 << 16) || cfg.live < 0 ||
        cfg.live > 2 || cfg.occupancy < 0 || cfg.occupancy > 2 ||
        (cfg.occupancy == 1 && cfg.wg_size > 256) || cfg.dep < 0 || cfg.dep > 2 ||
        cfg.trail_cap < 0 || cfg.trail_cap > (1 << 24))
        return fail(PCCP_E_INVALID_ARG, "bad config field");
    if (cfg.live == 1 && cfg.dep == 1)
        return fail(PCCP_E_INVALID_ARG, "item lists and dependency-driven propagation exclude each other");
    return PCCP_OK;
}

extern "C" int32_t pccp_solver_create(const pccp_model *m, const pccp_config *cfg, void *stream,
                                      pccp_solver **out)
{
    if (!m || !out) return fail(PCCP_E_INVALID_ARG, "pccp_solver_create: bad arguments");
    *out = nullptr;
    pccp_solver *s = new (std::nothrow) pccp_solver();
    if (!s) return fail(PCCP_E_NOMEM, "pccp_solver_create: out of memory");
    if (cfg) s->cfg = *cfg;
    fill_defaults(s->cfg);
    int32_t rc = check_cfg(s->cfg);
    if (rc == PCCP_OK) rc = compile_model(m, s->c);
    if (rc != PCCP_OK) { delete s; return rc; }
    s->stream = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = hipGetDevice(&s->device);
    hipDeviceProp_t prop;
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, s->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&s->wall_khz, hipDeviceAttributeWallClockRate, s->device);
    if (e != hipSuccess) { delete s; return fail(PCCP_E_DEVICE, std::string("device query: ") + hipGetErrorString(e)); }
    s->num_cus = prop.multiProcessorCount;
    s->lds_max = prop.sharedMemPerBlock;
    const Compiled &c = s->c;
    s->desc_bytes = model_desc_bytes((int)c.diff.size(), (int)c.reif.size(), (int)c.rows.size(),
                                     (int)c.terms.size(), c.ndec, (int)c.brows.size(),
                                     (int)c.bterms.size());
    if (propagate_lds_bytes(store_bytes(c.nI, c.nvars), 0, false) > s->lds_max) {
        delete s;
        return fail(PCCP_E_LDS_CAPACITY, "the store (8 bytes per variable) does not fit in LDS");
    }
    // one blob: lb0, ub0, diff, reif, rows, terms, dec (16-byte aligned pieces)
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t o_lb = 0, o_ub = o_lb + al(4 * (size_t)c.nvars);
    const size_t o_diff = o_ub + al(4 * (size_t)c.nvars);
    const size_t o_reif = o_diff + al(8 * c.diff.size());
    const size_t o_rows = o_reif + al(8 * c.reif.size());
    const size_t o_terms = o_rows + al(16 * c.rows.size());
    const size_t o_dec = o_terms + al(4 * c.terms.size());
    const size_t o_brows = o_dec + al(4 * (size_t)c.ndec);
    const size_t o_bterms = o_brows + al(8 * c.brows.size());
    const size_t o_fstat = o_bterms + al(4 * c.bterms.size());
    const size_t o_frp = o_fstat + al(4 * c.fstat.size());
    const size_t o_fr = o_frp + al(4 * c.fr_ptr.size());
    const size_t o_fbp = o_fr + al(8 * c.fr.size());
    const size_t o_fb = o_fbp + al(4 * c.fb_ptr.size());
    const size_t o_adjp = o_fb + al(4 * c.fb.size());
    const size_t o_adj = o_adjp + al(4 * c.adj_ptr.size());
    const size_t o_cmd = o_adj + al(4 * c.adj.size());
    const size_t o_ccnt = o_cmd + al(16 * c.cmds.size());
    const size_t o_cent = o_ccnt + al(4 * c.ccnt.size());
    const size_t o_vorig = o_cent + al(8 * c.cent.size());
    const size_t o_vnew = o_vorig + al(4 * c.vorig.size());
    const size_t total = o_vnew + al(4 * c.vnew.size()) + 256;
    rc = s->tables.ensure(total);
    if (rc == PCCP_OK) rc = s->dmodel.ensure(sizeof(DevModel));
    if (rc != PCCP_OK) { delete s; return rc; }
    char *base = s->tables.as<char>();
    std::vector<char> host(total, 0);
    auto put = [&](size_t off, const void *src, size_t n) { if (n) memcpy(host.data() + off, src, n); };
    put(o_lb, c.lb0.data(), 4 * (size_t)c.nvars);
    put(o_ub, c.ub0.data(), 4 * (size_t)c.nvars);
    put(o_diff, c.diff.data(), 8 * c.diff.size());
    put(o_reif, c.reif.data(), 8 * c.reif.size());
    put(o_rows, c.rows.data(), 16 * c.rows.size());
    put(o_terms, c.terms.data(), 4 * c.terms.size());
    put(o_dec, c.dec.data(), 4 * (size_t)c.ndec);
    put(o_brows, c.brows.data(), 8 * c.brows.size());
    put(o_bterms, c.bterms.data(), 4 * c.bterms.size());
    put(o_fstat, c.fstat.data(), 4 * c.fstat.size());
    put(o_frp, c.fr_ptr.data(), 4 * c.fr_ptr.size());
    put(o_fr, c.fr.data(), 8 * c.fr.size());
    put(o_fbp, c.fb_ptr.data(), 4 * c.fb_ptr.size());
    put(o_fb, c.fb.data(), 4 * c.fb.size());
    put(o_adjp, c.adj_ptr.data(), 4 * c.adj_ptr.size());
    put(o_adj, c.adj.data(), 4 * c.adj.size());
    put(o_cmd, c.cmds.data(), 16 * c.cmds.size());
    put(o_ccnt, c.ccnt.data(), 4 * c.ccnt.size());
    put(o_cent, c.cent.data(), 8 * c.cent.size());
    put(o_vorig, c.vorig.data(), 4 * c.vorig.size());
    put(o_vnew, c.vnew.data(), 4 * c.vnew.size());
    DevModel &dm = s->hmodel;
    dm.nvars = c.nvars;
    dm.nI = c.nI;
    dm.vorig = reinterpret_cast<const int32_t *>(base + o_vorig);
    dm.vnew = reinterpret_cast<const int32_t *>(base + o_vnew);
    dm.ndiff = (int32_t)c.diff.size();
    dm.nreif = (int32_t)c.reif.size();
    dm.nrows = (int32_t)c.rows.size();
    dm.nterms = (int32_t)c.terms.size();
    dm.ndec = c.ndec;
    dm.objective = c.objective;
    // lanes per linear row in a sweep: the smallest group (4, 8, 16) that
    // covers the longest row in at most two terms per lane, else 16
    int lmax = 0;
    for (const int4 &r : c.rows) lmax = std::max(lmax, r.y);
    dm.row_group = 16;
    for (int g : {4, 8, 16})
        if ((lmax + g - 1) / g <= 2) { dm.row_group = g; break; }
    dm.row_chunks = (lmax + dm.row_group - 1) / dm.row_group;
    dm.nbrows = (int32_t)c.brows.size();
    dm.bgroup = c.bgroup;
    dm.bchunks = c.bchunks;
    dm.nbterms = c.nbterms;
    dm.ncmd = (int32_t)c.cmds.size();
    dm.cmds = reinterpret_cast<const int4 *>(base + o_cmd);
    dm.ccnt = reinterpret_cast<const uint32_t *>(base + o_ccnt);
    dm.cent = reinterpret_cast<const int2 *>(base + o_cent);
    dm.brows = reinterpret_cast<const int2 *>(base + o_brows);
    dm.bterms = reinterpret_cast<const uint32_t *>(base + o_bterms);
    dm.lb0 = reinterpret_cast<const int32_t *>(base + o_lb);
    dm.ub0 = reinterpret_cast<const int32_t *>(base + o_ub);
    dm.diff = reinterpret_cast<const int2 *>(base + o_diff);
    dm.reif = reinterpret_cast<const int2 *>(base + o_reif);
    dm.rows = reinterpret_cast<const int4 *>(base + o_rows);
    dm.terms = reinterpret_cast<const uint32_t *>(base + o_terms);
    dm.dec = reinterpret_cast<const int32_t *>(base + o_dec);
    dm.fstat = reinterpret_cast<const float *>(base + o_fstat);
    dm.fr_ptr = reinterpret_cast<const int32_t *>(base + o_frp);
    dm.fr = reinterpret_cast<const int2 *>(base + o_fr);
    dm.fb_ptr = reinterpret_cast<const int32_t *>(base + o_fbp);
    dm.fb = reinterpret_cast<const int32_t *>(base + o_fb);
    dm.adj_ptr = reinterpret_cast<const int32_t *>(base + o_adjp);
    dm.adj = reinterpret_cast<const uint32_t *>(base + o_adj);
    e = hipMemcpyAsync(base, host.data(), total, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->dmodel.p, &dm, sizeof(DevModel), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e == hipSuccess) e = hipEventCreate(&s->ev0);
    if (e == hipSuccess) e = hipEventCreate(&s->ev1);
    if (e != hipSuccess) {
        pccp_solver_destroy(s);
        return fail(PCCP_E_DEVICE, std::string("upload: ") + hipGetErrorString(e));
    }
    s->best_vals.assign(std::max(c.ndec, 1), 0);
    *out = s;
    return PCCP_OK;
}

extern "C" int32_t pccp_solver_destroy(pccp_solver *s)
{
    if (!s) return PCCP_OK;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    if (s->stream || true) (void)hipStreamSynchronize(s->stream);
    s->tables.release();
    s->dmodel.release();
    s->box.release();
    s->ws.release();
    s->sols.release();
    if (s->ev0) (void)hipEventDestroy(s->ev0);
    if (s->ev1) (void)hipEventDestroy(s->ev1);
    (void)hipSetDevice(prev);
    delete s;
    return PCCP_OK;
}

// ------------------------------------------------------------------ propagate
static bool choose_prop_desc(const pccp_solver *s)
{
    const bool fits = propagate_lds_bytes(store_bytes(s->c.nI, s->c.nvars), s->desc_bytes, true) <= s->lds_max;
    if (s->cfg.desc_lds == 2) return false;
    return fits;
}

extern "C" int32_t pccp_propagate_batch(pccp_solver *s, int32_t nbox, const int32_t *lb_in,
                                        const int32_t *ub_in, int32_t *lb_out, int32_t *ub_out,
                                        int32_t *status, int32_t *sweeps)
{
    if (!s || nbox < 0 || (nbox > 0 && (!lb_in || !ub_in || !lb_out || !ub_out || !status)))
        return fail(PCCP_E_INVALID_ARG, "pccp_propagate_batch: bad arguments");
    if (nbox == 0) return PCCP_OK;
    if (s->cfg.desc_lds == 1 && !choose_prop_desc(s))
        return fail(PCCP_E_LDS_CAPACITY, "propagator tables do not fit in LDS next to the store");
    const bool dl = choose_prop_desc(s);
    const size_t lds = propagate_lds_bytes(store_bytes(s->c.nI, s->c.nvars), s->desc_bytes, dl);
    const int grid = std::min(nbox, std::max(1, s->num_cus * 8));
    HIPCHK(hipSetDevice(s->device));
    HIPCHK(launch_propagate_batch(reinterpret_cast<const DevModel *>(s->dmodel.p), nbox, lb_in,
                                  ub_in, lb_out, ub_out, status, sweeps, grid, s->cfg.wg_size, lds,
                                  dl, s->stream));
    return PCCP_OK;
}

extern "C" int32_t pccp_propagate(pccp_solver *s, const int32_t *lb_in, const int32_t *ub_in,
                                  int32_t *status)
{
    if (!s || !status || ((lb_in == nullptr) != (ub_in == nullptr)))
        return fail(PCCP_E_INVALID_ARG, "pccp_propagate: bad arguments");
    const size_t V = (size_t)s->c.nvars;
    int32_t rc = s->box.ensure(4 * (4 * V + 8) + 256);
    if (rc != PCCP_OK) return rc;
    int32_t *d = s->box.as<int32_t>();
    int32_t *dlb = d, *dub = d + V, *olb = d + 2 * V, *oub = d + 3 * V, *dst = d + 4 * V;
    HIPCHK(hipSetDevice(s->device));
    const int32_t *slb = lb_in ? lb_in : s->c.lb0_model.data();
    const int32_t *sub = ub_in ? ub_in : s->c.ub0_model.data();
    HIPCHK(hipMemcpyAsync(dlb, slb, 4 * V, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(dub, sub, 4 * V, hipMemcpyHostToDevice, s->stream));
    rc = pccp_propagate_batch(s, 1, dlb, dub, olb, oub, dst, dst + 1);
    if (rc != PCCP_OK) return rc;
    s->dom_lb.resize(V);
    s->dom_ub.resize(V);
    int32_t st[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(s->dom_lb.data(), olb, 4 * V, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipMemcpyAsync(s->dom_ub.data(), oub, 4 * V, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipMemcpyAsync(st, dst, 8, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    s->have_domains = true;
    *status = st[0] ? PCCP_FAILED : PCCP_FIXPOINT;
    return PCCP_OK;
}

extern "C" int32_t pccp_node_features(pccp_solver *s, int32_t nbox, const int32_t *lb,
                                      const int32_t *ub, float *feat)
{
    if (!s || nbox < 0 || (nbox > 0 && (!lb || !ub || !feat)))
        return fail(PCCP_E_INVALID_ARG, "pccp_node_features: bad arguments");
    if (nbox == 0 || s->c.ndec == 0) return PCCP_OK;
    HIPCHK(hipSetDevice(s->device));
    HIPCHK(launch_features(reinterpret_cast<const DevModel *>(s->dmodel.p), store_bytes(s->c.nI, s->c.nvars), nbox, lb, ub,
                           feat, s->stream));
    return PCCP_OK;
}

extern "C" int32_t pccp_get_domains(pccp_solver *s, int32_t *lb, int32_t *ub, int32_t cap)
{
    if (!s || !lb || !ub) return fail(PCCP_E_INVALID_ARG, "pccp_get_domains: bad arguments");
    if (!s->have_domains) return fail(PCCP_E_STATE, "pccp_get_domains: no propagation yet");
    if (cap < s->c.nvars) return fail(PCCP_E_INVALID_ARG, "pccp_get_domains: cap < nvars");
    memcpy(lb, s->dom_lb.data(), 4 * (size_t)s->c.nvars);
    memcpy(ub, s->dom_ub.data(), 4 * (size_t)s->c.nvars);
    return PCCP_OK;
}

// ------------------------------------------------------------------ search

// What a search launch has to hold: the largest instance, its tables and
// whether its propagator counts allow 16-bit list entries.
struct ShapeNeed {
    int max_vars = 0;
    size_t max_store = 0;     // bytes of the largest store (store_bytes)
    size_t max_desc = 0;
    int max_items[kDepKinds] = {0, 0, 0, 0, 0};   // per kind; [4] = guarded commands
    int feat_ndec = 0;        // learned branching: feature scratch per candidate
    bool lists_ok = false;    // item lists (every kind <= 65536 propagators)
    bool dep_ok = false;      // adjacency of every instance built
};

// LDS layout of dependency-driven propagation: variable bitmaps of the
// smallest power-of-two word count with 32 bits per word covering the
// store, one mark bit per propagator, work lists of 1/scale of each table
// (at least 64 entries; a sweep whose list would overflow runs the whole
// table of that kind).
struct DepLayout {
    int vshift = 0, qw = 0;
    int wcap[kDepKinds] = {0, 0, 0, 0, 0};
    int jcap = 0;       // two-phase expansion for workgroups of 8 or more wavefronts
};

static DepLayout dep_layout(int max_vars, const int items[kDepKinds], int scale)
{
    DepLayout d;
    const int Vp = (max_vars + 3) & ~3;
    while ((32 << d.vshift) < Vp) ++d.vshift;
    // queued bits for the kinds listed at most once (all but commands)
    const int64_t tot = (int64_t)items[0] + items[1] + items[2] + items[3];
    d.qw = (int)((tot + 31) / 32);
    for (int k = 0; k < kDepKinds; ++k)
        d.wcap[k] = std::min(items[k], std::max(64, (items[k] + scale - 1) / scale));
    return d;
}

struct LaunchShape {
    int block = 256, grid = 1, wgs_per_cu = 1;
    SearchShape k;
    size_t lds = 0;
    DepLayout dep;
};

// Launch shape of a search: the kernel variant (descriptor tables and
// subtree-root store in LDS or global memory) with the most resident
// workgroups.  Item lists (cfg.live == 1) and dependency-driven
// propagation (cfg.dep == 1) are used only when asked for.
static int32_t choose_shape(const pccp_config &cfg, const ShapeNeed &nd, int num_cus,
                            size_t lds_max, LaunchShape &sh)
{
    sh.block = cfg.wg_size;
    const int pm = cfg.dep == 1 ? 2 : (cfg.live == 1 ? 1 : 0);
    if (pm == 1 && !nd.lists_ok)
        return fail(PCCP_E_UNSUPPORTED, "item lists need at most 65536 propagators of each kind");
    if (pm == 2 && !nd.dep_ok)
        return fail(PCCP_E_UNSUPPORTED,
                    "dependency-driven propagation needs at most 65536 propagators of each kind");
    const int list_items = pm == 1 ? nd.max_items[0] + nd.max_items[1] + nd.max_items[2] + nd.max_items[3] : 0;
    struct Cand { bool d, r; };
    const Cand cands[4] = {{true, true}, {false, true}, {true, false}, {false, false}};
    int best_occ = -1, best_li = 1 << 30;
    for (const Cand &cd : cands) {
        if (cfg.desc_lds != 0 && cd.d != (cfg.desc_lds == 1)) continue;
        if (cfg.root_lds != 0 && cd.r != (cfg.root_lds == 1)) continue;
        const size_t base = search_lds_bytes(nd.max_store, cfg.max_depth, nd.max_desc, cd.d, cd.r,
                                             nd.feat_ndec, list_items, 0);
        if (base > lds_max) continue;
        SearchShape k;
        k.desc_lds = cd.d;
        k.root_lds = cd.r;
        k.learned = nd.feat_ndec > 0;
        k.live = pm == 1;
        k.dep = pm == 2;
        k.hi = cfg.occupancy == 1 || (cfg.occupancy == 0 && sh.block <= 256);
        // dependency-driven: the layouts from whole-table lists down to
        // short ones; the first with the most resident workgroups
        const int nlay = pm == 2 ? 8 : 1;
        for (int li = 0; li < nlay; ++li) {
            DepLayout dl;
            size_t depb = 0;
            if (pm == 2) {
                dl = dep_layout(nd.max_vars, nd.max_items, 1 << li);
                dl.jcap = sh.block >= 512 && !k.hi ? 512 : 0;
                depb = dep_lds_bytes(dl.vshift, dl.qw, dl.wcap, dl.jcap);
            }
            const size_t lds = search_lds_bytes(nd.max_store, cfg.max_depth, nd.max_desc, cd.d, cd.r,
                                                nd.feat_ndec, list_items, depb);
            if (lds > lds_max) continue;
            int occ = 0;
            hipError_t e = search_occupancy(sh.block, lds, k, &occ);
            if (e != hipSuccess)
                return fail(PCCP_E_DEVICE, std::string("occupancy: ") + hipGetErrorString(e));
            // the most resident workgroups, then the longest work lists,
            // then the candidates' order of preference
            if (occ > best_occ || (occ == best_occ && li < best_li)) {
                best_occ = occ;
                best_li = li;
                sh.k = k;
                sh.lds = lds;
                sh.dep = dl;
            }
        }
    }
    if (best_occ <= 0)
        return fail(PCCP_E_LDS_CAPACITY, "no store layout fits in LDS with this wg_size/max_depth");
    sh.wgs_per_cu = best_occ;
    const int resident = sh.wgs_per_cu * num_cus;
    sh.grid = cfg.num_wgs > 0 ? std::min(cfg.num_wgs, resident) : resident;
    return PCCP_OK;
}

static int32_t run_search(pccp_solver *const *sv, int32_t n, int32_t mode, const pccp_config *cfgp,
                          const pccp_limits *lim, int32_t *outcomes, bool noalloc = false)
{
    if (!sv || n < 1 || !outcomes || (mode != PCCP_ENUMERATE && mode != PCCP_MINIMIZE))
        return fail(PCCP_E_INVALID_ARG, "search: bad arguments");
    pccp_solver *s0 = sv[0];
    if (!s0) return fail(PCCP_E_INVALID_ARG, "search: solver is NULL");
    pccp_config cfg = cfgp ? *cfgp : s0->cfg;
    fill_defaults(cfg);
    int32_t rc = check_cfg(cfg);
    if (rc != PCCP_OK) return rc;
    int max_vars = 0, max_ndec = 1;
    size_t max_store = 0;
    int max_items[kDepKinds] = {0, 0, 0, 0, 0};
    size_t max_desc = 0;
    for (int i = 0; i < n; ++i) {
        if (!sv[i]) return fail(PCCP_E_INVALID_ARG, "search: solver is NULL");
        if (sv[i]->device != s0->device) return fail(PCCP_E_INVALID_ARG, "search: solvers on different devices");
        if (mode == PCCP_MINIMIZE && sv[i]->c.objective < 0)
            return fail(PCCP_E_STATE, "search: MINIMIZE without an objective");
        max_vars = std::max(max_vars, sv[i]->c.nvars);
        max_store = std::max(max_store, store_bytes(sv[i]->c.nI, sv[i]->c.nvars));
        max_ndec = std::max(max_ndec, sv[i]->c.ndec);
        max_desc = std::max(max_desc, sv[i]->desc_bytes);
        max_items[0] = std::max(max_items[0], (int)sv[i]->c.diff.size());
        max_items[1] = std::max(max_items[1], (int)sv[i]->c.reif.size());
        max_items[2] = std::max(max_items[2], (int)sv[i]->c.rows.size());
        max_items[3] = std::max(max_items[3], (int)sv[i]->c.brows.size());
        max_items[4] = std::max(max_items[4], (int)sv[i]->c.cmds.size());
    }
    HIPCHK(hipSetDevice(s0->device));
    const bool learned = s0->branching == PCCP_BRANCH_MLP && s0->mlp != nullptr;
    LaunchShape sh;
    ShapeNeed need;
    need.max_vars = max_vars;
    need.max_store = max_store;
    need.max_desc = max_desc;
    for (int k = 0; k < kDepKinds; ++k) need.max_items[k] = max_items[k];
    need.feat_ndec = learned ? max_ndec : 0;
    // list entries are 16-bit descriptor indices
    // item lists leave the guarded commands out; work lists hold them too
    need.lists_ok = *std::max_element(max_items, max_items + 4) <= 65536;
    need.dep_ok = *std::max_element(max_items, max_items + kDepKinds) <= 65536;
    rc = choose_shape(cfg, need, s0->num_cus, s0->lds_max, sh);
    if (rc != PCCP_OK) return rc;
    const int qcap = cfg.queue_cap > 0 ? std::max(cfg.queue_cap, n) : std::max(4 * sh.grid, n + sh.grid);
    const int slot_bytes = (int)(((size_t)sizeof(RecHdr) + sizeof(int2) * (size_t)cfg.max_depth + 15) & ~size_t(15));
    const int Vp = (max_vars + 3) & ~3;
    // trail: 8 entries of 16 bytes per store variable per workgroup, within
    // [4096, 2^18] entries; a path whose changes do not fit falls back to
    // recomputation
    const int tcap = !sh.k.dep ? 0 : cfg.trail_cap > 0 ? cfg.trail_cap
                                                       : std::min(std::max(8 * Vp, 4096), 1 << 18);
    // the pieces of the workspace, in bytes (0 = not used by this shape)
    const size_t z_models = sizeof(DevModel) * n, z_inst = sizeof(InstState) * n;
    const size_t z_glob = sizeof(SearchGlobals), z_qseq = sizeof(unsigned long long) * qcap;
    const size_t z_qdata = (size_t)slot_bytes * qcap, z_best = sizeof(int32_t) * (size_t)n * max_ndec;
    const size_t z_roots = sh.k.root_lds ? 0 : max_store * sh.grid;
    const size_t z_trail = sh.k.dep ? sizeof(int4) * (size_t)tcap * sh.grid : 0;
    const size_t z_gstack = sizeof(int4) * (size_t)cfg.max_depth * sh.grid;
    DevModel *w_models = nullptr;
    InstState *w_inst = nullptr;
    SearchGlobals *w_glob = nullptr;
    unsigned long long *w_qseq = nullptr;
    char *w_qdata = nullptr;
    int32_t *w_best = nullptr, *w_roots = nullptr;
    int4 *w_trail = nullptr, *w_gstack = nullptr;
    // the solution list is kept by the allocating form only
    const bool keep_sols = (!noalloc && mode == PCCP_ENUMERATE && n == 1 && cfg.sol_cap > 0);
    if (noalloc) {
        // carve every piece out of the library's static device array
        auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
        const size_t need = al(z_models) + al(z_inst) + al(z_glob) + al(z_qseq) + al(z_qdata) +
                            al(z_best) + al(z_roots) + al(z_trail) + al(z_gstack);
        if (need > kScratchBytes)
            return fail(PCCP_E_NOMEM, "pccp_solve_noalloc: the search needs " + std::to_string(need) +
                                          " bytes of workspace, more than the static " +
                                          std::to_string(kScratchBytes) +
                                          " (lower num_wgs, max_depth or trail_cap)");
        void *sp = nullptr;
        HIPCHK(scratch_address(&sp));
        char *base = reinterpret_cast<char *>(sp);
        size_t off = 0;
        auto carve = [&](size_t b) -> char * {
            if (b == 0) return nullptr;
            char *q = base + off;
            off += al(b);
            return q;
        };
        w_models = reinterpret_cast<DevModel *>(carve(z_models));
        w_inst = reinterpret_cast<InstState *>(carve(z_inst));
        w_glob = reinterpret_cast<SearchGlobals *>(carve(z_glob));
        w_qseq = reinterpret_cast<unsigned long long *>(carve(z_qseq));
        w_qdata = carve(z_qdata);
        w_best = reinterpret_cast<int32_t *>(carve(z_best));
        w_roots = reinterpret_cast<int32_t *>(carve(z_roots));
        w_trail = reinterpret_cast<int4 *>(carve(z_trail));
        w_gstack = reinterpret_cast<int4 *>(carve(z_gstack));
    } else {
        Workspace &ws = s0->ws;
        if ((rc = ws.models.ensure(z_models)) || (rc = ws.inst.ensure(z_inst)) ||
            (rc = ws.globals.ensure(z_glob)) || (rc = ws.qseq.ensure(z_qseq)) ||
            (rc = ws.qdata.ensure(z_qdata)) || (rc = ws.best.ensure(z_best)))
            return rc;
        if (z_roots && (rc = ws.roots.ensure(z_roots))) return rc;
        if (z_trail && (rc = ws.trail.ensure(z_trail))) return rc;
        if ((rc = ws.gstack.ensure(z_gstack))) return rc;
        if (keep_sols && (rc = s0->sols.ensure(sizeof(int32_t) * (size_t)cfg.sol_cap * std::max(s0->c.ndec, 1))))
            return rc;
        w_models = ws.models.as<DevModel>();
        w_inst = ws.inst.as<InstState>();
        w_glob = ws.globals.as<SearchGlobals>();
        w_qseq = ws.qseq.as<unsigned long long>();
        w_qdata = ws.qdata.as<char>();
        w_best = ws.best.as<int32_t>();
        w_roots = z_roots ? ws.roots.as<int32_t>() : nullptr;
        w_trail = z_trail ? ws.trail.as<int4>() : nullptr;
        w_gstack = ws.gstack.as<int4>();
    }
    std::vector<DevModel> hm(n);
    for (int i = 0; i < n; ++i) hm[i] = sv[i]->hmodel;
    HIPCHK(hipMemcpyAsync(w_models, hm.data(), sizeof(DevModel) * n, hipMemcpyHostToDevice, s0->stream));

    // zeroed bytewise: the struct's bytes, padding included, key the graph cache
    SearchParams P;
    memset(&P, 0, sizeof(P));
    P.models = w_models;
    P.inst = w_inst;
    P.ninst = n;
    P.mode = mode;
    P.branching = learned ? 2 : (s0->branching == PCCP_BRANCH_INPUT_ORDER ? 1 : 0);
    P.max_depth = cfg.max_depth;
    P.g = w_glob;
    P.q_seq = w_qseq;
    P.q_data = w_qdata;
    P.qcap = qcap;
    P.slot_bytes = slot_bytes;
    P.root_scratch = sh.k.root_lds ? nullptr : reinterpret_cast<char *>(w_roots);
    P.max_vars = max_vars;
    P.max_store = (long long)max_store;
    P.donate = sh.grid > 1 ? 1 : 0;
    P.node_limit = lim ? lim->node_limit : 0;
    P.inst_node_limit = lim ? lim->inst_node_limit : 0;
    P.t_limit_ticks = (lim && lim->time_limit_s > 0) ? (long long)(lim->time_limit_s * s0->wall_khz * 1000.0) : 0;
    P.cancel = lim ? lim->cancel : nullptr;
    P.sol_buf = keep_sols ? s0->sols.as<int32_t>() : nullptr;
    P.sol_cap = keep_sols ? cfg.sol_cap : 0;
    P.best_vals = w_best;
    P.max_ndec = max_ndec;
    P.mlp = learned ? reinterpret_cast<const uint16_t *>(s0->mlp) : nullptr;
    for (int k = 0; k < 4; ++k) P.max_items[k] = max_items[k];
    P.dep_vshift = sh.dep.vshift;
    P.dep_qw = sh.dep.qw;
    for (int k = 0; k < kDepKinds; ++k) P.dep_wcap[k] = sh.dep.wcap[k];
    P.dep_jcap = sh.dep.jcap;
    P.trail = sh.k.dep ? w_trail : nullptr;
    P.tcap = tcap;
    P.gstack = w_gstack;

    if (cfg.launch == 0 && !noalloc) {
        Workspace &ws = s0->ws;
        // the graph bakes in the launch parameters: rebuild it when they change
        std::vector<char> key(sizeof(P) + 8 * sizeof(int64_t));
        memcpy(key.data(), &P, sizeof(P));
        const int64_t extra[8] = {sh.grid, sh.block, (int64_t)sh.lds, sh.k.desc_lds, sh.k.root_lds,
                                  sh.k.learned, sh.k.live | (sh.k.dep << 1), sh.k.hi};
        memcpy(key.data() + sizeof(P), extra, sizeof(extra));
        if (!ws.graph || key != ws.graph_key) {
            if (ws.graph) (void)hipGraphExecDestroy(ws.graph);
            ws.graph = nullptr;
            HIPCHK(build_search_graph(P, sh.grid, sh.block, sh.lds, sh.k, &ws.graph));
            ws.graph_key = key;
        }
        HIPCHK(hipEventRecord(s0->ev0, s0->stream));
        HIPCHK(hipGraphLaunch(ws.graph, s0->stream));
        HIPCHK(hipEventRecord(s0->ev1, s0->stream));
    } else {
        HIPCHK(hipEventRecord(s0->ev0, s0->stream));
        HIPCHK(launch_search(P, sh.grid, sh.block, sh.lds, sh.k, s0->stream));
        HIPCHK(hipEventRecord(s0->ev1, s0->stream));
    }
    std::vector<InstState> st(n);
    SearchGlobals g{};
    std::vector<int32_t> bv((size_t)n * max_ndec);
    HIPCHK(hipMemcpyAsync(st.data(), P.inst, sizeof(InstState) * n, hipMemcpyDeviceToHost, s0->stream));
    HIPCHK(hipMemcpyAsync(&g, P.g, sizeof(SearchGlobals), hipMemcpyDeviceToHost, s0->stream));
    HIPCHK(hipMemcpyAsync(bv.data(), P.best_vals, sizeof(int32_t) * bv.size(), hipMemcpyDeviceToHost, s0->stream));
    HIPCHK(hipStreamSynchronize(s0->stream));
    float kms = 0.f;
    HIPCHK(hipEventElapsedTime(&kms, s0->ev0, s0->ev1));

    bool overflow = false;
    for (int i = 0; i < n; ++i) {
        pccp_solver *s = sv[i];
        const InstState &is = st[i];
        pccp_stats &o = s->stats;
        memset(&o, 0, sizeof(o));
        o.nodes = (int64_t)is.nodes;
        o.fails = (int64_t)is.fails;
        o.solutions = (int64_t)is.solutions;
        o.sweeps = (int64_t)is.sweeps;
        o.donations = (int64_t)is.donations;
        o.subtrees = (int64_t)is.pops;
        o.max_depth = (int64_t)is.max_depth;
        o.prop_linear2 = (int64_t)is.ex[0];
        o.prop_reified = (int64_t)is.ex[1];
        o.prop_linear = (int64_t)is.ex[2];
        o.prop_terms = (int64_t)is.ex[3];
        o.atomics = (int64_t)is.atomics;
        o.sol_hash = is.sol_hash;
        o.best = is.best;
        o.kernel_ms = kms;
        o.grid = sh.grid;
        o.block = sh.block;
        o.desc_lds = sh.k.desc_lds;
        o.root_lds = sh.k.root_lds;
        o.lds_bytes = (int64_t)sh.lds;
        o.live = sh.k.live;
        o.occupancy = sh.k.hi ? 1 : 2;
        o.dep = sh.k.dep;
        const bool done = is.outstanding == 0;
        o.ttpo_ms = done ? (double)(is.t_done - g.t_start) / (double)s->wall_khz : -1.0;
        if (done)
            o.outcome = mode == PCCP_ENUMERATE ? PCCP_OUT_ALL
                        : (is.best == INT32_MAX ? PCCP_OUT_UNSAT : PCCP_OUT_OPTIMAL);
        else
            o.outcome = g.abort == 3 ? PCCP_OUT_CANCELLED : PCCP_OUT_LIMIT;
        if (is.abandon) {
            o.outcome = PCCP_OUT_LIMIT;
            o.ttpo_ms = -1.0;
        }
        if (is.depth_overflow) overflow = true;
        outcomes[i] = o.outcome;
        s->best = is.best;
        for (int q = 0; q < s->c.ndec; ++q) s->best_vals[q] = bv[(size_t)i * max_ndec + q];
        s->sol_count = mode == PCCP_ENUMERATE ? (int64_t)is.solutions : 0;
        s->sol_kept = (keep_sols && i == 0) ? std::min<int64_t>(s->sol_count, cfg.sol_cap) : 0;
        s->have_stats = true;
    }
    if (overflow)
        return fail(PCCP_E_DEPTH, "a search path was deeper than max_depth");
    return PCCP_OK;
}

extern "C" int32_t pccp_solve(pccp_solver *s, int32_t mode, const pccp_limits *limits, int32_t *outcome)
{
    if (!s || !outcome) return fail(PCCP_E_INVALID_ARG, "pccp_solve: bad arguments");
    pccp_solver *sv[1] = {s};
    return run_search(sv, 1, mode, nullptr, limits, outcome);
}

extern "C" int32_t pccp_solve_noalloc(pccp_solver *s, int32_t mode, const pccp_limits *limits,
                                      int32_t *outcome)
{
    if (!s || !outcome) return fail(PCCP_E_INVALID_ARG, "pccp_solve_noalloc: bad arguments");
    pccp_solver *sv[1] = {s};
    return run_search(sv, 1, mode, nullptr, limits, outcome, true);
}

extern "C" int32_t pccp_batch_solve(pccp_solver *const *solvers, int32_t n, int32_t mode,
                                    const pccp_config *cfg, const pccp_limits *limits,
                                    int32_t *outcomes)
{
    return run_search(solvers, n, mode, cfg, limits, outcomes);
}

extern "C" int32_t pccp_get_stats(const pccp_solver *s, pccp_stats *st)
{
    if (!s || !st) return fail(PCCP_E_INVALID_ARG, "pccp_get_stats: bad arguments");
    if (!s->have_stats) return fail(PCCP_E_STATE, "pccp_get_stats: no search yet");
    *st = s->stats;
    return PCCP_OK;
}

extern "C" int32_t pccp_get_solution_hash(const pccp_solver *s, uint64_t *hash)
{
    if (!s || !hash) return fail(PCCP_E_INVALID_ARG, "pccp_get_solution_hash: bad arguments");
    if (!s->have_stats) return fail(PCCP_E_STATE, "pccp_get_solution_hash: no search yet");
    *hash = s->stats.sol_hash;
    return PCCP_OK;
}

extern "C" int32_t pccp_get_solution_count(const pccp_solver *s, int64_t *count)
{
    if (!s || !count) return fail(PCCP_E_INVALID_ARG, "pccp_get_solution_count: bad arguments");
    if (!s->have_stats) return fail(PCCP_E_STATE, "pccp_get_solution_count: no search yet");
    *count = s->sol_count;
    return PCCP_OK;
}

extern "C" int32_t pccp_get_solutions(pccp_solver *s, int64_t first, int64_t count, int32_t *vals)
{
    if (!s || first < 0 || count < 0 || (count > 0 && !vals))
        return fail(PCCP_E_INVALID_ARG, "pccp_get_solutions: bad arguments");
    if (first + count > s->sol_kept)
        return fail(PCCP_E_INVALID_ARG, "pccp_get_solutions: range beyond the kept solutions");
    if (count == 0) return PCCP_OK;
    const size_t nd = (size_t)std::max(s->c.ndec, 1);
    HIPCHK(hipSetDevice(s->device));
    HIPCHK(hipMemcpyAsync(vals, s->sols.as<int32_t>() + (size_t)first * nd, sizeof(int32_t) * nd * count,
                          hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return PCCP_OK;
}

extern "C" int32_t pccp_get_best(pccp_solver *s, int32_t *obj, int32_t *vals, int32_t cap)
{
    if (!s || !obj) return fail(PCCP_E_INVALID_ARG, "pccp_get_best: bad arguments");
    if (!s->have_stats) return fail(PCCP_E_STATE, "pccp_get_best: no search yet");
    *obj = s->best;
    if (vals) {
        if (cap < s->c.ndec) return fail(PCCP_E_INVALID_ARG, "pccp_get_best: cap < ndecision");
        memcpy(vals, s->best_vals.data(), sizeof(int32_t) * (size_t)s->c.ndec);
    }
    return PCCP_OK;
}

extern "C" int32_t pccp_set_branching(pccp_solver *s, int32_t kind, const void *weights)
{
    if (!s || kind < PCCP_BRANCH_FIRST_FAIL || kind > PCCP_BRANCH_MLP)
        return fail(PCCP_E_INVALID_ARG, "pccp_set_branching: bad arguments");
    s->branching = kind;
    s->mlp = weights;
    return PCCP_OK;
}

extern "C" int32_t pccp_solver_capacity(const pccp_solver *s, int32_t *wgs_per_cu, int32_t *num_cus)
{
    if (!s) return fail(PCCP_E_INVALID_ARG, "pccp_solver_capacity: bad arguments");
    pccp_config cfg = s->cfg;
    fill_defaults(cfg);
    LaunchShape sh;
    HIPCHK(hipSetDevice(s->device));
    ShapeNeed need;
    need.max_vars = s->c.nvars;
    need.max_store = store_bytes(s->c.nI, s->c.nvars);
    need.max_desc = s->desc_bytes;
    need.max_items[0] = (int)s->c.diff.size();
    need.max_items[1] = (int)s->c.reif.size();
    need.max_items[2] = (int)s->c.rows.size();
    need.max_items[3] = (int)s->c.brows.size();
    need.max_items[4] = (int)s->c.cmds.size();
    need.lists_ok = *std::max_element(need.max_items, need.max_items + 4) <= 65536;
    need.dep_ok = *std::max_element(need.max_items, need.max_items + kDepKinds) <= 65536;
    int32_t rc = choose_shape(cfg, need, s->num_cus, s->lds_max, sh);
    if (rc != PCCP_OK) return rc;
    if (wgs_per_cu) *wgs_per_cu = sh.wgs_per_cu;
    if (num_cus) *num_cus = s->num_cus;
    return PCCP_OK;
}

// ------------------------------------------------------------------ incremental propagation
extern "C" int32_t pccp_propagate_batch_incr(pccp_solver *s, int32_t nbox, const int32_t *lb_in,
                                             const int32_t *ub_in, const int32_t *dvar,
                                             const int32_t *dlo, const int32_t *dhi,
                                             int32_t *lb_out, int32_t *ub_out, int32_t *status,
                                             int32_t *sweeps)
{
    if (!s || nbox < 0 || (nbox > 0 && (!lb_in || !ub_in || !dvar || !dlo || !dhi || !lb_out ||
                                        !ub_out || !status)))
        return fail(PCCP_E_INVALID_ARG, "pccp_propagate_batch_incr: bad arguments");
    const Compiled &c = s->c;
    const int items[kDepKinds] = {(int)c.diff.size(), (int)c.reif.size(), (int)c.rows.size(),
                                  (int)c.brows.size(), (int)c.cmds.size()};
    if (*std::max_element(items, items + kDepKinds) > 65536)
        return fail(PCCP_E_UNSUPPORTED,
                    "dependency-driven propagation needs at most 65536 propagators of each kind");
    if (nbox == 0) return PCCP_OK;
    const int block = s->cfg.wg_size;
    // the longest work lists that fit next to the store (a sweep whose list
    // would overflow runs that kind's whole table)
    DepLayout dl;
    size_t lds = 0;
    bool fits = false;
    for (int li = 0; li < 8 && !fits; ++li) {
        dl = dep_layout(c.nvars, items, 1 << li);
        dl.jcap = block >= 512 ? 512 : 0;
        lds = propagate_lds_bytes(store_bytes(c.nI, c.nvars), 0, false) + dep_lds_bytes(dl.vshift, dl.qw, dl.wcap, dl.jcap);
        fits = lds <= s->lds_max;
    }
    if (!fits)
        return fail(PCCP_E_LDS_CAPACITY, "the store and the dependency bitmaps do not fit in LDS");
    IncrParams A;
    memset(&A, 0, sizeof(A));
    A.nbox = nbox;
    A.dep_vshift = dl.vshift;
    A.dep_qw = dl.qw;
    A.dep_jcap = dl.jcap;
    for (int k = 0; k < kDepKinds; ++k) A.dep_wcap[k] = dl.wcap[k];
    A.lb_in = lb_in;
    A.ub_in = ub_in;
    A.dvar = dvar;
    A.dlo = dlo;
    A.dhi = dhi;
    A.lb_out = lb_out;
    A.ub_out = ub_out;
    A.status = status;
    A.sweeps = sweeps;
    const int grid = std::min(nbox, std::max(1, s->num_cus * 8));
    HIPCHK(hipSetDevice(s->device));
    HIPCHK(launch_propagate_incr(reinterpret_cast<const DevModel *>(s->dmodel.p), A, grid, block, lds,
                                 s->stream));
    return PCCP_OK;
}

// ------------------------------------------------------------------ learned branching
// ------------------------------------------------------------------ launch tuning
namespace {
struct Probe {
    double nodes = 0, secs = 0;
    int32_t grid = 0;
};

// one time-limited batched search; nodes over all instances, device seconds
int32_t probe(pccp_solver *const *sv, int32_t n, int32_t mode, const pccp_config &cfg, double t,
              Probe &out)
{
    pccp_limits lim{};
    lim.time_limit_s = t;
    std::vector<int32_t> outc((size_t)n);
    const int32_t rc = run_search(sv, n, mode, &cfg, &lim, outc.data());
    if (rc != PCCP_OK) return rc;
    out.nodes = 0;
    for (int i = 0; i < n; ++i) out.nodes += (double)sv[i]->stats.nodes;
    out.secs = sv[0]->stats.kernel_ms / 1e3;
    out.grid = sv[0]->stats.grid;
    return PCCP_OK;
}

// node rate of a candidate (see pccp_tune_opts.whole_run)
int32_t cand_rate(pccp_solver *const *sv, int32_t n, int32_t mode, const pccp_config &cfg,
                  double budget, bool whole, double &rate, int32_t &grid)
{
    Probe a, b;
    // untimed first: the first launch of a kernel variant also loads its code
    int32_t rc = probe(sv, n, mode, cfg, std::min(0.05, budget / 4), a);
    if (rc == PCCP_OK && !whole) rc = probe(sv, n, mode, cfg, budget / 2, a);
    if (rc == PCCP_OK) rc = probe(sv, n, mode, cfg, budget, b);
    if (rc != PCCP_OK) return rc;
    grid = b.grid;
    if (whole || b.secs - a.secs < 0.25 * b.secs || b.nodes < a.nodes)
        rate = b.nodes / std::max(b.secs, 1e-9);       // finished early: the whole run
    else
        rate = (b.nodes - a.nodes) / (b.secs - a.secs);
    return PCCP_OK;
}
}  // namespace

extern "C" int32_t pccp_autotune(pccp_solver *const *solvers, int32_t n, int32_t mode,
                                 const pccp_tune_opts *opts, pccp_config *best,
                                 pccp_tune_result *results, int32_t cap, int32_t *nresults)
{
    if (!solvers || n < 1 || !best || cap < 0 || (cap > 0 && !results))
        return fail(PCCP_E_INVALID_ARG, "pccp_autotune: bad arguments");
    for (int i = 0; i < n; ++i)
        if (!solvers[i]) return fail(PCCP_E_INVALID_ARG, "pccp_autotune: solver is NULL");
    pccp_tune_opts o = opts ? *opts : pccp_tune_opts{};
    if (o.budget_s < 0 || o.finalists < 0 || o.modes < 0 || o.modes > 7 || o.wg_sizes < 0 ||
        o.wg_sizes > 31 || o.max_depth < 0)
        return fail(PCCP_E_INVALID_ARG, "pccp_autotune: bad options");
    const double budget = o.budget_s > 0 ? o.budget_s : 0.4;
    const int finalists = o.finalists > 0 ? o.finalists : 3;
    const int modes = o.modes ? o.modes : 3;
    const int wgs = o.wg_sizes ? o.wg_sizes : (2 | 4 | 8 | 16);
    struct Cand {
        pccp_config cfg;
        double rate = 0, rate_long = 0;
        int32_t grid = 0, status = PCCP_OK, order = 0;
    };
    std::vector<Cand> all;
    const pccp_config base = solvers[0]->cfg;
    for (int k = 0; k < 5; ++k) {
        if (!(wgs & (1 << k))) continue;
        const int wg = 64 << k;
        for (int place = 0; place < 4; ++place)
            for (int pm = 0; pm < 3; ++pm) {
                if (!(modes & (1 << pm))) continue;
                for (int occ = 1; occ <= 2; ++occ) {
                    if (occ == 1 && wg > 256) continue;
                    Cand c;
                    c.cfg = base;
                    c.cfg.wg_size = wg;
                    c.cfg.desc_lds = 1 + (place >> 1);
                    c.cfg.root_lds = 1 + (place & 1);
                    c.cfg.live = pm == 2 ? 1 : 2;
                    c.cfg.dep = pm == 1 ? 1 : 2;
                    c.cfg.occupancy = occ;
                    c.cfg.max_depth = o.max_depth > 0 ? o.max_depth : base.max_depth;
                    c.order = (int32_t)all.size();
                    all.push_back(c);
                }
            }
    }
    for (Cand &c : all) {
        c.status = cand_rate(solvers, n, mode, c.cfg, budget, o.whole_run != 0, c.rate, c.grid);
        if (c.status != PCCP_OK && c.status != PCCP_E_LDS_CAPACITY && c.status != PCCP_E_DEPTH)
            return c.status;
        if (c.status != PCCP_OK) c.rate = 0;
    }
    std::vector<Cand *> ok;
    for (Cand &c : all)
        if (c.status == PCCP_OK) ok.push_back(&c);
    if (ok.empty()) return fail(PCCP_E_LDS_CAPACITY, "pccp_autotune: no candidate fits");
    std::stable_sort(ok.begin(), ok.end(), [](const Cand *a, const Cand *b) { return a->rate > b->rate; });
    const size_t nf = std::min<size_t>(finalists, ok.size());
    double top = 0;
    for (size_t i = 0; i < nf; ++i) {
        int32_t g = 0;
        const int32_t rc = cand_rate(solvers, n, mode, ok[i]->cfg, 4 * budget, o.whole_run != 0,
                                     ok[i]->rate_long, g);
        if (rc == PCCP_E_DEPTH) ok[i]->rate_long = 0;
        else if (rc != PCCP_OK) return rc;
        top = std::max(top, ok[i]->rate_long);
    }
    const Cand *pick = ok[0];
    for (size_t i = 0; i < nf; ++i)
        if (ok[i]->rate_long >= 0.98 * top) { pick = ok[i]; break; }
    *best = pick->cfg;
    fill_defaults(*best);
    const int32_t nr = std::min<int32_t>(cap, (int32_t)all.size());
    for (int32_t i = 0; i < nr; ++i) {
        results[i].cfg = all[i].cfg;
        results[i].nodes_per_s = all[i].rate;
        results[i].nodes_per_s_long = all[i].rate_long;
        results[i].grid = all[i].grid;
        results[i].status = all[i].status;
    }
    if (nresults) *nresults = (int32_t)all.size();
    return PCCP_OK;
}

struct pccp_mlp {
    int device = 0;
    hipStream_t stream = nullptr;
    DevBuf state;      // params, m1, v1, grad (kNumParams each), bf16 copy, loss
    DevBuf work;       // per-candidate dL/ds + per-wave partials
    int64_t step = 0;
    float *params() { return state.as<float>(); }
    float *m1() { return state.as<float>() + 1 * 520; }
    float *v1() { return state.as<float>() + 2 * 520; }
    float *grad() { return state.as<float>() + 3 * 520; }
    float *loss() { return state.as<float>() + 4 * 520; }
    uint16_t *wbf() { return reinterpret_cast<uint16_t *>(state.as<float>() + 5 * 520); }
};

static uint64_t splitmix64(uint64_t &x)
{
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

extern "C" int32_t pccp_mlp_create(uint64_t seed, void *stream, pccp_mlp **out)
{
    if (!out) return fail(PCCP_E_INVALID_ARG, "pccp_mlp_create: out is NULL");
    *out = nullptr;
    pccp_mlp *m = new (std::nothrow) pccp_mlp();
    if (!m) return fail(PCCP_E_NOMEM, "pccp_mlp_create: out of memory");
    m->stream = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = hipGetDevice(&m->device);
    if (e != hipSuccess) { delete m; return fail(PCCP_E_DEVICE, hipGetErrorString(e)); }
    int32_t rc = m->state.ensure(sizeof(float) * 520 * 6);
    if (rc != PCCP_OK) { delete m; return rc; }
    // Glorot-uniform initial weights from a SplitMix64 stream, zero biases
    std::vector<float> host(520 * 5, 0.f);
    uint64_t st = seed;
    auto unif = [&](double a) {
        return (float)(a * (2.0 * ((splitmix64(st) >> 11) * (1.0 / 9007199254740992.0)) - 1.0));
    };
    const double a1 = std::sqrt(6.0 / (kNumFeat + kHidden)), a2 = std::sqrt(6.0 / (kHidden + 1));
    for (int i = 0; i < kHidden * kNumFeat; ++i) host[i] = unif(a1);
    for (int k = 0; k < kHidden; ++k) host[kHidden * kNumFeat + kHidden + k] = unif(a2);
    e = hipMemcpyAsync(m->state.p, host.data(), sizeof(float) * host.size(), hipMemcpyHostToDevice,
                       m->stream);
    if (e == hipSuccess) e = launch_mlp_sync_bf16(m->params(), m->wbf(), m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) {
        m->state.release();
        delete m;
        return fail(PCCP_E_DEVICE, std::string("pccp_mlp_create: ") + hipGetErrorString(e));
    }
    *out = m;
    return PCCP_OK;
}

extern "C" int32_t pccp_mlp_destroy(pccp_mlp *m)
{
    if (!m) return PCCP_OK;
    (void)hipStreamSynchronize(m->stream);
    m->state.release();
    m->work.release();
    delete m;
    return PCCP_OK;
}

extern "C" int32_t pccp_mlp_set_params(pccp_mlp *m, const float *params)
{
    if (!m || !params) return fail(PCCP_E_INVALID_ARG, "pccp_mlp_set_params: bad arguments");
    HIPCHK(hipSetDevice(m->device));
    HIPCHK(hipMemcpyAsync(m->params(), params, sizeof(float) * kNumParams, hipMemcpyHostToDevice, m->stream));
    HIPCHK(hipMemsetAsync(m->m1(), 0, sizeof(float) * 520 * 2, m->stream));
    HIPCHK(launch_mlp_sync_bf16(m->params(), m->wbf(), m->stream));
    HIPCHK(hipStreamSynchronize(m->stream));
    m->step = 0;
    return PCCP_OK;
}

extern "C" int32_t pccp_mlp_get_params(pccp_mlp *m, float *params)
{
    if (!m || !params) return fail(PCCP_E_INVALID_ARG, "pccp_mlp_get_params: bad arguments");
    HIPCHK(hipSetDevice(m->device));
    HIPCHK(hipMemcpyAsync(params, m->params(), sizeof(float) * kNumParams, hipMemcpyDeviceToHost, m->stream));
    HIPCHK(hipStreamSynchronize(m->stream));
    return PCCP_OK;
}

extern "C" int32_t pccp_mlp_get_grads(pccp_mlp *m, float *grads)
{
    if (!m || !grads) return fail(PCCP_E_INVALID_ARG, "pccp_mlp_get_grads: bad arguments");
    HIPCHK(hipSetDevice(m->device));
    HIPCHK(hipMemcpyAsync(grads, m->grad(), sizeof(float) * kNumParams, hipMemcpyDeviceToHost, m->stream));
    HIPCHK(hipStreamSynchronize(m->stream));
    return PCCP_OK;
}

extern "C" int32_t pccp_mlp_train_step(pccp_mlp *m, const float *feat, const int32_t *node_off,
                                       const float *target, int32_t nnodes, int32_t ncand,
                                       int32_t max_cand, float lr, float *loss)
{
    if (!m || !feat || !node_off || !target || nnodes < 1 || ncand < 1 || lr < 0.f)
        return fail(PCCP_E_INVALID_ARG, "pccp_mlp_train_step: bad arguments");
    if (max_cand > kMlpMaxCand || max_cand < 1)
        return fail(PCCP_E_UNSUPPORTED, "pccp_mlp_train_step: more than 256 candidates in a node");
    HIPCHK(hipSetDevice(m->device));
    const int rows = mlp_partial_rows();
    int32_t rc = m->work.ensure(sizeof(float) * ((size_t)ncand + (size_t)rows * 520 + 64));
    if (rc != PCCP_OK) return rc;
    float *g = m->work.as<float>();
    float *partial = g + (((size_t)ncand + 63) & ~size_t(63));
    if (lr > 0.f) m->step += 1;
    HIPCHK(launch_mlp_train(feat, node_off, target, nnodes, ncand, m->params(), m->m1(), m->v1(),
                            m->wbf(), m->grad(), g, partial, lr, (int)std::max<int64_t>(m->step, 1),
                            m->loss(), m->stream));
    if (loss) {
        HIPCHK(hipMemcpyAsync(loss, m->loss(), sizeof(float), hipMemcpyDeviceToHost, m->stream));
        HIPCHK(hipStreamSynchronize(m->stream));
    }
    return PCCP_OK;
}

extern "C" int32_t pccp_mlp_scores(pccp_mlp *m, const float *feat, int32_t ncand, float *scores,
                                   int32_t bf16)
{
    if (!m || ncand < 0 || (ncand > 0 && (!feat || !scores)))
        return fail(PCCP_E_INVALID_ARG, "pccp_mlp_scores: bad arguments");
    if (ncand == 0) return PCCP_OK;
    HIPCHK(hipSetDevice(m->device));
    HIPCHK(launch_mlp_scores(m->params(), m->wbf(), bf16 ? 1 : 0, feat, ncand, scores, m->stream));
    return PCCP_OK;
}

extern "C" int32_t pccp_mlp_weights(const pccp_mlp *m, const void **weights)
{
    if (!m || !weights) return fail(PCCP_E_INVALID_ARG, "pccp_mlp_weights: bad arguments");
    *weights = reinterpret_cast<const void *>(const_cast<pccp_mlp *>(m)->wbf());
    return PCCP_OK;
}

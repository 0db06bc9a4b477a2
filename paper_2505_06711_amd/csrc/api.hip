// C ABI entry points.  Every call converts library exceptions into a status code and a
// thread-local message; no exception crosses the boundary.
#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "runtime.hpp"

using namespace reann;

static thread_local std::string g_last_error;

static reann_status set_err(reann_status code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

namespace reann {
void set_last_error(const std::string &msg) { g_last_error = msg; }
}

template <class F> static reann_status guarded(F &&f) {
    try {
        f();
        g_last_error.clear();
        return REANN_OK;
    } catch (const Error &e) {
        return set_err(e.code, e.what());
    } catch (const std::bad_alloc &) {
        return set_err(REANN_E_NOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return set_err(REANN_E_DEVICE, e.what());
    } catch (...) {
        return set_err(REANN_E_DEVICE, "unknown error");
    }
}

#define REQUIRE(cond, msg) \
    do { if (!(cond)) fail(REANN_E_INVALID, msg); } while (0)

static void check_cell(const double *cell, const int32_t *pbc) {
    REQUIRE(cell && pbc, "cell and pbc are required");
    for (int k = 0; k < 9; ++k) REQUIRE(std::isfinite(cell[k]), "cell has a non-finite entry");
}

static void check_positions(const double *pos, int64_t n) {
    for (int64_t i = 0; i < 3 * n; ++i) REQUIRE(std::isfinite(pos[i]), "positions contain NaN or Inf");
}

static std::mutex g_ctx_mu;

static void ctx_destroy(reann_ctx *c) {
    (void)hipSetDevice(c->impl.device);
    (void)hipStreamSynchronize(c->impl.stream);
    c->impl.cached.reset();
    if (c->impl.own_stream) (void)hipStreamDestroy(c->impl.stream);
    delete c;
}

namespace reann {
void ctx_acquire(Ctx *c) {
    std::lock_guard<std::mutex> lk(g_ctx_mu);
    ++c->users;
}
void ctx_release(Ctx *c) {
    bool destroy = false;
    {
        std::lock_guard<std::mutex> lk(g_ctx_mu);
        destroy = --c->users == 0 && c->released;
    }
    if (destroy) ctx_destroy(reinterpret_cast<reann_ctx *>(c));
}
}  // namespace reann

extern "C" {

const char *reann_last_error(void) { return g_last_error.c_str(); }

reann_status reann_model_create(const reann_model_desc *d, reann_model **out) {
    return guarded([&] {
        REQUIRE(d && out, "NULL argument");
        REQUIRE(d->n_species >= 1 && d->n_species <= 64, "n_species must be in [1, 64]");
        REQUIRE(d->L >= 0 && d->K >= 1, "bad L or K");
        REQUIRE(d->form == REANN_FORM_REANN || d->form == REANN_FORM_RADIAL || d->form == REANN_FORM_DIAG,
                "unknown message form");
        const bool radial = d->form == REANN_FORM_RADIAL;
        REQUIRE(radial == (d->L == 0), "the radial form takes L = 0, the other forms L >= 1");
        const bool lk_ok = radial ? (d->K == 8 || d->K == 12)
                                  : ((d->L == 2 && (d->K == 8 || d->K == 12 || d->K == 4)) || (d->L == 1 && d->K == 4));
        if (!lk_ok) fail(REANN_E_UNSUPPORTED, "no kernels compiled for this (L, K)");
        REQUIRE(d->T_max >= 1 && d->T_max <= 16, "T_max must be in [1, 16]");
        REQUIRE(d->n_hidden >= 1 && d->n_hidden <= 4, "n_hidden must be in [1, 4]");
        REQUIRE(d->hidden >= 1 && d->hidden <= 256, "hidden must be in [1, 256]");
        REQUIRE(d->r_c > 0 && std::isfinite(d->r_c), "r_c must be > 0");
        REQUIRE(std::isfinite(d->ang_scale) && std::isfinite(d->energy_scale), "non-finite scale");
        REQUIRE(d->centres && d->alphas && d->c0 && d->en, "NULL parameter array");
        REQUIRE(d->T_max == 1 || d->msg, "message NN parameters required for T_max > 1");
        auto *m = new reann_model();
        Model &M = m->impl;
        M.n_species = d->n_species; M.L = d->L; M.K = d->K; M.T_max = d->T_max;
        M.nh = d->n_hidden; M.H = d->hidden;
        M.form = d->form;
        M.F = radial ? d->K : (d->form == REANN_FORM_DIAG ? (d->L + 1) * d->K : n_feat(d->L, d->K));
        M.NL = n_lambda(d->L);
        M.r_c = d->r_c; M.ang_scale = d->ang_scale; M.energy_scale = d->energy_scale;
        M.centres.assign(d->centres, d->centres + d->K);
        M.alphas.assign(d->alphas, d->alphas + d->K);
        M.c0.assign(d->c0, d->c0 + (size_t)d->n_species * d->K);
        M.msg_nn = nn_layout(M.F, M.H, M.nh, M.K);
        M.en_nn = nn_layout(M.F, M.H, M.nh, 1);
        const size_t nmsg = (size_t)(d->T_max - 1) * d->n_species * M.msg_nn.size;
        const size_t nen = (size_t)d->n_species * M.en_nn.size;
        if (nmsg) M.msg.assign(d->msg, d->msg + nmsg);
        M.en.assign(d->en, d->en + nen);
        for (double v : M.msg) if (!std::isfinite(v)) { delete m; fail(REANN_E_INVALID, "non-finite weight"); }
        for (double v : M.en) if (!std::isfinite(v)) { delete m; fail(REANN_E_INVALID, "non-finite weight"); }
        *out = m;
    });
}

// ---- model files: a JSON object of scalars next to a raw FP64 weight file ----
namespace {

// Top-level members of a JSON object whose values are numbers or strings (nested values are
// skipped).  Enough for the model spec; anything malformed is reported.
std::map<std::string, std::string> json_scalars(const std::string &t) {
    std::map<std::string, std::string> out;
    size_t i = 0;
    auto ws = [&] { while (i < t.size() && std::isspace((unsigned char)t[i])) ++i; };
    auto str = [&]() -> std::string {
        if (i >= t.size() || t[i] != '"') fail(REANN_E_INVALID, "model spec: string expected");
        std::string v;
        for (++i; i < t.size() && t[i] != '"'; ++i) {
            if (t[i] == '\\' && i + 1 < t.size()) ++i;
            v.push_back(t[i]);
        }
        if (i >= t.size()) fail(REANN_E_INVALID, "model spec: unterminated string");
        ++i;
        return v;
    };
    auto skip_nested = [&] {
        int depth = 0;
        bool in_str = false;
        for (; i < t.size(); ++i) {
            const char c = t[i];
            if (in_str) { if (c == '\\') ++i; else if (c == '"') in_str = false; continue; }
            if (c == '"') in_str = true;
            else if (c == '[' || c == '{') ++depth;
            else if (c == ']' || c == '}') { if (--depth == 0) { ++i; return; } }
        }
        fail(REANN_E_INVALID, "model spec: unbalanced brackets");
    };
    ws();
    if (i >= t.size() || t[i] != '{') fail(REANN_E_INVALID, "model spec: JSON object expected");
    ++i;
    for (;;) {
        ws();
        if (i < t.size() && t[i] == '}') break;
        const std::string key = str();
        ws();
        if (i >= t.size() || t[i] != ':') fail(REANN_E_INVALID, "model spec: ':' expected");
        ++i;
        ws();
        if (i < t.size() && t[i] == '"') {
            out[key] = str();
        } else if (i < t.size() && (t[i] == '[' || t[i] == '{')) {
            skip_nested();
        } else {
            const size_t b = i;
            while (i < t.size() && t[i] != ',' && t[i] != '}' && !std::isspace((unsigned char)t[i])) ++i;
            out[key] = t.substr(b, i - b);
        }
        ws();
        if (i < t.size() && t[i] == ',') { ++i; continue; }
        if (i < t.size() && t[i] == '}') break;
        fail(REANN_E_INVALID, "model spec: ',' or '}' expected");
    }
    return out;
}

size_t nn_doubles(int in, int hidden, int nh, int out) {
    size_t n = 0;
    int prev = in;
    for (int k = 0; k < nh; ++k) { n += (size_t)hidden * prev + hidden; prev = hidden; }
    return n + (size_t)out * prev + out;
}

}  // namespace

reann_status reann_model_load(const char *spec_json_path, reann_model **out) {
    return guarded([&] {
        REQUIRE(spec_json_path && out, "NULL argument");
        std::ifstream f(spec_json_path);
        if (!f) fail(REANN_E_INVALID, std::string("cannot open model spec ") + spec_json_path);
        std::stringstream ss;
        ss << f.rdbuf();
        const auto kv = json_scalars(ss.str());
        auto get = [&](const char *k) -> const std::string & {
            auto it = kv.find(k);
            if (it == kv.end()) fail(REANN_E_INVALID, std::string("model spec: missing \"") + k + "\"");
            return it->second;
        };
        auto num = [&](const char *k) {
            const std::string &v = get(k);
            char *end = nullptr;
            const double x = std::strtod(v.c_str(), &end);
            if (end == v.c_str() || *end != '\0') fail(REANN_E_INVALID, std::string("model spec: \"") + k + "\" is not a number");
            return x;
        };
        auto integer = [&](const char *k) {
            const double x = num(k);
            if (x != std::floor(x) || std::fabs(x) > 1e9) fail(REANN_E_INVALID, std::string("model spec: \"") + k + "\" is not an integer");
            return (int32_t)x;
        };
        if (get("format") != "reann-model") fail(REANN_E_INVALID, "model spec: \"format\" must be \"reann-model\"");
        if (integer("version") != 1) fail(REANN_E_UNSUPPORTED, "model spec: unsupported version");
        reann_model_desc d{};
        d.n_species = integer("n_species"); d.L = integer("L"); d.K = integer("K"); d.T_max = integer("T_max");
        d.n_hidden = integer("n_hidden"); d.hidden = integer("hidden");
        d.r_c = num("r_c"); d.ang_scale = num("ang_scale"); d.energy_scale = num("energy_scale");
        d.form = REANN_FORM_REANN;
        if (kv.count("form")) {
            const std::string &fm = kv.at("form");
            if (fm == "radial") d.form = REANN_FORM_RADIAL;
            else if (fm == "diag") d.form = REANN_FORM_DIAG;
            else if (fm != "reann") fail(REANN_E_INVALID, "model spec: \"form\" must be \"reann\", \"radial\" or \"diag\"");
        }
        REQUIRE(d.n_species >= 1 && d.n_species <= 64 && d.K >= 1 && d.K <= 64 && d.L >= 0 && d.L <= 4 &&
                    d.T_max >= 1 && d.T_max <= 16 && d.n_hidden >= 1 && d.n_hidden <= 4 && d.hidden >= 1 &&
                    d.hidden <= 256,
                "model spec: dimension out of range");
        // weight file: relative paths are taken from the spec's directory
        std::string wpath = get("weights");
        const std::string sp(spec_json_path);
        const size_t slash = sp.find_last_of('/');
        if (!wpath.empty() && wpath[0] != '/' && slash != std::string::npos) wpath = sp.substr(0, slash + 1) + wpath;
        const int F = d.form == REANN_FORM_RADIAL ? d.K : (d.form == REANN_FORM_DIAG ? (d.L + 1) * d.K : n_feat(d.L, d.K));
        const size_t nmsg = (size_t)(d.T_max - 1) * d.n_species * nn_doubles(F, d.hidden, d.n_hidden, d.K);
        const size_t nen = (size_t)d.n_species * nn_doubles(F, d.hidden, d.n_hidden, 1);
        const size_t total = 2 * (size_t)d.K + (size_t)d.n_species * d.K + nmsg + nen;
        std::ifstream w(wpath, std::ios::binary | std::ios::ate);
        if (!w) fail(REANN_E_INVALID, "cannot open model weights " + wpath);
        const std::streamoff bytes = w.tellg();
        if (bytes != (std::streamoff)(total * 8))
            fail(REANN_E_INVALID, "model weights: " + std::to_string((long long)bytes) + " bytes, expected " +
                                      std::to_string((unsigned long long)(total * 8)));
        std::vector<double> buf(total);
        w.seekg(0);
        if (!w.read(reinterpret_cast<char *>(buf.data()), (std::streamsize)(total * 8)))
            fail(REANN_E_INVALID, "model weights: read failed");
        const double *q = buf.data();
        d.centres = q; q += d.K;
        d.alphas = q; q += d.K;
        d.c0 = q; q += (size_t)d.n_species * d.K;
        d.msg = nmsg ? q : nullptr; q += nmsg;
        d.en = q;
        const reann_status st = reann_model_create(&d, out);
        if (st != REANN_OK) throw Error(st, reann_last_error());
    });
}

void reann_model_free(reann_model *m) { delete m; }

reann_status reann_ctx_create(int32_t device, void *hip_stream, reann_ctx **out) {
    return guarded([&] {
        REQUIRE(out, "NULL argument");
        int nd = 0;
        HIP_OK(hipGetDeviceCount(&nd));
        REQUIRE(device >= 0 && device < nd, "device index out of range");
        HIP_OK(hipSetDevice(device));
        auto *c = new reann_ctx();
        c->impl.device = device;
        if (hip_stream) {
            c->impl.stream = (hipStream_t)hip_stream;
        } else {
            hipError_t e = hipStreamCreateWithFlags(&c->impl.stream, hipStreamNonBlocking);
            if (e != hipSuccess) { delete c; HIP_OK(e); }
            c->impl.own_stream = true;
        }
        *out = c;
    });
}


void reann_ctx_free(reann_ctx *c) {
    if (!c) return;
    bool destroy = false;
    {
        std::lock_guard<std::mutex> lk(g_ctx_mu);
        c->impl.released = true;
        destroy = c->impl.users == 0;
    }
    if (destroy) ctx_destroy(c);
}

// ------------------------------------------------------------------ nlist --

struct reann_nlist {
    Plan plan;   // geometry and neighbour list only; no model attached
    Ctx *owner = nullptr;
    ~reann_nlist() {
        if (owner) ctx_release(owner);
    }
};

reann_status reann_build_neighbors(reann_ctx *ctx, const double *pos, int64_t n, const double cell[9],
                                   const int32_t pbc[3], double r_c, double skin, const int32_t decomp[3],
                                   reann_nlist **out) {
    return guarded([&] {
        REQUIRE(ctx && pos && out, "NULL argument");
        REQUIRE(n > 0, "n must be > 0");
        REQUIRE(r_c > 0 && std::isfinite(r_c), "r_c must be > 0");
        REQUIRE(skin >= 0 && std::isfinite(skin), "skin must be >= 0");
        check_cell(cell, pbc);
        check_positions(pos, n);
        HIP_OK(hipSetDevice(ctx->impl.device));
        auto *nl = new reann_nlist();
        ctx_acquire(&ctx->impl);
        nl->owner = &ctx->impl;
        try {
            Plan &p = nl->plan;
            p.ctx = &ctx->impl;
            p.n = n;
            int32_t P[3] = {1, 1, 1};
            if (decomp)
                for (int a = 0; a < 3; ++a) P[a] = decomp[a] > 0 ? decomp[a] : 1;
            geom_init(p.g, cell, pbc, P, r_c, skin);
            hipStream_t st = ctx->impl.stream;
            DevBuf dpos;
            dpos.ensure(n * 24);
            HIP_OK(hipMemcpyAsync(dpos.p, pos, n * 24, hipMemcpyHostToDevice, st));
            int32_t *ds = p.d_species.resize(n);
            zero(st, ds, n * 4);
            build_nlist(st, dpos.as<double>(), ds, n, 1, p.g, r_c, skin, p.nl, p.ns);
            p.built = true;
        } catch (...) {
            delete nl;
            throw;
        }
        *out = nl;
    });
}

reann_status reann_nlist_info(const reann_nlist *nl, int64_t *n_atoms, int64_t *n_ghosts, int64_t *n_pairs,
                              int64_t *n_local_pairs) {
    return guarded([&] {
        REQUIRE(nl, "NULL list");
        if (n_atoms) *n_atoms = nl->plan.nl.n;
        if (n_ghosts) *n_ghosts = nl->plan.nl.n_gh;
        if (n_pairs) *n_pairs = nl->plan.nl.n_pairs;
        if (n_local_pairs) *n_local_pairs = nl->plan.nl.n_local_pairs;
    });
}

reann_status reann_nlist_export(const reann_nlist *nlh, int64_t *n_pairs, int64_t *row, int64_t *j, int32_t *shift) {
    return guarded([&] {
        REQUIRE(nlh && n_pairs, "NULL argument");
        const NList &nl = nlh->plan.nl;
        const int64_t n = nl.n;
        if (!row) { *n_pairs = nl.n_local_pairs; return; }
        REQUIRE(j && shift, "NULL output array");
        HIP_OK(hipDeviceSynchronize());
        std::vector<int64_t> r(n + 1);
        std::vector<int32_t> col(std::max<int64_t>(nl.n_local_pairs, 1)), perm(n),
            owner(std::max<int64_t>(nl.n_gh, 1)), sh(std::max<int64_t>(nl.n_gh, 1) * 3);
        HIP_OK(hipMemcpy(r.data(), nl.row.ptr(), (n + 1) * 8, hipMemcpyDeviceToHost));
        if (nl.n_local_pairs) HIP_OK(hipMemcpy(col.data(), nl.col.ptr(), nl.n_local_pairs * 4, hipMemcpyDeviceToHost));
        HIP_OK(hipMemcpy(perm.data(), nl.perm.ptr(), n * 4, hipMemcpyDeviceToHost));
        if (nl.n_gh) {
            HIP_OK(hipMemcpy(owner.data(), nl.gh_owner.ptr(), nl.n_gh * 4, hipMemcpyDeviceToHost));
            HIP_OK(hipMemcpy(sh.data(), nl.gh_shift.ptr(), nl.n_gh * 12, hipMemcpyDeviceToHost));
        }
        std::vector<int32_t> inv(n);
        for (int64_t i = 0; i < n; ++i) inv[perm[i]] = (int32_t)i;
        struct E { int64_t j; int32_t s[3]; };
        int64_t o = 0;
        row[0] = 0;
        std::vector<E> buf;
        for (int64_t u = 0; u < n; ++u) {
            const int64_t x = inv[u];
            buf.clear();
            for (int64_t k = r[x]; k < r[x + 1]; ++k) {
                const int64_t e = col[k];
                E v;
                if (e < n) { v.j = perm[e]; v.s[0] = v.s[1] = v.s[2] = 0; }
                else {
                    const int64_t g = e - n;
                    v.j = perm[owner[g]];
                    for (int a = 0; a < 3; ++a) v.s[a] = sh[3 * g + a];
                }
                buf.push_back(v);
            }
            std::sort(buf.begin(), buf.end(), [](const E &a, const E &b) {
                if (a.j != b.j) return a.j < b.j;
                for (int q = 0; q < 3; ++q) if (a.s[q] != b.s[q]) return a.s[q] < b.s[q];
                return false;
            });
            for (const E &v : buf) {
                j[o] = v.j;
                for (int a = 0; a < 3; ++a) shift[3 * o + a] = v.s[a];
                ++o;
            }
            row[u + 1] = o;
        }
        *n_pairs = o;
    });
}

void reann_nlist_free(reann_nlist *nl) { delete nl; }

// ------------------------------------------------------------- evaluation --

static void check_eval_args(const reann_model *m, const double *pos, const int32_t *species, int64_t n,
                            const double *cell, const int32_t *pbc, int32_t T, const reann_opts *opt) {
    REQUIRE(m && species, "NULL argument");
    REQUIRE(n > 0, "n must be > 0");
    check_cell(cell, pbc);
    if (pos) check_positions(pos, n);
    REQUIRE(T >= 1 && T <= m->impl.T_max, "T must be in [1, T_max]");
    for (int64_t i = 0; i < n; ++i)
        REQUIRE(species[i] >= 0 && species[i] < m->impl.n_species, "species out of range");
    if (opt) {
        REQUIRE(opt->skin >= 0 && std::isfinite(opt->skin), "skin must be >= 0");
        if (opt->precision != REANN_FP64 && opt->precision != REANN_FP32 && opt->precision != REANN_BF16 &&
            opt->precision != REANN_FP8)
            fail(REANN_E_INVALID, "unknown precision");
    }
}

reann_status reann_energy_forces(reann_ctx *ctx, const reann_model *m, const double *pos, const int32_t *species,
                                 int64_t n, const double cell[9], const int32_t pbc[3], double r_c, int32_t T,
                                 const reann_opts *opt, double *energy, double *forces, double *virial) {
    return guarded([&] {
        REQUIRE(ctx && pos && energy, "NULL argument");
        check_eval_args(m, pos, species, n, cell, pbc, T, opt);
        REQUIRE(r_c == m->impl.r_c, "r_c must equal the model's cutoff");
        Ctx &c = ctx->impl;
        HIP_OK(hipSetDevice(c.device));
        if (!c.cached || !c.cached->same_system(&m->impl, species, n, cell, pbc, T, opt)) {
            c.cached.reset();
            auto p = std::make_unique<Plan>();
            p->init(&c, const_cast<Model *>(&m->impl), species, n, cell, pbc, T, opt);
            c.cached = std::move(p);
        }
        Plan &p = *c.cached;
        hipStream_t st = c.stream;
        double *dpos = static_cast<double *>(c.pos.ensure(n * 24));
        double *dF = static_cast<double *>(c.forces.ensure(n * 24));
        double *dsc = static_cast<double *>(c.scal.ensure(16 * 8));
        HIP_OK(hipMemcpyAsync(dpos, pos, n * 24, hipMemcpyHostToDevice, st));
        p.forward(dpos, dsc, nullptr, st);
        if (forces || virial) p.backward(nullptr, dF, dsc + 1, st);
        double h[10];
        HIP_OK(hipMemcpyAsync(h, dsc, 10 * 8, hipMemcpyDeviceToHost, st));
        if (forces) HIP_OK(hipMemcpyAsync(forces, dF, n * 24, hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
        *energy = h[0];
        if (virial) std::memcpy(virial, h + 1, 9 * 8);
    });
}

// ---------------------------------------------------------- allocation-free --
// Device memory of reann_energy_forces_noalloc: one static array per GPU, held from the load of
// the library's code object on that GPU until the process ends.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
struct ScratchSlot {
    std::mutex mu;            // one call at a time per GPU: every call shares the array
    char *ptr = nullptr;      // device address of `scratch` on this GPU
};
std::mutex g_scratch_mu;
std::map<int, std::unique_ptr<ScratchSlot>> g_scratch;

// The slot of `device` (current device), resolving the array's device address on the first
// call for that device.  In host code `scratch` names a host-side stand-in, never usable as a
// device address: every kernel and copy gets `ptr`.
ScratchSlot &scratch_slot(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto &slot = g_scratch[device];
    if (!slot) {
        auto s = std::make_unique<ScratchSlot>();
        void *p = nullptr;
        HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) fail(REANN_E_DEVICE, "no device address for the static scratch array");
        s->ptr = static_cast<char *>(p);
        slot = std::move(s);
    }
    return *slot;
}

// Installs an arena over the scratch for the current thread; uninstalls it on scope exit.
struct ArenaScope {
    Arena a;
    ArenaScope(char *base, size_t cap) { a.base = base; a.cap = cap; a.used = 0; current_arena() = &a; }
    ~ArenaScope() { current_arena() = nullptr; }
};
}  // namespace

reann_status reann_energy_forces_noalloc(reann_ctx *ctx, const reann_model *m, const double *pos,
                                         const int32_t *species, int64_t n, const double cell[9], const int32_t pbc[3],
                                         double r_c, int32_t T, const reann_opts *opt, double *energy, double *forces,
                                         double *virial) {
    return guarded([&] {
        REQUIRE(ctx && pos && energy, "NULL argument");
        check_eval_args(m, pos, species, n, cell, pbc, T, opt);
        REQUIRE(r_c == m->impl.r_c, "r_c must equal the model's cutoff");
        Ctx &c = ctx->impl;
        HIP_OK(hipSetDevice(c.device));
        const int prec = opt ? opt->precision : REANN_FP32;
        if (!const_cast<Model &>(m->impl).on_device(c.device, prec))
            fail(REANN_E_STATE, "reann_energy_forces_noalloc: the model's weights are not on this GPU at this "
                                "precision yet (run one reann_energy_forces or reann_plan_create with the same model, "
                                "GPU and precision first; those allocate them)");
        ScratchSlot &slot = scratch_slot(c.device);
        std::lock_guard<std::mutex> lk(slot.mu);
        hipStream_t st = c.stream;
        try {
            ArenaScope arena(slot.ptr, kScratchBytes);
            Plan p;   // every device buffer below comes from the arena
            p.init(&c, const_cast<Model *>(&m->impl), species, n, cell, pbc, T, opt);
            DevBuf bpos, bF, bsc;
            double *dpos = static_cast<double *>(bpos.ensure(n * 24));
            double *dF = static_cast<double *>(bF.ensure(n * 24));
            double *dsc = static_cast<double *>(bsc.ensure(16 * 8));
            HIP_OK(hipMemcpyAsync(dpos, pos, n * 24, hipMemcpyHostToDevice, st));
            p.forward(dpos, dsc, nullptr, st);
            if (forces || virial) p.backward(nullptr, dF, dsc + 1, st);
            double h[10];
            HIP_OK(hipMemcpyAsync(h, dsc, 10 * 8, hipMemcpyDeviceToHost, st));
            if (forces) HIP_OK(hipMemcpyAsync(forces, dF, n * 24, hipMemcpyDeviceToHost, st));
            HIP_OK(hipStreamSynchronize(st));
            *energy = h[0];
            if (virial) std::memcpy(virial, h + 1, 9 * 8);
        } catch (...) {
            // work already queued may still write the scratch: drain it before the next call
            (void)hipStreamSynchronize(st);
            throw;
        }
    });
}

reann_status reann_plan_create(reann_ctx *ctx, const reann_model *m, const int32_t *species, int64_t n,
                               const double cell[9], const int32_t pbc[3], int32_t T, const reann_opts *opt,
                               reann_plan **out) {
    return guarded([&] {
        REQUIRE(ctx && out, "NULL argument");
        check_eval_args(m, nullptr, species, n, cell, pbc, T, opt);
        HIP_OK(hipSetDevice(ctx->impl.device));
        auto *p = new reann_plan();
        try {
            p->impl.init(&ctx->impl, const_cast<Model *>(&m->impl), species, n, cell, pbc, T, opt);
        } catch (...) {
            delete p;
            throw;
        }
        ctx_acquire(&ctx->impl);
        *out = p;
    });
}

reann_status reann_plan_forward(reann_plan *p, const double *d_pos, double *d_energy, double *d_atom_energy,
                                void *hip_stream) {
    return guarded([&] {
        REQUIRE(p && d_pos && d_energy, "NULL argument");
        HIP_OK(hipSetDevice(p->impl.ctx->device));
        p->impl.forward(d_pos, d_energy, d_atom_energy, (hipStream_t)hip_stream);
    });
}

reann_status reann_plan_backward(reann_plan *p, const double *d_grad_energy, double *d_forces, double *d_virial,
                                 void *hip_stream) {
    return guarded([&] {
        REQUIRE(p && d_forces, "NULL argument");
        HIP_OK(hipSetDevice(p->impl.ctx->device));
        p->impl.backward(d_grad_energy, d_forces, d_virial, (hipStream_t)hip_stream);
    });
}

reann_status reann_forward_dev(reann_plan *p, const double *d_pos, double *d_energy, void *hip_stream) {
    return reann_plan_forward(p, d_pos, d_energy, nullptr, hip_stream);
}

reann_status reann_backward_dev(reann_plan *p, const double *d_grad_energy, double *d_forces, double *d_virial,
                                void *hip_stream) {
    return reann_plan_backward(p, d_grad_energy, d_forces, d_virial, hip_stream);
}

reann_status reann_plan_get(reann_plan *p, int32_t what, int32_t t, double *host_out) {
    return guarded([&] {
        REQUIRE(p && host_out, "NULL argument");
        HIP_OK(hipSetDevice(p->impl.ctx->device));
        p->impl.get(what, t, host_out);
    });
}

reann_status reann_plan_set_list_policy(reann_plan *p, int32_t auto_check) {
    return guarded([&] {
        REQUIRE(p, "NULL argument");
        REQUIRE(auto_check == 0 || auto_check == 1, "auto_check must be 0 or 1");
        p->impl.auto_list = auto_check != 0;
    });
}

reann_status reann_plan_update_list(reann_plan *p, const double *d_pos, void *hip_stream, int32_t *rebuilt) {
    return guarded([&] {
        REQUIRE(p && d_pos, "NULL argument");
        HIP_OK(hipSetDevice(p->impl.ctx->device));
        const bool r = p->impl.prepare(d_pos, (hipStream_t)hip_stream);
        if (rebuilt) *rebuilt = r ? 1 : 0;
    });
}

reann_status reann_plan_set_energy_weights(reann_plan *p, const double *w) {
    return guarded([&] {
        REQUIRE(p, "NULL argument");
        Plan &P = p->impl;
        HIP_OK(hipSetDevice(P.ctx->device));
        if (!w) {
            P.have_ew = false;
            return;
        }
        for (int64_t i = 0; i < P.n; ++i) REQUIRE(std::isfinite(w[i]), "non-finite energy weight");
        double *d = P.d_ew.resize(P.n);
        HIP_OK(hipMemcpyAsync(d, w, P.n * 8, hipMemcpyHostToDevice, P.ctx->stream));
        HIP_OK(hipStreamSynchronize(P.ctx->stream));
        P.have_ew = true;
    });
}

reann_status reann_plan_generation(const reann_plan *p, uint64_t *gen) {
    return guarded([&] {
        REQUIRE(p && gen, "NULL argument");
        *gen = p->impl.generation;
    });
}

reann_status reann_plan_set_timing(reann_plan *p, int32_t enable) {
    return guarded([&] {
        REQUIRE(p, "NULL argument");
        p->impl.timing = enable != 0;
    });
}

reann_status reann_plan_timing(reann_plan *p, double *ms, int64_t *launches, int64_t *steps) {
    return guarded([&] {
        REQUIRE(p && ms, "NULL argument");
        HIP_OK(hipSetDevice(p->impl.ctx->device));
        const int64_t s = p->impl.collect_timing(ms, launches);
        if (steps) *steps = s;
    });
}

void reann_plan_free(reann_plan *p) {
    if (!p) return;
    Ctx *c = p->impl.ctx;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();   // its work may sit on any stream the caller passed
    delete p;
    ctx_release(c);
}

}  // extern "C"

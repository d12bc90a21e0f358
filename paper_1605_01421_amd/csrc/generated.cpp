// generated.cpp -- models defined by transition strings (section 5.1): each
// "X -> propensity -> Y" is parsed, the state-change matrix S and the
// dependency graph G are derived from it, a device model type is generated
// from the propensities, and the kernels are compiled for that type at run
// time with hipRTC from the kernel sources built into this library (the
// counterpart of the paper's generated C compiled into a shared library).
//
// Expression language of a propensity: numbers, the names of compartments,
// of global data, of local data and of continuous state variables, the
// operators + - * / (binary, left-associative, * and / binding tighter) and
// unary - and +, and parentheses.  Every value is taken as binary64 and every
// operation is one IEEE operation in the order of the parse tree, so any
// other implementation that evaluates the same tree gets the same bits.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "models.h"
#include "siminf.h"

namespace siminf {

namespace {

// the kernel sources compiled into the library by the build (the device
// part of ssa_kernels.hip and the headers it includes)
#include "rtc_sources.inc"

struct Node {
    enum Kind { NUM, U, GD, LD, V, ADD, SUB, MUL, DIV, NEG } k;
    double v = 0.0;
    int idx = 0, a = -1, b = -1;
};

struct Names {
    std::map<std::string, std::pair<Node::Kind, int>> table;
};

// Recursive-descent parser of one propensity into nodes[]; returns the root
// index, or -1 with a message.
class Parser {
  public:
    Parser(const std::string& text, const Names& names, std::vector<Node>& out)
        : s_(text), names_(names), out_(out) {}
    int parse(std::string& err) {
        pos_ = 0;
        const int r = expr(err);
        if (r < 0) return -1;
        skip();
        if (pos_ != s_.size()) {
            err = "unexpected '" + s_.substr(pos_, 1) + "' in '" + s_ + "'";
            return -1;
        }
        return r;
    }

  private:
    void skip() {
        while (pos_ < s_.size() && std::isspace((unsigned char)s_[pos_])) ++pos_;
    }
    int add(Node n) {
        out_.push_back(n);
        return (int)out_.size() - 1;
    }
    int expr(std::string& err) {
        int l = term(err);
        if (l < 0) return -1;
        for (;;) {
            skip();
            if (pos_ < s_.size() && (s_[pos_] == '+' || s_[pos_] == '-')) {
                const char op = s_[pos_++];
                const int r = term(err);
                if (r < 0) return -1;
                Node n{op == '+' ? Node::ADD : Node::SUB};
                n.a = l;
                n.b = r;
                l = add(n);
            } else {
                return l;
            }
        }
    }
    int term(std::string& err) {
        int l = unary(err);
        if (l < 0) return -1;
        for (;;) {
            skip();
            if (pos_ < s_.size() && (s_[pos_] == '*' || s_[pos_] == '/')) {
                const char op = s_[pos_++];
                const int r = unary(err);
                if (r < 0) return -1;
                Node n{op == '*' ? Node::MUL : Node::DIV};
                n.a = l;
                n.b = r;
                l = add(n);
            } else {
                return l;
            }
        }
    }
    int unary(std::string& err) {
        skip();
        if (pos_ < s_.size() && (s_[pos_] == '-' || s_[pos_] == '+')) {
            const char op = s_[pos_++];
            const int x = unary(err);
            if (x < 0) return -1;
            if (op == '+') return x;
            Node n{Node::NEG};
            n.a = x;
            return add(n);
        }
        return primary(err);
    }
    int primary(std::string& err) {
        skip();
        if (pos_ >= s_.size()) {
            err = "expression ends early in '" + s_ + "'";
            return -1;
        }
        const char c = s_[pos_];
        if (c == '(') {
            ++pos_;
            const int x = expr(err);
            if (x < 0) return -1;
            skip();
            if (pos_ >= s_.size() || s_[pos_] != ')') {
                err = "missing ')' in '" + s_ + "'";
                return -1;
            }
            ++pos_;
            return x;
        }
        if (std::isdigit((unsigned char)c) || c == '.') {
            // a decimal literal: digits, an optional fraction, an optional exponent
            size_t e = pos_;
            while (e < s_.size() && std::isdigit((unsigned char)s_[e])) ++e;
            if (e < s_.size() && s_[e] == '.') {
                ++e;
                while (e < s_.size() && std::isdigit((unsigned char)s_[e])) ++e;
            }
            if (e < s_.size() && (s_[e] == 'e' || s_[e] == 'E')) {
                size_t f = e + 1;
                if (f < s_.size() && (s_[f] == '+' || s_[f] == '-')) ++f;
                if (f < s_.size() && std::isdigit((unsigned char)s_[f])) {
                    e = f;
                    while (e < s_.size() && std::isdigit((unsigned char)s_[e])) ++e;
                }
            }
            const std::string lit = s_.substr(pos_, e - pos_);
            if (!std::isdigit((unsigned char)lit[0]) && !(lit.size() > 1 && std::isdigit((unsigned char)lit[1]))) {
                err = "bad number in '" + s_ + "'";
                return -1;
            }
            Node n{Node::NUM};
            n.v = std::strtod(lit.c_str(), nullptr);  // correctly rounded
            if (!std::isfinite(n.v)) {
                err = "number out of range: " + lit;
                return -1;
            }
            pos_ = e;
            return add(n);
        }
        if (std::isalpha((unsigned char)c) || c == '_') {
            size_t e = pos_;
            while (e < s_.size() && (std::isalnum((unsigned char)s_[e]) || s_[e] == '_')) ++e;
            const std::string name = s_.substr(pos_, e - pos_);
            auto it = names_.table.find(name);
            if (it == names_.table.end()) {
                err = "unknown name '" + name + "' in '" + s_ + "'";
                return -1;
            }
            pos_ = e;
            Node n{it->second.first};
            n.idx = it->second.second;
            return add(n);
        }
        err = "unexpected '" + std::string(1, c) + "' in '" + s_ + "'";
        return -1;
    }

    const std::string& s_;
    const Names& names_;
    std::vector<Node>& out_;
    size_t pos_ = 0;
};

// C++ text of a parsed expression: fully parenthesised, every leaf binary64
std::string emit(const std::vector<Node>& t, int i) {
    const Node& n = t[i];
    char buf[64];
    switch (n.k) {
        case Node::NUM: std::snprintf(buf, sizeof buf, "%a", n.v); return buf;
        case Node::U: return "(double)u[" + std::to_string(n.idx) + "]";
        case Node::GD: return "gd[" + std::to_string(n.idx) + "]";
        case Node::LD: return "ld[" + std::to_string(n.idx) + "]";
        case Node::V: return "v[" + std::to_string(n.idx) + "]";
        case Node::NEG: return "(-" + emit(t, n.a) + ")";
        default: break;
    }
    const char* op = n.k == Node::ADD ? " + " : n.k == Node::SUB ? " - " : n.k == Node::MUL ? " * " : " / ";
    return "(" + emit(t, n.a) + op + emit(t, n.b) + ")";
}

void compartments_used(const std::vector<Node>& t, int i, std::vector<char>& used) {
    const Node& n = t[i];
    if (n.k == Node::U) used[n.idx] = 1;
    if (n.a >= 0) compartments_used(t, n.a, used);
    if (n.b >= 0) compartments_used(t, n.b, used);
}

std::string trim(const std::string& x) {
    size_t a = 0, b = x.size();
    while (a < b && std::isspace((unsigned char)x[a])) ++a;
    while (b > a && std::isspace((unsigned char)x[b - 1])) --b;
    return x.substr(a, b - a);
}

// One side of a transition: "@" (the empty set) or terms "X" / "k*X" joined
// by '+'; adds the counts to cnt.
bool parse_side(const std::string& side, const std::map<std::string, int>& comp, std::vector<int>& cnt,
                std::string& err) {
    const std::string s = trim(side);
    if (s == "@") return true;
    size_t start = 0;
    for (;;) {
        const size_t plus = s.find('+', start);
        std::string term = trim(s.substr(start, plus == std::string::npos ? std::string::npos : plus - start));
        int k = 1;
        const size_t star = term.find('*');
        if (star != std::string::npos) {
            const std::string num = trim(term.substr(0, star));
            char* end = nullptr;
            const long v = std::strtol(num.c_str(), &end, 10);
            if (num.empty() || *end != '\0' || v < 1 || v > 1000000) {
                err = "bad coefficient in '" + side + "'";
                return false;
            }
            k = (int)v;
            term = trim(term.substr(star + 1));
        }
        auto it = comp.find(term);
        if (it == comp.end()) {
            err = "unknown compartment '" + term + "' in '" + side + "'";
            return false;
        }
        cnt[it->second] += k;
        if (plus == std::string::npos) return true;
        start = plus + 1;
    }
}

struct DeviceModule {
    hipModule_t mod = nullptr;
    hipFunction_t fn[3][3] = {};  // [mode: free, barrier, dataflow][direct, pipelined direct, all events]
};

struct Generated {
    int id = 0;
    ModelShape shape{};
    std::vector<int32_t> S, G, E, N;  // column-major, as in siminf_spec
    int ecols = 0, ncols = 0;
    std::string source;
    std::vector<char> code;
    std::string lowered[3][3];
    std::map<int, DeviceModule> per_device;
};

std::mutex g_mu;         // the registry
std::mutex g_define_mu;  // one definition at a time (ids are handed out in order)
std::vector<std::unique_ptr<Generated>> g_models;

const char* const KERNEL_EXPR[3][3] = {
    {"siminf::free_kernel<siminf::ModelGen, false, false, false>", "siminf::free_kernel<siminf::ModelGen, true, false, false>",
     "siminf::free_kernel<siminf::ModelGen, false, false, true>"},
    {"siminf::sync_kernel<siminf::ModelGen, false, false>", "siminf::sync_kernel<siminf::ModelGen, true, false>",
     "siminf::sync_kernel<siminf::ModelGen, false, true>"},
    {"siminf::flow_kernel<siminf::ModelGen, false, false, false>", "siminf::flow_kernel<siminf::ModelGen, true, false, false>",
     "siminf::flow_kernel<siminf::ModelGen, false, false, true>"},
};

void put_message(char* msg, size_t cap, const std::string& text) {
    if (!msg || cap == 0) return;
    std::snprintf(msg, cap, "%s", text.c_str());
}

int mode_slot(int mode) { return mode == MODE_FREE ? 0 : mode == MODE_BARRIER ? 1 : 2; }

Generated* find(int id) {
    for (auto& g : g_models)
        if (g->id == id) return g.get();
    return nullptr;
}

// The module of a generated model on the current device (loaded on first use).
DeviceModule* module_on_device(Generated* g) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    auto it = g->per_device.find(dev);
    if (it != g->per_device.end()) return &it->second;
    DeviceModule dm;
    if (hipModuleLoadData(&dm.mod, g->code.data()) != hipSuccess) return nullptr;
    for (int m = 0; m < 3; ++m)
        for (int q = 0; q < 3; ++q)
            if (hipModuleGetFunction(&dm.fn[m][q], dm.mod, g->lowered[m][q].c_str()) != hipSuccess) {
                (void)hipModuleUnload(dm.mod);
                return nullptr;
            }
    return &(g->per_device[dev] = dm);
}

}  // namespace

bool generated_shape(int id, ModelShape* s) {
    std::lock_guard<std::mutex> lk(g_mu);
    Generated* g = find(id);
    if (!g) return false;
    *s = g->shape;
    return true;
}

int generated_check_spec(const siminf_spec& s) {
    std::lock_guard<std::mutex> lk(g_mu);
    Generated* g = find(s.model);
    if (!g) return SIMINF_E_UNSUPPORTED;
    const int nc = g->shape.nc, nt = g->shape.nt;
    for (int i = 0; i < nc * nt; ++i)
        if (s.S[i] != g->S[i]) return SIMINF_E_ARG;
    for (int i = 0; i < nt * nt; ++i)
        if ((s.G[i] != 0) != (g->G[i] != 0)) return SIMINF_E_ARG;
    // the event tables are compiled into the model
    if (s.Nev > 0) {
        if (s.Ecols != g->ecols || s.Ncols != g->ncols) return SIMINF_E_ARG;
        for (int i = 0; i < nc * g->ecols; ++i)
            if ((s.E[i] != 0) != (g->E[i] != 0)) return SIMINF_E_ARG;
        for (int i = 0; i < nc * g->ncols; ++i)
            if (s.N[i] != g->N[i]) return SIMINF_E_ARG;
    }
    return SIMINF_OK;
}

hipError_t generated_launch(int id, const KParams& p, int block, int blocks, size_t shmem, hipStream_t st) {
    DeviceModule* dm = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        Generated* g = find(id);
        if (!g) return hipErrorInvalidValue;
        dm = module_on_device(g);
    }
    if (!dm) return hipErrorInvalidImage;
    hipFunction_t fn = dm->fn[mode_slot(p.mode)][p.solver == 1 ? 2 : p.pipeline ? 1 : 0];
    KParams arg = p;
    void* args[] = {&arg};
    if (p.mode == MODE_FREE)
        return hipModuleLaunchKernel(fn, (unsigned)blocks, 1, 1, (unsigned)block, 1, 1, (unsigned)shmem, st, args,
                                     nullptr);
    return hipModuleLaunchCooperativeKernel(fn, (unsigned)blocks, 1, 1, (unsigned)block, 1, 1, (unsigned)shmem, st,
                                            args);
}

int generated_blocks_per_cu(int id, int mode, int pipeline, int block, size_t shmem, bool aem) {
    std::lock_guard<std::mutex> lk(g_mu);
    Generated* g = find(id);
    if (!g) return 0;
    DeviceModule* dm = module_on_device(g);
    if (!dm) return 0;
    int n = 0;
    if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&n, dm->fn[mode_slot(mode)][aem ? 2 : pipeline ? 1 : 0],
                                                           block, shmem) != hipSuccess)
        return 0;
    return n;
}

}  // namespace siminf

using namespace siminf;

extern "C" int siminf_define_model(const siminf_model_def* def, int32_t* model_id, int32_t* S_out, int32_t* G_out,
                                   char* msg, size_t msg_cap) {
    if (!def || !model_id) return SIMINF_E_ARG;
    *model_id = -1;
    std::lock_guard<std::mutex> define_lock(g_define_mu);
    const int nc = def->nc, nt = def->nt;
    if (nc < 1 || nc > SIMINF_GEN_MAX_NC || nt < 1 || nt > SIMINF_GEN_MAX_NT || def->ngd < 0 || def->nld < 0 ||
        def->nv < 0 || def->ngd > 64 || def->nld > 64 || def->nv > 16 || def->Ecols < 0 || def->Ncols < 0 ||
        def->Ecols > 1023 || def->Ncols > 1022 || !def->transitions || !def->compartments ||
        (def->ngd > 0 && !def->gdata_names) || (def->nld > 0 && !def->ldata_names) || (def->nv > 0 && !def->v_names) ||
        (def->Ecols > 0 && !def->E) || (def->Ncols > 0 && !def->N)) {
        put_message(msg, msg_cap, "invalid sizes or missing arrays");
        return SIMINF_E_ARG;
    }
    // names: unique across compartments, global data, local data and state
    Names names;
    std::map<std::string, int> comp;
    auto add_names = [&](const char* const* list, int count, Node::Kind kind) -> bool {
        for (int i = 0; i < count; ++i) {
            const std::string nm = list[i] ? list[i] : "";
            bool ok = !nm.empty() && (std::isalpha((unsigned char)nm[0]) || nm[0] == '_');
            for (char ch : nm) ok = ok && (std::isalnum((unsigned char)ch) || ch == '_');
            if (!ok || names.table.count(nm)) {
                put_message(msg, msg_cap, "bad or repeated name '" + nm + "'");
                return false;
            }
            names.table[nm] = {kind, i};
            if (kind == Node::U) comp[nm] = i;
        }
        return true;
    };
    if (!add_names(def->compartments, nc, Node::U) || !add_names(def->gdata_names, def->ngd, Node::GD) ||
        !add_names(def->ldata_names, def->nld, Node::LD) || !add_names(def->v_names, def->nv, Node::V))
        return SIMINF_E_ARG;
    // transitions: "from -> propensity -> to"
    auto gen = std::make_unique<Generated>();
    gen->shape = ModelShape{nc, nt, def->nv, def->nld, def->ngd};
    gen->S.assign((size_t)nc * nt, 0);
    gen->G.assign((size_t)nt * nt, 0);
    std::vector<std::string> rates(nt);
    std::vector<std::vector<char>> uses(nt, std::vector<char>(nc, 0));
    for (int j = 0; j < nt; ++j) {
        const std::string tr = def->transitions[j] ? def->transitions[j] : "";
        const size_t a = tr.find("->");
        const size_t b = a == std::string::npos ? a : tr.find("->", a + 2);
        if (a == std::string::npos || b == std::string::npos || tr.find("->", b + 2) != std::string::npos) {
            put_message(msg, msg_cap, "a transition needs the form 'from -> propensity -> to': '" + tr + "'");
            return SIMINF_E_ARG;
        }
        std::vector<int> from(nc, 0), to(nc, 0);
        std::string err;
        if (!parse_side(tr.substr(0, a), comp, from, err) || !parse_side(tr.substr(b + 2), comp, to, err)) {
            put_message(msg, msg_cap, err);
            return SIMINF_E_ARG;
        }
        for (int c = 0; c < nc; ++c) gen->S[(size_t)j * nc + c] = to[c] - from[c];
        std::vector<Node> tree;
        const std::string prop = trim(tr.substr(a + 2, b - a - 2));
        Parser ps(prop, names, tree);
        const int root = ps.parse(err);
        if (root < 0) {
            put_message(msg, msg_cap, err);
            return SIMINF_E_ARG;
        }
        rates[j] = emit(tree, root);
        compartments_used(tree, root, uses[j]);
    }
    // G: rate k is recomputed after transition j if its propensity reads a
    // compartment that transition j changes
    for (int j = 0; j < nt; ++j)
        for (int k = 0; k < nt; ++k)
            for (int c = 0; c < nc; ++c)
                if (uses[k][c] && gen->S[(size_t)j * nc + c] != 0) gen->G[(size_t)j * nt + k] = 1;
    // event tables; shifts must keep the compartment in range
    gen->ecols = def->Ecols;
    gen->ncols = def->Ncols;
    if (def->Ecols > 0) gen->E.assign(def->E, def->E + (size_t)nc * def->Ecols);
    if (def->Ncols > 0) gen->N.assign(def->N, def->N + (size_t)nc * def->Ncols);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (g_models.size() >= (size_t)(SIMINF_GEN_LAST - SIMINF_GEN_FIRST + 1)) {
            put_message(msg, msg_cap, "too many generated models in this process");
            return SIMINF_E_UNSUPPORTED;
        }
        gen->id = SIMINF_GEN_FIRST + (int)g_models.size();
    }
    // the device model type
    std::string src;
    src += "#include \"models.h\"\nnamespace siminf {\nstruct ModelGen {\n";
    src += "    static constexpr int ID = " + std::to_string(gen->id) + ", NC = " + std::to_string(nc) +
           ", NT = " + std::to_string(nt) + ", NV = " + std::to_string(def->nv) +
           ", NLD = " + std::to_string(def->nld) + ", NGD = " + std::to_string(def->ngd) + ";\n";
    src += "    static constexpr bool COUPLED = false, GENERATED = true;\n";
    src += "    __device__ static __forceinline__ double rate(int j, const int32_t* u, const double* v, "
           "const double* ld, const double* gd) {\n        switch (j) {\n";
    for (int j = 0; j < nt; ++j) src += "        case " + std::to_string(j) + ": return " + rates[j] + ";\n";
    src += "        }\n        return 0.0;\n    }\n";
    src += "    __device__ static __forceinline__ void apply(int n, int32_t* u) {\n        switch (n) {\n";
    for (int j = 0; j < nt; ++j) {
        src += "        case " + std::to_string(j) + ":";
        for (int c = 0; c < nc; ++c) {
            const int d = gen->S[(size_t)j * nc + c];
            if (d) src += " u[" + std::to_string(c) + "] += " + std::to_string(d) + ";";
        }
        src += " break;\n";
    }
    src += "        }\n    }\n";
    src += "    __device__ static __forceinline__ uint32_t deps(int n) {\n        switch (n) {\n";
    for (int j = 0; j < nt; ++j) {
        uint32_t mask = 0;
        for (int k = 0; k < nt; ++k)
            if (gen->G[(size_t)j * nt + k]) mask |= 1u << k;
        src += "        case " + std::to_string(j) + ": return " + std::to_string(mask) + "u;\n";
    }
    src += "        }\n        return 0u;\n    }\n";
    src += "    __device__ static __forceinline__ uint32_t select_mask(int col) {\n        switch (col) {\n";
    for (int q = 0; q < gen->ecols; ++q) {
        uint32_t mask = 0;
        for (int c = 0; c < nc; ++c)
            if (gen->E[(size_t)q * nc + c]) mask |= 1u << c;
        src += "        case " + std::to_string(q) + ": return " + std::to_string(mask) + "u;\n";
    }
    src += "        }\n        return 0u;\n    }\n";
    src += "    __device__ static __forceinline__ int shift_target(int col, int c) {\n        switch (col) {\n";
    for (int q = 0; q < gen->ncols; ++q) {
        src += "        case " + std::to_string(q) + ": switch (c) {";
        for (int c = 0; c < nc; ++c) {
            const int tg = c + gen->N[(size_t)q * nc + c];
            src += " case " + std::to_string(c) + ": return " + std::to_string(tg >= 0 && tg < nc ? tg : c) + ";";
        }
        src += " } break;\n";
    }
    src += "        }\n        return c;\n    }\n";
    src += "    __device__ static __forceinline__ bool pts(double*, const int32_t*, const double*, const double*, "
           "int64_t) { return true; }\n";
    src += "    __device__ static __forceinline__ bool pts_fixed(const double*, const int32_t*) { return true; }\n";
    src += "};\n}  // namespace siminf\n#include \"ssa_kernels.hip\"\n";
    gen->source = src;
    // compile
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "siminf_generated.hip", RTC_COUNT, RTC_TEXTS, RTC_NAMES) !=
        HIPRTC_SUCCESS) {
        put_message(msg, msg_cap, "hiprtcCreateProgram failed");
        return SIMINF_E_DEVICE;
    }
    for (int m = 0; m < 3; ++m)
        for (int q = 0; q < 3; ++q) hiprtcAddNameExpression(prog, KERNEL_EXPR[m][q]);
    const char* opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult rc = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
    if (rc != HIPRTC_SUCCESS) {
        size_t n = 0;
        hiprtcGetProgramLogSize(prog, &n);
        std::string log(n, '\0');
        if (n) hiprtcGetProgramLog(prog, &log[0]);
        put_message(msg, msg_cap, "compilation failed: " + log);
        hiprtcDestroyProgram(&prog);
        return SIMINF_E_DEVICE;
    }
    for (int m = 0; m < 3; ++m)
        for (int q = 0; q < 3; ++q) {
            const char* lowered = nullptr;
            if (hiprtcGetLoweredName(prog, KERNEL_EXPR[m][q], &lowered) != HIPRTC_SUCCESS || !lowered) {
                hiprtcDestroyProgram(&prog);
                put_message(msg, msg_cap, "kernel name lookup failed");
                return SIMINF_E_DEVICE;
            }
            gen->lowered[m][q] = lowered;
        }
    size_t code_size = 0;
    if (hiprtcGetCodeSize(prog, &code_size) != HIPRTC_SUCCESS || code_size == 0) {
        hiprtcDestroyProgram(&prog);
        put_message(msg, msg_cap, "no code object");
        return SIMINF_E_DEVICE;
    }
    gen->code.resize(code_size);
    if (hiprtcGetCode(prog, gen->code.data()) != HIPRTC_SUCCESS) {
        hiprtcDestroyProgram(&prog);
        put_message(msg, msg_cap, "no code object");
        return SIMINF_E_DEVICE;
    }
    hiprtcDestroyProgram(&prog);
    if (S_out) std::memcpy(S_out, gen->S.data(), sizeof(int32_t) * gen->S.size());
    if (G_out) std::memcpy(G_out, gen->G.data(), sizeof(int32_t) * gen->G.size());
    std::lock_guard<std::mutex> lk(g_mu);
    *model_id = gen->id;
    g_models.push_back(std::move(gen));
    put_message(msg, msg_cap, "");
    return SIMINF_OK;
}

extern "C" int siminf_generated_source(int32_t model_id, char* buf, size_t cap, size_t* needed) {
    std::lock_guard<std::mutex> lk(g_mu);
    Generated* g = find(model_id);
    if (!g) return SIMINF_E_ARG;
    if (needed) *needed = g->source.size() + 1;
    if (buf && cap) std::snprintf(buf, cap, "%s", g->source.c_str());
    return SIMINF_OK;
}

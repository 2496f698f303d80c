// Run-time specialisation of the sector integrand (hipRTC).
//
// The table-driven sector functor reads each monomial's factor list from
// wave-uniform memory and dispatches on it with scalar branches; on gfx950
// that dispatch costs more scalar-unit issue than the FP64 work it selects.
// For a single large sector the exponent structure is fixed for the whole
// estimate, so this module writes it out as straight-line FP64 code and
// compiles it once per structure: the monomials of U, F and z^nu become a
// shared-prefix product trie (each trie edge one multiply, each monomial one
// fused multiply-add with its coefficient), followed by the same tail as the
// table-driven functor.  Coefficients and powers are still read from the
// parameter blob, so one compiled kernel serves every coefficient set with
// the same exponents.  The kernel body is the same k_lattice template,
// compiled from the same headers (embedded into the library at build time).
#include <hip/hiprtc.h>

#include <algorithm>
#include <atomic>
#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <iterator>
#include <mutex>
#include <sstream>
#include <unordered_map>

#include <unistd.h>

#include "qmc_jit_headers.inc"
#include "qmc_runtime.hpp"
#include "qmc_cv.hpp"

namespace qmc {

namespace {

struct JitEntry {
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;
    std::string error;  // non-empty when compilation failed
};

std::mutex g_jit_mu;
std::map<std::string, JitEntry> g_jit_cache;

uint64_t word(const std::vector<double> &b, size_t i) {
    uint64_t v;
    std::memcpy(&v, &b[i], sizeof v);
    return v;
}

std::vector<int> factors_of(uint64_t code) {
    std::vector<int> f;
    const uint32_t cnt = (uint32_t)(code & 15u);
    for (uint32_t k = 0; k < cnt; ++k) f.push_back((int)((code >> (4 + 5 * k)) & 31u));
    return f;
}

// product trie over sorted factor lists
struct Trie {
    std::vector<std::pair<int, int>> node;  // (parent, variable); parent -1 = root
    std::map<std::pair<int, int>, int> index;
    int insert(const std::vector<int> &f) {
        int cur = -1;
        for (int v : f) {
            auto key = std::make_pair(cur, v);
            auto it = index.find(key);
            if (it == index.end()) {
                node.push_back(key);
                it = index.emplace(key, (int)node.size() - 1).first;
            }
            cur = it->second;
        }
        return cur;  // -1 for the empty product
    }
};

const char *transform_type(const qmc_transform &t) {
    static const char *kor[] = {"", "TrKorobov<1>", "TrKorobov<2>", "TrKorobov<3>",
                                "TrKorobov<4>", "TrKorobov<5>", "TrKorobov<6>"};
    static const char *sidi[] = {"", "TrSidi<1>", "TrSidi<2>", "TrSidi<3>", "TrSidi<4>", "TrSidi<5>", "TrSidi<6>"};
    if (t.kind == QMC_T_KOROBOV) return kor[t.alpha];
    if (t.kind == QMC_T_SIDI) return sidi[t.alpha];
    return t.kind == QMC_T_BAKER ? "TrBaker" : "TrNone";
}

}  // namespace

// Source of FamJit for a deformed contour (flag 8): straight-line code for
// the gradient and Hessian of F at the real point (their monomials share a
// real product trie), the deformed point z - i lam s grad F, the complex
// monomials of U, F and z^nu at that point (a complex product trie), the
// symmetrised Jacobian and its determinant, then sector_deformed; a last
// part counts the points where Im(F(z) - i delta) > 0.
static std::string deformed_source(uint32_t d, uint32_t flags, uint32_t orders,
                                   size_t eps_at, size_t lam_at, const std::vector<std::vector<int>> &fu,
                                   const std::vector<std::vector<int>> &ff, const std::vector<int> &nuf) {
    Trie rt, ct;  // real (derivative) and complex (deformed point) monomials
    const uint32_t nu = (uint32_t)fu.size(), nf = (uint32_t)ff.size();
    struct Term {
        int coef;   // index into cf
        int mult;   // integer factor from differentiation
        int mono;   // real trie node (-1: constant)
    };
    std::vector<std::vector<Term>> grad(d);
    std::vector<std::vector<Term>> hess(d * d);  // (i, j), j <= i, at i * d + j
    auto drop = [](std::vector<int> f, int v, int &mult) {
        int cnt = 0;
        for (int x : f) cnt += x == v;
        mult *= cnt;
        if (cnt) f.erase(std::find(f.begin(), f.end(), v));
        return f;
    };
    for (uint32_t t = 0; t < nf; ++t)
        for (uint32_t i = 0; i < d; ++i) {
            int mi = 1;
            const std::vector<int> gi = drop(ff[t], (int)i, mi);
            if (!mi) continue;
            grad[i].push_back({(int)t, mi, rt.insert(gi)});
            for (uint32_t j = 0; j <= i; ++j) {
                int mj = mi;
                const std::vector<int> hij = drop(gi, (int)j, mj);
                if (mj) hess[i * d + j].push_back({(int)t, mj, rt.insert(hij)});
            }
        }
    std::vector<int> cu(nu), cfm(nf);
    for (uint32_t t = 0; t < nu; ++t) cu[t] = ct.insert(fu[t]);
    for (uint32_t t = 0; t < nf; ++t) cfm[t] = ct.insert(ff[t]);
    const int cnu = ct.insert(nuf);

    const uint32_t no = orders >= 2 ? orders : 1u;
    const bool check = (flags & kSectorDeformCheck) != 0;
    std::ostringstream s;
    s << "struct FamJit {\n"
      << "    static constexpr int NP = " << (check ? 1u : 2 * no + 1) << ";\n"
      << "    template <class Tr, int D, int T>\n"
      << "    __device__ static void eval(const double *__restrict__ p, const double (&x)[T][D],"
         " double (&v)[T][NP]) {\n"
      << "        double z[T][D], jac[T];\n"
      << "        apply_transform<Tr, D, T, true>(x, z, jac);\n"
      << "        constexpr uint32_t flags = " << flags << "u;\n"
      << "        const __attribute__((address_space(4))) double *cp =\n"
      << "            (const __attribute__((address_space(4))) double *)p;\n"
      << "        asm volatile(\"\" : \"+s\"(cp));\n"
      << "        const double pow_u = cp[3], pow_f = cp[4], delta = cp[5], lam = cp[" << lam_at << "];\n"
      << "        const double eps_u = " << (orders >= 2 ? "cp[" + std::to_string(eps_at) + "]" : std::string("0.0"))
      << ", eps_f = " << (orders >= 2 ? "cp[" + std::to_string(eps_at + 1) + "]" : std::string("0.0")) << ";\n"
      << "        const __attribute__((address_space(4))) double *cu = cp + kSectorHeader;\n"
      << "        const __attribute__((address_space(4))) double *cf = cu + " << 2 * nu << ";\n"
      << "#pragma unroll\n"
      << "        for (int k = 0; k < T; ++k) {\n";
    // real monomials of the derivatives
    for (size_t id = 0; id < rt.node.size(); ++id) {
        const auto &nd = rt.node[id];
        s << "            const double r" << id << " = ";
        if (nd.first < 0) s << "z[k][" << nd.second << "];\n";
        else s << "r" << nd.first << " * z[k][" << nd.second << "];\n";
    }
    auto sum = [&](const std::string &name, const std::vector<Term> &terms) {
        s << "            double " << name << " = 0.0;\n";
        for (const Term &t : terms) {
            std::ostringstream c;
            if (t.mult == 1) c << "cf[" << t.coef << "]";
            else c << "(cf[" << t.coef << "] * " << t.mult << ".0)";
            if (t.mono < 0) s << "            " << name << " = " << name << " + " << c.str() << ";\n";
            else s << "            " << name << " = fma_(" << c.str() << ", r" << t.mono << ", " << name << ");\n";
        }
    };
    for (uint32_t i = 0; i < d; ++i) sum("g" + std::to_string(i), grad[i]);
    if (!check)
        for (uint32_t i = 0; i < d; ++i)
            for (uint32_t j = 0; j <= i; ++j) sum("h" + std::to_string(i) + "_" + std::to_string(j), hess[i * d + j]);
    // the deformed point: real part z, imaginary part y
    for (uint32_t i = 0; i < d; ++i)
        s << "            const double s" << i << " = z[k][" << i << "] * (1.0 - z[k][" << i << "]);\n"
          << "            const double y" << i << " = -lam * (s" << i << " * g" << i << ");\n";
    // complex monomials at the deformed point
    for (size_t id = 0; id < ct.node.size(); ++id) {
        const auto &nd = ct.node[id];
        const int v = nd.second;
        if (nd.first < 0) {
            s << "            const double c" << id << "r = z[k][" << v << "], c" << id << "i = y" << v << ";\n";
        } else {
            const int q = nd.first;
            s << "            const double c" << id << "r = fma_(c" << q << "r, z[k][" << v << "], -(c" << q << "i * y" << v
              << ")), c" << id << "i = fma_(c" << q << "r, y" << v << ", c" << q << "i * z[k][" << v << "]);\n";
        }
    }
    auto cpoly = [&](const char *name, const char *coef, const std::vector<int> &mono) {
        s << "            double " << name << "r = 0.0, " << name << "i = 0.0;\n";
        for (size_t t = 0; t < mono.size(); ++t) {
            if (mono[t] < 0) {
                s << "            " << name << "r = " << name << "r + " << coef << "[" << t << "];\n";
            } else {
                s << "            " << name << "r = fma_(" << coef << "[" << t << "], c" << mono[t] << "r, " << name
                  << "r);\n";
                s << "            " << name << "i = fma_(" << coef << "[" << t << "], c" << mono[t] << "i, " << name
                  << "i);\n";
            }
        }
    };
    if (check) {
        cpoly("F", "cf", cfm);
        s << "            v[k][0] = Fi - delta > 0.0 ? 1.0 : 0.0;\n"
          << "        }\n    }\n};\n";
        return s.str();
    }
    cpoly("U", "cu", cu);
    cpoly("F", "cf", cfm);
    if (cnu < 0) s << "            const double mr = jac[k], mi = 0.0;\n";
    else s << "            const double mr = jac[k] * c" << cnu << "r, mi = jac[k] * c" << cnu << "i;\n";
    // I + i Bs, packed lower triangle
    const uint32_t nt = d * (d + 1) / 2;
    s << "            double ar[" << nt << "], ai[" << nt << "];\n";
    // a transformed coordinate may round a few ulp outside [0, 1], making s
    // slightly negative: every term of det pairs q_k with itself (q_k^2
    // stands for s_k), so |s_k| changes det by O(|s_k|) only
    for (uint32_t i = 0; i < d; ++i)
        s << "            const double q" << i << " = __builtin_sqrt(__builtin_fabs(s" << i << "));\n";
    for (uint32_t i = 0; i < d; ++i)
        for (uint32_t j = 0; j <= i; ++j) {
            const uint32_t ij = i * (i + 1) / 2 + j;
            s << "            ar[" << ij << "] = " << (i == j ? "1.0" : "0.0") << ";\n";
            s << "            ai[" << ij << "] = -lam * ";
            if (i == j)
                s << "fma_(s" << i << ", h" << i << "_" << i << ", (1.0 - 2.0 * z[k][" << i << "]) * g" << i << ");\n";
            else
                s << "((q" << i << " * q" << j << ") * h" << i << "_" << j << ");\n";
        }
    // the value parts, then 1 where the contour is on the wrong side (the
    // sign check of the deformation, counted in the same pass)
    s << "            double dr, di, w[" << 2 * no << "];\n"
      << "            csym_det<D>(ar, ai, dr, di);\n"
      << "            sector_deformed<" << no
      << ">(mr, mi, dr, di, Ur, Ui, Fr, Fi, flags, pow_u, pow_f, delta, eps_u, eps_f, w);\n"
      << "#pragma unroll\n"
      << "            for (int j = 0; j < " << 2 * no << "; ++j) v[k][j] = w[j];\n"
      << "            v[k][" << 2 * no << "] = Fi - delta > 0.0 ? 1.0 : 0.0;\n"
      << "        }\n    }\n};\n";
    return s.str();
}

// Multivariate Horner form of sum_t coef[t] prod_i z_i^e[t][i]: split off
// the variable v that occurs in most non-constant terms, P = P0 + z_v P1,
// and recurse on P1 (exponents of v lowered) and P0.  Each split costs one
// FMA (one multiply when P0 is empty), so a polynomial of T terms takes
// about T operations instead of one multiply per product-trie edge plus one
// FMA per term.  Emits the temporaries (arrays over the thread's shifts k)
// into s and returns the expression of the value for shift k.
using HornerTerms = std::vector<std::pair<int, std::vector<int>>>;
static std::string horner(const char *coef, HornerTerms terms, std::ostringstream &s, int &tmp) {
    HornerTerms consts;
    for (const auto &t : terms)
        if (std::all_of(t.second.begin(), t.second.end(), [](int e) { return e == 0; })) consts.push_back(t);
    if (consts.size() == terms.size()) {
        std::ostringstream e;
        for (size_t c = 0; c < consts.size(); ++c) e << (c ? " + " : "") << coef << "[" << consts[c].first << "]";
        return consts.size() == 1 ? e.str() : "(" + e.str() + ")";
    }
    const size_t nv = terms[0].second.size();
    size_t v = 0;
    int best = -1;
    for (size_t i = 0; i < nv; ++i) {
        int c = 0;
        for (const auto &t : terms) c += t.second[i] > 0;
        if (c > best) {
            best = c;
            v = i;
        }
    }
    HornerTerms p1, p0;
    for (auto t : terms) {
        if (t.second[v] > 0) {
            t.second[v] -= 1;
            p1.push_back(t);
        } else {
            p0.push_back(t);
        }
    }
    const std::string a = horner(coef, p1, s, tmp);
    const std::string b = p0.empty() ? std::string() : horner(coef, p0, s, tmp);
    // one statement per line over the T shifts of the thread, so that a
    // coefficient is loaded once for all of them
    const std::string name = "h" + std::to_string(tmp++);
    s << "        double " << name << "[T]; _Pragma(\"unroll\") for (int k = 0; k < T; ++k) " << name << "[k] = ";
    if (b.empty()) s << a << " * z[k][" << v << "];\n";
    else s << "fma_(" << a << ", z[k][" << v << "], " << b << ");\n";
    return name + "[k]";
}

// Each coefficient of the Horner code is read once, in ascending order (the
// host stores the terms that way).  Left alone, the compiler issues all the
// scalar loads up front and spills the values it cannot keep in scalar
// registers (a large polynomial needs more than the 106 available).  A fresh
// laundered copy of the table pointer every kChunk coefficients, placed just
// before the first line that reads the chunk, keeps each chunk's loads after
// that point (volatile asm statements keep their order), so only a few
// chunks are live at a time.
static std::string launder_chunks(const std::string &text) {
    constexpr uint32_t kChunk = 8;
    std::istringstream in(text);
    std::ostringstream out;
    std::string line;
    int next[2] = {0, 0};  // next chunk start for cu, cf
    int ptr = 0;
    while (std::getline(in, line)) {
        std::string fixed;
        std::string pre;
        for (size_t i = 0; i < line.size();) {
            const bool is_u = line.compare(i, 3, "cu[") == 0, is_f = line.compare(i, 3, "cf[") == 0;
            if ((!is_u && !is_f) || (i > 0 && (std::isalnum((unsigned char)line[i - 1]) || line[i - 1] == '_'))) {
                fixed += line[i++];
                continue;
            }
            size_t j = i + 3;
            int v = 0;
            while (j < line.size() && std::isdigit((unsigned char)line[j])) v = 10 * v + (line[j++] - '0');
            const int w = is_u ? 0 : 1;
            const char *base = is_u ? "cu" : "cf";
            if (v >= next[w]) {
                ++ptr;
                pre += std::string("            const __attribute__((address_space(4))) double *q") +
                       std::to_string(ptr) + " = " + base + ";\n            asm volatile(\"\" : \"+s\"(q" +
                       std::to_string(ptr) + "));\n";
                next[w] = (v / kChunk + 1) * kChunk;
            }
            fixed += "q" + std::to_string(ptr) + "[" + std::to_string(v) + "]";
            i = j + 1;  // skip ']'
        }
        out << pre << fixed << "\n";
    }
    return out.str();
}

// The order in which the Horner form above first reads each coefficient.
// The host packer stores the terms in this order, so the generated code
// reads the coefficients in ascending address order and the compiler can
// fetch them with few scalar loads and few live scalar registers.
static std::vector<uint32_t> horner_term_order_uncached(const std::vector<uint64_t> &codes, uint32_t d) {
    HornerTerms terms;
    for (size_t t = 0; t < codes.size(); ++t) {
        std::vector<int> e(d, 0);
        for (int v : factors_of(codes[t])) e[v] += 1;
        terms.push_back({(int)t, e});
    }
    std::ostringstream s;
    int tmp = 0;
    const std::string top = horner("c", terms, s, tmp);
    s << top;
    const std::string text = s.str();
    std::vector<uint32_t> order;
    std::vector<bool> seen(codes.size(), false);
    for (size_t i = 0; i + 1 < text.size(); ++i) {
        if (text[i] != 'c' || text[i + 1] != '[') continue;
        size_t j = i + 2;
        uint32_t v = 0;
        while (j < text.size() && text[j] >= '0' && text[j] <= '9') v = 10 * v + (uint32_t)(text[j++] - '0');
        if (v < codes.size() && !seen[v]) {
            seen[v] = true;
            order.push_back(v);
        }
    }
    for (uint32_t t = 0; t < codes.size(); ++t)
        if (!seen[t]) order.push_back(t);
    return order;
}

// Remembered per (d, codes): a plan re-packs its integrand at every estimate.
std::vector<uint32_t> horner_term_order(const std::vector<uint64_t> &codes, uint32_t d) {
    static std::mutex mu;
    static std::unordered_map<std::string, std::vector<uint32_t>> memo;
    std::string key(sizeof(uint32_t) + codes.size() * sizeof(uint64_t), '\0');
    std::memcpy(&key[0], &d, sizeof(uint32_t));
    if (!codes.empty()) std::memcpy(&key[sizeof(uint32_t)], codes.data(), codes.size() * sizeof(uint64_t));
    {
        std::lock_guard<std::mutex> lock(mu);
        auto it = memo.find(key);
        if (it != memo.end()) return it->second;
    }
    std::vector<uint32_t> order = horner_term_order_uncached(codes, d);
    std::lock_guard<std::mutex> lock(mu);
    if (memo.size() >= 65536) memo.clear();  // bounded: structures of one run rarely exceed it
    memo.emplace(key, order);
    return order;
}


// A canonical description of everything the specialised functor of one
// sector blob depends on (dimension, complex flag, monomial codes, flags,
// expansion orders, nu): the key of its compiled code.  It is built without
// generating the source, so that a cached kernel is found cheaply.
static std::string sector_structure(const std::vector<double> &blob, uint32_t d, bool cplx) {
    const uint32_t nu = (uint32_t)word(blob, 0), nf = (uint32_t)word(blob, 1);
    const uint32_t flags = (uint32_t)word(blob, 2);
    const size_t eps_at = kSectorHeader + 2 * (size_t)nu + 2 * (size_t)nf;
    const uint32_t orders = (flags & kSectorOrders) ? (uint32_t)word(blob, eps_at + 2) : 0u;
    std::string st = "d" + std::to_string(d) + "c" + (cplx ? "1" : "0") + "|";
    st.reserve(st.size() + 21 * (size_t)(nu + nf) + 48);
    for (uint32_t t = 0; t < nu; ++t) (st += std::to_string(word(blob, kSectorHeader + nu + t))) += ',';
    st += '|';
    for (uint32_t t = 0; t < nf; ++t) (st += std::to_string(word(blob, kSectorHeader + 2 * nu + nf + t))) += ',';
    st += "|f" + std::to_string(flags) + "|o" + std::to_string(orders) + "|" + std::to_string(word(blob, 6));
    return st;
}

// Source of the specialised functor FamJit; `structure` receives a
// canonical description of what the code depends on.
static std::string functor_source(const std::vector<double> &blob, uint32_t d, bool cplx, std::string &structure) {
    const uint32_t nu = (uint32_t)word(blob, 0), nf = (uint32_t)word(blob, 1);
    // expansion orders (flag 4): three words after the F codes (eps_u,
    // eps_f, count); other blobs may carry other data there
    const size_t eps_at = kSectorHeader + 2 * (size_t)nu + 2 * (size_t)nf;
    const uint32_t orders = (word(blob, 2) & kSectorOrders) ? (uint32_t)word(blob, eps_at + 2) : 0u;
    Trie trie;  // the z^nu product
    HornerTerms hu, hf;
    auto exps = [d](uint64_t code) {
        std::vector<int> e(d, 0);
        for (int v : factors_of(code)) e[v] += 1;
        return e;
    };
    for (uint32_t t = 0; t < nu; ++t) {
        const uint64_t c = word(blob, kSectorHeader + nu + t);
        hu.push_back({(int)t, exps(c)});
    }
    for (uint32_t t = 0; t < nf; ++t) {
        const uint64_t c = word(blob, kSectorHeader + 2 * nu + nf + t);
        hf.push_back({(int)t, exps(c)});
    }
    const uint64_t nuc = word(blob, 6);
    const uint32_t flags = (uint32_t)word(blob, 2);
    std::vector<int> nuf;
    for (uint32_t i = 0; i < d; ++i)
        for (uint64_t r = 0; r < ((nuc >> (2 * i)) & 3u); ++r) nuf.push_back((int)i);
    const int mnu = trie.insert(nuf);
    structure = sector_structure(blob, d, cplx);
    if (flags & kSectorDeform) {
        // the deformation parameter follows the orders words (if any)
        const size_t lam_at = eps_at + ((flags & kSectorOrders) ? 3u : 0u);
        std::vector<std::vector<int>> fu(nu), ff(nf);
        for (uint32_t t = 0; t < nu; ++t) fu[t] = factors_of(word(blob, kSectorHeader + nu + t));
        for (uint32_t t = 0; t < nf; ++t) ff[t] = factors_of(word(blob, kSectorHeader + 2 * nu + nf + t));
        return deformed_source(d, flags, orders, eps_at, lam_at, fu, ff, nuf);
    }

    std::ostringstream s;
    const uint32_t np = (cplx ? 2u : 1u) * (orders >= 2 ? orders : 1u);
    s << "struct FamJit {\n"
      << "    static constexpr int NP = " << np << ";\n"
      << "    static constexpr bool kShiftsInVgprs = true;\n"
      << "    template <class Tr, int D, int T>\n"
      << "    __device__ static void eval(const double *__restrict__ p, const double (&x)[T][D],"
         " double (&v)[T][NP]) {\n"
      << "        double z[T][D], jac[T];\n"
      << "        apply_transform<Tr, D, T, true>(x, z, jac);\n"
      << "        constexpr uint32_t flags = " << flags << "u;\n"
      // the parameter words are read through a constant-address-space
      // pointer laundered per point: scalar loads inside the point loop
      // (SGPR operands of the FMAs) instead of vector loads hoisted into VGPRs
      << "        const __attribute__((address_space(4))) double *cp =\n"
      << "            (const __attribute__((address_space(4))) double *)p;\n"
      << "        asm volatile(\"\" : \"+s\"(cp));\n"
      << "        const double pow_u = cp[3], pow_f = cp[4], delta = cp[5];\n"
      << "        const __attribute__((address_space(4))) double *cu = cp + kSectorHeader;\n"
      << "        const __attribute__((address_space(4))) double *cf = cu + " << 2 * nu << ";\n";
    auto ref = [&](int id) {
        std::ostringstream r;
        if (trie.node[id].first < 0) r << "z[k][" << trie.node[id].second << "]";
        else r << "m" << id << "[k]";
        return r.str();
    };
    for (size_t id = 0; id < trie.node.size(); ++id) {
        const auto &nd = trie.node[id];
        if (nd.first < 0) continue;
        s << "        double m" << id << "[T]; _Pragma(\"unroll\") for (int k = 0; k < T; ++k) m" << id
          << "[k] = " << ref(nd.first) << " * z[k][" << nd.second << "];\n";
    }
    int tmp = 0;
    {
        std::ostringstream hs;
        const std::string ue = horner("cu", hu, hs, tmp);
        hs << "        double U[T]; _Pragma(\"unroll\") for (int k = 0; k < T; ++k) U[k] = " << ue << ";\n";
        const std::string fe = horner("cf", hf, hs, tmp);
        hs << "        double F[T]; _Pragma(\"unroll\") for (int k = 0; k < T; ++k) F[k] = " << fe << ";\n";
        s << launder_chunks(hs.str());
    }
    s << "#pragma unroll\n"
      << "        for (int k = 0; k < T; ++k) {\n"
      << "            const double mono = " << (mnu < 0 ? std::string("jac[k]") : "jac[k] * " + ref(mnu))
      << ";\n";
    if (orders >= 2)
        s << "            sector_orders<" << (cplx ? "true" : "false") << ", " << orders
          << ">(mono, U[k], F[k], flags, pow_u, pow_f, delta, cp[" << eps_at << "], cp[" << eps_at + 1
          << "], v[k]);\n";
    else
        s << "            sector_finish<" << (cplx ? "true" : "false")
          << ">(mono, U[k], F[k], flags, pow_u, pow_f, delta, v[k]);\n";
    s << "        }\n    }\n};\n";
    return s.str();
}

// FamJit for a sum of sectors of one dimension evaluated at the same points:
// the blob is the sectors' blobs one after another (offsets offs), each
// sector's code is the Horner form above in a scope of its own, and the
// values are accumulated before the kernel's per-shift sums.
// The key of a sum's functor: each sector's offset, flags, nu and monomial
// codes.
static std::string sum_structure(const std::vector<double> &blob, const std::vector<size_t> &offs, uint32_t d,
                                 bool cplx) {
    std::string st = "sum|d" + std::to_string(d) + "c" + (cplx ? "1" : "0");
    for (size_t o : offs) {
        const uint32_t nu = (uint32_t)word(blob, o), nf = (uint32_t)word(blob, o + 1);
        st += "|o" + std::to_string(o) + "f" + std::to_string((uint32_t)word(blob, o + 2)) + "n" +
              std::to_string(word(blob, o + 6)) + ":";
        for (uint32_t t = 0; t < nu; ++t) (st += std::to_string(word(blob, o + kSectorHeader + nu + t))) += ',';
        st += ';';
        for (uint32_t t = 0; t < nf; ++t)
            (st += std::to_string(word(blob, o + kSectorHeader + 2 * nu + nf + t))) += ',';
    }
    return st;
}

static std::string sum_source(const std::vector<double> &blob, const std::vector<size_t> &offs, uint32_t d,
                              bool cplx, std::string &structure) {
    const uint32_t np = cplx ? 2u : 1u;
    std::ostringstream s;
    s << "struct FamJit {\n"
      << "    static constexpr int NP = " << np << ";\n"
      << "    static constexpr bool kShiftsInVgprs = true;\n"
      << "    template <class Tr, int D, int T>\n"
      << "    __device__ static void eval(const double *__restrict__ p, const double (&x)[T][D],"
         " double (&v)[T][NP]) {\n"
      << "        double z[T][D], jac[T];\n"
      << "        apply_transform<Tr, D, T, true>(x, z, jac);\n"
      << "        double acc[T][NP];\n"
      << "        _Pragma(\"unroll\") for (int k = 0; k < T; ++k) _Pragma(\"unroll\") for (int q = 0; q < NP; ++q)"
         " acc[k][q] = 0.0;\n";
    auto exps = [d](uint64_t code) {
        std::vector<int> e(d, 0);
        for (int v : factors_of(code)) e[v] += 1;
        return e;
    };
    int tmp = 0;
    for (size_t o : offs) {
        const uint32_t nu = (uint32_t)word(blob, o), nf = (uint32_t)word(blob, o + 1);
        const uint32_t flags = (uint32_t)word(blob, o + 2);
        const uint64_t nuc = word(blob, o + 6);
        HornerTerms hu, hf;
        for (uint32_t t = 0; t < nu; ++t) {
            const uint64_t c = word(blob, o + kSectorHeader + nu + t);
            hu.push_back({(int)t, exps(c)});
        }
        for (uint32_t t = 0; t < nf; ++t) {
            const uint64_t c = word(blob, o + kSectorHeader + 2 * nu + nf + t);
            hf.push_back({(int)t, exps(c)});
        }
        Trie trie;
        std::vector<int> nuf;
        for (uint32_t i = 0; i < d; ++i)
            for (uint64_t r = 0; r < ((nuc >> (2 * i)) & 3u); ++r) nuf.push_back((int)i);
        const int mnu = trie.insert(nuf);
        s << "        {\n"
          << "        constexpr uint32_t flags = " << flags << "u;\n"
          << "        const __attribute__((address_space(4))) double *cp =\n"
          << "            (const __attribute__((address_space(4))) double *)(p + " << o << ");\n"
          << "        asm volatile(\"\" : \"+s\"(cp));\n"
          << "        const double pow_u = cp[3], pow_f = cp[4], delta = cp[5];\n"
          << "        const __attribute__((address_space(4))) double *cu = cp + kSectorHeader;\n"
          << "        const __attribute__((address_space(4))) double *cf = cu + " << 2 * nu << ";\n";
        auto ref = [&](int id) {
            std::ostringstream r;
            if (trie.node[id].first < 0) r << "z[k][" << trie.node[id].second << "]";
            else r << "m" << id << "[k]";
            return r.str();
        };
        for (size_t id = 0; id < trie.node.size(); ++id) {
            const auto &nd = trie.node[id];
            if (nd.first < 0) continue;
            s << "        double m" << id << "[T]; _Pragma(\"unroll\") for (int k = 0; k < T; ++k) m" << id
              << "[k] = " << ref(nd.first) << " * z[k][" << nd.second << "];\n";
        }
        std::ostringstream hs;
        const std::string ue = horner("cu", hu, hs, tmp);
        hs << "        double U[T]; _Pragma(\"unroll\") for (int k = 0; k < T; ++k) U[k] = " << ue << ";\n";
        const std::string fe = horner("cf", hf, hs, tmp);
        hs << "        double F[T]; _Pragma(\"unroll\") for (int k = 0; k < T; ++k) F[k] = " << fe << ";\n";
        s << launder_chunks(hs.str());
        s << "#pragma unroll\n"
          << "        for (int k = 0; k < T; ++k) {\n"
          << "            const double mono = " << (mnu < 0 ? std::string("jac[k]") : "jac[k] * " + ref(mnu))
          << ";\n"
          << "            double w[NP];\n"
          << "            sector_finish<" << (cplx ? "true" : "false")
          << ">(mono, U[k], F[k], flags, pow_u, pow_f, delta, w);\n"
          << "            _Pragma(\"unroll\") for (int q = 0; q < NP; ++q) acc[k][q] += w[q];\n"
          << "        }\n"
          << "        }\n";
    }
    s << "        _Pragma(\"unroll\") for (int k = 0; k < T; ++k) _Pragma(\"unroll\") for (int q = 0; q < NP; ++q)"
         " v[k][q] = acc[k][q];\n"
      << "    }\n};\n";
    structure = sum_structure(blob, offs, d, cplx);
    return s.str();
}

static std::string device_arch(int dev) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "gfx950";
    std::string a = prop.gcnArchName;
    return a.empty() ? std::string("gfx950") : a;
}

// Compile (or fetch from the process cache) `src`, returning the function
// named by name_expr; nullptr and `err` on failure.
// Optional on-disk store of compiled code objects (directory in QMC_JIT_CACHE):
// one file per (architecture, kernel name expression, source), holding the
// lowered kernel name and the code object, so that other processes (or a
// later run) load the kernel instead of compiling it again.
static uint64_t fnv1a(const std::string &s) {
    uint64_t h = 1469598103934665603ull;
    for (unsigned char c : s) {
        h ^= c;
        h *= 1099511628211ull;
    }
    return h;
}

static std::string disk_path(const std::string &arch, const std::string &name_expr, const std::string &src) {
    const char *dir = std::getenv("QMC_JIT_CACHE");
    if (!dir || !*dir) return std::string();
    // the embedded headers are part of what the code depends on
    static const uint64_t headers = [] {
        std::string all;
        for (int i = 0; i < kJitHeaderCount; ++i) all += kJitHeaderText[i];
        return fnv1a(all);
    }();
    char buf[48];
    std::snprintf(buf, sizeof buf, "%016llx_%016llx", (unsigned long long)headers,
                  (unsigned long long)fnv1a(arch + "\n" + name_expr + "\n" + src));
    return std::string(dir) + "/qmc_" + buf + ".co";
}

// file: u32 length of the lowered name, the name, then the code object
static bool disk_load(const std::string &path, std::string &lowered, std::vector<char> &code) {
    if (path.empty()) return false;
    std::ifstream f(path, std::ios::binary);
    if (!f) return false;
    uint32_t len = 0;
    if (!f.read(reinterpret_cast<char *>(&len), 4) || len == 0 || len > 4096) return false;
    lowered.resize(len);
    if (!f.read(&lowered[0], len)) return false;
    code.assign(std::istreambuf_iterator<char>(f), std::istreambuf_iterator<char>());
    return !code.empty();
}

static void disk_store(const std::string &path, const std::string &lowered, const std::vector<char> &code) {
    if (path.empty()) return;
    static std::atomic<unsigned> counter{0};
    const std::string tmp = path + ".tmp." + std::to_string((long)getpid()) + "." + std::to_string(counter++);
    {
        std::ofstream f(tmp, std::ios::binary);
        if (!f) return;
        const uint32_t len = (uint32_t)lowered.size();
        f.write(reinterpret_cast<const char *>(&len), 4);
        f.write(lowered.data(), len);
        f.write(code.data(), (std::streamsize)code.size());
        if (!f) return;
    }
    std::rename(tmp.c_str(), path.c_str());  // atomic within one file system
}

static hipFunction_t compile_cached(const std::string &src, const std::string &name_expr, const std::string &key,
                                    int dev, std::string &err) {
    if (const char *dump = std::getenv("QMC_JIT_DUMP")) {  // write the generated source for inspection
        std::ofstream(std::string(dump) + "/" + std::to_string(std::hash<std::string>()(key)) + ".hip") << src;
    }
    {
        std::lock_guard<std::mutex> lock(g_jit_mu);
        auto it = g_jit_cache.find(key);
        if (it != g_jit_cache.end()) {
            err = it->second.error;
            return it->second.fn;
        }
    }
    // compile without holding the lock, so that several threads can compile
    // different programs at once; the first result stored for a key wins
    JitEntry e;
    const std::string arch = "--offload-arch=" + device_arch(dev);
    const std::string path = disk_path(arch, name_expr, src);
    {
        std::string low;
        std::vector<char> code;
        if (disk_load(path, low, code)) {
            hipError_t he = hipModuleLoadData(&e.mod, code.data());
            if (he == hipSuccess) he = hipModuleGetFunction(&e.fn, e.mod, low.c_str());
            if (he == hipSuccess) {
                std::lock_guard<std::mutex> lock(g_jit_mu);
                auto ins = g_jit_cache.emplace(key, e);
                if (!ins.second) (void)hipModuleUnload(e.mod);
                err = ins.first->second.error;
                return ins.first->second.fn;
            }
            if (e.mod) (void)hipModuleUnload(e.mod);  // unreadable entry: compile instead
            e = JitEntry{};
        }
    }
    hiprtcProgram prog = nullptr;
    hiprtcResult r = hiprtcCreateProgram(&prog, src.c_str(), "qmc_sector_jit.hip", kJitHeaderCount, kJitHeaderText,
                                         kJitHeaderName);
    if (r == HIPRTC_SUCCESS) r = hiprtcAddNameExpression(prog, name_expr.c_str());
    const char *opts[] = {arch.c_str(), "-O3", "-std=c++17", "-ffp-contract=off", "-Xclang", "-target-feature",
                          "-Xclang", "-packed-fp32-ops"};
    if (r == HIPRTC_SUCCESS) r = hiprtcCompileProgram(prog, 8, opts);
    if (r != HIPRTC_SUCCESS) {
        size_t ls = 0;
        std::string log;
        if (prog && hiprtcGetProgramLogSize(prog, &ls) == HIPRTC_SUCCESS && ls > 1) {
            log.resize(ls);
            hiprtcGetProgramLog(prog, &log[0]);
        }
        e.error = std::string("hipRTC: ") + hiprtcGetErrorString(r) + ": " + log.substr(0, 2000);
    } else {
        const char *lowered = nullptr;
        size_t cs = 0;
        std::vector<char> code;
        if (hiprtcGetLoweredName(prog, name_expr.c_str(), &lowered) != HIPRTC_SUCCESS || !lowered ||
            hiprtcGetCodeSize(prog, &cs) != HIPRTC_SUCCESS) {
            e.error = "hipRTC: no lowered name / code";
        } else {
            code.resize(cs);
            hiprtcGetCode(prog, code.data());
            std::string low = lowered;
            hipError_t he = hipModuleLoadData(&e.mod, code.data());
            if (he == hipSuccess) he = hipModuleGetFunction(&e.fn, e.mod, low.c_str());
            if (he != hipSuccess) {
                e.error = std::string("module load: ") + hipGetErrorString(he);
                e.fn = nullptr;
            } else {
                disk_store(path, low, code);
            }
        }
    }
    if (prog) hiprtcDestroyProgram(&prog);
    std::lock_guard<std::mutex> lock(g_jit_mu);
    auto ins = g_jit_cache.emplace(key, e);
    if (!ins.second && e.mod) (void)hipModuleUnload(e.mod);  // another thread stored this key first
    err = ins.first->second.error;
    return ins.first->second.fn;
}

// The kernel stored under key (or the error its compile gave), if any.
static bool jit_lookup(const std::string &key, hipFunction_t &fn, std::string &err) {
    std::lock_guard<std::mutex> lock(g_jit_mu);
    auto it = g_jit_cache.find(key);
    if (it == g_jit_cache.end()) return false;
    fn = it->second.fn;
    err = it->second.error;
    return true;
}

// The getters below build the key from the blob's structure first and
// generate the source only when no kernel is stored under it: the
// repeated estimates of one integrand pay a key, not a code generation.

// The lattice kernel with the specialised sector functor.
hipFunction_t jit_kernel(const std::vector<double> &blob, uint32_t d, const qmc_transform &tr, uint32_t T,
                         bool cplx, int dev, std::string &err) {
    std::ostringstream key;
    key << dev << "#lattice#T" << T << "t" << tr.kind << "a" << tr.alpha << "#" << sector_structure(blob, d, cplx);
    hipFunction_t fn = nullptr;
    if (jit_lookup(key.str(), fn, err)) return fn;
    std::string structure;
    const std::string fam = functor_source(blob, d, cplx, structure);
    std::ostringstream ne, src;
    ne << "qmc::k_lattice<qmc::FamJit, qmc::" << transform_type(tr) << ", " << d << ", " << T << ">";
    src << "#include \"qmc_cv.hpp\"\nnamespace qmc {\n" << fam << "template __global__ void k_lattice<FamJit, "
        << transform_type(tr) << ", " << d << ", " << T << ">(const LatticeArgs);\n}  // namespace qmc\n";
    return compile_cached(src.str(), ne.str(), key.str(), dev, err);
}

// The lattice kernel with the functor of a sum of sectors.
hipFunction_t jit_sum_kernel(const std::vector<double> &blob, const std::vector<size_t> &offs, uint32_t d,
                             const qmc_transform &tr, uint32_t T, bool cplx, int dev, std::string &err) {
    std::ostringstream key;
    key << dev << "#sum#T" << T << "t" << tr.kind << "a" << tr.alpha << "#" << sum_structure(blob, offs, d, cplx);
    hipFunction_t fn = nullptr;
    if (jit_lookup(key.str(), fn, err)) return fn;
    std::string structure;
    const std::string fam = sum_source(blob, offs, d, cplx, structure);
    std::ostringstream ne, src;
    ne << "qmc::k_lattice<qmc::FamJit, qmc::" << transform_type(tr) << ", " << d << ", " << T << ">";
    src << "#include \"qmc_cv.hpp\"\nnamespace qmc {\n" << fam << "template __global__ void k_lattice<FamJit, "
        << transform_type(tr) << ", " << d << ", " << T << ">(const LatticeArgs);\n}  // namespace qmc\n";
    return compile_cached(src.str(), ne.str(), key.str(), dev, err);
}

// The lattice kernel with the control-variate residual around the
// specialised functor (parts: fhat, fhat - J g).
hipFunction_t jit_cv_kernel(const std::vector<double> &blob, size_t cv_off, uint32_t d, const qmc_transform &tr,
                            uint32_t R, uint32_t K, bool cplx, int dev, std::string &err) {
    std::ostringstream key;
    key << dev << "#cv#R" << R << "K" << K << "o" << cv_off << "c" << cplx << "t" << tr.kind << "a" << tr.alpha << "#"
        << sector_structure(blob, d, cplx);
    hipFunction_t fn = nullptr;
    if (jit_lookup(key.str(), fn, err)) return fn;
    std::string structure;
    const std::string fam = functor_source(blob, d, cplx, structure);
    std::ostringstream ne, src, cvt;
    cvt << "FamCvResidual<FamJit, " << R << ", " << K << ", " << cv_off << ">";
    // real integrands up to R = 32 fit two waves per SIMD without spills
    const char *kern = R <= 32 && !cplx ? "k_lattice_w2" : "k_lattice";
    ne << "qmc::" << kern << "<qmc::FamCvResidual<qmc::FamJit, " << R << ", " << K << ", " << cv_off << ">, qmc::"
       << transform_type(tr) << ", " << d << ", 1>";
    src << "#include \"qmc_cv.hpp\"\nnamespace qmc {\n" << fam << "template __global__ void " << kern << "<" << cvt.str()
        << ", " << transform_type(tr) << ", " << d << ", 1>(const LatticeArgs);\n}  // namespace qmc\n";
    return compile_cached(src.str(), ne.str(), key.str(), dev, err);
}

// The training-lattice sampler with the specialised functor.
hipFunction_t jit_sample_kernel(const std::vector<double> &blob, uint32_t d, const qmc_transform &tr, bool cplx,
                                int dev, std::string &err) {
    std::ostringstream key;
    key << dev << "#sample#c" << cplx << "t" << tr.kind << "a" << tr.alpha << "#" << sector_structure(blob, d, cplx);
    hipFunction_t fn = nullptr;
    if (jit_lookup(key.str(), fn, err)) return fn;
    std::string structure;
    const std::string fam = functor_source(blob, d, cplx, structure);
    std::ostringstream ne, src;
    ne << "qmc::k_cv_sample<qmc::FamJit, qmc::" << transform_type(tr) << ", " << d << ">";
    src << "#include \"qmc_cv.hpp\"\nnamespace qmc {\n" << fam << "template __global__ void k_cv_sample<FamJit, "
        << transform_type(tr) << ", " << d << ">(const CvSampleArgs);\n}  // namespace qmc\n";
    return compile_cached(src.str(), ne.str(), key.str(), dev, err);
}

hipError_t jit_launch_sample(hipFunction_t fn, const CvSampleArgs &a, uint32_t blocks, hipStream_t s) {
    CvSampleArgs copy = a;
    void *args[] = {&copy};
    return hipModuleLaunchKernel(fn, blocks, 1, 1, kBlock, 1, 1, 0, s, args, nullptr);
}

hipError_t jit_launch(hipFunction_t fn, const LatticeArgs &a, dim3 grid, hipStream_t s) {
    LatticeArgs copy = a;
    void *args[] = {&copy};
    return hipModuleLaunchKernel(fn, grid.x, grid.y, 1, kBlock, 1, 1, 0, s, args, nullptr);
}

}  // namespace qmc

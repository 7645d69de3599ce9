// Host-side construction of the screening tables; see tables.hpp.
#include "tables.hpp"

#include <algorithm>
#include <cmath>
#include <unordered_map>

namespace vmc {
namespace {

inline int64_t pair_index(int64_t p, int64_t q) {
    int64_t hi = p > q ? p : q, lo = p > q ? q : p;
    return hi * (hi + 1) / 2 + lo;
}
inline uint64_t quad_index(int p, int q, int r, int s) {
    int64_t a = pair_index(p, q), b = pair_index(r, s);
    int64_t hi = a > b ? a : b, lo = a > b ? b : a;
    return (uint64_t)(hi * (hi + 1) / 2 + lo);
}

struct Integrals {
    int n = 0;
    const double* h1 = nullptr;
    std::unordered_map<uint64_t, double> eri;

    double spatial(int p, int q, int r, int s) const {
        auto it = eri.find(quad_index(p, q, r, s));
        return it == eri.end() ? 0.0 : it->second;
    }
    // chemist (pq|rs) over spin-orbitals (block ordered)
    double so(int p, int q, int r, int s) const {
        if ((p >= n) != (q >= n) || (r >= n) != (s >= n)) return 0.0;
        return spatial(p % n, q % n, r % n, s % n);
    }
    double h(int p, int q) const {
        if ((p >= n) != (q >= n)) return 0.0;
        return h1[(p % n) * n + (q % n)];
    }
};

inline uint64_t pack_key(int i, int j, int a, int b) {
    return ((uint64_t)i << 48) | ((uint64_t)j << 32) | ((uint64_t)a << 16) | (uint64_t)b;
}

}  // namespace

std::string build_host_tables(int n, int na, int nb, const double* h1, int64_t n_nz, const int32_t* pqrs,
                              const double* val, double eps, HostTables& T) {
    if (n <= 0 || 2 * n > 1024) return "n_orb must be in 1..512";
    if (na < 0 || nb < 0 || na > n || nb > n || na + nb == 0) return "electron counts out of range";
    if (!(eps >= 0.0) || !std::isfinite(eps)) return "eps must be finite and >= 0";
    if (!h1) return "h1 is NULL";
    if (n_nz < 0 || (n_nz > 0 && (!pqrs || !val))) return "bad integral list";
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q) {
            if (!std::isfinite(h1[p * n + q])) return "h1 has a non-finite entry";
            if (h1[p * n + q] != h1[q * n + p]) return "h1 is not symmetric";
        }
    Integrals I;
    I.n = n;
    I.h1 = h1;
    I.eri.reserve((size_t)n_nz * 2 + 16);
    for (int64_t k = 0; k < n_nz; ++k) {
        int p = pqrs[4 * k], q = pqrs[4 * k + 1], r = pqrs[4 * k + 2], s = pqrs[4 * k + 3];
        if (p < 0 || q < 0 || r < 0 || s < 0 || p >= n || q >= n || r >= n || s >= n)
            return "integral index out of range at entry " + std::to_string(k);
        if (p < q || r < s || pair_index(p, q) < pair_index(r, s))
            return "integral entry " + std::to_string(k) + " is not in canonical order";
        if (!std::isfinite(val[k])) return "non-finite integral at entry " + std::to_string(k);
        if (!I.eri.emplace(quad_index(p, q, r, s), val[k]).second)
            return "duplicate integral entry " + std::to_string(k);
    }
    const int nso = 2 * n;
    T.n = n;
    T.n_so = nso;
    T.na = na;
    T.nb = nb;
    T.ne = na + nb;
    T.eps = eps;

    // ---------------------------------------------------------------- singles
    // per spatial (I, A): Coulomb C[J] = (IA|JJ), exchange X[J] = (IJ|JA)
    T.s_off.assign(nso + 1, 0);
    T.sa.clear();
    T.sS.clear();
    T.sh.clear();
    T.sV.clear();
    std::vector<double> C(n), X(n), S(nso), Vrow((size_t)nso * nso);
    std::vector<std::pair<double, int>> order;
    for (int i = 0; i < nso; ++i) {
        const int sig = i / n, Ii = i % n;
        order.clear();
        for (int A = 0; A < n; ++A) {
            const int a = A + sig * n;
            if (a == i) continue;
            for (int J = 0; J < n; ++J) {
                C[J] = I.spatial(Ii, A, J, J);
                X[J] = I.spatial(Ii, J, J, A);
            }
            double acc = std::fabs(I.h(i, a));
            double* V = &Vrow[(size_t)a * nso];
            for (int j = 0; j < nso; ++j) {
                const double c = C[j % n];
                const double x = (j / n == sig) ? X[j % n] : 0.0;
                V[j] = c - x;
                acc += std::fabs(c - x);
            }
            if (acc > eps) order.emplace_back(acc, a);
        }
        std::sort(order.begin(), order.end(), [](const std::pair<double, int>& u, const std::pair<double, int>& w) {
            if (u.first != w.first) return u.first > w.first;
            return u.second < w.second;
        });
        // V of the row's entries, j-major: V_e[j] at (s_off[i] nso + j len + e)
        const size_t len = order.size(), v0 = T.sV.size();
        T.sV.resize(v0 + len * (size_t)nso);
        for (size_t e = 0; e < len; ++e) {
            const int a = order[e].second;
            T.sa.push_back(a);
            T.sS.push_back(order[e].first);
            T.sh.push_back(I.h(i, a));
            const double* V = &Vrow[(size_t)a * nso];
            for (int j = 0; j < nso; ++j) T.sV[v0 + (size_t)j * len + e] = V[j];
        }
        T.s_off[i + 1] = (int64_t)T.sa.size();
    }

    // ---------------------------------------------------------------- doubles
    std::vector<uint64_t> keys;
    keys.reserve((size_t)n_nz * 12 + 16);
    for (int64_t k = 0; k < n_nz; ++k) {
        const int p = pqrs[4 * k], q = pqrs[4 * k + 1], r = pqrs[4 * k + 2], s = pqrs[4 * k + 3];
        if (val[k] == 0.0) continue;
        const int img[8][4] = {{p, q, r, s}, {q, p, r, s}, {p, q, s, r}, {q, p, s, r},
                               {r, s, p, q}, {s, r, p, q}, {r, s, q, p}, {s, r, q, p}};
        for (int m = 0; m < 8; ++m) {
            // (A I | B J) = <A B | I J>
            const int A = img[m][0], Ii = img[m][1], B = img[m][2], J = img[m][3];
            if (A != Ii && B != J) keys.push_back(pack_key(Ii, J + n, A, B + n));  // alpha-beta pair
            if (A != B && Ii != J && A != Ii && A != J && B != Ii && B != J) {
                const int i0 = std::min(Ii, J), j0 = std::max(Ii, J);
                const int a0 = std::min(A, B), b0 = std::max(A, B);
                for (int sg = 0; sg < 2; ++sg)
                    keys.push_back(pack_key(i0 + sg * n, j0 + sg * n, a0 + sg * n, b0 + sg * n));
            }
        }
    }
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    struct Ent {
        int32_t i, j, a, b;
        double v;
    };
    std::vector<Ent> ents;
    ents.reserve(keys.size());
    for (uint64_t key : keys) {
        const int i = (int)(key >> 48), j = (int)((key >> 32) & 0xFFFF), a = (int)((key >> 16) & 0xFFFF),
                  b = (int)(key & 0xFFFF);
        const double v = I.so(a, i, b, j) - I.so(a, j, b, i);
        if (std::fabs(v) > eps) ents.push_back({i, j, a, b, v});
    }
    std::sort(ents.begin(), ents.end(), [](const Ent& u, const Ent& w) {
        if (u.i != w.i) return u.i < w.i;
        if (u.j != w.j) return u.j < w.j;
        const double au = std::fabs(u.v), aw = std::fabs(w.v);
        if (au != aw) return au > aw;
        if (u.a != w.a) return u.a < w.a;
        return u.b < w.b;
    });
    T.row_off.assign((size_t)nso * nso + 1, 0);
    T.dab.resize(ents.size() * 2);
    T.dv.resize(ents.size());
    std::vector<int64_t> cnt((size_t)nso * nso, 0);
    for (size_t e = 0; e < ents.size(); ++e) {
        cnt[(size_t)ents[e].i * nso + ents[e].j]++;
        T.dab[2 * e] = ents[e].a;
        T.dab[2 * e + 1] = ents[e].b;
        T.dv[e] = ents[e].v;
    }
    for (size_t k = 0; k < (size_t)nso * nso; ++k) T.row_off[k + 1] = T.row_off[k] + cnt[k];

    // --------------------------------------------------------------- diagonal
    T.D.assign((size_t)nso * nso, 0.0);
    T.hdiag.assign(nso, 0.0);
    for (int i = 0; i < nso; ++i) {
        T.hdiag[i] = I.h(i, i);
        for (int j = 0; j < nso; ++j)
            if (j != i) T.D[(size_t)i * nso + j] = I.so(i, i, j, j) - I.so(i, j, j, i);
    }
    return std::string();
}

}  // namespace vmc

// Host-side planning for SparStencil on gfx950 (arXiv 2506.22969, Section 3).
#include "planner.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <queue>

namespace ss {

Geometry make_geometry(int ndim, int k, int r1, int r2) {
    Geometry gm;
    gm.ndim = ndim;
    gm.k = k;
    gm.r1 = r1;
    gm.r2 = (ndim == 1) ? 1 : r2;
    gm.g = k + r1 - 1;
    gm.m_b = (ndim == 1) ? 1 : k + gm.r2 - 1;
    gm.planes = (ndim == 3) ? k : 1;
    return gm;
}

// Column c of A' is patch element (pz, pr, pc) with c = (pz*m_b + pr)*g + pc;
// row t is output (ty, tx) with t = ty*r1 + tx.  Horizontal crush shifts the
// kernel row by one column per output of a row; vertical crush shifts by one
// row segment per output row (Section 3.1), so the entry is nonzero inside
// the bounding box: 0 <= pc - tx < k and 0 <= pr - ty < k.
bool structural(const Geometry &gm, int row, int col) {
    const int ty = row / gm.r1, tx = row % gm.r1;
    const int within = col % (gm.m_b * gm.g);
    const int pr = within / gm.g, pc = within % gm.g;
    const int dx = pc - tx;
    if (dx < 0 || dx >= gm.k) return false;
    if (gm.ndim == 1) return true;
    const int dy = pr - ty;
    return dy >= 0 && dy < gm.k;
}

std::vector<double> morph_matrix(const Geometry &gm, const std::vector<double> &w) {
    const int mp = gm.m_prime(), kp = gm.k_prime(), k = gm.k;
    std::vector<double> a((size_t)mp * kp, 0.0);
    for (int row = 0; row < mp; ++row) {
        const int ty = row / gm.r1, tx = row % gm.r1;
        for (int col = 0; col < kp; ++col) {
            if (!structural(gm, row, col)) continue;
            const int pz = col / (gm.m_b * gm.g);
            const int within = col % (gm.m_b * gm.g);
            const int dy = within / gm.g - ty, dx = within % gm.g - tx;
            size_t widx;
            if (gm.ndim == 1) widx = dx;
            else if (gm.ndim == 2) widx = (size_t)dy * k + dx;
            else widx = ((size_t)pz * k + dy) * k + dx;
            a[(size_t)row * kp + col] = w[widx];
        }
    }
    return a;
}

// Algorithm 1 (hierarchical two-level matching), stated in closed form.
// Level 1: two blocks (row segments) s1 = max(floor(m/2), k) apart never
// share an output row (Theorem 1), so block i takes block i + s1 for every
// i below n1 = min(s1, m - s1); past n1 a block is either the partner of an
// earlier one or has none.  Level 2, inside every block left over: column u
// takes column u + s2 (s2 = max(floor(g/2), k)) for u below
// n2 = min(s2, g - s2), and each of the block's other columns that is no
// such partner gets a zero node.  Output order: the block pairs expanded
// column by column, then the leftover blocks' pairs by (block, column).
PairList two_level_matching(int m_blocks, int g, int k) {
    PairList out;
    const int s1 = std::max(m_blocks / 2, k);
    const int n1 = std::max(0, std::min(s1, m_blocks - s1));
    for (int i = 0; i < n1; ++i)
        for (int t = 0; t < g; ++t) out.pairs.emplace_back(i * g + t, (i + s1) * g + t);
    const int s2 = std::max(g / 2, k);
    const int n2 = std::max(0, std::min(s2, g - s2));
    for (int x = 0; x < m_blocks; ++x) {
        if (x < n1 || (x >= s1 && x < s1 + n1)) continue;
        for (int u = 0; u < g; ++u) {
            if (u < n2) {
                out.pairs.emplace_back(x * g + u, x * g + u + s2);
            } else if (u < s2 || u >= s2 + n2) {
                out.pairs.emplace_back(x * g + u, kZeta);
                ++out.zeros;
            }
        }
    }
    return out;
}

PairList matrix_pairs(const Geometry &gm) {
    const PairList one = two_level_matching(gm.m_b, gm.g, gm.k);
    PairList all;
    const int plane = gm.m_b * gm.g;
    for (int pz = 0; pz < gm.planes; ++pz) {
        for (const auto &p : one.pairs)
            all.pairs.emplace_back(p.first + pz * plane, p.second == kZeta ? kZeta : p.second + pz * plane);
        all.zeros += one.zeros;
    }
    return all;
}

std::vector<int> group_pairs(const PairList &pl, int kfrag) {
    std::vector<std::pair<int, int>> ps = pl.pairs;
    if (ps.size() % 2) ps.emplace_back(kZeta, kZeta);
    while ((2 * ps.size()) % (size_t)kfrag) ps.emplace_back(kZeta, kZeta);
    std::vector<int> perm;
    perm.reserve(2 * ps.size());
    for (size_t j = 0; j < ps.size(); j += 2) {
        perm.push_back(ps[j].first);
        perm.push_back(ps[j + 1].first);
        perm.push_back(ps[j].second);
        perm.push_back(ps[j + 1].second);
    }
    return perm;
}

static std::vector<char> used_columns(const Geometry &gm, const std::vector<double> &amat) {
    const int mp = gm.m_prime(), kp = gm.k_prime();
    std::vector<char> used(kp, 0);
    for (int row = 0; row < mp; ++row)
        for (int c = 0; c < kp; ++c)
            if (amat[(size_t)row * kp + c] != 0.0) used[c] = 1;
    return used;
}

// Maximum-cardinality matching in a general graph (Edmonds' blossom
// algorithm, the general matcher the paper's Section 3.2 names for
// structures that are not staircases): grow an alternating tree from each
// free vertex by breadth-first search; an edge between two outer vertices of
// the tree closes an odd cycle (a blossom), whose vertices are then treated
// as its base; an edge to a free vertex outside the tree completes an
// augmenting path, which is flipped.  mate[v] = v's partner or -1.
static std::vector<int> max_matching(int n, const std::vector<std::vector<int>> &adj) {
    std::vector<int> mate(n, -1), parent(n), base(n), label(n);
    std::vector<char> in_blossom(n), on_path(n);
    auto lca = [&](int a, int b) {
        std::fill(on_path.begin(), on_path.end(), 0);
        for (;;) {
            a = base[a];
            on_path[a] = 1;
            if (mate[a] < 0) break;
            a = parent[mate[a]];
        }
        for (;;) {
            b = base[b];
            if (on_path[b]) return b;
            b = parent[mate[b]];
        }
    };
    auto mark_path = [&](int v, int b, int child) {
        while (base[v] != b) {
            in_blossom[base[v]] = in_blossom[base[mate[v]]] = 1;
            parent[v] = child;
            child = mate[v];
            v = parent[mate[v]];
        }
    };
    auto find_path = [&](int root) -> int {
        std::fill(label.begin(), label.end(), 0);        // 0 unreached, 1 outer
        std::fill(parent.begin(), parent.end(), -1);
        std::iota(base.begin(), base.end(), 0);
        std::queue<int> q;
        label[root] = 1;
        q.push(root);
        while (!q.empty()) {
            const int v = q.front();
            q.pop();
            for (int u : adj[v]) {
                if (base[v] == base[u] || mate[v] == u) continue;
                if (u == root || (mate[u] >= 0 && parent[mate[u]] >= 0)) {
                    // u is an outer vertex: a blossom closes
                    const int b = lca(v, u);
                    std::fill(in_blossom.begin(), in_blossom.end(), 0);
                    mark_path(v, b, u);
                    mark_path(u, b, v);
                    for (int i = 0; i < n; ++i)
                        if (in_blossom[base[i]]) {
                            base[i] = b;
                            if (!label[i]) {
                                label[i] = 1;
                                q.push(i);
                            }
                        }
                } else if (parent[u] < 0) {
                    parent[u] = v;
                    if (mate[u] < 0) return u;               // augmenting path found
                    label[mate[u]] = 1;
                    q.push(mate[u]);
                }
            }
        }
        return -1;
    };
    for (int v = 0; v < n; ++v) {
        if (mate[v] >= 0) continue;
        const int u = find_path(v);
        for (int x = u; x >= 0;) {          // flip the path
            const int pv = parent[x], ppv = mate[pv];
            mate[x] = pv;
            mate[pv] = x;
            x = ppv;
        }
    }
    return mate;
}

std::vector<int> compact_groups(const Geometry &gm, const std::vector<double> &amat, const std::vector<int> &perm,
                                int kfrag) {
    const int mp = gm.m_prime(), kp = gm.k_prime();
    const std::vector<char> used = used_columns(gm, amat);
    auto is_used = [&](int c) { return c != kZeta && used[c]; };
    // columns a and b may share a 2:4 half when no row is nonzero in both
    auto apart = [&](int a, int b) {
        if (a == kZeta || b == kZeta) return true;
        for (int row = 0; row < mp; ++row)
            if (amat[(size_t)row * kp + a] != 0.0 && amat[(size_t)row * kp + b] != 0.0) return false;
        return true;
    };
    // with an even row length every half of a kept group is a domino
    // (pc, pc+1), pc even; a group with another half is taken apart into such
    // dominoes (each once, in order of first appearance)
    const bool aligned_only = gm.g % 2 == 0;
    auto aligned = [&](int a, int b) {
        if (a == kZeta && b == kZeta) return true;
        return a != kZeta && b == a + 1 && (a % gm.g) % 2 == 0;
    };
    std::vector<char> seen(aligned_only ? kp : 0, 0);
    std::vector<int> out;
    std::vector<std::pair<int, int>> half;   // used dominoes set aside for re-pairing
    for (size_t j = 0; j + 3 < perm.size(); j += 4) {
        if (aligned_only && !(aligned(perm[j], perm[j + 1]) && aligned(perm[j + 2], perm[j + 3]))) {
            for (size_t i = j; i < j + 4; ++i) {
                const int c = perm[i];
                if (c == kZeta) continue;
                const int d0 = c - (c % gm.g) % 2;
                if (seen[d0]) continue;
                seen[d0] = 1;
                if (is_used(d0) || is_used(d0 + 1)) half.emplace_back(d0, d0 + 1);
            }
            continue;
        }
        const bool ua = is_used(perm[j]) || is_used(perm[j + 1]);
        const bool ub = is_used(perm[j + 2]) || is_used(perm[j + 3]);
        if (ua && ub) out.insert(out.end(), perm.begin() + j, perm.begin() + j + 4);
        else if (ua) half.emplace_back(perm[j], perm[j + 1]);
        else if (ub) half.emplace_back(perm[j + 2], perm[j + 3]);
    }
    // re-pair the set-aside dominoes by a maximum matching of the graph
    // whose edges join two dominoes that may share a 4-group: their first
    // columns and their second columns are conflict-free pairs (Definition
    // 1), the pairing Algorithm 1's own groups have.  Each matched couple is
    // one group, at its smaller index; an unmatched domino gets a zero one.
    const int nh = (int)half.size();
    std::vector<std::vector<int>> adj(nh);
    for (int i = 0; i < nh; ++i)
        for (int j = i + 1; j < nh; ++j)
            if (apart(half[i].first, half[j].first) && apart(half[i].second, half[j].second)) {
                adj[i].push_back(j);
                adj[j].push_back(i);
            }
    const std::vector<int> mate = max_matching(nh, adj);
    for (int i = 0; i < nh; ++i) {
        if (mate[i] >= 0 && mate[i] < i) continue;
        out.push_back(half[i].first);
        out.push_back(half[i].second);
        out.push_back(mate[i] >= 0 ? half[mate[i]].first : kZeta);
        out.push_back(mate[i] >= 0 ? half[mate[i]].second : kZeta);
    }
    while (out.size() % (size_t)kfrag) out.push_back(kZeta);
    return out;
}

std::vector<int> dense_order(const Geometry &gm, const std::vector<double> &amat, int kfrag) {
    const int kp = gm.k_prime();
    const std::vector<char> used = used_columns(gm, amat);
    std::vector<int> out;
    for (int c = 0; c < kp; c += 2) {
        const bool u = used[c] || (c + 1 < kp && used[c + 1]);
        if (!u) continue;
        out.push_back(c);
        out.push_back(c + 1 < kp ? c + 1 : kZeta);
    }
    while (out.size() % (size_t)kfrag) out.push_back(kZeta);
    return out;
}

bool compress(const Geometry &gm, const std::vector<double> &amat, const std::vector<int> &perm,
              Compressed *out, bool by_value) {
    const int mp = gm.m_prime(), kp = gm.k_prime();
    const int groups = (int)perm.size() / 4;
    auto live_at = [&](int row, int c) {
        if (c == kZeta) return false;
        return by_value ? amat[(size_t)row * kp + c] != 0.0 : structural(gm, row, c);
    };
    out->values.assign((size_t)mp * groups * 2, 0.0);
    out->meta.assign((size_t)mp * groups * 2, 0);
    for (int row = 0; row < mp; ++row) {
        for (int j = 0; j < groups; ++j) {
            int live[4], nlive = 0;
            for (int p = 0; p < 4; ++p) {
                const int c = perm[4 * j + p];
                if (live_at(row, c)) live[nlive++] = p;
            }
            if (nlive > 2) return false;
            int pos[2], n = 0;
            for (int t = 0; t < nlive; ++t) pos[n++] = live[t];
            for (int p = 0; p < 4 && n < 2; ++p) {
                bool taken = false;
                for (int t = 0; t < nlive; ++t) taken |= (live[t] == p);
                if (!taken) pos[n++] = p;
            }
            if (pos[0] > pos[1]) std::swap(pos[0], pos[1]);
            for (int t = 0; t < 2; ++t) {
                const int c = perm[4 * j + pos[t]];
                double v = 0.0;
                if (live_at(row, c)) v = amat[(size_t)row * kp + c];
                out->values[((size_t)row * groups + j) * 2 + t] = v;
                out->meta[((size_t)row * groups + j) * 2 + t] = (uint8_t)pos[t];
            }
        }
    }
    return true;
}

// Round |x| to the nearest multiple of 2^q with ties to even, q chosen from
// the binade (subnormals share the minimum exponent's spacing).  man = stored
// mantissa bits, emin = minimum normal exponent, bias = exponent bias.
static bool round_bits(double x, int man, int emin, int emax, int bias, uint16_t *bits) {
    const uint16_t sign = std::signbit(x) ? (uint16_t)(1u << (man + (bias == 15 ? 5 : 8))) : 0;
    const double ax = std::fabs(x);
    if (std::isnan(x)) return false;
    if (ax == 0.0) { *bits = sign; return true; }
    int e2;
    std::frexp(ax, &e2);                  // ax = f * 2^e2, f in [0.5, 1)
    int e = e2 - 1;                       // ax in [2^e, 2^(e+1))
    if (e < emin) e = emin;
    const int q = e - man;                // spacing exponent
    double n = std::nearbyint(std::ldexp(ax, -q));  // exact scaling, RNE
    // n in [2^man, 2^(man+1)] for normals, [0, 2^(man+1)] for subnormals
    long long ni = (long long)n;
    int biased;
    if (ni >= (1LL << (man + 1))) { ni >>= 1; ++e; }  // carried into next binade
    if (ni < (1LL << man)) {
        biased = 0;                      // subnormal (or zero after rounding)
    } else {
        biased = e + bias;
        ni -= (1LL << man);
    }
    if (e > emax) return false;
    *bits = (uint16_t)(sign | (uint16_t)(biased << man) | (uint16_t)ni);
    return true;
}

bool to_f16_bits(double x, uint16_t *bits) { return round_bits(x, 10, -14, 15, 15, bits); }
bool to_bf16_bits(double x, uint16_t *bits) { return round_bits(x, 7, -126, 127, 127, bits); }

double f16_value(uint16_t b) {
    const int s = b >> 15, e = (b >> 10) & 31, m = b & 1023;
    double v;
    if (e == 0) v = std::ldexp((double)m, -24);
    else if (e == 31) v = m ? NAN : INFINITY;
    else v = std::ldexp((double)(m + 1024), e - 25);
    return s ? -v : v;
}

double bf16_value(uint16_t b) {
    uint32_t u = (uint32_t)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return (double)f;
}

// c = a composed with w: c[o] = sum over a's offsets p (row-major) of
// a[p] * w[o - p], outputs visited row-major.
static std::vector<double> compose2(const std::vector<double> &a, int ka, const std::vector<double> &w,
                                    int kw, int ndim) {
    const int kc = ka + kw - 1;
    const int na = (ndim >= 3 ? ka : 1), nw = (ndim >= 3 ? kw : 1), nc = (ndim >= 3 ? kc : 1);
    const int ma = (ndim >= 2 ? ka : 1), mw = (ndim >= 2 ? kw : 1), mc = (ndim >= 2 ? kc : 1);
    std::vector<double> c((size_t)nc * mc * kc, 0.0);
    for (int oz = 0; oz < nc; ++oz)
        for (int oy = 0; oy < mc; ++oy)
            for (int ox = 0; ox < kc; ++ox) {
                double acc = 0.0;
                for (int az = 0; az < na; ++az)
                    for (int ay = 0; ay < ma; ++ay)
                        for (int ax = 0; ax < ka; ++ax) {
                            const int bz = oz - az, by = oy - ay, bx = ox - ax;
                            if (bz < 0 || bz >= nw || by < 0 || by >= mw || bx < 0 || bx >= kw) continue;
                            acc += a[((size_t)az * ma + ay) * ka + ax] * w[((size_t)bz * mw + by) * kw + bx];
                        }
                c[((size_t)oz * mc + oy) * kc + ox] = acc;
            }
    return c;
}

std::vector<double> compose(const std::vector<double> &w, int ndim, int k, int steps, int *k_out) {
    std::vector<double> c = w;
    int kc = k;
    for (int s = 1; s < steps; ++s) {
        c = compose2(c, kc, w, k, ndim);
        kc = kc + k - 1;
    }
    *k_out = kc;
    return c;
}

// MI355X constants of the analytical model: 2.4 GHz, 256 CUs x 4 matrix
// cores, 16 cycles per 16x16x64 sparse (or 16x16x32 dense) f16 MMA (the
// dense 2.5 PFLOP/s peak), 8 TB/s HBM, 128 B/clk/CU of LDS.
static constexpr double kFreq = 2.4e9;
static constexpr double kNtcu = 1024.0;
static constexpr double kCpi = 16.0;
static constexpr double kBwGlobal = 8.0e12;
static constexpr double kBwShared = 256.0 * 128.0 * 2.4e9;

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

ModelRow model_time(const ModelParams &mp, int r1, int r2) {
    const Geometry gm = make_geometry(mp.ndim, mp.k, r1, r2);
    const std::vector<int> perm = group_pairs(matrix_pairs(gm), mp.kfrag);
    const int kpad = (int)perm.size();
    int64_t tiles, points;
    if (mp.ndim == 1) {
        tiles = ceil_div(mp.dims[0], r1);
        points = mp.dims[0];
    } else if (mp.ndim == 2) {
        tiles = ceil_div(mp.dims[0], r2) * ceil_div(mp.dims[1], r1);
        points = mp.dims[0] * mp.dims[1];
    } else {
        tiles = mp.dims[0] * ceil_div(mp.dims[1], r2) * ceil_div(mp.dims[2], r1);
        points = mp.dims[0] * mp.dims[1] * mp.dims[2];
    }
    // Eq. 9 with the converted column count
    const double n_mma = (double)(ceil_div(gm.m_prime(), 16) * ceil_div(kpad, mp.kfrag) * ceil_div(tiles, 16));
    ModelRow r;
    r.r1 = r1;
    r.r2 = gm.r2;
    r.k_pad = kpad;
    r.t_compute = n_mma * mp.passes * kCpi / (kFreq * kNtcu);                         // Eq. 7
    const double data_r = (double)points * mp.elem_bytes * mp.planes_state;
    const double data_w = data_r;
    r.t_global = (data_r + data_w) / kBwGlobal;
    // Eq. 10, reading 'm/2' as m'/2 (A' is held compressed to half width)
    const double trans = (double)gm.k_prime() * (gm.m_prime() / 2.0 + (double)tiles);
    // each part of the operands moves through LDS: one (plain), two (hi and
    // lo: three products), three (hi, mid and lo: six products)
    const int parts = mp.passes >= 6 ? 3 : mp.passes > 1 ? 2 : 1;
    const double trans_rw = trans * mp.coef_bytes * parts;
    r.t_shared = (trans_rw + trans_rw) / kBwShared;
    r.t = std::max(r.t_compute, std::max(r.t_global, r.t_shared));                     // Eqs. 6, 8
    return r;
}

static bool close_rel(double a, double b) { return std::fabs(a - b) <= 1e-12 * std::max(std::fabs(a), std::fabs(b)); }

// Eq. 11 tie-break: T, then T_compute (the matrix work separates layouts
// that tie on an HBM-bound T), then T_shared, then K_pad, then r1*r2, then r1.
bool model_better(const ModelRow &a, const ModelRow &b) {
    if (!close_rel(a.t, b.t)) return a.t < b.t;
    if (!close_rel(a.t_compute, b.t_compute)) return a.t_compute < b.t_compute;
    if (!close_rel(a.t_shared, b.t_shared)) return a.t_shared < b.t_shared;
    if (a.k_pad != b.k_pad) return a.k_pad < b.k_pad;
    if (a.r1 * a.r2 != b.r1 * b.r2) return a.r1 * a.r2 < b.r1 * b.r2;
    return a.r1 < b.r1;
}

bool pair_aligned(const Geometry &gm, const std::vector<int> &perm) {
    for (size_t kk = 0; kk + 1 < perm.size(); kk += 2) {
        const int a = perm[kk], b = perm[kk + 1];
        if (a == kZeta && b == kZeta) continue;
        if (a == kZeta || b == kZeta) return false;
        if (b != a + 1) return false;
        const int pc = a % gm.g;
        if (pc % 2 != 0 || pc + 1 >= gm.g) return false;
    }
    return true;
}

}  // namespace ss

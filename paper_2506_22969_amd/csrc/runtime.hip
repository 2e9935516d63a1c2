// C ABI of libsparstencil: plan construction (host tables + device upload),
// sweeps, runs and read-back.  See include/sparstencil.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/sparstencil.h"
#include "kargs.hpp"
#include "kgeom.hpp"
#include "plan.hpp"
#include "planner.hpp"

using namespace ss;

namespace {

const int64_t kMaxDim = (int64_t)1 << 30;

size_t state_bytes(int dtype) {
    switch (dtype) {
        case SS_F64: return 8;
        case SS_F32: case SS_F32_SPLIT_F16: case SS_F32_SPLIT_BF16: return 4;
        case SS_F16: return 2;
        case SS_SPLIT_BF16: return 4;  // two 2-byte planes
        case SS_SPLIT3_BF16: return 6; // three 2-byte planes
        default: return 0;
    }
}

int64_t points(const ss_plan_ *p) { return p->dims[0] * p->dims[1] * p->dims[2]; }

bool valid_star(const std::vector<double> &w, int ndim, int r) {
    const int k = 2 * r + 1;
    const int nz = ndim == 3 ? k : 1, ny = ndim >= 2 ? k : 1;
    for (int a = 0; a < nz; ++a)
        for (int b = 0; b < ny; ++b)
            for (int c = 0; c < k; ++c) {
                int off = 0;
                if (ndim == 3 && a != r) ++off;
                if (ndim >= 2 && b != r) ++off;
                if (c != r) ++off;
                if (off > 1 && w[((size_t)a * ny + b) * k + c] != 0.0) return false;
            }
    return true;
}

// Fill the MMA kernel tables for the kernel's K order `kperm` (A' column per
// K slot, kZeta for zero columns).  Sparse: compressed A'' in the SMFMAC
// operand layout with its index words; dense: A' columns in kperm order.
// Gather offsets are in bytes from the tile's patch origin within one input
// plane of the slab: FP32 rows `pitch` values apart (the 3-D kernel picks the
// plane per K chunk), bfloat16 planes rows of interleaved hi/lo dword pairs
// `pitch` bytes apart, or (pw > 0) converted rows `pitch` dwords apart whose
// pair j sits at dword pw * (j + j / padg).
ss_status build_mma_tables(ss_plan_ *p, const Geometry &gm, const std::vector<int> &kperm, int mode, int part,
                           int kc_count, int pitch, bool planes, int pw, int padg, std::vector<uint8_t> *blob,
                           size_t *off_hi, size_t *off_lo, size_t *off_mid, size_t *off_idx, size_t *off_boff,
                           size_t *off_zero) {
    const int MB = gm.m_prime() / 16;
    const std::vector<double> amat = morph_matrix(gm, p->w);
    const int kp = gm.k_prime();
    // coefficient parts: hi + lo (binary16 lo scaled by sigma = 2^11), or for
    // a three-part state bfloat16 hi + mid + lo, each part the rounding of
    // what the parts before it leave
    const bool three = p->dtype == SS_SPLIT3_BF16;
    auto split = [&](double c, uint16_t *h, uint16_t *l, uint16_t *m) -> bool {
        *m = 0;
        if (part == kPartF16) {
            if (!to_f16_bits(c, h)) return false;
            return to_f16_bits((c - f16_value(*h)) * 2048.0, l);
        }
        if (!to_bf16_bits(c, h)) return false;
        if (!three) return to_bf16_bits(c - bf16_value(*h), l);
        const double r = c - bf16_value(*h);
        if (!to_bf16_bits(r, m)) return false;
        return to_bf16_bits(r - bf16_value(*m), l);
    };
    const int VPK = mode == kSparse ? 8 : 4;
    if ((int)kperm.size() != kc_count * (mode == kSparse ? 64 : 32)) return SS_E_UNSUPPORTED;
    std::vector<uint16_t> ahi((size_t)MB * kc_count * 64 * 8), alo(ahi.size()), amid(three ? ahi.size() : 0);
    uint16_t mid_unused = 0;
    auto mid_at = [&](size_t t) -> uint16_t * { return three ? &amid[t] : &mid_unused; };
    std::vector<uint32_t> aidx((size_t)MB * kc_count * 64, 0);
    std::vector<int32_t> boff((size_t)kc_count * 4 * VPK, 0);
    if (mode == kSparse) {
        Compressed cm;
        if (!compress(gm, amat, kperm, &cm, true)) return SS_E_UNSUPPORTED;
        const int groups = (int)kperm.size() / 4;
        for (int mb = 0; mb < MB; ++mb)
            for (int kc = 0; kc < kc_count; ++kc)
                for (int l = 0; l < 64; ++l) {
                    const int r = mb * 16 + (l & 15), qa = l >> 4;
                    uint32_t word = 0;
                    for (int ea = 0; ea < 8; ++ea) {
                        const int gl = ea >> 1, s = ea & 1;
                        const int qb = 2 * (qa & 1) + (gl >> 1);
                        const int m = 2 * (qa >> 1) + (gl & 1);
                        const int j = kc * 16 + 4 * qb + m;     // 4-group of the K order
                        const size_t vi = ((size_t)r * groups + j) * 2 + s;
                        const size_t t = (((size_t)mb * kc_count + kc) * 64 + l) * 8 + ea;
                        if (!split(cm.values[vi], &ahi[t], &alo[t], mid_at(t))) return SS_E_UNSUPPORTED;
                        word |= (uint32_t)cm.meta[vi] << (2 * ea);
                    }
                    aidx[((size_t)mb * kc_count + kc) * 64 + l] = word;
                }
    } else {
        for (int mb = 0; mb < MB; ++mb)
            for (int kc = 0; kc < kc_count; ++kc)
                for (int l = 0; l < 64; ++l)
                    for (int e = 0; e < 8; ++e) {
                        const int r = mb * 16 + (l & 15);
                        const int col = kperm[kc * 32 + 8 * (l >> 4) + e];
                        const double c = col != kZeta && col < kp ? amat[(size_t)r * kp + col] : 0.0;
                        const size_t t = (((size_t)mb * kc_count + kc) * 64 + l) * 8 + e;
                        if (!split(c, &ahi[t], &alo[t], mid_at(t))) return SS_E_UNSUPPORTED;
                    }
    }
    // gather offsets: K slot pair (kk, kk+1) of B register v of lane group qb
    const int plane = gm.m_b * gm.g;
    for (int kc = 0; kc < kc_count; ++kc)
        for (int qb = 0; qb < 4; ++qb)
            for (int v = 0; v < VPK; ++v) {
                const int kk = mode == kSparse ? kc * 64 + 16 * qb + 2 * v : kc * 32 + 8 * qb + 2 * v;
                const int col = kperm[kk];
                int32_t o = 0;
                if (col != kZeta) {
                    const int pr = (col % plane) / gm.g, pc = col % gm.g;
                    if (pw > 0) {
                        // the register's pair starts at an even patch column
                        if (pc % 2) return SS_E_UNSUPPORTED;
                        const int j = pc / 2;
                        o = 4 * (pr * pitch + pw * (j + j / padg));
                    } else if (planes) {
                        // slab rows of interleaved hi/lo dword pairs (pitch
                        // in bytes): value column c sits at byte
                        // 8 * (c / 2) + 2 * (c % 2) of the row (hi; lo 4
                        // bytes on), counted from the dword pair of the tile
                        // origin, whose parity is that of the radius (the
                        // slab margin is even)
                        const int c = (p->rad & 1) + pc;
                        o = pr * pitch + (c >> 1) * 8 + (c & 1) * 2;
                    } else {
                        o = (pr * pitch + pc) * 4;
                    }
                }
                // the kernels keep two offsets per 32-bit register
                if (o >= 65536) return SS_E_UNSUPPORTED;
                boff[((size_t)kc * 4 + qb) * VPK + v] = o;
            }
    // pack: a_hi | a_lo | a_mid | a_idx | boff | 1 KiB of zeros, each
    // 256-byte aligned (a_mid empty but for three-part states)
    auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
    *off_hi = 0;
    *off_lo = align(*off_hi + ahi.size() * 2);
    *off_mid = align(*off_lo + alo.size() * 2);
    *off_idx = align(*off_mid + amid.size() * 2);
    *off_boff = align(*off_idx + aidx.size() * 4);
    *off_zero = align(*off_boff + boff.size() * 4);
    blob->assign(*off_zero + 1024, 0);
    std::memcpy(blob->data() + *off_hi, ahi.data(), ahi.size() * 2);
    std::memcpy(blob->data() + *off_lo, alo.data(), alo.size() * 2);
    if (three) std::memcpy(blob->data() + *off_mid, amid.data(), amid.size() * 2);
    std::memcpy(blob->data() + *off_idx, aidx.data(), aidx.size() * 4);
    std::memcpy(blob->data() + *off_boff, boff.data(), boff.size() * 4);
    p->kernel_lut = boff;
    // read-back copy of the A fragments (SS_Q_KERNEL_FRAGS)
    const int32_t head[4] = {MB, kc_count, mode, three ? 3 : 2};
    std::vector<uint8_t> &fr = p->kernel_frags;
    fr.assign((const uint8_t *)head, (const uint8_t *)head + sizeof head);
    auto put = [&](const void *d, size_t n) { fr.insert(fr.end(), (const uint8_t *)d, (const uint8_t *)d + n); };
    put(ahi.data(), ahi.size() * 2);
    put(alo.data(), alo.size() * 2);
    if (three) put(amid.data(), amid.size() * 2);
    if (mode == kSparse) put(aidx.data(), aidx.size() * 4);
    return SS_OK;
}

// Canonical tables of the sparse layout: perm, compressed values, metadata,
// hi/lo parts, gather LUT.
ss_status build_canonical(ss_plan_ *p, const Geometry &gm, int part, int kfrag) {
    const std::vector<double> amat = morph_matrix(gm, p->w);
    const PairList pl = matrix_pairs(gm);
    std::vector<int> perm = group_pairs(pl, kfrag);
    Compressed cm;
    if (!compress(gm, amat, perm, &cm)) return SS_E_UNSUPPORTED;
    p->perm.assign(perm.begin(), perm.end());
    p->values = cm.values;
    p->meta = cm.meta;
    p->hi.resize(cm.values.size());
    p->lo.resize(cm.values.size());
    const bool three = p->dtype == SS_SPLIT3_BF16;
    p->mid.assign(three ? cm.values.size() : 0, 0);
    for (size_t i = 0; i < cm.values.size(); ++i) {
        const double c = cm.values[i];
        bool ok;
        if (part == kPartF16) {
            ok = to_f16_bits(c, &p->hi[i]) && to_f16_bits((c - f16_value(p->hi[i])) * 2048.0, &p->lo[i]);
        } else if (three) {
            ok = to_bf16_bits(c, &p->hi[i]);
            const double r = ok ? c - bf16_value(p->hi[i]) : 0.0;
            ok = ok && to_bf16_bits(r, &p->mid[i]) && to_bf16_bits(r - bf16_value(p->mid[i]), &p->lo[i]);
        } else {
            ok = to_bf16_bits(c, &p->hi[i]) && to_bf16_bits(c - bf16_value(p->hi[i]), &p->lo[i]);
        }
        if (!ok) return SS_E_UNSUPPORTED;
    }
    p->lut.assign(perm.size() * 3, -1);
    const int plane = gm.m_b * gm.g;
    for (size_t kk = 0; kk < perm.size(); ++kk) {
        const int c = perm[kk];
        if (c == kZeta) continue;
        p->lut[kk * 3 + 0] = c / plane;
        p->lut[kk * 3 + 1] = (c % plane) / gm.g;
        p->lut[kk * 3 + 2] = c % gm.g;
    }
    p->info.zeros = pl.zeros;
    return SS_OK;
}

ss_status upload(ss_plan_ *p, const std::vector<uint8_t> &blob) {
    if (p->host_only) return SS_OK;
    if (hipGetDevice(&p->device) != hipSuccess) return SS_E_DEVICE;
    if (blob.empty()) return SS_OK;
    if (hipMalloc(&p->dev, blob.size()) != hipSuccess) {
        p->dev = nullptr;
        return SS_E_NOMEM;
    }
    if (hipMemcpy(p->dev, blob.data(), blob.size(), hipMemcpyHostToDevice) != hipSuccess) return SS_E_DEVICE;
    return SS_OK;
}

// State layout of a dtype on the MMA path.
int mma_state(int dtype) {
    return dtype == SS_SPLIT_BF16    ? kStatePlanes
           : dtype == SS_SPLIT3_BF16 ? kStatePlanes3
           : dtype == SS_F16         ? kStateF16
                                     : kStateF32;
}

// The slab-pipelined kernels (matrix-core and LDS direct) address a work
// item's rows, and a 3-D plane's rows, with 32-bit offsets: a 2-D item of
// kItemRows rows, or a 3-D plane, must span fewer than 2^31 bytes.  Larger
// grids run on the plain direct kernel (64-bit indexing).
bool slab_offsets_fit(const ss_plan_ *p) {
    const int64_t nx = p->dims[2], ny = p->dims[1];
    const int64_t bytes =
        p->dtype == SS_F64 ? 8 : (p->dtype == SS_SPLIT_BF16 || p->dtype == SS_SPLIT3_BF16 || p->dtype == SS_F16) ? 2 : 4;
    const int64_t limit = (int64_t)1 << 31;
    if (p->ndim == 3) return ny * nx * bytes < limit;
    return (int64_t)kItemRows * nx * bytes < limit;
}

// K order of a 2-D matrix-core kernel: Algorithm 1's groups compacted to the
// columns the stencil uses (sparse), or the used column pairs in natural
// order (dense).
std::vector<int> kernel_order(const ss_plan_ *p, const Geometry &gm, int mode) {
    const std::vector<double> amat = morph_matrix(gm, p->w);
    if (mode == kSparse) return compact_groups(gm, amat, group_pairs(matrix_pairs(gm), 64), 64);
    return dense_order(gm, amat, 32);
}

ss_status plan_mma2d(ss_plan_ *p, int engine) {
    const int part = (p->dtype == SS_F32_SPLIT_F16 || p->dtype == SS_F16) ? kPartF16 : kPartBF16;
    const int state = mma_state(p->dtype);
    const int mode = engine == SS_ENGINE_SMFMAC ? kSparse : kDense;
    // plain binary16: one product of the rounded coefficients and state;
    // three-part states: hi*hi, hi*mid, mid*hi, hi*lo, lo*hi, mid*mid
    const int passes = state == kStateF16 ? 1 : state == kStatePlanes3 ? 6 : 3;
    if (!slab_offsets_fit(p)) return SS_E_UNSUPPORTED;
    // the planes and binary16 kernels move rows in 8-value (16-byte) pieces
    if (state != kStateF32 && p->dims[2] % 8 != 0) return SS_E_UNSUPPORTED;
    ModelParams mp{};
    mp.ndim = p->ndim;
    mp.k = p->k;
    for (int d = 0; d < 3; ++d) mp.dims[d] = d < p->ndim ? p->dims[3 - p->ndim + d] : 1;
    mp.elem_bytes = state == kStateF32 ? 4 : 2;
    mp.planes_state = state == kStatePlanes3 ? 3 : state == kStatePlanes ? 2 : 1;
    mp.coef_bytes = 2;
    mp.passes = passes;
    mp.kfrag = 64;
    // tiles with instantiated kernels
    MmaKey keys[32];
    const int nkeys = mma2d_keys(p->rad, mode, part, state, keys, 32);
    std::vector<MmaKey> cands;
    for (int i = 0; i < nkeys; ++i) {
        const MmaKey &c = keys[i];
        if (p->info.r1 && (c.r1 != p->info.r1 || c.r2 != p->info.r2)) continue;
        const Geometry gm = make_geometry(2, p->k, c.r1, c.r2);
        if (mode == kDense && gm.g % 2) continue;
        const std::vector<int> order = kernel_order(p, gm, mode);
        if (mode == kSparse && !pair_aligned(gm, order)) continue;
        if ((int)order.size() != (mode == kSparse ? 64 : 32) * c.kc) continue;
        cands.push_back(c);
    }
    if (cands.empty()) return SS_E_UNSUPPORTED;
    ModelRow best{};
    MmaKey key{};
    bool have = false;
    p->model.clear();
    for (const MmaKey &c : cands) {
        const ModelRow r = model_time(mp, c.r1, c.r2);
        const double row[7] = {(double)r.r1, (double)r.r2, r.t, r.t_compute, r.t_global, r.t_shared,
                               (double)r.k_pad};
        p->model.insert(p->model.end(), row, row + 7);
        if (!have || model_better(r, best)) {
            best = r;
            key = c;
            have = true;
        }
    }
    const Geometry gm = make_geometry(2, p->k, key.r1, key.r2);
    ss_status st = build_canonical(p, gm, part, 64);
    if (st != SS_OK) return st;
    const std::vector<int> kperm = kernel_order(p, gm, mode);
    if (mode == kSparse && !pair_aligned(gm, kperm)) return SS_E_UNSUPPORTED;
    p->kperm.assign(kperm.begin(), kperm.end());
    int wgh, row, pw, padg;
    if (!mma2d_geometry(key, &wgh, &row, &pw, &padg)) return SS_E_UNSUPPORTED;
    std::vector<uint8_t> blob;
    size_t o_hi, o_lo, o_mid, o_idx, o_boff, o_zero;
    st = build_mma_tables(p, gm, kperm, mode, part, key.kc, row, state == kStatePlanes, pw, padg, &blob, &o_hi,
                          &o_lo, &o_mid, &o_idx, &o_boff, &o_zero);
    if (st != SS_OK) return st;
    // the planes kernels of an even radius read each B register's hi and lo
    // parts as one dword each: every gather offset must be a whole dword
    if (state == kStatePlanes && p->rad % 2 == 0)
        for (int32_t o : p->kernel_lut)
            if (o % 4) return SS_E_UNSUPPORTED;
    st = upload(p, blob);
    if (st != SS_OK) return st;
    char *d = static_cast<char *>(p->dev);
    p->mma = find_mma2d(key);
    p->margs.periodic = p->boundary == SS_BC_PERIODIC;
    p->margs.inv_sigma = part == kPartF16 && passes == 3 ? 1.0f / 2048.0f : 1.0f;
    p->margs.a_hi = reinterpret_cast<const uint4 *>(d + o_hi);
    p->margs.a_lo = reinterpret_cast<const uint4 *>(d + o_lo);
    p->margs.a_mid = reinterpret_cast<const uint4 *>(d + o_mid);
    p->margs.a_idx = reinterpret_cast<const uint32_t *>(d + o_idx);
    p->margs.boff = reinterpret_cast<const int32_t *>(d + o_boff);
    p->margs.zeros = d + o_zero;
    p->engine = engine;
    p->info.r1 = gm.r1;
    p->info.r2 = gm.r2;
    p->info.m_b = gm.m_b;
    p->info.g = gm.g;
    p->info.planes = gm.planes;
    p->info.m_prime = gm.m_prime();
    p->info.k_prime = gm.k_prime();
    p->info.k_pad = (int)p->perm.size();
    p->info.passes = passes;
    p->info.sigma = part == kPartF16 && passes == 3 ? 2048.0 : 1.0;
    return SS_OK;
}

// The FP32 gather reads each B register's two values from adjacent columns
// of one patch row (two dword reads, any alignment).
bool pairs_adjacent(const Geometry &gm, const std::vector<int> &perm) {
    for (size_t kk = 0; kk + 1 < perm.size(); kk += 2) {
        const int a = perm[kk], b = perm[kk + 1];
        if (a == kZeta && b == kZeta) continue;
        if (a == kZeta || b == kZeta || b != a + 1 || a % gm.g + 1 >= gm.g) return false;
    }
    return true;
}

// 3-D MMA engines (FP32 state).  The kernel's K order keeps every input
// plane in whole chunks, one order for all planes (the kernel gathers an
// input plane once for every plane offset): the 2-D order of a plane's block
// staircase, compacted to the union of the columns any plane offset uses --
// Algorithm 1's groups re-paired (sparse, 64-column chunks) or the used
// column pairs (dense, 32-column chunks).  A 27-point box uses every
// column; a 7-point star composed over two sweeps uses at most a radius-2
// diamond in any plane, which takes half the sparse chunks.  The canonical
// tables (queries) are those of the plain 3-D reading: plane lists
// concatenated, then grouped and padded once.
ss_status plan_mma3d(ss_plan_ *p, int engine) {
    const int part = p->dtype == SS_F32_SPLIT_F16 ? kPartF16 : kPartBF16;
    const int mode = engine == SS_ENGINE_SMFMAC ? kSparse : kDense;
    if (!slab_offsets_fit(p)) return SS_E_UNSUPPORTED;
    MmaKey keys[16];
    const int nkeys = mma3d_keys(p->rad, mode, part, keys, 16);
    const MmaKey *key = nullptr;
    std::vector<int> kperm;
    for (int i = 0; i < nkeys && !key; ++i) {
        const MmaKey &c = keys[i];
        if (p->info.r1 && (c.r1 != p->info.r1 || c.r2 != p->info.r2)) continue;
        const Geometry g2 = make_geometry(2, p->k, c.r1, c.r2);
        const int plane = g2.m_b * g2.g, cpp = c.kc / p->k;
        if (mode == kDense && g2.g % 2) continue;
        // |A'| summed over the plane offsets: nonzero where any plane is
        const size_t kk = (size_t)p->k * p->k;
        std::vector<double> u((size_t)g2.m_prime() * plane, 0.0);
        for (int pz = 0; pz < p->k; ++pz) {
            std::vector<double> wz(p->w.begin() + pz * kk, p->w.begin() + (pz + 1) * kk);
            for (double &v : wz) v = std::fabs(v);
            const std::vector<double> a = morph_matrix(g2, wz);
            for (size_t i = 0; i < u.size(); ++i) u[i] += a[i];
        }
        const std::vector<int> one = mode == kSparse ? compact_groups(g2, u, group_pairs(matrix_pairs(g2), 64), 64)
                                                     : dense_order(g2, u, 32);
        if (!pair_aligned(g2, one)) continue;
        if ((int)one.size() != (mode == kSparse ? 64 : 32) * cpp) continue;
        kperm.clear();
        for (int pz = 0; pz < p->k; ++pz)
            for (int x : one) kperm.push_back(x == kZeta ? kZeta : x + pz * plane);
        key = &keys[i];
    }
    if (!key) return SS_E_UNSUPPORTED;
    const Geometry gm = make_geometry(3, p->k, key->r1, key->r2);
    ss_status st = build_canonical(p, gm, part, 64);
    if (st != SS_OK) return st;
    if (mode == kDense) {
        p->perm.clear();
        const int kd = (gm.k_prime() + 31) / 32 * 32;
        for (int c = 0; c < kd; ++c) p->perm.push_back(c < gm.k_prime() ? c : kZeta);
    }
    // model rows of the one candidate (Eqs. 6-10 for the record)
    ModelParams mp{};
    mp.ndim = 3;
    mp.k = p->k;
    for (int d = 0; d < 3; ++d) mp.dims[d] = p->dims[d];
    mp.elem_bytes = 4;
    mp.planes_state = 1;
    mp.coef_bytes = 2;
    mp.passes = 3;
    mp.kfrag = 64;
    const ModelRow r = model_time(mp, key->r1, key->r2);
    p->model.assign({(double)r.r1, (double)r.r2, r.t, r.t_compute, r.t_global, r.t_shared, (double)r.k_pad});
    int wgh, pitch, pw, padg;
    if (!mma3d_geometry(*key, &wgh, &pitch, &pw, &padg)) return SS_E_UNSUPPORTED;
    std::vector<uint8_t> blob;
    size_t o_hi, o_lo, o_mid, o_idx, o_boff, o_zero;
    p->kperm.assign(kperm.begin(), kperm.end());
    st = build_mma_tables(p, gm, kperm, mode, part, key->kc, pitch, false, pw, padg, &blob, &o_hi, &o_lo, &o_mid,
                          &o_idx, &o_boff, &o_zero);
    if (st != SS_OK) return st;
    st = upload(p, blob);
    if (st != SS_OK) return st;
    char *d = static_cast<char *>(p->dev);
    p->mma = find_mma3d(*key);
    p->margs.periodic = p->boundary == SS_BC_PERIODIC;
    p->margs.inv_sigma = part == kPartF16 ? 1.0f / 2048.0f : 1.0f;
    p->margs.a_hi = reinterpret_cast<const uint4 *>(d + o_hi);
    p->margs.a_lo = reinterpret_cast<const uint4 *>(d + o_lo);
    p->margs.a_idx = reinterpret_cast<const uint32_t *>(d + o_idx);
    p->margs.boff = reinterpret_cast<const int32_t *>(d + o_boff);
    p->margs.zeros = d + o_zero;
    p->engine = engine;
    p->info.r1 = gm.r1;
    p->info.r2 = gm.r2;
    p->info.m_b = gm.m_b;
    p->info.g = gm.g;
    p->info.planes = gm.planes;
    p->info.m_prime = gm.m_prime();
    p->info.k_prime = gm.k_prime();
    p->info.k_pad = (int)p->perm.size();
    p->info.passes = 3;
    p->info.sigma = part == kPartF16 ? 2048.0 : 1.0;
    return SS_OK;
}

// Dense FP64 MMA engine (2-D): A' in FP64, natural column order, one tile
// shape (8,4); gather offsets per K chunk and lane group.
ss_status plan_mma2d_f64(ss_plan_ *p) {
    const int r1 = 8, r2 = 4;
    if (p->info.r1 && (p->info.r1 != r1 || p->info.r2 != r2)) return SS_E_UNSUPPORTED;
    const Geometry gm = make_geometry(2, p->k, r1, r2);
    const int kp = gm.k_prime(), kc_count = (kp + 3) / 4, MB = gm.m_prime() / 16;
    const MmaLaunch fn = find_mma2d_f64(p->rad, kc_count);
    const int pitch = mma2d_f64_pitch(p->rad);
    if (!fn || pitch == 0) return SS_E_UNSUPPORTED;
    const std::vector<double> amat = morph_matrix(gm, p->w);
    std::vector<double> a((size_t)MB * kc_count * 64, 0.0);
    for (int mb = 0; mb < MB; ++mb)
        for (int kc = 0; kc < kc_count; ++kc)
            for (int l = 0; l < 64; ++l) {
                const int row = mb * 16 + (l & 15), col = kc * 4 + (l >> 4);
                a[((size_t)mb * kc_count + kc) * 64 + l] = col < kp ? amat[(size_t)row * kp + col] : 0.0;
            }
    std::vector<int32_t> boff((size_t)kc_count * 4, 0);
    for (int kc = 0; kc < kc_count; ++kc)
        for (int q = 0; q < 4; ++q) {
            const int col = kc * 4 + q;
            boff[(size_t)kc * 4 + q] = col < kp ? (col / gm.g) * pitch + col % gm.g : 0;
        }
    p->perm.clear();
    for (int c = 0; c < kc_count * 4; ++c) p->perm.push_back(c < kp ? c : kZeta);
    p->kernel_lut = boff;
    auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t o_b = align(a.size() * 8), o_z = align(o_b + boff.size() * 4);
    std::vector<uint8_t> blob(o_z + 1024, 0);
    std::memcpy(blob.data(), a.data(), a.size() * 8);
    std::memcpy(blob.data() + o_b, boff.data(), boff.size() * 4);
    ss_status st = upload(p, blob);
    if (st != SS_OK) return st;
    char *d = static_cast<char *>(p->dev);
    p->mma = fn;
    p->margs.periodic = p->boundary == SS_BC_PERIODIC;
    p->margs.inv_sigma = 1.0f;
    p->margs.a_hi = reinterpret_cast<const uint4 *>(d);
    p->margs.boff = reinterpret_cast<const int32_t *>(d + o_b);
    p->margs.zeros = d + o_z;
    p->engine = SS_ENGINE_MFMA;
    p->info.r1 = r1;
    p->info.r2 = r2;
    p->info.m_b = gm.m_b;
    p->info.g = gm.g;
    p->info.planes = gm.planes;
    p->info.m_prime = gm.m_prime();
    p->info.k_prime = kp;
    p->info.k_pad = kc_count * 4;
    p->info.passes = 1;
    p->info.sigma = 1.0;
    return SS_OK;
}

// K order of the 1-D kernels (tile of 16 outputs, g = 15 + k patch
// columns, g even).  Sparse: adjacent column pairs (2j, 2j+1), so that one
// B register holds two neighbouring inputs, each 4-group two such pairs at
// least k + 1 columns apart (then no row of the band has more than the two
// values of one pair in a group), unmatched pairs beside zero columns.
// Dense: natural order.  Both padded with zero columns to one K chunk.
std::vector<int> order_1d(const Geometry &gm, int k, int mode) {
    std::vector<int> order;
    if (mode == kDense) {
        for (int c = 0; c < gm.g; ++c) order.push_back(c);
        order.resize(32, kZeta);
        return order;
    }
    const int npairs = gm.g / 2, gap = (k + 2) / 2;   // 2 * gap >= k + 1
    std::vector<char> used(npairs, 0);
    for (int a = 0; a < npairs; ++a) {
        if (used[a]) continue;
        used[a] = 1;
        int b = -1;
        for (int t = a + gap; t < npairs && b < 0; ++t)
            if (!used[t]) b = t;
        if (b >= 0) used[b] = 1;
        order.push_back(2 * a);
        order.push_back(2 * a + 1);
        order.push_back(b >= 0 ? 2 * b : kZeta);
        order.push_back(b >= 0 ? 2 * b + 1 : kZeta);
    }
    order.resize(64, kZeta);
    return order;
}

// 1-D MMA engines (FP32 state, binary16 or bfloat16 split): tile (16, 1),
// one K chunk, composed radius up to 8.
ss_status plan_mma1d(ss_plan_ *p, int engine) {
    if (p->ndim != 1 || p->rad > 8) return SS_E_UNSUPPORTED;
    if (p->info.r1 && (p->info.r1 != 16 || p->info.r2 != 1)) return SS_E_UNSUPPORTED;
    const int part = p->dtype == SS_F32_SPLIT_F16 ? kPartF16 : kPartBF16;
    const int mode = engine == SS_ENGINE_SMFMAC ? kSparse : kDense;
    const Geometry gm = make_geometry(1, p->k, 16, 1);
    ModelParams mp{};
    mp.ndim = 1;
    mp.k = p->k;
    mp.dims[0] = p->dims[2];
    mp.dims[1] = mp.dims[2] = 1;
    mp.elem_bytes = 4;
    mp.planes_state = 1;
    mp.coef_bytes = 2;
    mp.passes = 3;
    mp.kfrag = 64;
    const ModelRow r = model_time(mp, 16, 1);
    const double row[7] = {(double)r.r1, (double)r.r2, r.t, r.t_compute, r.t_global, r.t_shared, (double)r.k_pad};
    p->model.assign(row, row + 7);
    ss_status st = build_canonical(p, gm, part, 64);
    if (st != SS_OK) return st;
    const std::vector<int> kperm = order_1d(gm, p->k, mode);
    p->kperm.assign(kperm.begin(), kperm.end());
    std::vector<uint8_t> blob;
    size_t o_hi, o_lo, o_mid, o_idx, o_boff, o_zero;
    st = build_mma_tables(p, gm, kperm, mode, part, 1, 0, false, 0, 0, &blob, &o_hi, &o_lo, &o_mid, &o_idx, &o_boff,
                          &o_zero);
    if (st != SS_OK) return st;
    const MmaLaunch fn = find_mma1d(p->rad, mode, part);
    if (!fn) return SS_E_UNSUPPORTED;
    st = upload(p, blob);
    if (st != SS_OK) return st;
    char *d = static_cast<char *>(p->dev);
    p->mma = fn;
    p->margs.periodic = p->boundary == SS_BC_PERIODIC;
    p->margs.inv_sigma = part == kPartF16 ? 1.0f / 2048.0f : 1.0f;
    p->margs.a_hi = reinterpret_cast<const uint4 *>(d + o_hi);
    p->margs.a_lo = reinterpret_cast<const uint4 *>(d + o_lo);
    p->margs.a_idx = reinterpret_cast<const uint32_t *>(d + o_idx);
    p->margs.boff = reinterpret_cast<const int32_t *>(d + o_boff);
    p->margs.zeros = d + o_zero;
    p->engine = engine;
    p->info.r1 = gm.r1;
    p->info.r2 = gm.r2;
    p->info.m_b = gm.m_b;
    p->info.g = gm.g;
    p->info.planes = gm.planes;
    p->info.m_prime = gm.m_prime();
    p->info.k_prime = gm.k_prime();
    p->info.k_pad = (int)p->perm.size();
    p->info.passes = 3;
    p->info.sigma = part == kPartF16 ? 2048.0 : 1.0;
    return SS_OK;
}

ss_status plan_direct(ss_plan_ *p) {
    const bool f64 = p->dtype == SS_F64;
    // 2-D FP32-state or plane grids, 3-D and 1-D FP32-state grids run on the
    // LDS-staged kernels (planes need rows of a multiple of 8 values);
    // FP64, 1-D planes and the rest on the plain one
    const int state = mma_state(p->dtype);
    MmaLaunch lds = nullptr;
    if (!f64 && p->ndim == 2 && (state != kStatePlanes || p->dims[2] % 8 == 0) && slab_offsets_fit(p))
        lds = find_lds_direct2d(p->rad, state);
    if (!f64 && p->ndim == 3 && state == kStateF32 && slab_offsets_fit(p)) lds = find_lds_direct3d(p->rad);
    if (!f64 && p->ndim == 1 && state == kStateF32) lds = find_lds_direct1d(p->rad);
    if (!lds && p->rad > kDirectMaxRad) return SS_E_UNSUPPORTED;
    // a fused zero-halo 1-D or 3-D sweep needs the staged kernel's band pass
    if (!lds && p->ndim != 2 && p->edge_rad) return SS_E_UNSUPPORTED;
    const size_t wbytes = p->w.size() * (f64 ? 8 : 4);
    const size_t o_zero = (wbytes + 255) & ~(size_t)255;
    std::vector<uint8_t> blob(o_zero + 1024, 0);
    if (f64) {
        std::memcpy(blob.data(), p->w.data(), wbytes);
    } else {
        std::vector<float> wf(p->w.begin(), p->w.end());
        std::memcpy(blob.data(), wf.data(), wbytes);
    }
    ss_status st = upload(p, blob);
    if (st != SS_OK) return st;
    p->dargs.rz = p->ndim == 3 ? p->rad : 0;
    p->dargs.ry = p->ndim >= 2 ? p->rad : 0;
    p->dargs.rx = p->rad;
    p->dargs.periodic = p->boundary == SS_BC_PERIODIC;
    p->dargs.w = p->dev;
    if (lds) {
        char *d = static_cast<char *>(p->dev);
        p->mma = lds;
        p->margs.periodic = p->boundary == SS_BC_PERIODIC;
        p->margs.w = reinterpret_cast<const float *>(d);
        p->margs.zeros = d + o_zero;
        p->margs.inv_sigma = 1.0f;
    }
    p->engine = SS_ENGINE_DIRECT;
    p->info.passes = 1;
    p->info.sigma = 1.0;
    // a small 2-D FP64 grid (a sweep takes a few microseconds, about what a
    // launch costs) runs several sweeps per launch in LDS
    if (f64 && p->ndim == 2 && p->fuse == 1 && p->rad <= 4 && p->dims[1] * p->dims[2] <= (int64_t)1 << 20)
        p->tb = kTbHalo / p->rad;
    return SS_OK;
}

void free_plan(ss_plan_ *p) {
    if (!p) return;
    free_plan(p->rem);
    if (p->dev) (void)hipFree(p->dev);
    if (p->edge_w) (void)hipFree(p->edge_w);
    delete p;
}

ss_status make_plan(ss_plan_ **out, int shape, int radius, const double *coeffs, int ndim,
                    const int64_t *grid_dims, int dtype, const ss_plan_opts *opts, bool allow_fuse) {
    if (!out || !coeffs || !grid_dims) return SS_E_INVALID;
    if (shape != SS_SHAPE_BOX && shape != SS_SHAPE_STAR && shape != SS_SHAPE_CUSTOM) return SS_E_INVALID;
    if (ndim < 1 || ndim > 3 || radius < 1 || radius > 16) return SS_E_INVALID;
    if (state_bytes(dtype) == 0) return SS_E_INVALID;
    ss_plan_opts o{sizeof(ss_plan_opts), SS_BC_ZERO, 1, 0, 0, SS_ENGINE_AUTO, 0};
    if (opts) {
        if (opts->struct_size < sizeof(ss_plan_opts)) return SS_E_INVALID;
        o = *opts;
    }
    if (o.boundary != SS_BC_ZERO && o.boundary != SS_BC_PERIODIC) return SS_E_INVALID;
    if (o.fuse_steps < 1 || o.fuse_steps > 8) return SS_E_INVALID;
    if (o.engine < SS_ENGINE_AUTO || o.engine > SS_ENGINE_DIRECT) return SS_E_INVALID;
    if ((o.r1 == 0) != (o.r2 == 0) || o.r1 < 0 || o.r2 < 0) return SS_E_INVALID;
    // a zero halo fuses sweeps of an FP32 state -- 2-D: two of any radius,
    // or three of radius 1; 3-D: two of radius 1; 1-D: r*S <= 8 -- with the
    // band along the edges recomputed (the composed stencil is exact only
    // farther than r(S-1) from the edges)
    const bool edge_fused = o.fuse_steps > 1 && o.boundary == SS_BC_ZERO;
    const bool f32_split = dtype == SS_F32_SPLIT_F16 || dtype == SS_F32_SPLIT_BF16;
    if (edge_fused && !(f32_split && ((ndim == 2 && (o.fuse_steps == 2 || (o.fuse_steps == 3 && radius == 1))) ||
                                      (ndim == 3 && o.fuse_steps == 2 && radius == 1) ||
                                      (ndim == 1 && radius * o.fuse_steps <= 8))))
        return SS_E_UNSUPPORTED;
    if (o.fuse_steps > 1 && !allow_fuse) return SS_E_INVALID;
    if (o.flags & ~SS_FLAG_HOST_ONLY) return SS_E_INVALID;

    auto t0 = std::chrono::steady_clock::now();
    ss_plan_ *p = new (std::nothrow) ss_plan_();
    if (!p) return SS_E_NOMEM;
    p->ndim = ndim;
    for (int d = 0; d < ndim; ++d) {
        if (grid_dims[d] < 1 || grid_dims[d] > kMaxDim) {
            delete p;
            return SS_E_INVALID;
        }
        p->dims[3 - ndim + d] = grid_dims[d];
    }
    p->dtype = dtype;
    p->host_only = (o.flags & SS_FLAG_HOST_ONLY) != 0;
    p->boundary = o.boundary;
    p->fuse = o.fuse_steps;
    const int k0 = 2 * radius + 1;
    size_t nw = 1;
    for (int d = 0; d < ndim; ++d) nw *= (size_t)k0;
    std::vector<double> w(coeffs, coeffs + nw);
    for (double c : w)
        if (!std::isfinite(c)) {
            delete p;
            return SS_E_INVALID;
        }
    if (shape == SS_SHAPE_STAR && !valid_star(w, ndim, radius)) {
        delete p;
        return SS_E_INVALID;
    }
    int kf = k0;
    p->w = o.fuse_steps > 1 ? compose(w, ndim, k0, o.fuse_steps, &kf) : w;
    if (edge_fused) {
        p->w1 = w;
        p->edge_rad = radius;
    }
    p->k = kf;
    p->rad = (kf - 1) / 2;
    // a periodic grid must be at least as wide as the composed stencil
    if (o.boundary == SS_BC_PERIODIC)
        for (int d = 3 - ndim; d < 3; ++d)
            if (p->dims[d] < p->rad) {
                delete p;
                return SS_E_UNSUPPORTED;
            }
    p->info.r1 = o.r1;
    p->info.r2 = o.r2;

    ss_status st = SS_E_UNSUPPORTED;
    const bool split = dtype == SS_F32_SPLIT_F16 || dtype == SS_F32_SPLIT_BF16 || dtype == SS_SPLIT_BF16 ||
                       dtype == SS_SPLIT3_BF16;
    int engine = o.engine;
    // 3-D and 1-D kernels take an FP32 state
    const bool split3 = split && dtype != SS_SPLIT_BF16 && dtype != SS_SPLIT3_BF16;
    const bool mma2 = split || dtype == SS_F16;   // state types of the 2-D matrix kernels
    if (mma2 && ndim == 2 && (engine == SS_ENGINE_AUTO || engine == SS_ENGINE_SMFMAC)) {
        st = plan_mma2d(p, SS_ENGINE_SMFMAC);
        if (st != SS_OK && engine == SS_ENGINE_AUTO) st = plan_mma2d(p, SS_ENGINE_MFMA);
    } else if (mma2 && ndim == 2 && engine == SS_ENGINE_MFMA) {
        st = plan_mma2d(p, SS_ENGINE_MFMA);
    } else if (split3 && ndim == 3 && (engine == SS_ENGINE_AUTO || engine == SS_ENGINE_SMFMAC)) {
        st = plan_mma3d(p, SS_ENGINE_SMFMAC);
        if (st != SS_OK && engine == SS_ENGINE_AUTO) st = plan_mma3d(p, SS_ENGINE_MFMA);
    } else if (split3 && ndim == 3 && engine == SS_ENGINE_MFMA) {
        st = plan_mma3d(p, SS_ENGINE_MFMA);
    } else if (split3 && ndim == 1 && (engine == SS_ENGINE_AUTO || engine == SS_ENGINE_SMFMAC)) {
        st = plan_mma1d(p, SS_ENGINE_SMFMAC);
        if (st != SS_OK && engine == SS_ENGINE_AUTO) st = plan_mma1d(p, SS_ENGINE_MFMA);
    } else if (split3 && ndim == 1 && engine == SS_ENGINE_MFMA) {
        st = plan_mma1d(p, SS_ENGINE_MFMA);
    } else if (dtype == SS_F64 && ndim == 2 && engine == SS_ENGINE_MFMA) {
        st = plan_mma2d_f64(p);
    }
    if (st != SS_OK && (engine == SS_ENGINE_DIRECT || engine == SS_ENGINE_AUTO) &&
        (dtype == SS_F32 || dtype == SS_F64 || split) && dtype != SS_SPLIT3_BF16 && o.r1 == 0)
        st = plan_direct(p);
    if (st != SS_OK) {
        free_plan(p);
        return st;
    }
    if (edge_fused && !p->host_only) {
        // the unfused coefficients in FP64, then in FP32 (one allocation)
        const size_t n = p->w1.size();
        std::vector<uint8_t> blob(n * (sizeof(double) + sizeof(float)));
        std::vector<float> w32(p->w1.begin(), p->w1.end());
        std::memcpy(blob.data(), p->w1.data(), n * sizeof(double));
        std::memcpy(blob.data() + n * sizeof(double), w32.data(), n * sizeof(float));
        if (hipMalloc(&p->edge_w, blob.size()) != hipSuccess) {
            p->edge_w = nullptr;
            free_plan(p);
            return SS_E_NOMEM;
        }
        p->edge_w32 = reinterpret_cast<float *>(p->edge_w + n);
        if (hipMemcpy(p->edge_w, blob.data(), blob.size(), hipMemcpyHostToDevice) != hipSuccess) {
            free_plan(p);
            return SS_E_DEVICE;
        }
    }
    if (o.fuse_steps > 1) {
        ss_plan_opts ro = o;
        ro.fuse_steps = 1;
        ro.r1 = ro.r2 = 0;
        ro.engine = p->engine;
        st = make_plan(&p->rem, shape, radius, coeffs, ndim, grid_dims, dtype, &ro, false);
        if (st != SS_OK) {
            free_plan(p);
            return st;
        }
    }
    ss_plan_info &inf = p->info;
    inf.ndim = ndim;
    inf.radius = p->rad;
    inf.k = p->k;
    inf.fuse_steps = p->fuse;
    inf.engine = p->engine;
    inf.dtype = dtype;
    inf.boundary = p->boundary;
    inf.launches_per_sweep = p->edge_rad && !band_in_launch(p) ? 2 : 1;
    for (int d = 0; d < 3; ++d) inf.dims[d] = p->dims[d];
    // plans with the same class share device-table contents: their grids can
    // be swept by one launch
    uint64_t h = 1469598103934665603ull;
    auto mix = [&h](const void *d, size_t n) {
        const unsigned char *c = static_cast<const unsigned char *>(d);
        for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
    };
    const int32_t key[8] = {p->engine, p->dtype, p->boundary, p->k, inf.r1, inf.r2, ndim, p->fuse};
    mix(key, sizeof key);
    // the kernel the plan picked (the direct engine picks by grid size)
    mix(&p->mma, sizeof p->mma);
    mix(p->w.data(), p->w.size() * sizeof(double));
    mix(p->w1.data(), p->w1.size() * sizeof(double));
    p->klass = h;
    inf.plan_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = p;
    return SS_OK;
}

template <class T>
ss_status copy_out(const std::vector<T> &v, void *buf, size_t *nbytes) {
    const size_t need = v.size() * sizeof(T);
    if (!nbytes) return SS_E_INVALID;
    if (!buf) {
        *nbytes = need;
        return SS_OK;
    }
    if (*nbytes < need) return SS_E_INVALID;
    if (need) std::memcpy(buf, v.data(), need);
    *nbytes = need;
    return SS_OK;
}

}  // namespace

namespace ss {
// The band of a fused zero-halo sweep is computed inside the sweep launch by
// the 1-D and 3-D kernels and the 2-D matrix kernels (radius-1 sweeps,
// S <= 3); the 2-D direct engine, and 2-D sweeps of larger radius, use a
// second launch.
bool band_in_launch(const ss_plan_ *p) {
    if (!p->mma || !p->edge_rad) return false;
    if (p->ndim != 2) return true;
    return p->engine != SS_ENGINE_DIRECT && p->edge_rad == 1 && p->fuse <= 3;
}

// One sweep of the plan over n grids of its own shape class (same tables,
// same boundary): one kernel launch.  dims_j = (nz, ny, nx) of grid j.
hipError_t sweep_grids(const ss_plan_ *p, int n, const void *const *in, void *const *out,
                       const int64_t (*dims)[3], hipStream_t s) {
    if (n < 1 || n > kMaxJobs) return hipErrorInvalidValue;
    hipError_t e;
    if (!p->mma) {
        DirectArgs a = p->dargs;
        a.njobs = n;
        for (int j = 0; j < n; ++j)
            a.job[j] = DirectJob{in[j], out[j], (int)dims[j][0], (int)dims[j][1], (int)dims[j][2], 0};
        const int kind = p->dtype == SS_F64 ? kDirectF64 : p->dtype == SS_SPLIT_BF16 ? kDirectPlanes : kDirectF32;
        e = launch_direct(a, kind, s);
    } else {
        MmaArgs a = p->margs;
        a.njobs = n;
        for (int j = 0; j < n; ++j)
            a.job[j] = MmaJob{in[j], out[j], (int)dims[j][1], (int)dims[j][2], 0, (int)dims[j][0], 0};
        // the 1-D and 3-D kernels and the 2-D matrix kernels recompute the
        // band of a fused zero-halo sweep in the same launch
        if (p->edge_w && band_in_launch(p)) {
            a.edge_w = p->edge_w;
            a.edge_w32 = p->edge_w32;
            a.edge_rad = p->edge_rad;
            a.edge_steps = p->fuse;
        }
        e = p->mma(a, s);
        if (band_in_launch(p)) return e;
    }
    // zero-halo fused sweeps of the 2-D direct engine: exact values for the
    // band along the edges, by a second launch
    if (e != hipSuccess || !p->edge_w) return e;
    EdgeArgs ea{};
    ea.njobs = n;
    ea.rad = p->edge_rad;
    ea.steps = p->fuse;
    ea.w = p->edge_w;
    for (int j = 0; j < n; ++j)
        ea.job[j] = EdgeJob{static_cast<const float *>(in[j]), static_cast<float *>(out[j]), (int)dims[j][1],
                            (int)dims[j][2], 0};
    return launch_edge2d(ea, s);
}

hipError_t sweep_one(const ss_plan_ *p, const void *in, void *out, hipStream_t s) {
    void *o = out;
    return sweep_grids(p, 1, &in, &o, &p->dims, s);
}


size_t plan_state_bytes(const ss_plan_ *p) { return state_bytes(p->dtype); }

bool same_class(const ss_plan_ *a, const ss_plan_ *b) {
    return a->klass == b->klass && a->mma == b->mma && a->engine == b->engine && a->dtype == b->dtype &&
           a->boundary == b->boundary && a->k == b->k && a->ndim == b->ndim && a->fuse == b->fuse &&
           a->info.r1 == b->info.r1 && a->info.r2 == b->info.r2 && a->w == b->w && a->w1 == b->w1;
}

}  // namespace ss

extern "C" {

ss_status sparstencil_plan(ss_plan_t *out, int32_t shape, int32_t radius, const double *coeffs, int32_t ndim,
                           const int64_t *grid_dims, int32_t dtype, const ss_plan_opts *opts) {
    if (out) *out = nullptr;
    try {
        return make_plan(out, shape, radius, coeffs, ndim, grid_dims, dtype, opts, true);
    } catch (...) {
        return SS_E_NOMEM;
    }
}

ss_status sparstencil_plan_points(ss_plan_t *out, int32_t ndim, int32_t npoints, const int32_t *offsets,
                                  const double *coeffs, const int64_t *grid_dims, int32_t dtype,
                                  const ss_plan_opts *opts) {
    if (out) *out = nullptr;
    if (!out || !offsets || !coeffs || !grid_dims || ndim < 1 || ndim > 3 || npoints < 1) return SS_E_INVALID;
    try {
        int r = 1;
        for (int64_t i = 0; i < (int64_t)npoints * ndim; ++i) {
            if (offsets[i] < -16 || offsets[i] > 16) return SS_E_INVALID;
            r = std::max(r, std::abs(offsets[i]));
        }
        const int k = 2 * r + 1;
        size_t n = 1;
        for (int d = 0; d < ndim; ++d) n *= (size_t)k;
        std::vector<double> w(n, 0.0);
        std::vector<char> seen(n, 0);
        for (int i = 0; i < npoints; ++i) {
            size_t at = 0;
            for (int d = 0; d < ndim; ++d) at = at * k + (size_t)(offsets[(size_t)i * ndim + d] + r);
            if (seen[at]) return SS_E_INVALID;
            seen[at] = 1;
            w[at] = coeffs[i];
        }
        return make_plan(out, SS_SHAPE_CUSTOM, r, w.data(), ndim, grid_dims, dtype, opts, true);
    } catch (...) {
        return SS_E_NOMEM;
    }
}

ss_status sparstencil_plan_destroy(ss_plan_t plan) {
    free_plan(plan);
    return SS_OK;
}

size_t sparstencil_grid_bytes(ss_plan_t p) {
    if (!p) return 0;
    return (size_t)points(p) * state_bytes(p->dtype);
}

int64_t sparstencil_launch_count(ss_plan_t p, int64_t steps) {
    if (!p || steps <= 0) return 0;
    if (p->tb) return (steps + p->tb - 1) / p->tb;
    return steps / p->fuse + steps % p->fuse;
}

ss_status sparstencil_run(ss_plan_t p, void *in, void *out, int64_t steps, void *stream) {
    if (!p || !in || !out || in == out || steps < 0 || p->host_only) return SS_E_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t bytes = sparstencil_grid_bytes(p);
    if (steps == 0)
        return hipMemcpyAsync(out, in, bytes, hipMemcpyDeviceToDevice, s) == hipSuccess ? SS_OK : SS_E_DEVICE;
    const int64_t fused = steps / p->fuse, rest = steps % p->fuse;
    const int64_t total = sparstencil_launch_count(p, steps);
    // Ping-pong between the two meshes so that the last launch writes `out`;
    // with an even number of launches the input is first copied into `out`.
    void *src = in, *dst = out;
    if (total % 2 == 0) {
        if (hipMemcpyAsync(out, in, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess) return SS_E_DEVICE;
        src = out;
        dst = in;
    }
    for (int64_t i = 0; i < total; ++i) {
        if (p->tb) {
            // the steps shared out evenly over the launches
            ss::DirectArgs a = p->dargs;
            a.njobs = 1;
            a.job[0] = ss::DirectJob{src, dst, 1, (int)p->dims[1], (int)p->dims[2], 0};
            a.steps = (int)(steps / total + (i < steps % total ? 1 : 0));
            if (ss::launch_direct_tb(a, s) != hipSuccess) return SS_E_DEVICE;
        } else {
            const ss_plan_ *q = i < fused ? p : p->rem;
            if (ss::sweep_one(q, src, dst, s) != hipSuccess) return SS_E_DEVICE;
        }
        std::swap(src, dst);
    }
    return SS_OK;
}

ss_status sparstencil_sweep(ss_plan_t p, const void *in, void *out, void *stream) {
    if (!p || !in || !out || in == out || p->host_only) return SS_E_INVALID;
    return ss::sweep_one(p, in, out, static_cast<hipStream_t>(stream)) == hipSuccess ? SS_OK : SS_E_DEVICE;
}

ss_status sparstencil_sweep_batch(ss_plan_t p, int32_t n, const void *const *in, void *const *out, void *stream) {
    if (!p || !in || !out || n < 1 || n > kMaxJobs || p->host_only) return SS_E_INVALID;
    const size_t bytes = sparstencil_grid_bytes(p);
    for (int i = 0; i < n; ++i) {
        if (!in[i] || !out[i]) return SS_E_INVALID;
        // no output may overlap any grid of the launch
        const char *o = static_cast<const char *>(out[i]);
        for (int j = 0; j < n; ++j) {
            const char *a = static_cast<const char *>(in[j]), *b = static_cast<const char *>(out[j]);
            if (o < a + bytes && a < o + bytes) return SS_E_INVALID;
            if (j != i && o < b + bytes && b < o + bytes) return SS_E_INVALID;
        }
    }
    int64_t dims[kMaxJobs][3];
    for (int i = 0; i < n; ++i) std::memcpy(dims[i], p->dims, sizeof dims[i]);
    return ss::sweep_grids(p, n, in, out, dims, static_cast<hipStream_t>(stream)) == hipSuccess ? SS_OK
                                                                                             : SS_E_DEVICE;
}

ss_status sparstencil_plan_query(ss_plan_t p, int32_t what, void *buf, size_t *nbytes) {
    if (!p || !nbytes) return SS_E_INVALID;
    switch (what) {
        case SS_Q_INFO: {
            std::vector<ss_plan_info> v{p->info};
            return copy_out(v, buf, nbytes);
        }
        case SS_Q_COEFFS: return copy_out(p->w, buf, nbytes);
        case SS_Q_PERM: return copy_out(p->perm, buf, nbytes);
        case SS_Q_VALUES: return copy_out(p->values, buf, nbytes);
        case SS_Q_META: return copy_out(p->meta, buf, nbytes);
        case SS_Q_HI: return copy_out(p->hi, buf, nbytes);
        case SS_Q_LO: return copy_out(p->lo, buf, nbytes);
        case SS_Q_MID: return copy_out(p->mid, buf, nbytes);
        case SS_Q_LUT: return copy_out(p->lut, buf, nbytes);
        case SS_Q_MODEL: return copy_out(p->model, buf, nbytes);
        case SS_Q_KERNEL_LUT: return copy_out(p->kernel_lut, buf, nbytes);
        case SS_Q_KERNEL_PERM: return copy_out(p->kperm, buf, nbytes);
        case SS_Q_KERNEL_FRAGS: return copy_out(p->kernel_frags, buf, nbytes);
        default: return SS_E_INVALID;
    }
}

const char *sparstencil_status_string(int32_t s) {
    switch (s) {
        case SS_OK: return "ok";
        case SS_PENDING: return "pending";
        case SS_E_INVALID: return "invalid argument";
        case SS_E_UNSUPPORTED: return "unsupported";
        case SS_E_NOMEM: return "out of memory";
        case SS_E_DEVICE: return "device error";
        case SS_E_NOT_FOUND: return "not found";
        case SS_E_BUSY: return "busy";
        default: return "unknown status";
    }
}

}  // extern "C"

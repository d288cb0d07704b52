// Level schedule of a plan and its execution on a HIP stream.
//
// One level (paper Sec. 2.2): u = dx0^2 * G * f on the level's blocks, one
// blockwise convolution per component.
//
// K levels (paper Sec. 3.4, revised FLGF-AMR, in the paper's order):
//   f^_k  = f_k restricted to Omega_k (octants covered by level k+1 zeroed)
//   F_k   = f^_k + P_{k+1->k} F_{k+1}                 (fine -> coarse, mean of 8)
//   psi_0 = L_0^-1 f^_0 on dom(psi_0),  phi_0 = L_0^-1 F_0 on Omega_0
//   k >= 1, on R_k = Omega_k u Omega_k^E (level-k blocks dilated by ne blocks):
//     P psi_{k-1}, S_k = (P L_{k-1} - L_k P) psi_{k-1}
//     phi_k = P psi_{k-1} + L_k^-1 (S_k + F_k)        on Omega_k
//     psi_k = P psi_{k-1} + L_k^-1 (S_k + f^_k)       on dom(psi_k), k < K-1
// dom(psi_{k-1}) = level-(k-1) blocks holding any coarse cell within two
// cells of a parent of R_k (trilinear P and L_{k-1} each reach one cell).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "lgf_runtime.hpp"

namespace lgf {

namespace {

using Key = std::tuple<int, int, int>;

int fdiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

template <typename T> void upload(lgf_context *ctx, DeviceBuffer &d, const std::vector<T> &h, const char *what) {
    d.alloc(ctx, sizeof(T) * std::max<size_t>(1, h.size()), what);
    if (!h.empty()) hip_check(hipMemcpy(d.ptr, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice), "upload");
}

std::vector<Key> dilate(const std::vector<Key> &in, int layers) {
    std::map<Key, int> seen;
    std::vector<Key> out;
    auto add = [&](Key k) {
        if (seen.emplace(k, 0).second) out.push_back(k);
    };
    for (const Key &k : in) add(k);
    for (const Key &k : in)
        for (int dz = -layers; dz <= layers; ++dz)
            for (int dy = -layers; dy <= layers; ++dy)
                for (int dx = -layers; dx <= layers; ++dx)
                    add(Key(std::get<0>(k) + dx, std::get<1>(k) + dy, std::get<2>(k) + dz));
    return out;
}

}  // namespace

void build_schedule(lgf_plan *p) {
    lgf_context *ctx = p->ctx;
    const bool refine = p->prec == LGF_FP32_REFINE;
    const int nb = p->nb, K = p->K;
    const int64_t nb3 = (int64_t)nb * nb * nb;
    p->mac_nc = std::min(p->nc, kMacComponents);
    const bool fif = p->if_a0 > 0.0;
    p->build_ka = p->kernel0;
    if (fif) p->build_ka.a = p->if_a0;
    if (K == 1) {
        p->op0 = build_op(p, p->levels[0], p->levels[0], refine);
        plan_alloc_refine(p, {p->op0.get()});
        plan_alloc_spectral(p);
        std::map<Key, int64_t> at;
        std::vector<int64_t> off, back;
        p->src_ijk.assign(1, {});
        for (const auto &b : p->levels[0]) {
            at[Key(b.ijk[0], b.ijk[1], b.ijk[2])] = b.off;
            off.push_back(b.off);
            p->src_ijk[0].insert(p->src_ijk[0].end(), b.ijk, b.ijk + 3);
        }
        upload(ctx, p->d_blk_off, off, "block offsets");
        if (p->flgf_D >= 0) {   // the far field: the same blocks on the node lattice (nb/2), far band, G(2n)
            auto c = std::make_unique<lgf_plan>();
            c->ctx = ctx;
            c->K = 1;
            c->nb = nb / 2;
            c->nc = p->nc;
            c->prec = LGF_FP64;
            c->ne = 1;
            c->dx0 = p->dx0;
            const int64_t h3 = (int64_t)c->nb * c->nb * c->nb;
            std::vector<Blk> cb = p->levels[0];
            for (size_t i = 0; i < cb.size(); ++i) cb[i].off = (int64_t)i * h3;
            c->levels.push_back(cb);
            c->level_base.push_back(0);
            c->comp_len = (int64_t)cb.size() * h3;
            c->cell_mask.assign(1, {});
            c->kernel0.stride = 2;
            c->kernel0.band = 2;
            c->kernel0.D = p->flgf_D;
            build_schedule(c.get());
            p->ws_fc.alloc(ctx, sizeof(double) * c->comp_len * p->nc, "node-lattice source");
            p->ws_uc.alloc(ctx, sizeof(double) * c->comp_len * p->nc, "node-lattice field");
            p->flgf_coarse = std::move(c);
        }
        if (p->nc == 3) {      // the velocity refresh's curl reads backward neighbours
            for (const auto &b : p->levels[0])
                for (int a = 0; a < 3; ++a) {
                    int q[3] = {b.ijk[0], b.ijk[1], b.ijk[2]};
                    --q[a];
                    auto it = at.find(Key(q[0], q[1], q[2]));
                    back.push_back(it == at.end() ? -1 : it->second);
                }
            upload(ctx, p->d_blk_back, back, "backward neighbours");
        }
        if (!p->cell_mask[0].empty()) {
            upload(ctx, p->d_cmask0, p->cell_mask[0], "cell mask");
            p->ws_masked.alloc(ctx, sizeof(double) * p->comp_len * p->nc, "masked source");
        }
        p->ind_base = {0};
        p->ind_total = (int64_t)p->levels[0].size();
        p->d_ind.alloc(ctx, sizeof(double) * 2 * p->ind_total * p->nc, "indicator statistics");
        return;
    }
    for (int k = 0; k < K; ++k) p->lv.push_back(std::make_unique<LevelSched>());
    std::vector<std::map<Key, int>> index(K);
    for (int k = 0; k < K; ++k)
        for (size_t i = 0; i < p->levels[k].size(); ++i) {
            const auto &b = p->levels[k][i];
            index[k][Key(b.ijk[0], b.ijk[1], b.ijk[2])] = (int)i;
        }
    // cover bits and coarsening pairs
    for (int k = 0; k < K; ++k) {
        LevelSched &L = *p->lv[k];
        const auto &B = p->levels[k];
        std::vector<unsigned char> cover(B.size(), 0);
        std::vector<int64_t> own(B.size());
        for (size_t i = 0; i < B.size(); ++i) own[i] = B[i].off;
        std::vector<int64_t> cf_f, cf_c;
        std::vector<unsigned char> cf_o;
        if (k + 1 < K) {
            for (const auto &fb : p->levels[k + 1]) {
                const int px = fdiv(fb.ijk[0], 2), py = fdiv(fb.ijk[1], 2), pz = fdiv(fb.ijk[2], 2);
                const int ci = index[k].at(Key(px, py, pz));
                const int oct = (fb.ijk[0] - 2 * px) | ((fb.ijk[1] - 2 * py) << 1) | ((fb.ijk[2] - 2 * pz) << 2);
                cover[ci] |= (unsigned char)(1u << oct);
                cf_f.push_back(fb.off);
                cf_c.push_back(B[ci].off);
                cf_o.push_back((unsigned char)oct);
            }
        }
        L.n_own = (int)B.size();
        L.any_cover = std::any_of(cover.begin(), cover.end(), [](unsigned char c) { return c != 0; });
        upload(ctx, L.d_cover, cover, "cover bits");
        if (!p->cell_mask[k].empty()) upload(ctx, L.d_cmask, p->cell_mask[k], "cell mask");
        upload(ctx, L.d_own_off, own, "offsets");
        L.n_cf = (int)cf_f.size();
        upload(ctx, L.d_cf_fine, cf_f, "coarsen pairs");
        upload(ctx, L.d_cf_coarse, cf_c, "coarsen pairs");
        upload(ctx, L.d_cf_oct, cf_o, "coarsen pairs");
    }
    // extension R_k (k >= 1) and psi domains dom(psi_{k-1})
    std::vector<std::vector<Key>> ext(K), dom(K);
    for (int k = 1; k < K; ++k) {
        std::vector<Key> own;
        for (const auto &b : p->levels[k]) own.push_back(Key(b.ijk[0], b.ijk[1], b.ijk[2]));
        ext[k] = dilate(own, p->ne);
        std::map<Key, int> dseen;
        const int H = nb / 2;
        for (const Key &f : ext[k]) {
            int lo[3], hi[3];
            const int fc[3] = {std::get<0>(f), std::get<1>(f), std::get<2>(f)};
            for (int a = 0; a < 3; ++a) {
                lo[a] = fdiv(fc[a] * H - 2, nb);
                hi[a] = fdiv(fc[a] * H + H + 1, nb);
            }
            for (int z = lo[2]; z <= hi[2]; ++z)
                for (int y = lo[1]; y <= hi[1]; ++y)
                    for (int x = lo[0]; x <= hi[0]; ++x)
                        if (dseen.emplace(Key(x, y, z), 0).second) dom[k - 1].push_back(Key(x, y, z));
        }
    }
    // field layout helpers
    auto as_blk = [&](const std::vector<Key> &ks) {
        std::vector<Blk> v(ks.size());
        for (size_t i = 0; i < ks.size(); ++i) {
            v[i].ijk[0] = std::get<0>(ks[i]);
            v[i].ijk[1] = std::get<1>(ks[i]);
            v[i].ijk[2] = std::get<2>(ks[i]);
            v[i].off = (int64_t)i * nb3;           // compact workspace offset
        }
        return v;
    };
    int64_t max_ext = 0, max_dom = 0;
    for (int k = 0; k < K; ++k) {
        LevelSched &L = *p->lv[k];
        // convolution of the phi right-hand side: sources -> Omega_k targets
        // (the integrating factor of level k has a_k = 4^k a_0)
        std::vector<Blk> src = (k == 0) ? p->levels[0] : as_blk(ext[k]);
        if (fif) p->build_ka.a = p->if_a0 * (double)(1 << (2 * k));
        L.convF = build_op(p, src, p->levels[k], refine);
        if (k + 1 < K) {
            std::vector<Blk> tgt = as_blk(dom[k]);
            if (!fif) L.convPsi = build_op(p, src, tgt, refine);
            L.n_dom = (int)dom[k].size();
            max_dom = std::max<int64_t>(max_dom, L.n_dom);
            // dense map of dom(psi_k) for the level-(k+1) correction
            int lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
            for (const Key &d : dom[k]) {
                const int c[3] = {std::get<0>(d), std::get<1>(d), std::get<2>(d)};
                for (int a = 0; a < 3; ++a) {
                    lo[a] = std::min(lo[a], c[a]);
                    hi[a] = std::max(hi[a], c[a]);
                }
            }
            CorrGeom &g = p->lv[k + 1]->corr;
            g.dxc = p->dx0 / (double)(1 << k);
            g.dxf = p->dx0 / (double)(1 << (k + 1));
            for (int a = 0; a < 3; ++a) {
                g.mlo[a] = lo[a];
                g.mdim[a] = hi[a] - lo[a] + 1;
            }
            std::vector<int> map((size_t)g.mdim[0] * g.mdim[1] * g.mdim[2], -1);
            for (size_t i = 0; i < dom[k].size(); ++i) {
                const Key &d = dom[k][i];
                map[((size_t)(std::get<2>(d) - lo[2]) * g.mdim[1] + (std::get<1>(d) - lo[1])) * g.mdim[0] +
                    (std::get<0>(d) - lo[0])] = (int)i;
            }
            upload(ctx, p->lv[k + 1]->d_cmap, map, "psi block map");
        }
        if (k >= 1) {
            L.n_ext = (int)ext[k].size();
            max_ext = std::max<int64_t>(max_ext, L.n_ext);
            std::vector<int> fblk;
            std::vector<int64_t> own_off;
            std::map<Key, int> eidx;
            for (size_t e = 0; e < ext[k].size(); ++e) {
                const Key &q = ext[k][e];
                fblk.push_back(std::get<0>(q));
                fblk.push_back(std::get<1>(q));
                fblk.push_back(std::get<2>(q));
                auto it = index[k].find(q);
                own_off.push_back(it == index[k].end() ? -1 : p->levels[k][it->second].off);
                eidx[q] = (int)e;
            }
            upload(ctx, L.d_fblk, fblk, "extension blocks");
            upload(ctx, L.d_ext_own, own_off, "extension offsets");
            // P psi_{k-1} copies: R_k -> Omega_k targets (in u) and R_k -> dom(psi_k)
            std::vector<int64_t> cu_s, cu_d, cp_s, cp_d;
            for (const auto &b : p->levels[k]) {
                cu_s.push_back((int64_t)eidx.at(Key(b.ijk[0], b.ijk[1], b.ijk[2])) * nb3);
                cu_d.push_back(b.off);
            }
            if (k + 1 < K)
                for (size_t i = 0; i < dom[k].size(); ++i) {
                    auto it = eidx.find(dom[k][i]);
                    if (it == eidx.end())
                        throw Failure(LGF_E_UNSUPPORTED, "psi domain leaves the extended region (nb < 4?)");
                    cp_s.push_back((int64_t)it->second * nb3);
                    cp_d.push_back((int64_t)i * nb3);
                }
            upload(ctx, L.d_cu_src, cu_s, "copy offsets");
            upload(ctx, L.d_cu_dst, cu_d, "copy offsets");
            upload(ctx, L.d_cp_src, cp_s, "copy offsets");
            upload(ctx, L.d_cp_dst, cp_d, "copy offsets");
        }
    }
    if (fif) {      // q_0 = f^_0 on dom(psi_0): the level-0 blocks inside it, the rest 0
        std::map<Key, int> didx;
        for (size_t i = 0; i < dom[0].size(); ++i) didx[dom[0][i]] = (int)i;
        std::vector<int64_t> qs, qd;
        for (const auto &b : p->levels[0]) {
            auto it = didx.find(Key(b.ijk[0], b.ijk[1], b.ijk[2]));
            if (it == didx.end()) continue;
            qs.push_back(b.off);
            qd.push_back((int64_t)it->second * nb3);
        }
        p->n_q0 = (int)qs.size();
        upload(ctx, p->d_q0_src, qs, "q0 offsets");
        upload(ctx, p->d_q0_dst, qd, "q0 offsets");
        for (int k = 1; k < K; ++k) p->lv[k]->corr.interp_only = 1;
    }
    // refinement-indicator bookkeeping: R_0 = level 0's blocks, R_k = ext[k]
    p->src_ijk.assign(K, {});
    for (const auto &b : p->levels[0]) p->src_ijk[0].insert(p->src_ijk[0].end(), b.ijk, b.ijk + 3);
    for (int k = 1; k < K; ++k)
        for (const Key &q : ext[k]) {
            p->src_ijk[k].push_back(std::get<0>(q));
            p->src_ijk[k].push_back(std::get<1>(q));
            p->src_ijk[k].push_back(std::get<2>(q));
        }
    p->ind_base.clear();
    p->ind_total = 0;
    for (int k = 0; k < K; ++k) {
        p->ind_base.push_back(p->ind_total);
        p->ind_total += (int64_t)p->src_ijk[k].size() / 3;
    }
    p->d_ind.alloc(ctx, sizeof(double) * 2 * p->ind_total * p->nc, "indicator statistics");
    // workspaces: mac_nc component regions each (the components of one MAC group)
    const int64_t m = p->mac_nc;
    p->dom_len = std::max<int64_t>(1, max_dom) * nb3;
    p->ext_len = std::max<int64_t>(1, max_ext) * nb3;
    p->ws_fhat.alloc(ctx, sizeof(double) * p->comp_len * m, "masked sources");
    p->ws_F.alloc(ctx, sizeof(double) * p->comp_len * m, "cumulative sources");
    p->ws_psi[0].alloc(ctx, sizeof(double) * p->dom_len * m, "psi");
    p->ws_psi[1].alloc(ctx, sizeof(double) * p->dom_len * m, "psi");
    p->ws_ppsi.alloc(ctx, sizeof(double) * p->ext_len * m, "P psi");
    p->ws_srcF.alloc(ctx, sizeof(double) * p->ext_len * m, "sources");
    p->ws_srcf.alloc(ctx, sizeof(double) * p->ext_len * m, "sources");
    std::vector<const ConvOp *> ops;
    for (int k = 0; k < K; ++k) {
        ops.push_back(p->lv[k]->convF.get());
        ops.push_back(p->lv[k]->convPsi.get());
    }
    plan_alloc_refine(p, ops);
    plan_alloc_spectral(p);
}

// The components run in groups of up to kMacComponents: every step of the
// recursion is applied to each component of the group, and each
// convolution takes the whole group in one MAC launch.
static void enqueue_composite(lgf_plan *p, const double *f, double *u, hipStream_t s) {
    const int K = p->K, nb = p->nb;
    const int64_t CL = p->comp_len, DL = p->dom_len, EL = p->ext_len;
    double *FH = (double *)p->ws_fhat.ptr, *FC = (double *)p->ws_F.ptr;
    double *PP = (double *)p->ws_ppsi.ptr, *SF = (double *)p->ws_srcF.ptr, *Sf = (double *)p->ws_srcf.ptr;
    for (int c0 = 0; c0 < p->nc; c0 += kMacComponents) {
        const int ng = std::min(kMacComponents, p->nc - c0);
        const double *fg = f + (size_t)c0 * CL;
        double *ug = u + (size_t)c0 * CL;
        StageTimer tm(p->ctx, 3, s);
        // f^_k and F_k
        for (int c = 0; c < ng; ++c)
            for (int k = 0; k < K; ++k) {
                const LevelSched &L = *p->lv[k];
                hip_check(mask_blocks(nb, fg + c * CL, FH + c * CL, (const int64_t *)L.d_own_off.ptr,
                                      (const int64_t *)L.d_own_off.ptr, (const unsigned char *)L.d_cover.ptr, L.n_own,
                                      s, (const unsigned char *)L.d_cmask.ptr),
                          "mask sources");
                hip_check(copy_blocks(nb, FH + c * CL, FC + c * CL, (const int64_t *)L.d_own_off.ptr,
                                      (const int64_t *)L.d_own_off.ptr, L.n_own, s),
                          "copy sources");
            }
        for (int c = 0; c < ng; ++c)
            for (int k = K - 2; k >= 0; --k) {
                const LevelSched &L = *p->lv[k];
                hip_check(coarsen_mean8(nb, FC + c * CL, FC + c * CL, (const int64_t *)L.d_cf_fine.ptr,
                                        (const int64_t *)L.d_cf_coarse.ptr, (const unsigned char *)L.d_cf_oct.ptr,
                                        L.n_cf, s),
                          "coarsen");
            }
        int cur = 0;   // psi ping-pong
        for (int k = 0; k < K; ++k) {
            const LevelSched &L = *p->lv[k];
            const double dxk = p->dx0 / (double)(1 << k);
            double *psi_prev = (double *)p->ws_psi[cur].ptr;
            double *psi_next = (double *)p->ws_psi[cur ^ 1].ptr;
            double *ind = (double *)p->d_ind.ptr;
            if (k == 0) {
                if (p->collect)
                    for (int c = 0; c < ng; ++c)
                        hip_check(block_stats(nb, FC + c * CL, (const int64_t *)L.d_own_off.ptr, L.n_own,
                                              ind + 2 * ((c0 + c) * p->ind_total + p->ind_base[0]), s),
                                  "indicator");
                run_op(p, *L.convF, FC, CL, ug, CL, ng, dxk, 0, s);
                if (L.convPsi) run_op(p, *L.convPsi, FH, CL, psi_next, DL, ng, dxk, 0, s);
            } else {
                for (int c = 0; c < ng; ++c) {
                    hip_check(correction_source(nb, L.corr, psi_prev + c * DL, (const int *)L.d_cmap.ptr,
                                                (const int *)L.d_fblk.ptr, (const int64_t *)L.d_ext_own.ptr,
                                                FC + c * CL, FH + c * CL, PP + c * EL, SF + c * EL, Sf + c * EL,
                                                L.n_ext, s),
                              "correction source");
                    hip_check(copy_blocks(nb, PP + c * EL, ug + c * CL, (const int64_t *)L.d_cu_src.ptr,
                                          (const int64_t *)L.d_cu_dst.ptr, L.n_own, s),
                              "P psi -> phi");
                    if (p->collect)
                        hip_check(block_stats(nb, SF + c * EL, nullptr, L.n_ext,
                                              ind + 2 * ((c0 + c) * p->ind_total + p->ind_base[k]), s),
                                  "indicator");
                }
                run_op(p, *L.convF, SF, EL, ug, CL, ng, dxk, 1, s);
                if (L.convPsi) {
                    for (int c = 0; c < ng; ++c)
                        hip_check(copy_blocks(nb, PP + c * EL, psi_next + c * DL, (const int64_t *)L.d_cp_src.ptr,
                                              (const int64_t *)L.d_cp_dst.ptr, L.n_dom, s),
                                  "P psi -> psi");
                    run_op(p, *L.convPsi, Sf, EL, psi_next, DL, ng, dxk, 1, s);
                }
            }
            if (L.any_cover || L.d_cmask.ptr)
                for (int c = 0; c < ng; ++c)
                    hip_check(mask_blocks(nb, ug + c * CL, ug + c * CL, (const int64_t *)L.d_own_off.ptr,
                                          (const int64_t *)L.d_own_off.ptr, (const unsigned char *)L.d_cover.ptr,
                                          L.n_own, s, (const unsigned char *)L.d_cmask.ptr),
                              "restrict phi");
            cur ^= 1;
        }
    }
}

// Integrating factor on the composite mesh (paper Sec. 3.5, eq. FIF-AMR):
// phi = Gamma H P f^.  Per level k the composite source P f^ on R_k is the
// cumulative F_k (f^_k plus the coarsening of finer levels) plus the
// interpolation P q_{k-1} of the coarser-level sources, q_0 = f^_0,
// q_k = P q_{k-1} + f^_k; then phi_k = H(a_k) of it on Omega_k.
static void enqueue_fif(lgf_plan *p, const double *f, double *u, hipStream_t s) {
    const int K = p->K, nb = p->nb;
    const int64_t CL = p->comp_len, DL = p->dom_len, EL = p->ext_len;
    double *FH = (double *)p->ws_fhat.ptr, *FC = (double *)p->ws_F.ptr;
    double *PP = (double *)p->ws_ppsi.ptr, *SF = (double *)p->ws_srcF.ptr, *Sf = (double *)p->ws_srcf.ptr;
    for (int c0 = 0; c0 < p->nc; c0 += kMacComponents) {
        const int ng = std::min(kMacComponents, p->nc - c0);
        const double *fg = f + (size_t)c0 * CL;
        double *ug = u + (size_t)c0 * CL;
        StageTimer tm(p->ctx, 3, s);
        for (int c = 0; c < ng; ++c)
            for (int k = 0; k < K; ++k) {
                const LevelSched &L = *p->lv[k];
                hip_check(mask_blocks(nb, fg + c * CL, FH + c * CL, (const int64_t *)L.d_own_off.ptr,
                                      (const int64_t *)L.d_own_off.ptr, (const unsigned char *)L.d_cover.ptr, L.n_own,
                                      s, (const unsigned char *)L.d_cmask.ptr),
                          "mask sources");
                hip_check(copy_blocks(nb, FH + c * CL, FC + c * CL, (const int64_t *)L.d_own_off.ptr,
                                      (const int64_t *)L.d_own_off.ptr, L.n_own, s),
                          "copy sources");
            }
        for (int c = 0; c < ng; ++c)
            for (int k = K - 2; k >= 0; --k) {
                const LevelSched &L = *p->lv[k];
                hip_check(coarsen_mean8(nb, FC + c * CL, FC + c * CL, (const int64_t *)L.d_cf_fine.ptr,
                                        (const int64_t *)L.d_cf_coarse.ptr, (const unsigned char *)L.d_cf_oct.ptr,
                                        L.n_cf, s),
                          "coarsen");
            }
        int cur = 0;
        for (int k = 0; k < K; ++k) {
            const LevelSched &L = *p->lv[k];
            const double dxk = p->dx0 / (double)(1 << k);
            double *q_prev = (double *)p->ws_psi[cur].ptr;
            double *q_next = (double *)p->ws_psi[cur ^ 1].ptr;
            if (k == 0) {
                run_op(p, *L.convF, FC, CL, ug, CL, ng, dxk, 0, s);
                hip_check(zero_fill(q_next, sizeof(double) * (size_t)DL * ng, s), "clear q");
                for (int c = 0; c < ng; ++c)
                    hip_check(copy_blocks(nb, FH + c * CL, q_next + c * DL, (const int64_t *)p->d_q0_src.ptr,
                                          (const int64_t *)p->d_q0_dst.ptr, p->n_q0, s),
                              "q0");
            } else {
                for (int c = 0; c < ng; ++c)
                    hip_check(correction_source(nb, L.corr, q_prev + c * DL, (const int *)L.d_cmap.ptr,
                                                (const int *)L.d_fblk.ptr, (const int64_t *)L.d_ext_own.ptr,
                                                FC + c * CL, FH + c * CL, PP + c * EL, SF + c * EL, Sf + c * EL,
                                                L.n_ext, s),
                              "interpolate q");
                run_op(p, *L.convF, SF, EL, ug, CL, ng, dxk, 0, s);
                if (k + 1 < K)
                    for (int c = 0; c < ng; ++c)
                        hip_check(copy_blocks(nb, Sf + c * EL, q_next + c * DL, (const int64_t *)L.d_cp_src.ptr,
                                              (const int64_t *)L.d_cp_dst.ptr, L.n_dom, s),
                                  "q");
            }
            if (L.any_cover || L.d_cmask.ptr)
                for (int c = 0; c < ng; ++c)
                    hip_check(mask_blocks(nb, ug + c * CL, ug + c * CL, (const int64_t *)L.d_own_off.ptr,
                                          (const int64_t *)L.d_own_off.ptr, (const unsigned char *)L.d_cover.ptr,
                                          L.n_own, s, (const unsigned char *)L.d_cmask.ptr),
                              "restrict phi");
            cur ^= 1;
        }
    }
}

static void enqueue(lgf_plan *p, const double *f, double *u, hipStream_t s) {
    if (p->K > 1) {
        if (p->if_a0 > 0.0)
            enqueue_fif(p, f, u, s);
        else
            enqueue_composite(p, f, u, s);
        return;
    }
    const int nblk = (int)p->levels[0].size();
    const int64_t *boff = (const int64_t *)p->d_blk_off.ptr;
    const unsigned char *cm = (const unsigned char *)p->d_cmask0.ptr;
    if (cm) {            // the caller's cell mask: Omega_0 only
        double *fm = (double *)p->ws_masked.ptr;
        for (int c = 0; c < p->nc; ++c)
            hip_check(mask_blocks(p->nb, f + (size_t)c * p->comp_len, fm + (size_t)c * p->comp_len, boff, boff,
                                  nullptr, nblk, s, cm),
                      "mask sources");
        f = fm;
    }
    if (p->collect)      // one level: the combined source is the source itself
        for (int c = 0; c < p->nc; ++c)
            hip_check(block_stats(p->nb, f + (size_t)c * p->comp_len, boff, nblk,
                                  (double *)p->d_ind.ptr + 2 * c * p->ind_total, s),
                      "indicator");
    run_op(p, *p->op0, f, p->comp_len, u, p->comp_len, p->nc, p->dx0, 0, s);
    if (lgf_plan *c = p->flgf_coarse.get()) {   // + I (far convolution on the node lattice) A f
        double *Fc = (double *)p->ws_fc.ptr, *Uc = (double *)p->ws_uc.ptr;
        for (int k = 0; k < p->nc; ++k)
            hip_check(flgf_anterpolate(p->nb, f + (size_t)k * p->comp_len, boff, nblk, Fc + (size_t)k * c->comp_len, s),
                      "anterpolate");
        run_op(c, *c->op0, Fc, c->comp_len, Uc, c->comp_len, c->nc, c->dx0, 0, s);
        for (int k = 0; k < p->nc; ++k)
            hip_check(flgf_interpolate_add(p->nb, Uc + (size_t)k * c->comp_len, boff, nblk, u + (size_t)k * p->comp_len,
                                           s),
                      "interpolate");
    }
    if (cm)
        for (int c = 0; c < p->nc; ++c)
            hip_check(mask_blocks(p->nb, u + (size_t)c * p->comp_len, u + (size_t)c * p->comp_len, boff, boff, nullptr,
                                  nblk, s, cm),
                      "restrict u");
}

void run_plan(lgf_plan *p, const double *f, double *u, hipStream_t s, lgf_report *rep) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (rep) {
        hip_check(hipEventCreate(&e0), "event");
        hip_check(hipEventCreate(&e1), "event");
        hip_check(hipEventRecord(e0, s), "event record");
    }
    enqueue(p, f, u, s);
    if (rep) {
        hip_check(hipEventRecord(e1, s), "event record");
        hip_check(hipEventSynchronize(e1), "event sync");
        float ms = 0.f;
        hip_check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
        rep->device_ms = ms;
        rep->refine_rel_l2 = 0.0;
        rep->passes = (int)p->convs_view.size();
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
}

// Record one solve of plan p on fixed f / u into a graph: the launches that
// lgf_solve would enqueue, captured on a private stream.  Stage timing is
// off while capturing (no event nodes), and the spectral workspace is
// cleared at the start of the graph whatever the host believes it holds.
hipGraph_t capture_solve(lgf_plan *p, const double *f, double *u) {
    hipStream_t cs = nullptr;
    hip_check(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "capture stream");
    const bool timing = p->ctx->timing;
    p->ctx->timing = false;
    p->fhat_conv = nullptr;
    hipGraph_t g = nullptr;
    try {
        hip_check(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed), "begin capture");
        enqueue(p, f, u, cs);
        hip_check(hipStreamEndCapture(cs, &g), "end capture");
    } catch (...) {
        hipGraph_t partial = nullptr;
        (void)hipStreamEndCapture(cs, &partial);
        if (partial) (void)hipGraphDestroy(partial);
        p->ctx->timing = timing;
        p->fhat_conv = nullptr;
        (void)hipStreamDestroy(cs);
        throw;
    }
    p->ctx->timing = timing;
    p->fhat_conv = nullptr;
    (void)hipStreamDestroy(cs);
    return g;
}

thread_local std::vector<std::unique_ptr<DeviceBuffer>> *g_job_sink = nullptr;

namespace {

// One convolution of a batch: plan workspace, sources -> destination.
struct ConvCall {
    lgf_plan *p;
    const Conv *c;
    const double *src;
    double *dst;
    double dx;
    int accumulate;
};

// Copy a job table into the next ring slot (pinned host -> device, on s).
template <typename T> const T *stage_jobs(lgf_context *ctx, const std::vector<T> &jobs, hipStream_t s, int &slot) {
    JobRing &r = ctx->ring;
    const size_t bytes = sizeof(T) * jobs.size();
    if (g_job_sink) {   // graph capture: a table of its own, filled now, read by every replay
        auto b = std::make_unique<DeviceBuffer>();
        b->alloc(ctx, std::max<size_t>(bytes, 16), "captured job table");
        // on the context's own stream, which is not being captured (a copy
        // on the legacy stream would join the capture)
        hip_check(hipMemcpyAsync(b->ptr, jobs.data(), bytes, hipMemcpyHostToDevice, ctx->stream),
                  "captured job table copy");
        hip_check(hipStreamSynchronize(ctx->stream), "captured job table sync");
        const T *d = (const T *)b->ptr;
        g_job_sink->push_back(std::move(b));
        slot = -1;
        return d;
    }
    if (bytes > JobRing::kSlotBytes) throw Failure(LGF_E_UNSUPPORTED, "batch job table larger than 256 KiB");
    std::lock_guard<std::mutex> lk(r.mu);
    const int k = r.next;
    r.next = (r.next + 1) % JobRing::kSlots;
    hip_check(hipEventSynchronize(r.done[k]), "ring slot wait");
    char *h = (char *)r.host + (size_t)k * JobRing::kSlotBytes;
    char *d = (char *)r.dev + (size_t)k * JobRing::kSlotBytes;
    std::memcpy(h, jobs.data(), bytes);
    hip_check(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s), "job table copy");
    slot = k;
    return (const T *)d;
}

// The slot may be reused once the launch that reads it has completed.
void ring_mark(lgf_context *ctx, int slot, hipStream_t s) {
    if (slot < 0) return;   // a captured table, not a ring slot
    JobRing &r = ctx->ring;
    std::lock_guard<std::mutex> lk(r.mu);
    hip_check(hipEventRecord(r.done[slot], s), "ring event record");
}

// Every call runs its forward FFTs, spectral MAC and inverse FFTs; calls with
// the same block size / row template / precision share one launch per stage.
void run_conv_batch(lgf_context *ctx, const std::vector<ConvCall> &calls, hipStream_t s) {
    if (calls.empty()) return;
    for (const ConvCall &k : calls)
        if (k.p->fhat_conv != k.c) {
            const bool needs_zeros = !fhat_full(*k.c) && k.c->method != kMethodLattice;
            if (needs_zeros) hip_check(zero_fill(k.p->Fhat.ptr, k.p->Fhat.bytes, s), "clear Fhat");
            k.p->fhat_conv = needs_zeros ? k.c : nullptr;
        }
    const int nb = calls[0].p->nb;
    for (const ConvCall &k : calls)
        if (k.p->nb != nb) throw Failure(LGF_E_INVALID, "internal: mixed block sizes in one batch group");
    const double N3 = 8.0 * nb * nb * nb;
    for (int fp = 0; fp < 2; ++fp) {
        std::vector<FftJob> fj;
        int total = 0;
        for (const ConvCall &k : calls) {
            if ((int)k.c->fp32 != fp || k.c->n_src == 0) continue;
            FftJob j{};
            j.src = k.src;
            j.blk_off = (const int64_t *)k.c->d_src_off.ptr;
            j.slot = (const int *)k.c->d_src_slot.ptr;
            j.spec = k.p->Fhat.ptr;
            j.n_slots = k.c->n_slots;
            j.block_major = k.c->method == kMethodLattice;
            j.scale = 1.0;
            j.blk_begin = total;
            total += k.c->n_src;
            fj.push_back(j);
        }
        if (fj.empty()) continue;
        StageTimer t(ctx, 0, s);
        int slot = 0;
        hip_check(block_fft_forward_batch(nb, fp == 1, stage_jobs(ctx, fj, s, slot), (int)fj.size(), total, s),
                  "batched forward FFT");
        ring_mark(ctx, slot, s);
    }
    std::vector<const void *> uhat2(calls.size(), nullptr);   // second terms of one-pass lattice MACs
    for (size_t i = 0; i < calls.size(); ++i) {
        const ConvCall &k = calls[i];
        if (k.c->method == kMethodLattice) {
            uhat2[i] = lattice_mac(ctx, *k.c, lat_geom(*k.c, 1), k.p->Fhat.ptr, k.p->ws_lat.ptr, k.p->Uhat.ptr, s);
        } else if (k.c->parts.empty()) {
            hip_check(zero_fill(k.p->Uhat.ptr, k.p->Uhat.bytes, s), "clear Uhat");
        }
    }
    // parts of one target segment are in different phases: one launch per
    // (phase, precision, template, sparse flag)
    int n_phase = 0;
    for (const ConvCall &k : calls)
        for (const auto &pt : k.c->parts) n_phase = std::max(n_phase, pt->phase + 1);
    // one launch per (phase, precision, template, tile shape, sparsity)
    std::set<std::tuple<int, int, int>> shapes;   // (bx, ty, tz)
    for (const ConvCall &k : calls) shapes.insert({k.c->bx, k.c->ty, k.c->tz});
    for (int ph = 0; ph < n_phase; ++ph)
        for (int fp = 0; fp < 2; ++fp)
            for (const auto &shape : shapes)
                for (int sp = 0; sp < 2; ++sp) {
                    const int bx = std::get<0>(shape), ty = std::get<1>(shape), tz = std::get<2>(shape);
                    std::vector<SmacJob> sj;
                    int64_t total = 0;
                    for (const ConvCall &k : calls) {
                        if ((int)k.c->fp32 != fp || k.c->bx != bx || k.c->ty != ty || k.c->tz != tz) continue;
                        for (const auto &pt : k.c->parts) {
                            if (pt->phase != ph || (int)pt->sparse != sp || pt->n_rows == 0 || pt->n_tiles == 0)
                                continue;
                            SmacJob j{};
                            j.g = conv_geom(*k.c, *pt);
                            j.F = k.p->Fhat.ptr;
                            j.U = k.p->Uhat.ptr;
                            j.K = k.c->spec->data.ptr;
                            j.rows = (const SmacRow *)pt->d_rows.ptr;
                            j.tiles = (const SmacTile *)pt->d_tiles.ptr;
                            j.wg_begin = total;
                            total += (int64_t)j.g.n_freq * j.g.n_tiles;
                            sj.push_back(j);
                        }
                    }
                    if (sj.empty()) continue;
                    StageTimer t(ctx, 1, s);
                    int slot = 0;
                    hip_check(smac_batch_launch(bx, ty, tz, fp == 1, sp == 1, stage_jobs(ctx, sj, s, slot), (int)sj.size(),
                                                total, s),
                              "batched spectral MAC");
                    ring_mark(ctx, slot, s);
                }
    for (int fp = 0; fp < 2; ++fp) {
        std::vector<FftJob> fj;
        int total = 0;
        for (size_t i = 0; i < calls.size(); ++i) {
            const ConvCall &k = calls[i];
            if ((int)k.c->fp32 != fp || k.c->n_tgt == 0) continue;
            FftJob j{};
            j.dst = k.dst;
            j.blk_off = (const int64_t *)k.c->d_tgt_off.ptr;
            j.slot = (const int *)k.c->d_tgt_slot.ptr;
            j.spec = k.p->Uhat.ptr;
            j.spec2 = uhat2[i];
            j.n_slots = k.c->n_slots;
            j.block_major = k.c->method == kMethodLattice;
            j.scale = conv_scale(k.p, k.dx) / N3;
            j.accumulate = k.accumulate;
            j.blk_begin = total;
            total += k.c->n_tgt;
            fj.push_back(j);
        }
        if (fj.empty()) continue;
        StageTimer t(ctx, 2, s);
        int slot = 0;
        hip_check(block_fft_inverse_batch(nb, fp == 1, stage_jobs(ctx, fj, s, slot), (int)fj.size(), total, s),
                  "batched inverse FFT");
        ring_mark(ctx, slot, s);
    }
}

}  // namespace

// One L^-1 application of a batch, for one component: plan, op, source ->
// destination (accumulate: add into it).  The plans of one batch call are
// distinct, so each call owns its plan's spectral and refinement workspaces.
struct OpCall {
    lgf_plan *p;
    const ConvOp *op;
    const double *src;
    double *dst;
    double dx;
    int accumulate;
};

// The ops of one batch step: plain ones and the float32 pass of refined ones
// in common launches, then the refined ones' residual step, cut passes (rows
// along x, then along y) and float32 residual pass, each in common launches.
void run_ops_batch(lgf_context *ctx, const std::vector<OpCall> &calls, hipStream_t s) {
    std::vector<ConvCall> a, b1, b1y, b2;
    for (const OpCall &k : calls) {
        const ConvOp &op = *k.op;
        if (!op.refined) {
            a.push_back(ConvCall{k.p, op.c64.get(), k.src, k.dst, k.dx, k.accumulate});
            continue;
        }
        a.push_back(ConvCall{k.p, op.c32.get(), k.src, (double *)k.p->ws_ut.ptr, k.dx, 0});
        if (op.c64) b1.push_back(ConvCall{k.p, op.c64.get(), (const double *)k.p->ws_ush.ptr, k.dst, k.dx, 1});
        if (op.c64y) b1y.push_back(ConvCall{k.p, op.c64y.get(), (const double *)k.p->ws_ush.ptr, k.dst, k.dx, 1});
        b2.push_back(ConvCall{k.p, op.ccorr.get(), (const double *)k.p->ws_rho.ptr, k.dst, k.dx, 1});
    }
    run_conv_batch(ctx, a, s);
    for (const OpCall &k : calls)
        if (k.op->refined)
            refine_middle(k.p, *k.op, k.src, k.dst, (const double *)k.p->ws_ut.ptr, (double *)k.p->ws_rho.ptr,
                          (double *)k.p->ws_ush.ptr, k.dx, k.accumulate, s);
    run_conv_batch(ctx, b1, s);
    run_conv_batch(ctx, b1y, s);
    run_conv_batch(ctx, b2, s);
}

// Composite plans of one block size, level by level (the order of the
// paper's Sec. 3.4 within each plan): per component group, every plan's
// source restriction and coarsening, then for k = 0, 1, ...: every plan's
// correction source at level k, the phi_k convolutions of all plans in
// common launches, then their psi_k convolutions, then the restriction.
void run_composite_batch(lgf_context *ctx, const std::vector<lgf_plan *> &ps, const std::vector<const double *> &fs,
                         const std::vector<double *> &us, hipStream_t s) {
    int n_groups = 0, k_max = 0;
    for (lgf_plan *p : ps) {
        n_groups = std::max(n_groups, (p->nc + kMacComponents - 1) / kMacComponents);
        k_max = std::max(k_max, p->K);
    }
    const size_t n = ps.size();
    for (int g = 0; g < n_groups; ++g) {
        const int c0 = g * kMacComponents;
        std::vector<int> ng(n, 0), cur(n, 0);
        for (size_t i = 0; i < n; ++i) {
            lgf_plan *p = ps[i];
            if (c0 >= p->nc) continue;
            ng[i] = std::min(kMacComponents, p->nc - c0);
            const int64_t CL = p->comp_len;
            const double *fg = fs[i] + (size_t)c0 * CL;
            double *FH = (double *)p->ws_fhat.ptr, *FC = (double *)p->ws_F.ptr;
            StageTimer tm(ctx, 3, s);
            for (int c = 0; c < ng[i]; ++c)
                for (int k = 0; k < p->K; ++k) {
                    const LevelSched &L = *p->lv[k];
                    hip_check(mask_blocks(p->nb, fg + c * CL, FH + c * CL, (const int64_t *)L.d_own_off.ptr,
                                          (const int64_t *)L.d_own_off.ptr, (const unsigned char *)L.d_cover.ptr,
                                          L.n_own, s, (const unsigned char *)L.d_cmask.ptr),
                              "mask sources");
                    hip_check(copy_blocks(p->nb, FH + c * CL, FC + c * CL, (const int64_t *)L.d_own_off.ptr,
                                          (const int64_t *)L.d_own_off.ptr, L.n_own, s),
                              "copy sources");
                }
            for (int c = 0; c < ng[i]; ++c)
                for (int k = p->K - 2; k >= 0; --k) {
                    const LevelSched &L = *p->lv[k];
                    hip_check(coarsen_mean8(p->nb, FC + c * CL, FC + c * CL, (const int64_t *)L.d_cf_fine.ptr,
                                            (const int64_t *)L.d_cf_coarse.ptr, (const unsigned char *)L.d_cf_oct.ptr,
                                            L.n_cf, s),
                              "coarsen");
                }
        }
        for (int k = 0; k < k_max; ++k) {
            std::vector<OpCall> opF[kMacComponents], opPsi[kMacComponents];
            for (size_t i = 0; i < n; ++i) {
                lgf_plan *p = ps[i];
                if (ng[i] == 0 || k >= p->K) continue;
                const LevelSched &L = *p->lv[k];
                const int nb = p->nb;
                const int64_t CL = p->comp_len, DL = p->dom_len, EL = p->ext_len;
                double *FH = (double *)p->ws_fhat.ptr, *FC = (double *)p->ws_F.ptr;
                double *PP = (double *)p->ws_ppsi.ptr, *SF = (double *)p->ws_srcF.ptr, *Sf = (double *)p->ws_srcf.ptr;
                double *ug = us[i] + (size_t)c0 * CL;
                const double dxk = p->dx0 / (double)(1 << k);
                double *psi_prev = (double *)p->ws_psi[cur[i]].ptr;
                double *psi_next = (double *)p->ws_psi[cur[i] ^ 1].ptr;
                if (k > 0) {
                    StageTimer tm(ctx, 3, s);
                    for (int c = 0; c < ng[i]; ++c) {
                        hip_check(correction_source(nb, L.corr, psi_prev + c * DL, (const int *)L.d_cmap.ptr,
                                                    (const int *)L.d_fblk.ptr, (const int64_t *)L.d_ext_own.ptr,
                                                    FC + c * CL, FH + c * CL, PP + c * EL, SF + c * EL, Sf + c * EL,
                                                    L.n_ext, s),
                                  "correction source");
                        hip_check(copy_blocks(nb, PP + c * EL, ug + c * CL, (const int64_t *)L.d_cu_src.ptr,
                                              (const int64_t *)L.d_cu_dst.ptr, L.n_own, s),
                                  "P psi -> phi");
                        if (L.convPsi)
                            hip_check(copy_blocks(nb, PP + c * EL, psi_next + c * DL, (const int64_t *)L.d_cp_src.ptr,
                                                  (const int64_t *)L.d_cp_dst.ptr, L.n_dom, s),
                                      "P psi -> psi");
                    }
                }
                for (int c = 0; c < ng[i]; ++c) {
                    const double *srcF = k == 0 ? FC + c * CL : SF + c * EL;
                    opF[c].push_back(OpCall{p, L.convF.get(), srcF, ug + c * CL, dxk, k > 0});
                    if (L.convPsi) {
                        const double *srcf = k == 0 ? FH + c * CL : Sf + c * EL;
                        opPsi[c].push_back(OpCall{p, L.convPsi.get(), srcf, psi_next + c * DL, dxk, k > 0});
                    }
                }
            }
            for (int c = 0; c < kMacComponents; ++c) run_ops_batch(ctx, opF[c], s);
            for (int c = 0; c < kMacComponents; ++c) run_ops_batch(ctx, opPsi[c], s);
            for (size_t i = 0; i < n; ++i) {
                lgf_plan *p = ps[i];
                if (ng[i] == 0 || k >= p->K) continue;
                const LevelSched &L = *p->lv[k];
                double *ug = us[i] + (size_t)c0 * p->comp_len;
                if (L.any_cover || L.d_cmask.ptr)
                    for (int c = 0; c < ng[i]; ++c)
                        hip_check(mask_blocks(p->nb, ug + c * p->comp_len, ug + c * p->comp_len,
                                              (const int64_t *)L.d_own_off.ptr, (const int64_t *)L.d_own_off.ptr,
                                              (const unsigned char *)L.d_cover.ptr, L.n_own, s, (const unsigned char *)L.d_cmask.ptr),
                                  "restrict phi");
                cur[i] ^= 1;
            }
        }
    }
}

void run_batch(lgf_context *ctx, int n, lgf_plan *const *plans, const double *const *f, double *const *u,
               hipStream_t s, lgf_report *reps) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (reps) {
        hip_check(hipEventCreate(&e0), "event");
        hip_check(hipEventCreate(&e1), "event");
        hip_check(hipEventRecord(e0, s), "event record");
    }
    // per block size: single-level plans component by component, then the
    // composite plans level by level
    std::map<int, std::vector<int>> by_nb;
    for (int i = 0; i < n; ++i) by_nb[plans[i]->nb].push_back(i);
    for (auto &kv : by_nb) {
        std::vector<int> single;
        std::vector<lgf_plan *> cps;
        std::vector<const double *> cfs;
        std::vector<double *> cus;
        for (int i : kv.second) {
            if (plans[i]->K == 1 && (plans[i]->d_cmask0.ptr || plans[i]->flgf_coarse)) {   // own extra steps
                enqueue(plans[i], f[i], u[i], s);
            } else if (plans[i]->K == 1) {
                single.push_back(i);
            } else if (plans[i]->if_a0 > 0.0) {   // integrating factor on a composite mesh: its own schedule
                enqueue(plans[i], f[i], u[i], s);
            } else {
                cps.push_back(plans[i]);
                cfs.push_back(f[i]);
                cus.push_back(u[i]);
            }
        }
        int max_nc = 0;
        for (int i : single) max_nc = std::max(max_nc, plans[i]->nc);
        for (int comp = 0; comp < max_nc; ++comp) {
            std::vector<OpCall> calls;
            for (int i : single) {
                lgf_plan *p = plans[i];
                if (comp >= p->nc) continue;
                calls.push_back(OpCall{p, p->op0.get(), f[i] + (size_t)comp * p->comp_len,
                                       u[i] + (size_t)comp * p->comp_len, p->dx0, 0});
            }
            run_ops_batch(ctx, calls, s);
        }
        if (!cps.empty()) run_composite_batch(ctx, cps, cfs, cus, s);
    }
    if (reps) {
        hip_check(hipEventRecord(e1, s), "event record");
        hip_check(hipEventSynchronize(e1), "event sync");
        float ms = 0.f;
        hip_check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
        for (int i = 0; i < n; ++i) {
            reps[i].device_ms = ms;
            reps[i].refine_rel_l2 = 0.0;
            reps[i].passes = (int)plans[i]->convs_view.size();
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
}

}  // namespace lgf

namespace lgf {

// Record one lgf_solve_batch of these plans on fixed buffers into a graph,
// as capture_solve does for one plan; the job tables of the batched
// launches go to buffers of their own (kept in `tables`) instead of the ring.
hipGraph_t capture_batch(lgf_context *ctx, int n, lgf_plan *const *plans, const double *const *f, double *const *u,
                         std::vector<std::unique_ptr<DeviceBuffer>> &tables) {
    hipStream_t cs = nullptr;
    hip_check(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "capture stream");
    for (int i = 0; i < n; ++i) plans[i]->fhat_conv = nullptr;
    g_no_timing = true;
    g_job_sink = &tables;
    hipGraph_t g = nullptr;
    auto reset = [&]() {
        g_no_timing = false;
        g_job_sink = nullptr;
        for (int i = 0; i < n; ++i) plans[i]->fhat_conv = nullptr;
        (void)hipStreamDestroy(cs);
    };
    try {
        hip_check(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed), "begin capture");
        run_batch(ctx, n, plans, f, u, cs, nullptr);
        hip_check(hipStreamEndCapture(cs, &g), "end capture");
    } catch (...) {
        hipGraph_t partial = nullptr;
        (void)hipStreamEndCapture(cs, &partial);
        if (partial) (void)hipGraphDestroy(partial);
        (void)hipGetLastError();
        reset();
        throw;
    }
    reset();
    return g;
}

}  // namespace lgf

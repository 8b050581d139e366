// Local expectation values by direct boundary-MPS contraction (Results,
// Fig. 4: <Z_i> from <psi|Z_i|psi> / <psi|psi>).
//
// Boundaries from below come from the bottom-up set, boundaries from above from
// the same fit on the vertically mirrored lattice view.  Within row r, the
// double-layer row environments [p, h, k, g] between the boundary above (bond
// p) and below (bond g) give the one-site density matrix with the site open
// (ket s, bra t), and the diagonal of the two-site marginal of horizontal
// neighbours.  Vertical neighbours use a two-row environment
// [p, h1, k1, h2, k2, g] between the boundary above row r and the boundary
// below row r+1.  Environments are renormalised per column (the outputs are
// ratios).
#include <vector>

#include "tn_core.hpp"

namespace tnb {

namespace {

Ten row_left(Engine &E, const Ten &Le, const Ten &U, const SiteRef &a, const Ten &B, int s = -1, int t = -1) {
    Ten x1 = E.contract_new(op(Le, "phkg"), op(U, "puvP"), "hkguvP");
    Ten x3;
    if (s < 0) {
        Ten x2 = E.contract_new(op(x1, "hkguvP"), sop(a, "suhdH"), "kgvPsdH");
        E.drop(x1);
        x3 = E.contract_new(op(x2, "kgvPsdH"), sop(a, "svkeK", true), "gPdHeK");
        E.drop(x2);
    } else {
        Ten x2 = E.contract_new(op(x1, "hkguvP"), sop_proj(a, s, "uhdH"), "kgvPdH");
        E.drop(x1);
        x3 = E.contract_new(op(x2, "kgvPdH"), sop_proj(a, t, "vkeK", true), "gPdHeK");
        E.drop(x2);
    }
    Ten out = E.contract_new(op(x3, "gPdHeK"), op(B, "gdeG"), "PHKG");
    E.drop(x3);
    return out;
}

Ten row_right(Engine &E, const Ten &Re, const Ten &U, const SiteRef &a, const Ten &B) {
    Ten x1 = E.contract_new(op(U, "puvP"), op(Re, "PHKG"), "puvHKG");
    Ten x2 = E.contract_new(op(x1, "puvHKG"), sop(a, "suhdH"), "pvKGshd");
    E.drop(x1);
    Ten x3 = E.contract_new(op(x2, "pvKGshd"), sop(a, "svkeK", true), "pGhdke");
    E.drop(x2);
    Ten out = E.contract_new(op(x3, "pGhdke"), op(B, "gdeG"), "phkg");
    E.drop(x3);
    return out;
}

// letters of the two-row environment: a = h1, b = k1, c = h2, d = k2
Ten two_left(Engine &E, const Ten &Le, const Ten &U, const SiteRef &a1, const SiteRef &a2, const Ten &B, int s = -1,
             int t = -1) {
    Ten x1 = E.contract_new(op(Le, "pabcdg"), op(U, "puvP"), "abcdguvP");
    Ten x3;
    if (s < 0) {
        Ten x2 = E.contract_new(op(x1, "abcdguvP"), sop(a1, "suamH"), "bcdgvPsmH");
        E.drop(x1);
        x3 = E.contract_new(op(x2, "bcdgvPsmH"), sop(a1, "svbnK", true), "cdgPmHnK");
        E.drop(x2);
    } else {
        Ten x2 = E.contract_new(op(x1, "abcdguvP"), sop_proj(a1, s, "uamH"), "bcdgvPmH");
        E.drop(x1);
        x3 = E.contract_new(op(x2, "bcdgvPmH"), sop_proj(a1, s, "vbnK", true), "cdgPmHnK");
        E.drop(x2);
    }
    Ten x5;
    if (t < 0) {
        Ten x4 = E.contract_new(op(x3, "cdgPmHnK"), sop(a2, "tmcxJ"), "dgPHnKtxJ");
        E.drop(x3);
        x5 = E.contract_new(op(x4, "dgPHnKtxJ"), sop(a2, "tndeL", true), "gPHKxJeL");
        E.drop(x4);
    } else {
        Ten x4 = E.contract_new(op(x3, "cdgPmHnK"), sop_proj(a2, t, "mcxJ"), "dgPHnKxJ");
        E.drop(x3);
        x5 = E.contract_new(op(x4, "dgPHnKxJ"), sop_proj(a2, t, "ndeL", true), "gPHKxJeL");
        E.drop(x4);
    }
    Ten out = E.contract_new(op(x5, "gPHKxJeL"), op(B, "gxeG"), "PHKJLG");
    E.drop(x5);
    return out;
}

Ten two_right(Engine &E, const Ten &Re, const Ten &U, const SiteRef &a1, const SiteRef &a2, const Ten &B) {
    Ten x1 = E.contract_new(op(U, "puvP"), op(Re, "PHKJLG"), "puvHKJLG");
    Ten x2 = E.contract_new(op(x1, "puvHKJLG"), sop(a1, "suamH"), "pvKJLGsam");
    E.drop(x1);
    Ten x3 = E.contract_new(op(x2, "pvKJLGsam"), sop(a1, "svbnK", true), "pJLGambn");
    E.drop(x2);
    Ten x4 = E.contract_new(op(x3, "pJLGambn"), sop(a2, "tmcxJ"), "pLGabntcx");
    E.drop(x3);
    Ten x5 = E.contract_new(op(x4, "pLGabntcx"), sop(a2, "tndeL", true), "pGabcxde");
    E.drop(x4);
    Ten out = E.contract_new(op(x5, "pGabcxde"), op(B, "gxeG"), "pabcdg");
    E.drop(x5);
    return out;
}

void unit1(Engine &E, Ten &t) { E.normalise(t.p, t.esz, t.numel(), 1, 0, nullptr, false, nullptr); }

}  // namespace

void environments(Engine &E, const PepsDev &P, const FitOpts &o, const BoundarySet *below_in, double *rho1,
                  double *zz_h, double *zz_v, double *p2_h, double *p2_v) {
    const int rows = P.rows, cols = P.cols;
    const double nan = __builtin_nan("");
    TN_HIP(tnk::launch_fill_f64(rho1, (int64_t)rows * cols * 8, nan, E.s));
    if (zz_h && cols > 1) TN_HIP(tnk::launch_fill_f64(zz_h, (int64_t)rows * (cols - 1), nan, E.s));
    if (zz_v && rows > 1) TN_HIP(tnk::launch_fill_f64(zz_v, (int64_t)(rows - 1) * cols, nan, E.s));
    const bool want_h = zz_h || p2_h, want_v = zz_v || p2_v;
    if (p2_h && cols > 1) TN_HIP(tnk::launch_fill_f64(p2_h, (int64_t)rows * (cols - 1) * 4, nan, E.s));
    if (p2_v && rows > 1) TN_HIP(tnk::launch_fill_f64(p2_v, (int64_t)(rows - 1) * cols * 4, nan, E.s));
    const LView V = make_view(P, 0);
    const LView F = make_view(P, 1);
    BoundarySet own;
    if (!below_in) own = boundary_set(E, V, o, 0);
    const BoundarySet &below = below_in ? *below_in : own;
    BoundarySet fb = boundary_set(E, F, o, 1);
    auto above = [&](int r) -> const DMps & { return fb.below[rows - 1 - r]; };
    double *dots = reinterpret_cast<double *>(E.raw(8 * 8));
    try {
        for (int r = 0; r < rows; ++r) {
            const DMps &U = above(r);
            const DMps &B = below.below[r];
            std::vector<Ten> Le(cols + 1), Ri(cols + 1);
            Le[0] = ones(E, {1, 1, 1, 1});
            for (int c = 0; c < cols; ++c) {
                Le[c + 1] = row_left(E, Le[c], U.site[c], V.at(r, c), B.site[c]);
                unit1(E, Le[c + 1]);
            }
            Ri[cols] = ones(E, {1, 1, 1, 1});
            for (int c = cols - 1; c >= 0; --c) {
                Ri[c] = row_right(E, Ri[c + 1], U.site[c], V.at(r, c), B.site[c]);
                unit1(E, Ri[c]);
            }
            for (int c = 0; c < cols; ++c) {
                if (P.phys[(size_t)r * cols + c] != 2) continue;
                for (int s = 0; s < 2; ++s)
                    for (int t = 0; t < 2; ++t) {
                        Ten x = row_left(E, Le[c], U.site[c], V.at(r, c), B.site[c], s, t);
                        E.dot(x.p, Ri[c + 1].p, x.esz, x.numel(), 1, 0, dots + 2 * (2 * s + t));
                        E.drop(x);
                    }
                TN_HIP(tnk::launch_env_rho(dots, rho1 + ((size_t)r * cols + c) * 8, E.s));
            }
            for (int c = 0; want_h && c + 1 < cols; ++c) {
                if (P.phys[(size_t)r * cols + c] != 2 || P.phys[(size_t)r * cols + c + 1] != 2) continue;
                for (int s = 0; s < 2; ++s) {
                    Ten x = row_left(E, Le[c], U.site[c], V.at(r, c), B.site[c], s, s);
                    for (int t = 0; t < 2; ++t) {
                        Ten y = row_left(E, x, U.site[c + 1], V.at(r, c + 1), B.site[c + 1], t, t);
                        E.dot(y.p, Ri[c + 2].p, y.esz, y.numel(), 1, 0, dots + 2 * (2 * s + t));
                        E.drop(y);
                    }
                    E.drop(x);
                }
                const size_t b = (size_t)r * (cols - 1) + c;
                TN_HIP(tnk::launch_env_p2(dots, p2_h ? p2_h + 4 * b : nullptr, zz_h ? zz_h + b : nullptr, E.s));
            }
            for (auto &x : Le) E.drop(x);
            for (auto &x : Ri) E.drop(x);
        }
        for (int r = 0; want_v && r + 1 < rows; ++r) {
            const DMps &U = above(r);
            const DMps &B = below.below[r + 1];
            std::vector<Ten> Le(cols + 1), Ri(cols + 1);
            Le[0] = ones(E, {1, 1, 1, 1, 1, 1});
            for (int c = 0; c < cols; ++c) {
                Le[c + 1] = two_left(E, Le[c], U.site[c], V.at(r, c), V.at(r + 1, c), B.site[c]);
                unit1(E, Le[c + 1]);
            }
            Ri[cols] = ones(E, {1, 1, 1, 1, 1, 1});
            for (int c = cols - 1; c >= 0; --c) {
                Ri[c] = two_right(E, Ri[c + 1], U.site[c], V.at(r, c), V.at(r + 1, c), B.site[c]);
                unit1(E, Ri[c]);
            }
            for (int c = 0; c < cols; ++c) {
                if (P.phys[(size_t)r * cols + c] != 2 || P.phys[(size_t)(r + 1) * cols + c] != 2) continue;
                for (int s = 0; s < 2; ++s)
                    for (int t = 0; t < 2; ++t) {
                        Ten x = two_left(E, Le[c], U.site[c], V.at(r, c), V.at(r + 1, c), B.site[c], s, t);
                        E.dot(x.p, Ri[c + 1].p, x.esz, x.numel(), 1, 0, dots + 2 * (2 * s + t));
                        E.drop(x);
                    }
                const size_t b = (size_t)r * cols + c;
                TN_HIP(tnk::launch_env_p2(dots, p2_v ? p2_v + 4 * b : nullptr, zz_v ? zz_v + b : nullptr, E.s));
            }
            for (auto &x : Le) E.drop(x);
            for (auto &x : Ri) E.drop(x);
        }
    } catch (...) {
        E.unraw(dots);
        free_set(E, own);
        free_set(E, fb);
        throw;
    }
    E.sync();
    E.unraw(dots);
    free_set(E, own);
    free_set(E, fb);
}

}  // namespace tnb

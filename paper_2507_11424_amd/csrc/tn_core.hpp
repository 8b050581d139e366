// Boundary-MPS contraction and sampling on the engine (host orchestration).
#pragma once

#include "engine.hpp"

namespace tnb {

// Site tensors staged in the compute precision, dims {p, u, l, d, r}.
struct PepsDev {
    int rows = 0, cols = 0, nq = 0;
    std::vector<Ten> site;
    std::vector<int> phys, site_index;
    const Ten &at(int r, int c) const { return site[(size_t)r * cols + c]; }
};

// A site seen through a lattice transformation: view slot i (0..4 = s,u,l,d,r)
// reads slot perm[i] of the stored tensor.  No data is moved.
struct SiteRef {
    const Ten *t = nullptr;
    int perm[5] = {0, 1, 2, 3, 4};
    int dim(int i) const { return t->d[perm[i]]; }
};

struct LView {
    int rows = 0, cols = 0;
    std::vector<SiteRef> s;
    const SiteRef &at(int r, int c) const { return s[(size_t)r * cols + c]; }
};

// direction 0: rows as stored; 1: mirrored top-bottom; 2: rows and columns
// exchanged; 3: exchanged then mirrored.
LView make_view(const PepsDev &P, int direction);
Op sop(const SiteRef &a, const std::string &letters5, bool conj = false);
// Physical index fixed to s: letters for (u, l, d, r).
Op sop_proj(const SiteRef &a, int s, const std::string &letters4, bool conj = false);

struct FitOpts {
    int chi = 16;
    int sweeps = 2;
    bool force_fit = false;
    uint64_t seed = 0;
};

// Double-layer boundary MPS, site c dims {yl, u, v, yr} (ket phys u, bra phys v).
struct DMps {
    std::vector<Ten> site;
};

struct BoundarySet {
    std::vector<DMps> below;   // below[r] approximates the rows under row r
    double *logs = nullptr;    // device [rows]: log of the norm divided out of below[r]
    std::vector<int> mode;     // per r: 1 exact product, 2 fitted
    int rows = 0;
};

void free_mps(Engine &E, DMps &m);
Ten ones(Engine &E, const std::vector<int> &dims);
// QR of T as batch x m x n (first nb dims batch, n = last dim); R optional.
// TN_PROGRESS=1: long loops synchronise per row and report it on stderr.
bool progress_enabled();
void qr_left(Engine &E, const Ten &T, int nb, Ten &Q, Ten *R, bool well_conditioned = false);
// LQ of T as batch x m x n (m = dim nb, n = the rest); L optional.
void lq_right(Engine &E, const Ten &T, int nb, Ten &Q, Ten *L, bool well_conditioned = false);
// Canonical form by QR then LQ sweeps, centre (site 0) normalised into logscale.
void canonicalise(Engine &E, std::vector<Ten> &Y, int nb, double *logscale, bool acc);
void right_canonicalise(Engine &E, std::vector<Ten> &Y, int nb);
void free_set(Engine &E, BoundarySet &b);

void plan_bonds(const std::vector<int> &phys, const std::vector<int64_t> &bond_in, int chi,
                bool &exact_ok, std::vector<int> &t);

BoundarySet boundary_set(Engine &E, const LView &V, const FitOpts &o, uint64_t tag);
// log|Z| and arg Z from closing row 0 of the view against below[0]; synchronises.
void norm_close(Engine &E, const LView &V, const BoundarySet &B, double *logabs, double *arg);

// below: the bottom-up boundary set of P with the same options (computed here if null).
void environments(Engine &E, const PepsDev &P, const FitOpts &o, const BoundarySet *below, double *rho1,
                  double *zz_h, double *zz_v, double *p2_h, double *p2_v);

struct SampleOpts {
    int chi_x = 16;
    int sweeps = 2;
    bool force_fit = false;
    uint64_t init_seed = 0;
    uint64_t seed = 0;
    int wave = 0;  // samples per wave (0 = automatic)
    int init_tag = 2;  // Philox stream of the fit's random initial guesses
    double svd_cutoff = 0;  // > 0: SVD truncation of every fitted amplitude boundary
    int chi_x_min = 1;      // lower clamp of the truncation
    // test hooks: stop after rows_limit rows (0 = all rows); log_cond (device
    // [n][N] doubles) receives every drawn qubit's log P(x_q | earlier qubits)
    int rows_limit = 0;
    double *log_cond = nullptr;
    // replay full waves after the second from a captured graph (0: run every wave directly)
    int graphs = 1;
};

// chi_used (optional, device [n][rows] int32): largest kept bond of the
// amplitude boundary conditioning each row (1 for the first row).
void sample(Engine &E, const PepsDev &P, const BoundarySet &B, const SampleOpts &o, uint64_t first,
            int64_t n, const double *uniforms, uint8_t *bits, double *log_q, double *log_p, int *chi_used);

// <x|psi> for given bitstrings bits [n][nq] (device) by single-layer boundary
// MPSs of bond <= o.chi_x from the top row down; log_p [n] = 2 log|<x|psi>|,
// arg [n] (optional) = its phase.  Sample index first + i keys the Philox
// stream (tag o.init_tag) of the fits' initial guesses.
void amplitude(Engine &E, const PepsDev &P, const SampleOpts &o, uint64_t first, int64_t n, const uint8_t *bits,
               double *log_p, double *arg);

// Belief propagation on the norm network and the loop BP error (FP64).
struct BpOpts {
    int max_sweeps = 1000;
    double tol = 1e-13;
    bool loops = true;          // also the loop BP error of every primitive loop
    void *messages = nullptr;   // optional device copy of the final messages [N][4][Dm][Dm]
    // optional device messages to start from (same layout, those of an earlier
    // state of the same lattice); identity / sqrt(D) on every bond otherwise
    const void *init_messages = nullptr;
};
struct BpResult {
    double log_abs = 0, arg = 0, delta = 0, eps_mean = 0;
    int sweeps = 0, eig_info = 0;
    std::vector<double> eps;    // per primitive loop, ordered by the loop's first site
};
void bp_contract(Engine &E, const PepsDev &P, const BpOpts &o, BpResult &res);

// Simple-update circuit simulation (FP64).  A gate acts on the qubits at
// (r, c) and (r2, c2) = (r, c + 1) or (r + 1, c); the BP messages are refreshed
// whenever `group` changes along the list.
struct SuGate {
    int group, r, c, r2, c2;
};
struct SuOpts {
    int bp_max_sweeps = 1000;
    double bp_tol = 1e-13;
};
// P's complex128 site tensors are replaced in place; gmat (host) holds the
// 4 x 4 complex128 gate matrices, gstride = 16 complex numbers per gate or 0
// (one matrix for every gate); eps_host [gates] receives the gate errors.
// msg_in (optional, device [rows*cols][4][Dm][Dm] complex128, the BpOpts
// message layout): the first group's BP starts from these messages instead of
// identity / sqrt(D); msg_out (optional, same layout, may alias msg_in)
// receives the last group's converged messages, so that a circuit split over
// several calls runs as one.
void simple_update(Engine &E, PepsDev &P, const std::vector<SuGate> &gates, const double *gmat, int gstride,
                   const SuOpts &o, double *eps_host, const void *msg_in = nullptr, void *msg_out = nullptr);

}  // namespace tnb

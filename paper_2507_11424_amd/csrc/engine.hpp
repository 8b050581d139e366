// Host-side execution engine: device memory pool, tensor views, the
// einsum-style contraction planner on top of the GETT kernel, QR and norm
// wrappers.  All work is enqueued on one HIP stream.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

#include "kernels.hpp"

namespace tnb {

enum : int { ST_INVALID = 1, ST_SHAPE = 2, ST_OOM = 3, ST_HIP = 4, ST_NUMERIC = 5, ST_UNSUPPORTED = 6 };

struct TnError : std::runtime_error {
    int code;
    TnError(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define TN_HIP(x)                                                                          \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess)                                                              \
            throw ::tnb::TnError(::tnb::ST_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Dense row-major complex tensor in device memory.
struct Ten {
    void *p = nullptr;
    std::vector<int> d;
    int esz = 16;
    int64_t numel() const {
        int64_t n = 1;
        for (int x : d) n *= x;
        return n;
    }
    size_t bytes() const { return (size_t)numel() * esz; }
    int dim(int i) const { return d[i < 0 ? (int)d.size() + i : i]; }
};

// One operand of a contraction: letters, dims and element strides.  A letter
// may have stride 0 (broadcast over that index).
struct Op {
    const void *p = nullptr;
    int esz = 16;
    std::string idx;
    std::vector<int> dims;
    std::vector<int64_t> str;
    bool conj = false;
};

Op op(const Ten &t, const std::string &idx, bool conj = false);
// The same tensor seen with an extra broadcast letter in front (stride 0).
Op op_bcast(const Ten &t, char letter, int size, const std::string &idx, bool conj = false);

class Pool {
  public:
    explicit Pool(size_t cap) : cap_(cap) {}
    ~Pool();
    void *get(size_t bytes);
    void put(void *p);
    size_t held() const { return held_; }
    void trim();
    // Arena mode (stream capture): between begin_arena and end_arena every block
    // handed out -- taken from the free list or newly allocated -- is recorded,
    // and blocks put back are reused only within the arena.  end_arena returns
    // them all: they belong to the captured graph, whose replays use the same
    // addresses, until release() hands them back to the pool.
    void begin_arena();
    std::vector<void *> end_arena();
    void release(const std::vector<void *> &blocks);

  private:
    size_t cap_;
    size_t held_ = 0;
    std::multimap<size_t, void *> free_;
    std::unordered_map<void *, size_t> size_;
    bool arena_ = false;
    std::multimap<size_t, void *> afree_;
    std::vector<void *> ablocks_;
    void *take(std::multimap<size_t, void *> &fl, size_t bytes);
};

struct Plan {
    tnk::GettArgs base;  // pointers to tables filled in; data pointers per call
    int cfg = 0;
    bool swapped = false;
    void *dev = nullptr;  // table storage
    double flops = 0;     // 8 * M * N * K * batch
    std::string desc;     // "A,B->C M=.. N=.. K=.. batch=.. cfg=.. split=.."
    std::string key;      // cache key (shape signature)
    double ms = 0;        // device time accumulated in timing mode
    int64_t calls = 0;
    bool tuned = false;   // tile configuration chosen by measurement
    int64_t kM = 0, kN = 0, K = 0, Z = 0;
    bool pack = false;    // split-BF16 on packed operand planes (else split while staging)
    bool can_pack = false;  // packing is offered (both matrix sides above 128); the tuner decides
    bool fp32 = false;      // split-BF16 modes: this shape runs on the FP32 kernel (chosen by the tuner)
    // letters of the batch, kernel-M and kernel-N index spaces, slowest first,
    // and every letter's extent (for masked launches)
    std::string bl, kml, knl;
    std::map<char, int> ldim;
};

struct Counters {
    double gemm_flops = 0;
    int64_t gemm_launches = 0;
    double gemm_ms = 0;
    double qr_ms = 0;
    int64_t qr_launches = 0;
    double qr_gemm_flops = 0;  // part of gemm_flops issued inside orthonormalisations
    // masked launches (tiles of masked items skipped): neither their flops nor
    // their time enter gemm_flops / gemm_ms
    double masked_ms = 0;
    int64_t masked_launches = 0;
    // algorithmic operand bytes of the (unmasked) launches: every element of A
    // and B read once, C written once (read too when accumulating)
    double gemm_bytes = 0;
    // replays of captured launch graphs (their launches are counted above too)
    int64_t graph_launches = 0;
    void reset() { *this = Counters(); }
};

class Engine {
  public:
    Engine(int device, hipStream_t s, size_t cap);
    ~Engine();

    hipStream_t s;
    int device;
    int prec = tnk::P_FP64;
    int esz = 16;  // element size of compute tensors
    // test hook: run contractions with this tile configuration / K-slice count
    // instead of the plan's (-1: the plan's choice)
    int force_cfg = -1, force_ksplit = 0;
    Counters ctr;
    bool timing = false;
    // orthonormalise() by Householder QR instead of CholeskyQR: set while the
    // sampler truncates its amplitude boundaries, whose zero-padded bonds make
    // the fit's matrices rank-deficient (CholeskyQR needs full column rank)
    bool householder_only = false;
    // Contractions issued while a mask is set skip the tiles of the items z of
    // letter `letter` with mask[z] == skip (device int array over that letter's
    // extent) when the letter is the slowest of the batch, M or N index space;
    // otherwise they compute everything.  Skipped parts of the output keep
    // whatever they held.
    void set_mask(const int *mask, char letter, int skip = 0) {
        mask_ = mask;
        mask_letter_ = letter;
        mask_skip_ = skip;
    }
    void clear_mask() { mask_ = nullptr; }

    void set_prec(int p) { prec = p; esz = (p == tnk::P_FP64) ? 16 : 8; }

    Ten make(const std::vector<int> &dims, int esz_override = 0);
    void drop(Ten &t);

    // C[ic] (+)= sum A[ia] * B[ib]; C must be allocated with the dims of ic.
    void contract(const Op &A, const Op &B, const Op &C, bool accumulate = false);
    // Allocates C with the letters of ic (dims taken from A and B).
    Ten contract_new(const Op &A, const Op &B, const std::string &ic);

    // Reduced QR (FP64) of `batch` matrices; see tnk::QrArgs.
    void qr(const tnk::QrArgs &a);
    // Orthonormal Q for m >= n (else Householder): shifted CholeskyQR3 in
    // FP64 -- three passes of Gram matrix (MFMA), Cholesky and R^{-1} (one
    // workgroup), Q <- Q R^{-1} (MFMA); the first pass adds the shift
    // 11 (mn + n(n+1)) u tr(G), the others only clamp non-positive pivots;
    // an item with a clamped pivot (numerically rank deficient: singular values
    // below ~1e-11 of the largest) is refactored by Householder on the device,
    // so Q has orthonormal columns for any rank.  If
    // a.R is set, R = R_3 R_2 R_1 (A = Q R to about u cond(A); meant for
    // well-conditioned A such as random initial guesses).  n > 64: blocks of 64
    // columns, each orthogonalised against the previous ones by three passes of
    // block Gram-Schmidt before its CholeskyQR3.
    void orthonormalise(const tnk::QrArgs &a);
    void ortho_impl(const tnk::QrArgs &a, bool householder_blocks);
    // norm2 per batch item into dev[batch]; normalise in place; logscale +=.
    void norm2(const void *x, int e, int64_t n, int batch, int64_t bs, double *out);
    void normalise(void *x, int e, int64_t n, int batch, int64_t bs, double *logscale, bool acc,
                   int *flags);
    void dot(const void *x, const void *y, int e, int64_t n, int batch, int64_t bs, double *out,
             const int *mask = nullptr, int mask_skip = 0);

    // Raw device memory from the pool (stream-ordered reuse after unraw).
    void *raw(size_t bytes) { return pool_.get(bytes); }
    void unraw(void *p) { pool_.put(p); }
    size_t held() const { return pool_.held(); }

    void sync() { TN_HIP(hipStreamSynchronize(s)); }

    // Event pair around one timed launch; kind 0 = contraction, 1 = QR, 2 = masked.
    struct EvPair { hipEvent_t a, b; int kind; Plan *plan; };
    // Stream capture of a launch sequence into a graph: the launches issued
    // between begin_capture and end_capture are recorded (not run), device
    // memory taken from the pool meanwhile stays with the graph, timing event
    // pairs are recorded as graph nodes (owned by the graph), and the host-side
    // counters they added are returned so that each replay can add them again.
    struct Captured {
        hipGraphExec_t exec = nullptr;
        std::vector<void *> blocks;
        std::deque<EvPair> pairs;
        Counters delta;
    };
    void begin_capture(Captured &g);
    // Ends the capture; false (and nothing kept) if the capture failed.
    bool end_capture(Captured &g, bool ok);
    void launch(const Captured &g);  // one replay (counters and event pairs included)
    void collect_graph_timing(const std::deque<EvPair> &pairs);  // after the replay has finished
    void release(Captured &g);  // synchronises, frees the graph, returns its memory to the pool
    bool capturing() const { return cap_pairs_ != nullptr; }
    // Waits for the stream and adds the elapsed times of the event pairs recorded
    // since the last collection to the counters (timing mode).
    void collect_timing();
    // Text table of the contraction plans by accumulated device time (timing mode).
    std::string plan_report(int top) const;
    // Autotuning: on the first call of a contraction shape, every tile
    // configuration (and split-K choice) is timed on the real operands and the
    // fastest kept.  Choices are read from / appended to `cache_path` if given.
    void set_autotune(bool on, const std::string &cache_path);

  private:
    Pool pool_;
    std::unordered_map<std::string, std::unique_ptr<Plan>> plans_;
    Plan *plan(const Op &A, const Op &B, const Op &C);
    // event pairs recorded around launches in timing mode
    std::deque<EvPair> ev_;
    size_t ev_used_ = 0;
    std::deque<EvPair> *cap_pairs_ = nullptr;  // set while capturing
    hipStream_t cap_stream_ = nullptr, user_stream_ = nullptr;
    Counters cap_ctr0_;
    void add_pair_time(const EvPair &e);
    void destroy_pairs(std::deque<EvPair> &pairs);
    bool in_qr_ = false;  // contractions issued by the QR: flops booked as qr_gemm_flops
    const int *mask_ = nullptr;
    char mask_letter_ = 0;
    int mask_skip_ = 0;
    bool autotune_ = false;
    std::string tune_path_;
    struct TuneChoice { int cfg, ks, pack, fp32; };
    std::map<std::string, TuneChoice> tune_cache_;  // key -> tile configuration, K slices, packing
    std::map<std::string, int64_t> qr_shapes_;               // factorisation calls by shape
    void set_split(Plan *P, int cfg, int ksplit_hint);
    void pack_bf16(tnk::GettArgs &g, void **pa, void **pb);
    void tune(Plan *P, tnk::GettArgs g);
    EvPair *next_pair(int kind);
};

}  // namespace tnb

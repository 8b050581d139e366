#include "engine.hpp"

#include <algorithm>
#include <cstring>
#include <set>
#include <fstream>
#include <sstream>

namespace tnb {

// ---------------------------------------------------------------- operands

Op op(const Ten &t, const std::string &idx, bool conj) {
    if (idx.size() != t.d.size())
        throw TnError(ST_SHAPE, "operand letters '" + idx + "' do not match tensor rank");
    Op o;
    o.p = t.p;
    o.esz = t.esz;
    o.idx = idx;
    o.dims = t.d;
    o.str.assign(t.d.size(), 1);
    for (int i = (int)t.d.size() - 2; i >= 0; --i) o.str[i] = o.str[i + 1] * t.d[i + 1];
    o.conj = conj;
    return o;
}

Op op_bcast(const Ten &t, char letter, int size, const std::string &idx, bool conj) {
    Op o = op(t, idx, conj);
    o.idx = std::string(1, letter) + o.idx;
    o.dims.insert(o.dims.begin(), size);
    o.str.insert(o.str.begin(), 0);
    return o;
}

// ---------------------------------------------------------------- pool

Pool::~Pool() {
    for (auto &kv : size_) (void)hipFree(kv.first);
}

void *Pool::take(std::multimap<size_t, void *> &fl, size_t bytes) {
    auto it = fl.lower_bound(bytes);
    if (it != fl.end() && it->first <= 2 * bytes + (1 << 20)) {
        void *p = it->second;
        fl.erase(it);
        return p;
    }
    return nullptr;
}

void *Pool::get(size_t bytes) {
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~size_t(255);
    if (arena_) {
        if (void *p = take(afree_, bytes)) return p;
        if (void *p = take(free_, bytes)) {
            ablocks_.push_back(p);
            return p;
        }
    } else if (void *p = take(free_, bytes)) {
        return p;
    }
    size_t alloc = bytes;
    if (alloc > (1 << 20)) alloc = (alloc + (1 << 20) - 1) & ~size_t((1 << 20) - 1);
    if (cap_ && held_ + alloc > cap_) {
        if (!arena_) trim();  // (trim synchronises the device: not while capturing)
        if (held_ + alloc > cap_)
            throw TnError(ST_OOM, "workspace cap reached (" + std::to_string(held_ + alloc) + " > " +
                                      std::to_string(cap_) + " bytes)");
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, alloc);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (arena_) throw TnError(ST_OOM, "hipMalloc of " + std::to_string(alloc) + " bytes failed (capture)");
        trim();
        e = hipMalloc(&p, alloc);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw TnError(ST_OOM, "hipMalloc of " + std::to_string(alloc) + " bytes failed");
        }
    }
    held_ += alloc;
    size_[p] = alloc;
    if (arena_) ablocks_.push_back(p);
    return p;
}

void Pool::put(void *p) {
    if (!p) return;
    auto it = size_.find(p);
    if (it == size_.end()) return;
    if (arena_ && std::find(ablocks_.begin(), ablocks_.end(), p) != ablocks_.end()) {
        afree_.emplace(it->second, p);
        return;
    }
    free_.emplace(it->second, p);
}

void Pool::begin_arena() {
    arena_ = true;
    afree_.clear();
    ablocks_.clear();
}

std::vector<void *> Pool::end_arena() {
    arena_ = false;
    afree_.clear();
    std::vector<void *> b;
    b.swap(ablocks_);
    return b;
}

void Pool::release(const std::vector<void *> &blocks) {
    for (void *p : blocks) {
        auto it = size_.find(p);
        if (it != size_.end()) free_.emplace(it->second, p);
    }
}

void Pool::trim() {
    if (free_.empty()) return;
    (void)hipDeviceSynchronize();
    for (auto &kv : free_) {
        held_ -= size_[kv.second];
        size_.erase(kv.second);
        (void)hipFree(kv.second);
    }
    free_.clear();
}

// ---------------------------------------------------------------- engine

Engine::Engine(int dev, hipStream_t st, size_t cap) : s(st), device(dev), pool_(cap) {}

Engine::~Engine() {
    (void)hipStreamSynchronize(s);
    if (cap_stream_) (void)hipStreamDestroy(cap_stream_);
    for (auto &kv : plans_)
        if (kv.second->dev) (void)hipFree(kv.second->dev);
    for (auto &e : ev_) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
}

// A fresh event pair (deque storage: nested calls that add pairs keep references valid).
Engine::EvPair *Engine::next_pair(int kind) {
    if (cap_pairs_) {  // stream capture: the pair belongs to the graph being captured
        EvPair e{};
        TN_HIP(hipEventCreate(&e.a));
        TN_HIP(hipEventCreate(&e.b));
        e.kind = kind;
        e.plan = nullptr;
        cap_pairs_->push_back(e);
        return &cap_pairs_->back();
    }
    if (ev_used_ == ev_.size()) {
        EvPair e{};
        TN_HIP(hipEventCreate(&e.a));
        TN_HIP(hipEventCreate(&e.b));
        ev_.push_back(e);
    }
    EvPair &e = ev_[ev_used_];
    e.kind = kind;
    e.plan = nullptr;
    ++ev_used_;
    return &e;
}

void Engine::add_pair_time(const EvPair &e) {
    float ms = 0.f;
    TN_HIP(hipEventElapsedTime(&ms, e.a, e.b));
    if (e.kind == 0) ctr.gemm_ms += ms;
    else if (e.kind == 2) ctr.masked_ms += ms;
    else ctr.qr_ms += ms;
    if (e.plan && e.kind != 2) {
        e.plan->ms += ms;
        e.plan->calls += 1;
    }
}

void Engine::collect_timing() {
    if (ev_used_ == 0) return;
    sync();
    for (size_t i = 0; i < ev_used_; ++i) add_pair_time(ev_[i]);
    ev_used_ = 0;
}

namespace {
Counters count_delta(const Counters &a, const Counters &b) {  // a - b, counts only (no times)
    Counters d;
    d.gemm_flops = a.gemm_flops - b.gemm_flops;
    d.gemm_launches = a.gemm_launches - b.gemm_launches;
    d.qr_launches = a.qr_launches - b.qr_launches;
    d.qr_gemm_flops = a.qr_gemm_flops - b.qr_gemm_flops;
    d.masked_launches = a.masked_launches - b.masked_launches;
    d.gemm_bytes = a.gemm_bytes - b.gemm_bytes;
    return d;
}
}  // namespace

void Engine::begin_capture(Captured &g) {
    if (cap_pairs_) throw TnError(ST_INVALID, "nested stream capture");
    g = Captured();
    // the null stream cannot be captured: record on a private stream (nothing
    // runs during the capture) and launch the graph on the handle's stream
    if (!cap_stream_) TN_HIP(hipStreamCreateWithFlags(&cap_stream_, hipStreamNonBlocking));
    user_stream_ = s;
    const hipError_t e = hipStreamBeginCapture(cap_stream_, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw TnError(ST_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
    }
    s = cap_stream_;
    pool_.begin_arena();
    cap_ctr0_ = ctr;
    cap_pairs_ = &g.pairs;
}

bool Engine::end_capture(Captured &g, bool ok) {
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(cap_stream_, &graph);
    s = user_stream_;
    cap_pairs_ = nullptr;
    std::vector<void *> blocks = pool_.end_arena();
    const Counters d = count_delta(ctr, cap_ctr0_);
    ctr = cap_ctr0_;  // nothing ran yet: each launch adds the delta
    if (ok && e == hipSuccess && graph) {
        e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        graph = nullptr;
        if (e == hipSuccess) {
            g.blocks = std::move(blocks);
            g.delta = d;
            return true;
        }
    }
    (void)hipGetLastError();
    if (graph) (void)hipGraphDestroy(graph);
    g.exec = nullptr;
    destroy_pairs(g.pairs);
    pool_.release(blocks);
    return false;
}

void Engine::launch(const Captured &g) {
    TN_HIP(hipGraphLaunch(g.exec, s));
    ctr.graph_launches += 1;
    ctr.gemm_flops += g.delta.gemm_flops;
    ctr.gemm_launches += g.delta.gemm_launches;
    ctr.qr_launches += g.delta.qr_launches;
    ctr.qr_gemm_flops += g.delta.qr_gemm_flops;
    ctr.masked_launches += g.delta.masked_launches;
    ctr.gemm_bytes += g.delta.gemm_bytes;
}

void Engine::release(Captured &g) {
    (void)hipStreamSynchronize(s);
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
    destroy_pairs(g.pairs);
    pool_.release(g.blocks);
    g.blocks.clear();
}

void Engine::collect_graph_timing(const std::deque<EvPair> &pairs) {
    for (const EvPair &e : pairs) add_pair_time(e);
}

void Engine::destroy_pairs(std::deque<EvPair> &pairs) {
    for (EvPair &e : pairs) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    pairs.clear();
}

std::string Engine::plan_report(int top) const {
    std::vector<const Plan *> v;
    for (auto &kv : plans_) v.push_back(kv.second.get());
    std::sort(v.begin(), v.end(), [](const Plan *a, const Plan *b) { return a->ms > b->ms; });
    std::ostringstream os;
    os << "ms\tcalls\tTFLOP/s\tplan\n";
    for (int i = 0; i < (int)v.size() && i < top; ++i) {
        const Plan *p = v[i];
        if (p->calls == 0) continue;
        const double tf = p->ms > 0 ? p->flops * p->calls / (p->ms * 1e-3) / 1e12 : 0.0;
        os << p->ms << '\t' << p->calls << '\t' << tf << '\t' << p->desc << (p->pack ? " packed" : "")
           << (p->fp32 ? " fp32" : "") << " cfg=" << p->cfg
           << " split=" << p->base.ksplit << (p->tuned ? " tuned" : "") << '\n';
    }
    os << "calls\tfactorisation\n";
    std::vector<std::pair<int64_t, std::string>> q;
    for (auto &kv : qr_shapes_) q.push_back({kv.second, kv.first});
    std::sort(q.rbegin(), q.rend());
    for (int i = 0; i < (int)q.size() && i < top; ++i) os << q[i].first << '\t' << q[i].second << '\n';
    return os.str();
}

Ten Engine::make(const std::vector<int> &dims, int e) {
    Ten t;
    t.d = dims;
    t.esz = e ? e : esz;
    t.p = pool_.get(t.bytes());
    return t;
}

void Engine::drop(Ten &t) {
    pool_.put(t.p);
    t.p = nullptr;
}

static Op squeeze(const Op &o) {
    Op r = o;
    r.idx.clear();
    r.dims.clear();
    r.str.clear();
    for (size_t i = 0; i < o.idx.size(); ++i) {
        if (o.dims[i] == 1) continue;
        r.idx.push_back(o.idx[i]);
        r.dims.push_back(o.dims[i]);
        r.str.push_back(o.str[i]);
    }
    return r;
}

// Rows of o as a matrix against the other input x: the product of the letters
// x does not carry (batch letters, shared by all three operands, are excluded).
static int64_t op_rows(const Op &o, const Op &x) {
    int64_t rows = 1;
    for (size_t i = 0; i < o.idx.size(); ++i)
        if (x.idx.find(o.idx[i]) == std::string::npos) rows *= o.dims[i];
    return rows;
}

// Split-BF16 packs both operands into bf16 part planes once when each is
// re-read by several output tiles (both matrix sides above 128); otherwise the
// kernel splits the gathered elements while staging, which reads each operand
// once instead of three times.
static bool pack_pays(const Op &A, const Op &B) {
    return op_rows(A, B) > 128 && op_rows(B, A) > 128;
}

Plan *Engine::plan(const Op &A0, const Op &B0, const Op &C0) {
    const Op A = squeeze(A0), B = squeeze(B0), C = squeeze(C0);
    std::ostringstream ks;
    auto addk = [&](const Op &o) {
        ks << o.idx << ':';
        for (size_t i = 0; i < o.idx.size(); ++i) ks << o.dims[i] << '/' << o.str[i] << ',';
        ks << '|';
    };
    addk(A); addk(B); addk(C);
    const std::string key = std::to_string(prec) + '#' + ks.str();  // plans are per precision
    auto it = plans_.find(key);
    if (it != plans_.end()) return it->second.get();

    std::map<char, int> dim;
    auto note = [&](const Op &o) {
        for (size_t i = 0; i < o.idx.size(); ++i) {
            auto f = dim.find(o.idx[i]);
            if (f != dim.end() && f->second != o.dims[i])
                throw TnError(ST_SHAPE, std::string("dimension mismatch on letter ") + o.idx[i] + " in " + key);
            dim[o.idx[i]] = o.dims[i];
        }
    };
    note(A); note(B); note(C);
    auto has = [](const Op &o, char c) { return o.idx.find(c) != std::string::npos; };
    auto stride = [](const Op &o, char c) -> int64_t {
        const size_t i = o.idx.find(c);
        return i == std::string::npos ? 0 : o.str[i];
    };
    std::string bl, ml, nl, kl;
    for (char c : C.idx) {
        const bool a = has(A, c), b = has(B, c);
        if (a && b) bl.push_back(c);
        else if (a) ml.push_back(c);
        else if (b) nl.push_back(c);
        else throw TnError(ST_SHAPE, std::string("output letter ") + c + " not in inputs: " + key);
    }
    for (char c : A.idx) {
        if (has(C, c)) continue;
        if (!has(B, c)) throw TnError(ST_SHAPE, std::string("letter ") + c + " summed on one operand only: " + key);
        kl.push_back(c);
    }
    for (char c : B.idx)
        if (!has(C, c) && !has(A, c))
            throw TnError(ST_SHAPE, std::string("letter ") + c + " summed on one operand only: " + key);
    // order K letters to follow whichever operand is contiguous along K
    if (!kl.empty()) {
        const char lastA = A.idx.empty() ? 0 : A.idx.back();
        const char lastB = B.idx.empty() ? 0 : B.idx.back();
        std::string order;
        if (lastB && kl.find(lastB) != std::string::npos && stride(B, lastB) == 1 &&
            !(lastA && kl.find(lastA) != std::string::npos && stride(A, lastA) == 1)) {
            for (char c : B.idx) if (kl.find(c) != std::string::npos) order.push_back(c);
        } else {
            for (char c : A.idx) if (kl.find(c) != std::string::npos) order.push_back(c);
        }
        kl = order;
    }
    auto total = [&](const std::string &l) {
        int64_t t = 1;
        for (char c : l) t *= dim[c];
        return t;
    };
    const int64_t M = total(ml), N = total(nl), K = total(kl), Z = total(bl);
    if (M > INT32_MAX || N > INT32_MAX || K > INT32_MAX || Z > INT32_MAX)
        throw TnError(ST_UNSUPPORTED, "contraction extent too large: " + key);
    // offset tables
    auto table = [&](const std::string &l, const Op &o, std::vector<int64_t> &out) {
        const int64_t n = total(l);
        out.assign((size_t)n, 0);
        std::vector<int> idx(l.size(), 0);
        std::vector<int64_t> st(l.size());
        for (size_t i = 0; i < l.size(); ++i) st[i] = stride(o, l[i]);
        int64_t off = 0;
        for (int64_t e = 0; e < n; ++e) {
            out[(size_t)e] = off;
            for (int i = (int)l.size() - 1; i >= 0; --i) {
                idx[i]++;
                off += st[i];
                if (idx[i] < dim[l[i]]) break;
                off -= st[i] * idx[i];
                idx[i] = 0;
            }
        }
    };
    std::vector<int64_t> am, ak, bk, bn, cm, cn, ab, bb, cb;
    table(ml, A, am); table(kl, A, ak); table(bl, A, ab);
    table(kl, B, bk); table(nl, B, bn); table(bl, B, bb);
    table(ml, C, cm); table(nl, C, cn); table(bl, C, cb);
    auto fits = [](const std::vector<int64_t> &v) {
        for (int64_t x : v)
            if (x < 0 || x > INT32_MAX) return false;
        return true;
    };
    if (!fits(am) || !fits(ak) || !fits(bk) || !fits(bn) || !fits(cm) || !fits(cn))
        throw TnError(ST_UNSUPPORTED, "tensor offsets exceed 2^31 elements: " + key);

    auto P = std::make_unique<Plan>();
    // kernel N dimension should be C's contiguous letter for coalesced stores
    const char cfast = C.idx.empty() ? 0 : C.idx.back();
    const bool swap = cfast && ml.find(cfast) != std::string::npos;
    P->swapped = swap;
    const std::vector<int64_t> &kam = swap ? bn : am, &kak = swap ? bk : ak, &kbk = swap ? ak : bk,
                               &kbn = swap ? am : bn, &kcm = swap ? cn : cm, &kcn = swap ? cm : cn,
                               &kab = swap ? bb : ab, &kbb = swap ? ab : bb;
    const Op &opA = swap ? B : A;
    const Op &opB = swap ? A : B;
    const std::string &kml = swap ? nl : ml, &knl = swap ? ml : nl;
    const int64_t kM = swap ? N : M, kN = swap ? M : N;
    // upload: int32 tables then int64 batch tables
    const size_t n32 = kam.size() + kak.size() + kbk.size() + kbn.size() + kcm.size() + kcn.size();
    const size_t bytes = n32 * 4 + 3 * (size_t)Z * 8 + 64;
    std::vector<char> host(bytes, 0);
    size_t off = 0;
    int32_t *t32[6];
    const std::vector<int64_t> *src32[6] = {&kam, &kak, &kbk, &kbn, &kcm, &kcn};
    for (int i = 0; i < 6; ++i) {
        t32[i] = reinterpret_cast<int32_t *>(host.data() + off);
        for (size_t j = 0; j < src32[i]->size(); ++j) t32[i][j] = (int32_t)(*src32[i])[j];
        off += src32[i]->size() * 4;
    }
    off = (off + 7) & ~size_t(7);
    const size_t off64 = off;
    const std::vector<int64_t> *src64[3] = {&kab, &kbb, &cb};
    for (int i = 0; i < 3; ++i) {
        std::memcpy(host.data() + off, src64[i]->data(), src64[i]->size() * 8);
        off += src64[i]->size() * 8;
    }
    if (hipMalloc(&P->dev, bytes) != hipSuccess) {
        // the pool's cached blocks may hold the memory: return them and retry
        (void)hipGetLastError();
        if (!capturing()) pool_.trim();
        TN_HIP(hipMalloc(&P->dev, bytes));
    }
    TN_HIP(hipMemcpy(P->dev, host.data(), bytes, hipMemcpyHostToDevice));
    char *d = reinterpret_cast<char *>(P->dev);
    size_t o2 = 0;
    const int32_t *dt[6];
    for (int i = 0; i < 6; ++i) {
        dt[i] = reinterpret_cast<const int32_t *>(d + o2);
        o2 += src32[i]->size() * 4;
    }
    const int64_t *db[3];
    o2 = off64;
    for (int i = 0; i < 3; ++i) {
        db[i] = reinterpret_cast<const int64_t *>(d + o2);
        o2 += src64[i]->size() * 8;
    }
    tnk::GettArgs &g = P->base;
    std::memset(&g, 0, sizeof(g));
    g.M = (int)kM; g.N = (int)kN; g.K = (int)K; g.batch = (int)Z;
    g.a_moff = dt[0]; g.a_koff = dt[1]; g.b_koff = dt[2]; g.b_noff = dt[3]; g.c_moff = dt[4]; g.c_noff = dt[5];
    g.a_boff = db[0]; g.b_boff = db[1]; g.c_boff = db[2];
    // load direction: along k when the operand's fastest letter is a K letter with stride 1
    const char la = opA.idx.empty() ? 0 : opA.idx.back();
    const char lb = opB.idx.empty() ? 0 : opB.idx.back();
    g.a_kfast = (la && kl.find(la) != std::string::npos && stride(opA, la) == 1) ? 1 : 0;
    g.b_kfast = (lb && kl.find(lb) != std::string::npos && stride(opB, lb) == 1) ? 1 : 0;
    // affine k tables need no table reads in the kernel
    auto affine = [](const std::vector<int64_t> &t, int *ks) {
        const int64_t s1 = t.size() > 1 ? t[1] : 0;
        for (size_t k = 0; k < t.size(); ++k)
            if (t[k] != (int64_t)k * s1) return false;
        *ks = (int)s1;
        return true;
    };
    g.a_ks = g.b_ks = 0;
    g.a_kaff = affine(kak, &g.a_ks) ? 1 : 0;
    g.b_kaff = affine(kbk, &g.b_ks) ? 1 : 0;
    // operand windows (bytes) reachable from a batch item's base
    auto window = [&](const std::vector<int64_t> &r, const std::vector<int64_t> &k) {
        int64_t mr = 0, mk = 0;
        for (int64_t x : r) mr = std::max(mr, x);
        for (int64_t x : k) mk = std::max(mk, x);
        return (mr + mk + 1) * (int64_t)esz;
    };
    const int64_t wa = window(kam, kak), wb = window(kbn, kbk);
    if (wa > (int64_t)tnk::GETT_MAX_WINDOW || wb > (int64_t)tnk::GETT_MAX_WINDOW)
        throw TnError(ST_UNSUPPORTED, "contraction operand spans more than 2 GiB per batch item: " + key);
    g.a_bytes = (uint32_t)wa;
    g.b_bytes = (uint32_t)wb;
    (void)kml; (void)knl;
    P->kM = kM; P->kN = kN; P->K = K; P->Z = Z;
    P->can_pack = (prec == tnk::P_BF16X3 || prec == tnk::P_BF16X6) && pack_pays(A, B);
    P->pack = P->can_pack;
    P->bl = bl;
    P->kml = swap ? nl : ml;
    P->knl = swap ? ml : nl;
    P->ldim = dim;
    P->key = key;
    P->flops = 8.0 * (double)M * (double)N * (double)K * (double)Z;
    {
        std::ostringstream d;
        d << A.idx << ',' << B.idx << "->" << C.idx << " M=" << M << " N=" << N << " K=" << K << " batch=" << Z
          << (swap ? " swapped" : "");
        P->desc = d.str();
    }
    auto tc = tune_cache_.find(P->key);
    if (tc != tune_cache_.end()) {
        P->pack = P->can_pack && tc->second.pack;
        P->fp32 = (prec == tnk::P_BF16X3 || prec == tnk::P_BF16X6) && tc->second.fp32 && !P->pack;
        set_split(P.get(), tc->second.cfg, tc->second.ks);
        P->tuned = true;
    } else {
        int cfg;
        if (kN <= 16) cfg = tnk::CFG_64x16;
        else if (kM >= 8192 && kN >= 128 && K >= 16) cfg = tnk::CFG_128x64;
        else cfg = tnk::CFG_64x64;
        set_split(P.get(), cfg, 0);
    }
    Plan *raw = P.get();
    plans_[key] = std::move(P);
    return raw;
}

// ksplit_hint: 0 = heuristic (split K when the output tiles alone cannot fill
// the chip and K is long), otherwise the number of K slices wanted.
void Engine::set_split(Plan *P, int cfg, int ksplit_hint) {
    tnk::GettArgs &g = P->base;
    P->cfg = cfg;
    const int64_t K = P->K;
    int64_t ks = 1;
    if (ksplit_hint > 0) {
        ks = std::min<int64_t>(ksplit_hint, std::max<int64_t>(K / 32, 1));
    } else {
        int bm = 64, bn = 64;
        tnk::gett_tile(cfg, prec, &bm, &bn);
        const int64_t tiles = ((P->kM + bm - 1) / bm) * ((P->kN + bn - 1) / bn) * P->Z;
        if (tiles < 512 && K >= 256) ks = std::min<int64_t>((1024 + tiles - 1) / tiles, K / 128);
    }
    // a k table staged in LDS bounds the K slice of a block (the packed
    // split-BF16 kernel reads no tables)
    if (!P->pack && (!g.a_kaff || !g.b_kaff)) ks = std::max<int64_t>(ks, (K + tnk::GETT_KTAB - 1) / tnk::GETT_KTAB);
    g.ksplit = 1;
    g.kchunk = (int)K;
    if (ks > 1) {
        int64_t chunk = (K + ks - 1) / ks;
        chunk = (chunk + 31) / 32 * 32;
        g.kchunk = (int)chunk;
        g.ksplit = (int)((K + chunk - 1) / chunk);
    }
}

void Engine::set_autotune(bool on, const std::string &cache_path) {
    autotune_ = on;
    tune_path_ = cache_path;
    if (!on || cache_path.empty()) return;
    std::ifstream f(cache_path);
    std::string k;
    int cfg, ks, pk, f32;
    while (f >> k >> cfg >> ks >> pk >> f32)
        if (cfg >= 0 && cfg < tnk::CFG_COUNT && ks >= 1) tune_cache_[k] = {cfg, ks, pk ? 1 : 0, f32 ? 1 : 0};
}

// Times every candidate (tile configuration x split-K choice) on the call's own
// operands; only for calls that overwrite C, so repeated launches leave the
// same result.  The last launch of the caller then runs with the winner.
void Engine::tune(Plan *P, tnk::GettArgs g) {
    // candidates: tile configuration x K slices, and for split-BF16 shapes that
    // may pack, packed or split while staging (the packing is timed with it)
    // In the split-BF16 modes the FP32 kernel (same complex64 storage, at least
    // as accurate) is a candidate too: it can win on shapes whose short K or
    // narrow N leave the split products little to amortise.
    struct Cand { int cfg, ks; bool pack, fp32; };
    std::vector<Cand> cands;
    const bool bf16 = prec == tnk::P_BF16X3 || prec == tnk::P_BF16X6;
    const int cfgs[5] = {tnk::CFG_64x16, tnk::CFG_64x64, tnk::CFG_128x64, tnk::CFG_128x64W, tnk::CFG_128x128W};
    for (int pk = 0; pk < 3; ++pk) {
        const bool pack = pk == 1, f32 = pk == 2;
        if (pack && !P->can_pack) continue;
        if (f32 && !bf16) continue;
        for (int c : cfgs) {
            if ((c == tnk::CFG_128x64 || c == tnk::CFG_128x64W || c == tnk::CFG_128x128W) && P->kM < 128) continue;
            if (c == tnk::CFG_128x128W && (!pack || P->kN < 128)) continue;  // packed split-BF16 only
            if (c == tnk::CFG_64x16 && P->kN > 64) continue;
            int bm = 64, bn = 64;
            tnk::gett_tile(c, prec, &bm, &bn);
            const int64_t tiles = ((P->kM + bm - 1) / bm) * ((P->kN + bn - 1) / bn) * P->Z;
            cands.push_back({c, 1, pack, f32});
            // K slices only pay when the output tiles leave CUs idle
            if (tiles >= 1024) continue;
            for (int64_t ks = 2; ks <= 16; ks *= 2) {
                if (P->K < 64 * ks) break;
                if (tiles * ks > 4096) break;
                cands.push_back({c, (int)ks, pack, f32});
            }
        }
    }
    hipEvent_t e0, e1;
    TN_HIP(hipEventCreate(&e0));
    TN_HIP(hipEventCreate(&e1));
    const tnk::GettArgs saved = P->base;
    const bool saved_pack = P->pack, saved_fp32 = P->fp32;
    const Cand start{P->cfg, std::max(P->base.ksplit, 1), P->pack, P->fp32};
    auto run = [&](const Cand &c, int reps) {
        P->pack = c.pack;
        P->fp32 = c.fp32;
        set_split(P, c.cfg, c.ks);
        tnk::GettArgs t = g;
        t.ksplit = P->base.ksplit;
        t.kchunk = P->base.kchunk;
        void *part = t.ksplit > 1 ? pool_.get((size_t)t.ksplit * t.batch * (size_t)t.M * t.N * esz) : nullptr;
        t.part = part;
        TN_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < reps; ++r) {
            tnk::GettArgs u = t;
            void *pa = nullptr, *pb = nullptr;
            if (c.pack) pack_bf16(u, &pa, &pb);
            TN_HIP(tnk::launch_gett(u, c.fp32 ? (int)tnk::P_FP32 : prec, c.cfg, s));
            if (pa) pool_.put(pa);
            if (pb) pool_.put(pb);
        }
        TN_HIP(hipEventRecord(e1, s));
        TN_HIP(hipEventSynchronize(e1));
        float ms = 0;
        TN_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (part) pool_.put(part);
        return ms / reps;
    };
    Cand win = start;
    try {
        // the planner's choice first (also warms the caches); short launches are
        // timed over three repetitions, long ones once
        float best = run(start, 1);
        const int reps = best < 0.05f ? 3 : 1;
        if (reps > 1) best = run(start, reps);
        for (const Cand &c : cands) {
            if (c.cfg == start.cfg && c.ks == start.ks && c.pack == start.pack && c.fp32 == start.fp32) continue;
            const float ms = run(c, reps);
            if (ms < best) { best = ms; win = c; }
        }
    } catch (...) {
        P->base = saved;
        P->pack = saved_pack;
        P->fp32 = saved_fp32;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    P->base = saved;
    P->pack = win.pack;
    P->fp32 = win.fp32;
    set_split(P, win.cfg, win.ks);
    P->tuned = true;
    tune_cache_[P->key] = {win.cfg, win.ks, win.pack ? 1 : 0, win.fp32 ? 1 : 0};
    if (!tune_path_.empty()) {
        std::ofstream f(tune_path_, std::ios::app);
        f << P->key << ' ' << win.cfg << ' ' << win.ks << ' ' << (win.pack ? 1 : 0) << ' ' << (win.fp32 ? 1 : 0)
          << '\n';
    }
}

// Bytes an operand spans per batch item (letters shared by all three operands
// index the batch and are applied through the batch base).
static int64_t op_window(const Op &o, const Op &x, const Op &y) {
    int64_t w = 0;
    for (size_t i = 0; i < o.idx.size(); ++i) {
        const char c = o.idx[i];
        if (x.idx.find(c) != std::string::npos && y.idx.find(c) != std::string::npos) continue;
        w += (int64_t)(o.dims[i] - 1) * o.str[i];
    }
    return (w + 1) * (int64_t)o.esz;
}

// Elements of the dense rows x kpad matrix a packed operand becomes (kpad = K
// rounded up to 32; letters shared by all three operands index the batch).
// x is the other input, y the output.
static int64_t op_dense(const Op &o, const Op &x, const Op &y) {
    int64_t rows = 1, k = 1;
    for (size_t i = 0; i < o.idx.size(); ++i) {
        const char c = o.idx[i];
        const bool in_x = x.idx.find(c) != std::string::npos, in_y = y.idx.find(c) != std::string::npos;
        if (in_x && in_y) continue;
        if (in_x) k *= o.dims[i];
        else rows *= o.dims[i];
    }
    return rows * ((k + 31) / 32 * 32);
}

// Restricts letter c of o (if present) to [i0, i0 + n).
static Op slice(const Op &o, char c, int i0, int n) {
    Op r = o;
    const size_t i = o.idx.find(c);
    if (i == std::string::npos) return r;
    r.p = static_cast<const char *>(o.p) + (int64_t)i0 * o.str[i] * o.esz;
    r.dims[i] = n;
    return r;
}

// Split-BF16: packs A and B into bf16 part planes (see tnk::launch_pack_bf16)
// and points g at them.  The buffers come from the pool; the caller returns them.
void Engine::pack_bf16(tnk::GettArgs &g, void **pa, void **pb) {
    const int np = prec == tnk::P_BF16X3 ? 2 : 3;
    const int kpad = (std::max(g.K, 1) + 31) / 32 * 32;
    const int64_t ba = (int64_t)np * 4 * g.M * kpad, bb = (int64_t)np * 4 * g.N * kpad;
    if (ba > (int64_t)tnk::GETT_MAX_WINDOW || bb > (int64_t)tnk::GETT_MAX_WINDOW)
        throw TnError(ST_UNSUPPORTED, "packed split-BF16 operand above 2 GiB per batch item");
    *pa = pool_.get((size_t)ba * g.batch);
    *pb = pool_.get((size_t)bb * g.batch);
    TN_HIP(tnk::launch_pack_bf16(np, g.A, g.a_boff, g.a_moff, g.a_koff, g.a_kaff, g.a_ks, g.M, g.K, kpad, g.batch,
                                 g.conjA, *pa, s));
    TN_HIP(tnk::launch_pack_bf16(np, g.B, g.b_boff, g.b_noff, g.b_koff, g.b_kaff, g.b_ks, g.N, g.K, kpad, g.batch,
                                 g.conjB, *pb, s));
    g.A = *pa;
    g.B = *pb;
    g.kpad = kpad;
    g.a_bytes = (uint32_t)ba;
    g.b_bytes = (uint32_t)bb;
    g.conjA = g.conjB = 0;
    g.a_kaff = g.b_kaff = 1;  // no tables in the packed kernel
}

void Engine::contract(const Op &A, const Op &B, const Op &C, bool accumulate) {
    if (A.esz != esz || B.esz != esz || C.esz != esz)
        throw TnError(ST_INVALID, "operand element size does not match the compute precision");
    // The kernel addresses A and B through buffer resources of < 2 GiB per
    // batch item; a larger operand is cut along its widest-stride letter into
    // slices that fit (a summed letter accumulates over its slices).
    const bool bf16 = prec == tnk::P_BF16X3 || prec == tnk::P_BF16X6;
    const int64_t lim = (int64_t)tnk::GETT_MAX_WINDOW;
    // The output's row and column offsets are int32 tables: an output spanning
    // 2^31 elements or more (outside its batch letters) is cut along its
    // widest-stride letter into equal slices that fit.
    {
        const int64_t winc = op_window(C, A, B) / C.esz;  // elements reachable through the tables
        if (winc > (int64_t)INT32_MAX) {
            int best = -1;
            int64_t span = 0;
            for (size_t i = 0; i < C.idx.size(); ++i) {
                const char c = C.idx[i];
                if (C.dims[i] < 2) continue;
                if (A.idx.find(c) != std::string::npos && B.idx.find(c) != std::string::npos) continue;
                const int64_t sp = (int64_t)(C.dims[i] - 1) * C.str[i];
                if (sp > span) { span = sp; best = (int)i; }
            }
            if (best < 0) throw TnError(ST_UNSUPPORTED, "contraction output cannot be cut below 2^31 elements");
            const char c = C.idx[best];
            const int dim = C.dims[best];
            const int64_t rest = winc - (int64_t)(dim - 1) * C.str[best];
            int chunk = (int)std::max<int64_t>(1, std::min<int64_t>(dim / 2, ((int64_t)INT32_MAX - rest) / C.str[best] + 1));
            const int nsl = (dim + chunk - 1) / chunk;
            chunk = (dim + nsl - 1) / nsl;
            const int *mask = mask_;
            for (int i0 = 0; i0 < dim; i0 += chunk) {
                const int n = std::min(chunk, dim - i0);
                if (mask && c == mask_letter_) mask_ = mask + i0;
                contract(slice(A, c, i0, n), slice(B, c, i0, n), slice(C, c, i0, n), accumulate);
                mask_ = mask;
            }
            return;
        }
    }
    const int64_t wina = op_window(A, B, C), winb = op_window(B, A, C);
    int64_t wa = wina, wb = winb;
    if (bf16 && pack_pays(A, B)) {
        // packed split-BF16 reads packed operands: dense rows x K planes, 4 * parts bytes
        // per complex element (the window of a strided or broadcast operand can
        // be smaller than that)
        const int64_t per = prec == tnk::P_BF16X3 ? 8 : 12;
        wa = std::max(wa, op_dense(A, B, C) * per);
        wb = std::max(wb, op_dense(B, A, C) * per);
    }
    if (wa > lim || wb > lim) {
        const Op &X = wa > lim ? A : B;
        const Op &Y = wa > lim ? B : A;
        const int64_t w = wa > lim ? wa : wb;
        const int64_t win = wa > lim ? wina : winb;
        // widest-stride letter
        int best = -1;
        int64_t span = 0;
        for (size_t i = 0; i < X.idx.size(); ++i) {
            const char c = X.idx[i];
            if (X.dims[i] < 2) continue;
            if (Y.idx.find(c) != std::string::npos && C.idx.find(c) != std::string::npos) continue;
            const int64_t sp = (int64_t)(X.dims[i] - 1) * X.str[i];
            if (sp > span) { span = sp; best = (int)i; }
        }
        if (best < 0) throw TnError(ST_UNSUPPORTED, "contraction operand cannot be cut below 2 GiB");
        const char c = X.idx[best];
        const int dim = X.dims[best];
        int chunk;
        if (win >= w) {  // the strided window is the binding limit
            const int64_t step = X.str[best] * (int64_t)X.esz;
            const int64_t rest = w - (int64_t)(dim - 1) * step;
            chunk = (int)std::max<int64_t>(1, std::min<int64_t>(dim / 2, (lim - rest) / step + 1));
        } else {         // the packed size is: it shrinks in proportion to the letter
            chunk = (int)std::max<int64_t>(1, std::min<int64_t>(dim / 2, dim * lim / w));
        }
        {   // equal slices (a short last slice wastes a launch on a thin GEMM)
            const int nsl = (dim + chunk - 1) / chunk;
            chunk = (dim + nsl - 1) / nsl;
        }
        const bool summed = C.idx.find(c) == std::string::npos;
        const int *mask = mask_;
        for (int i0 = 0; i0 < dim; i0 += chunk) {
            const int n = std::min(chunk, dim - i0);
            if (mask && c == mask_letter_) mask_ = mask + i0;
            contract(slice(A, c, i0, n), slice(B, c, i0, n), slice(C, c, i0, n),
                     summed ? (accumulate || i0 > 0) : accumulate);
            mask_ = mask;
        }
        return;
    }
    Plan *P = plan(A, B, C);
    tnk::GettArgs g = P->base;
    g.A = P->swapped ? B.p : A.p;
    g.B = P->swapped ? A.p : B.p;
    g.C = const_cast<void *>(C.p);
    g.conjA = (P->swapped ? B.conj : A.conj) ? 1 : 0;
    g.conjB = (P->swapped ? A.conj : B.conj) ? 1 : 0;
    g.accumulate = accumulate ? 1 : 0;
    int cfg = P->cfg;
    if (force_cfg == tnk::CFG_128x128W && !P->pack)
        throw TnError(ST_UNSUPPORTED, "the 128x128 tile serves packed split-BF16 operands only");
    if (force_cfg >= 0) {
        Plan tmp = *P;  // shares the tables, owns nothing
        set_split(&tmp, force_cfg, force_ksplit);
        tmp.dev = nullptr;
        g.ksplit = tmp.base.ksplit;
        g.kchunk = tmp.base.kchunk;
        cfg = force_cfg;
    } else if (autotune_ && !P->tuned && !accumulate) {
        tune(P, g);
        g.ksplit = P->base.ksplit;
        g.kchunk = P->base.kchunk;
        cfg = P->cfg;
    }
    bool masked = false;
    if (mask_) {
        auto div = [&](const std::string &l) {
            int64_t d = 1;
            for (size_t i = 1; i < l.size(); ++i) d *= P->ldim.at(l[i]);
            return d;
        };
        int mode = 0;
        int64_t d = 0;
        if (!P->bl.empty() && P->bl[0] == mask_letter_) { mode = 1; d = div(P->bl); }
        else if (!P->kml.empty() && P->kml[0] == mask_letter_) { mode = 2; d = div(P->kml); }
        else if (!P->knl.empty() && P->knl[0] == mask_letter_) { mode = 3; d = div(P->knl); }
        if (mode && d <= INT32_MAX) {
            g.mask = mask_;
            g.mask_mode = mode;
            g.mask_div = (int)d;
            g.mask_skip = mask_skip_;
            masked = true;
        }
    }
    void *part = nullptr;
    if (g.ksplit > 1) {
        part = pool_.get((size_t)g.ksplit * g.batch * (size_t)g.M * g.N * esz);
        g.part = part;
    }
    // contractions inside the orthonormalisation are timed too (their QR-level
    // pair also covers them); their flops are booked separately.  The pair
    // covers the split-BF16 packing of the operands.
    EvPair *ev = timing ? next_pair(masked ? 2 : 0) : nullptr;
    if (ev) {
        ev->plan = P;
        TN_HIP(hipEventRecord(ev->a, s));
    }
    void *pka = nullptr, *pkb = nullptr;
    if (P->pack) pack_bf16(g, &pka, &pkb);
    TN_HIP(tnk::launch_gett(g, P->fp32 ? (int)tnk::P_FP32 : prec, cfg, s));
    if (ev) TN_HIP(hipEventRecord(ev->b, s));
    if (part) pool_.put(part);
    if (pka) pool_.put(pka);
    if (pkb) pool_.put(pkb);
    if (masked) {
        ctr.masked_launches += 1;
        return;
    }
    if (in_qr_) ctr.qr_gemm_flops += P->flops;
    ctr.gemm_flops += P->flops;
    ctr.gemm_launches += 1;
    ctr.gemm_bytes += (double)P->Z * ((double)P->kM * P->K + (double)P->K * P->kN +
                                      (double)P->kM * P->kN * (accumulate ? 2.0 : 1.0)) * esz;
}

Ten Engine::contract_new(const Op &A, const Op &B, const std::string &ic) {
    std::vector<int> dims;
    for (char c : ic) {
        size_t i = A.idx.find(c);
        if (i != std::string::npos) { dims.push_back(A.dims[i]); continue; }
        i = B.idx.find(c);
        if (i != std::string::npos) { dims.push_back(B.dims[i]); continue; }
        throw TnError(ST_SHAPE, std::string("output letter ") + c + " not found");
    }
    Ten C = make(dims);
    contract(A, B, op(C, ic));
    return C;
}

void Engine::qr(const tnk::QrArgs &a) {
    if (a.n > 64 && a.m >= a.n && (int64_t)a.m * a.n > 8192) {
        // one workgroup per matrix would factor it alone: blocks of 64 columns,
        // block Gram-Schmidt between them and Householder TSQR within
        ortho_impl(a, true);
        return;
    }
    const size_t ws = tnk::qr_workspace_bytes(a.m, a.n, a.batch);
    void *w = pool_.get(ws);
    {
        std::ostringstream k;
        k << "householder m=" << a.m << " n=" << a.n << " batch=" << a.batch << (a.R ? " R" : "");
        qr_shapes_[k.str()] += 1;
    }
    // inside a wider factorisation the outer call's pair covers this one
    EvPair *ev = (timing && !in_qr_) ? next_pair(1) : nullptr;
    if (ev) TN_HIP(hipEventRecord(ev->a, s));
    TN_HIP(tnk::launch_qr(a, w, s));
    if (ev) TN_HIP(hipEventRecord(ev->b, s));
    if (!in_qr_) ctr.qr_launches += 1;
    pool_.put(w);
}

// A strided complex128 view as a contraction operand.
static Op view(void *p, const std::string &idx, std::vector<int> dims, std::vector<int64_t> str, bool conj = false) {
    Op o;
    o.p = p;
    o.esz = 16;
    o.idx = idx;
    o.dims = std::move(dims);
    o.str = std::move(str);
    o.conj = conj;
    return o;
}

void Engine::orthonormalise(const tnk::QrArgs &a) {
    const int m = a.m, n = a.n, Z = a.batch;
    {
        std::ostringstream k;
        k << "orthonormalise m=" << m << " n=" << n << " batch=" << Z;
        qr_shapes_[k.str()] += 1;
    }
    if (m < n || householder_only) {
        qr(a);
        return;
    }
    ortho_impl(a, false);
}

// CholeskyQR3 (n <= 64) or the blocked scheme (n > 64) behind orthonormalise;
// with householder_blocks the blocks of the wide case are factored by
// Householder TSQR (exact for rank-deficient input) instead of CholeskyQR3.
void Engine::ortho_impl(const tnk::QrArgs &a, bool householder_blocks) {
    const int m = a.m, n = a.n, Z = a.batch;
    const int saved = prec;
    const bool nested = in_qr_;  // a block of a wider orthonormalisation
    set_prec(tnk::P_FP64);
    in_qr_ = true;
    EvPair *ev = (timing && !nested) ? next_pair(1) : nullptr;
    std::vector<Ten> tmp;
    tmp.reserve(8);  // references into tmp are taken below: no reallocation
    auto cleanup = [&]() {
        for (auto &t : tmp)
            if (t.p) drop(t);
        in_qr_ = nested;
        set_prec(saved);
    };
    try {
        if (ev) TN_HIP(hipEventRecord(ev->a, s));
        if (n <= 64) {
            // Three CholeskyQR passes (the first shifted), each one launch over
            // row blocks (rows times the previous inverse factor, their partial
            // Gram matrices), one ordered sum of the partials and one
            // factorisation; a last row launch writes Q = X_2 R_3^{-1}.
            const int rb = tnk::cqr_rows_per_block(m);
            const int nblk = (m + rb - 1) / rb;
            tmp.push_back(make({Z, m, n}, 16));        // X_1 = A R_1^{-1}
            tmp.push_back(make({Z, m, n}, 16));        // X_2 = X_1 R_2^{-1}
            tmp.push_back(make({Z, nblk, n, n}, 16));  // partial Gram matrices
            tmp.push_back(make({Z, n, n}, 16));        // R^{-1} of the current pass
            tmp.push_back(make({Z, n, n}, 16));        // Gram matrix of the current pass
            Ten &X1 = tmp[0], &X2 = tmp[1], &Pg = tmp[2], &Ri = tmp[3], &G = tmp[4];
            // with R requested: the passes factor R_1, R_2, R_3 (A = Q R_3 R_2 R_1)
            const size_t r0 = tmp.size();
            if (a.R)
                for (int i = 0; i < 3; ++i) tmp.push_back(make({Z, n, n}, 16));
            const double u = 1.1102230246251565e-16;
            // a clamped pivot in any pass flags the item for the Householder fallback
            int *flags = static_cast<int *>(raw((size_t)Z * sizeof(int)));
            TN_HIP(tnk::launch_fill_i32(flags, Z, 0, s));
            for (int pass = 0; pass <= 3; ++pass) {
                tnk::CqrPass c{};
                c.m = m; c.n = n; c.batch = Z; c.rb = rb;
                if (pass < 2) {
                    c.src = a.A; c.s_esz = a.a_esz; c.s_bs = a.a_bs; c.s_rs = a.a_rs; c.s_cs = a.a_cs;
                    c.s_conj = a.a_conj;
                } else {
                    const Ten &Xs = pass == 2 ? X1 : X2;
                    c.src = Xs.p; c.s_esz = 16; c.s_bs = (int64_t)m * n; c.s_rs = n; c.s_cs = 1; c.s_conj = 0;
                }
                c.Ri = pass > 0 ? reinterpret_cast<const double *>(Ri.p) : nullptr;
                if (pass == 1) c.X = reinterpret_cast<double *>(X1.p);
                if (pass == 2) c.X = reinterpret_cast<double *>(X2.p);
                if (pass == 3) {
                    c.dst = a.Q; c.d_esz = a.q_esz; c.d_bs = a.q_bs; c.d_rs = a.q_rs; c.d_cs = a.q_cs;
                    c.d_conj = a.q_conj;
                } else {
                    c.part = reinterpret_cast<double *>(Pg.p);
                }
                TN_HIP(tnk::launch_cqr_pass(c, s));
                if (pass == 3) break;
                // shift relative to tr(G)/n; tr(G) bounds ||A||_2^2
                const double shift = pass == 0 ? 11.0 * ((double)m * n + (double)n * (n + 1)) * u * n : 0.0;
                const double clamp = pass == 0 ? 1e-300 : 1e-14;
                TN_HIP(tnk::launch_sum_parts(reinterpret_cast<const double *>(Pg.p), nblk, n, Z,
                                             reinterpret_cast<double *>(G.p), s));
                TN_HIP(tnk::launch_chol_inv(reinterpret_cast<const double *>(G.p), n, Z, shift, clamp,
                                            reinterpret_cast<double *>(Ri.p),
                                            a.R ? reinterpret_cast<double *>(tmp[r0 + pass].p) : nullptr, flags,
                                            s));
            }
            if (a.R) {
                contract(op(tmp[r0 + 2], "bij"), op(tmp[r0 + 1], "bjk"), op(G, "bik"));
                contract(op(G, "bij"), op(tmp[r0], "bjk"), op(Ri, "bik"));
                TN_HIP(tnk::launch_strided_copy(Ri.p, 16, (int64_t)n * n, n, 1, a.R, a.r_esz, a.r_bs, a.r_rs, a.r_cs, n,
                                                n, Z, a.r_conj, s));
            }
            // Numerically rank-deficient items (a pivot clamped: the passes cannot
            // complete a basis from dependent columns) are refactored by Householder,
            // which returns orthonormal columns for any rank; the others skip it.
            void *ws = raw(tnk::qr_fallback_workspace_bytes(m, n, Z));
            TN_HIP(tnk::launch_qr_fallback(a, flags, ws, s));
            unraw(ws);
            unraw(flags);
        } else {
            // Wider than one Cholesky block: columns in blocks of 64; each block is
            // made orthogonal to the finished ones by three passes of block
            // Gram-Schmidt (W = Q_prev^H X_j, X_j -= Q_prev W; the later passes
            // remove what rounding left of ill-conditioned blocks), then
            // CholeskyQR3'd.  R = [[R_prev, sum of the W], [0, R_jj]] blockwise.
            tmp.push_back(make({Z, m, n}, 16));  // X (the input, updated)
            tmp.push_back(make({Z, m, n}, 16));  // Q
            Ten &X = tmp[0], &Q = tmp[1];
            Ten *R = nullptr;
            if (a.R) {
                tmp.push_back(make({Z, n, n}, 16));
                R = &tmp.back();
                TN_HIP(tnk::launch_fill(R->p, 16, (int64_t)Z * n * n, 0.0, 0.0, s));
            }
            TN_HIP(tnk::launch_strided_copy(a.A, a.a_esz, a.a_bs, a.a_rs, a.a_cs, X.p, 16, (int64_t)m * n, n, 1, m, n,
                                            Z, a.a_conj, s));
            char *xp = static_cast<char *>(X.p), *qp = static_cast<char *>(Q.p);
            const int64_t bs = (int64_t)m * n;
            for (int j0 = 0; j0 < n; j0 += 64) {
                const int nb = std::min(64, n - j0);
                const Op Xj = view(xp + (int64_t)j0 * 16, "bik", {Z, m, nb}, {bs, n, 1});
                if (j0 > 0) {
                    const Op Qp = view(qp, "bij", {Z, m, j0}, {bs, n, 1});
                    const Op Qpc = view(qp, "bij", {Z, m, j0}, {bs, n, 1}, true);
                    Ten W = make({Z, j0, nb}, 16);
                    for (int pass = 0; pass < 3; ++pass) {
                        contract(Qpc, Xj, op(W, "bjk"));
                        if (R) {
                            const Op Rb = view(static_cast<char *>(R->p) + (int64_t)j0 * 16, "bjk", {Z, j0, nb},
                                               {(int64_t)n * n, n, 1});
                            contract(Qpc, Xj, Rb, pass > 0);
                        }
                        TN_HIP(tnk::launch_scale(W.p, W.numel(), -1.0, 0.0, s));
                        contract(Qp, op(W, "bjk"), Xj, true);
                    }
                    drop(W);
                }
                tnk::QrArgs b{};
                b.m = m; b.n = nb; b.batch = Z;
                b.A = xp + (int64_t)j0 * 16; b.a_esz = 16; b.a_bs = bs; b.a_rs = n; b.a_cs = 1; b.a_conj = 0;
                b.Q = qp + (int64_t)j0 * 16; b.q_esz = 16; b.q_bs = bs; b.q_rs = n; b.q_cs = 1; b.q_conj = 0;
                if (R) {
                    b.R = static_cast<char *>(R->p) + ((int64_t)j0 * n + j0) * 16;
                    b.r_esz = 16; b.r_bs = (int64_t)n * n; b.r_rs = n; b.r_cs = 1; b.r_conj = 0;
                }
                if (householder_blocks) {
                    qr(b);
                    if (j0 > 0) {
                        // Householder completes a rank-deficient block with
                        // directions built from unit vectors, which the finished
                        // blocks know nothing about: project them out of Q_j and
                        // factor it again, Q_j = Q' R2, and fold R2 into R_jj
                        const Op Qp = view(qp, "bij", {Z, m, j0}, {bs, n, 1});
                        const Op Qpc = view(qp, "bij", {Z, m, j0}, {bs, n, 1}, true);
                        const Op Qj = view(qp + (int64_t)j0 * 16, "bik", {Z, m, nb}, {bs, n, 1});
                        Ten W = make({Z, j0, nb}, 16);
                        contract(Qpc, Qj, op(W, "bjk"));
                        TN_HIP(tnk::launch_scale(W.p, W.numel(), -1.0, 0.0, s));
                        contract(Qp, op(W, "bjk"), Qj, true);
                        drop(W);
                        Ten R2 = make({Z, nb, nb}, 16);
                        tnk::QrArgs c2 = b;
                        c2.A = qp + (int64_t)j0 * 16;
                        c2.R = R2.p; c2.r_esz = 16; c2.r_bs = (int64_t)nb * nb; c2.r_rs = nb; c2.r_cs = 1;
                        c2.r_conj = 0;
                        qr(c2);  // in place: the factorisation reads A before it writes Q
                        if (R) {
                            const Op Rjj = view(static_cast<char *>(R->p) + ((int64_t)j0 * n + j0) * 16, "bjk",
                                                {Z, nb, nb}, {(int64_t)n * n, n, 1});
                            Ten T = make({Z, nb, nb}, 16);
                            contract(op(R2, "bij"), Rjj, op(T, "bik"));
                            TN_HIP(tnk::launch_strided_copy(T.p, 16, (int64_t)nb * nb, nb, 1,
                                                            static_cast<char *>(R->p) + ((int64_t)j0 * n + j0) * 16,
                                                            16, (int64_t)n * n, n, 1, nb, nb, Z, 0, s));
                            drop(T);
                        }
                        drop(R2);
                    }
                } else {
                    orthonormalise(b);
                    if (j0 > 0 && !R) {
                        // the block's factor scales what the projection left of
                        // the finished blocks in it by up to its condition number:
                        // project once more and orthonormalise again (Q only;
                        // with R the inputs are well conditioned)
                        const Op Qp = view(qp, "bij", {Z, m, j0}, {bs, n, 1});
                        const Op Qpc = view(qp, "bij", {Z, m, j0}, {bs, n, 1}, true);
                        const Op Qj = view(qp + (int64_t)j0 * 16, "bik", {Z, m, nb}, {bs, n, 1});
                        Ten W = make({Z, j0, nb}, 16);
                        contract(Qpc, Qj, op(W, "bjk"));
                        TN_HIP(tnk::launch_scale(W.p, W.numel(), -1.0, 0.0, s));
                        contract(Qp, op(W, "bjk"), Qj, true);
                        drop(W);
                        tnk::QrArgs c2 = b;
                        c2.A = qp + (int64_t)j0 * 16;  // in place: read before Q is written
                        orthonormalise(c2);
                    }
                }
            }
            TN_HIP(tnk::launch_strided_copy(Q.p, 16, bs, n, 1, a.Q, a.q_esz, a.q_bs, a.q_rs, a.q_cs, m, n, Z, a.q_conj,
                                            s));
            if (R)
                TN_HIP(tnk::launch_strided_copy(R->p, 16, (int64_t)n * n, n, 1, a.R, a.r_esz, a.r_bs, a.r_rs, a.r_cs,
                                                n, n, Z, a.r_conj, s));
        }
        if (ev) TN_HIP(hipEventRecord(ev->b, s));
    } catch (...) {
        cleanup();
        throw;
    }
    cleanup();
    if (!nested) ctr.qr_launches += 1;
}

void Engine::norm2(const void *x, int e, int64_t n, int batch, int64_t bs, double *out) {
    const int P = tnk::reduce_partial_count(n);
    void *w = pool_.get((size_t)P * batch * 8);
    TN_HIP(tnk::launch_norm2(x, e, n, batch, bs, reinterpret_cast<double *>(w), out, s));
    pool_.put(w);
}

void Engine::normalise(void *x, int e, int64_t n, int batch, int64_t bs, double *logscale, bool acc,
                       int *flags) {
    void *q = pool_.get((size_t)batch * 8);
    norm2(x, e, n, batch, bs, reinterpret_cast<double *>(q));
    TN_HIP(tnk::launch_normalise(x, e, n, batch, bs, reinterpret_cast<double *>(q), logscale, acc ? 1 : 0,
                                 flags, s));
    pool_.put(q);
}

void Engine::dot(const void *x, const void *y, int e, int64_t n, int batch, int64_t bs, double *out,
                 const int *mask, int mask_skip) {
    const int P = tnk::reduce_partial_count(n);
    void *w = pool_.get((size_t)P * batch * 16);
    TN_HIP(tnk::launch_dot(x, y, e, n, batch, bs, reinterpret_cast<double *>(w), out, s, mask, mask_skip));
    pool_.put(w);
}

}  // namespace tnb

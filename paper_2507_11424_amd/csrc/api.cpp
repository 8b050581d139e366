// C ABI of the library (declared in include/tn.h): validation, staging of the
// site tensors into the compute precision, the cached norm boundary set, and
// error reporting.  No exception crosses this boundary.
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>

#include "../../include/tn.h"
#include "tn_core.hpp"
#include "kernels.hpp"

using namespace tnb;

// Fixed device scratch of tn_sample_stats_noalloc: the partial results of the
// metric kernels.  Each device holds its own copy until the process ends; host
// code uses only the device address obtained by hipGetSymbolAddress (the
// array's name is a host-side stand-in).
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(4) << 20;
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_ptr[MAX_DEVICES] = {};

// Address of `scratch` on `device` (current), looked up once per device.
void *scratch_on(int device) {
    if (device < 0 || device >= MAX_DEVICES) throw TnError(ST_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            throw TnError(ST_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        scratch_ptr[device] = ptr;
    }
    return scratch_ptr[device];
}

}  // namespace

struct tn_handle {
    int device = 0;
    hipStream_t stream = nullptr;
    std::unique_ptr<Engine> E;
    std::string err;
    size_t cap = 0;
    // cached bottom-up boundary set of the last state
    BoundarySet cache;
    std::string cache_key;
    PepsDev cache_peps;
    // sampler test hooks (tn_test_sample_config)
    int sample_wave = 0, sample_rows_limit = 0, sample_graphs = 1;
    double *sample_log_cond = nullptr;
};

namespace {

std::string peps_key(const tn_peps *p, const tn_opts *o) {
    std::string k;
    auto add = [&](const void *d, size_t n) { k.append(reinterpret_cast<const char *>(d), n); };
    add(&p->rows, 4); add(&p->cols, 4); add(&p->dtype, sizeof(p->dtype));
    const int n = p->rows * p->cols;
    add(p->phys, (size_t)n * 4);
    if (p->cols > 1) add(p->dim_h, (size_t)p->rows * (p->cols - 1) * 4);
    if (p->rows > 1) add(p->dim_v, (size_t)(p->rows - 1) * p->cols * 4);
    add(p->site_index, (size_t)n * 4);
    add(p->site, (size_t)n * sizeof(void *));
    add(&o->chi, 4); add(&o->sweeps, 4); add(&o->init, 4); add(&o->prec, sizeof(o->prec));
    add(&o->init_seed, 8);
    return k;
}

void validate(const tn_peps *p, const tn_opts *o) {
    if (!p || !o) throw TnError(ST_INVALID, "null peps or opts");
    if (p->rows < 1 || p->cols < 1) throw TnError(ST_SHAPE, "rows and cols must be >= 1");
    if (!p->phys || !p->site_index || !p->site) throw TnError(ST_INVALID, "null lattice array");
    if (p->cols > 1 && !p->dim_h) throw TnError(ST_INVALID, "null dim_h");
    if (p->rows > 1 && !p->dim_v) throw TnError(ST_INVALID, "null dim_v");
    if (p->dtype != TN_C128 && p->dtype != TN_C64) throw TnError(ST_INVALID, "bad dtype");
    if (o->chi < 1 || o->chi_x < 1 || o->sweeps < 1) throw TnError(ST_INVALID, "chi, chi_x and sweeps must be >= 1");
    if (o->direction < 0 || o->direction > 3) throw TnError(ST_INVALID, "direction must be 0..3");
    if (o->init != 0 && o->init != 1) throw TnError(ST_INVALID, "init must be 0 or 1");
    if (o->prec < TN_PREC_FP64 || o->prec > TN_PREC_BF16X6) throw TnError(ST_INVALID, "bad precision");
    if (!(o->svd_cutoff >= 0.0 && o->svd_cutoff <= 1.0)) throw TnError(ST_INVALID, "svd_cutoff must be in [0, 1]");
    if (o->chi_x_min < 1) throw TnError(ST_INVALID, "chi_x_min must be >= 1");
    const int n = p->rows * p->cols;
    int nq = 0;
    std::vector<int> seen(n, 0);
    for (int i = 0; i < n; ++i) {
        if (p->phys[i] != 1 && p->phys[i] != 2) throw TnError(ST_SHAPE, "phys must be 1 or 2");
        if (!p->site[i]) throw TnError(ST_INVALID, "null site tensor pointer");
        if (p->phys[i] == 2) {
            const int q = p->site_index[i];
            if (q < 0 || q >= n || seen[q]) throw TnError(ST_SHAPE, "site_index must be a permutation of the qubits");
            seen[q] = 1;
            ++nq;
        } else if (p->site_index[i] != -1) {
            throw TnError(ST_SHAPE, "non-qubit sites (phys 1) must have site_index -1");
        }
    }
    for (int q = 0; q < nq; ++q)
        if (!seen[q]) throw TnError(ST_SHAPE, "site_index must cover 0..N-1");
    for (int i = 0; i < p->rows * (p->cols - 1); ++i)
        if (p->dim_h[i] < 1) throw TnError(ST_SHAPE, "bond dimensions must be >= 1");
    for (int i = 0; i < (p->rows - 1) * p->cols; ++i)
        if (p->dim_v[i] < 1) throw TnError(ST_SHAPE, "bond dimensions must be >= 1");
}

PepsDev stage(Engine &E, const tn_peps *p) {
    PepsDev P;
    P.rows = p->rows;
    P.cols = p->cols;
    const int n = p->rows * p->cols;
    P.phys.assign(p->phys, p->phys + n);
    P.site_index.assign(p->site_index, p->site_index + n);
    P.nq = 0;
    for (int i = 0; i < n; ++i) P.nq += p->phys[i] == 2;
    const int src_esz = p->dtype == TN_C128 ? 16 : 8;
    for (int r = 0; r < p->rows; ++r)
        for (int c = 0; c < p->cols; ++c) {
            const int i = r * p->cols + c;
            const int u = r > 0 ? p->dim_v[(r - 1) * p->cols + c] : 1;
            const int d = r + 1 < p->rows ? p->dim_v[r * p->cols + c] : 1;
            const int l = c > 0 ? p->dim_h[r * (p->cols - 1) + c - 1] : 1;
            const int rr = c + 1 < p->cols ? p->dim_h[r * (p->cols - 1) + c] : 1;
            Ten t = E.make({p->phys[i], u, l, d, rr});
            TN_HIP(tnk::launch_convert(p->site[i], src_esz, t.p, t.esz, t.numel(), E.s));
            P.site.push_back(t);
        }
    return P;
}

void unstage(Engine &E, PepsDev &P) {
    for (auto &t : P.site)
        if (t.p) E.drop(t);
    P.site.clear();
}

tn_status fail(tn_handle *h, const TnError &e) {
    if (h) h->err = e.what();
    return (tn_status)e.code;
}

void begin(tn_handle *h, const tn_opts *o) {
    if (!h) throw TnError(ST_INVALID, "null handle");
    h->err.clear();
    TN_HIP(hipSetDevice(h->device));
    if (o) h->E->set_prec((int)o->prec);
    h->E->collect_timing();
    h->E->ctr.reset();
}

FitOpts fit_opts(const tn_opts *o) {
    FitOpts f;
    f.chi = o->chi;
    f.sweeps = o->sweeps;
    f.force_fit = o->init == 1;
    f.seed = o->init_seed;
    return f;
}

// 64-bit fingerprint of the bytes of every site tensor (device-side sum of
// mixed words, read back to the host: synchronises the stream).  Part of the
// cache key, so a state overwritten in place, or a new state placed at the
// freed addresses of an old one, is never served the old boundary set.
uint64_t fingerprint(Engine &E, const tn_peps *p) {
    const int n = p->rows * p->cols;
    const int esz = p->dtype == TN_C128 ? 16 : 8;
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(E.raw(8));
    try {
        TN_HIP(tnk::launch_fill_f64(reinterpret_cast<double *>(acc), 1, 0.0, E.s));
        tnk::FingerprintSet f{};
        for (int i = 0; i < n; ++i) {
            const int r = i / p->cols, c = i % p->cols;
            const int64_t u = r > 0 ? p->dim_v[(r - 1) * p->cols + c] : 1;
            const int64_t d = r + 1 < p->rows ? p->dim_v[r * p->cols + c] : 1;
            const int64_t l = c > 0 ? p->dim_h[r * (p->cols - 1) + c - 1] : 1;
            const int64_t rr = c + 1 < p->cols ? p->dim_h[r * (p->cols - 1) + c] : 1;
            f.ptr[f.count] = p->site[i];
            f.words[f.count] = p->phys[i] * u * l * d * rr * esz / 8;
            f.salt[f.count] = (uint64_t)i << 40;
            if (++f.count == tnk::FP_MAX || i + 1 == n) {
                TN_HIP(tnk::launch_fingerprint(f, acc, E.s));
                f.count = 0;
            }
        }
        unsigned long long hv = 0;
        TN_HIP(hipMemcpyAsync(&hv, acc, 8, hipMemcpyDeviceToHost, E.s));
        E.sync();
        E.unraw(acc);
        return hv;
    } catch (...) {
        E.unraw(acc);
        throw;
    }
}

// Bottom-up boundary set of the state, cached in the handle.  The key holds the
// lattice, the options that shape the set, the site pointers and the content
// fingerprint of the site tensors.
const BoundarySet &cached_set(tn_handle *h, const tn_peps *p, const tn_opts *o, bool recompute) {
    std::string key = peps_key(p, o);
    const uint64_t fp = fingerprint(*h->E, p);
    key.append(reinterpret_cast<const char *>(&fp), 8);
    if (!recompute && key == h->cache_key && !h->cache.below.empty()) return h->cache;
    free_set(*h->E, h->cache);
    unstage(*h->E, h->cache_peps);
    h->cache_key.clear();
    h->cache_peps = stage(*h->E, p);
    LView V = make_view(h->cache_peps, 0);
    h->cache = boundary_set(*h->E, V, fit_opts(o), 0);
    h->cache_key = key;
    return h->cache;
}

}  // namespace

extern "C" {

void tn_default_opts(tn_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->chi = 16;
    o->chi_x = 16;
    o->sweeps = 2;
    o->direction = 0;
    o->init = 0;
    o->prec = TN_PREC_FP64;
    o->init_seed = 0;
    o->workspace_cap = 0;
    o->svd_cutoff = 0.0;
    o->chi_x_min = 1;
}

tn_status tn_create(tn_handle **out, int device, void *stream) {
    if (!out) return TN_ERR_INVALID;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        return TN_ERR_HIP;
    }
    if (device < 0 || device >= n) return TN_ERR_INVALID;
    try {
        auto h = std::make_unique<tn_handle>();
        h->device = device;
        h->stream = reinterpret_cast<hipStream_t>(stream);
        TN_HIP(hipSetDevice(device));
        h->E = std::make_unique<Engine>(device, h->stream, 0);
        (void)scratch_on(device);  // the device's scratch address, once per device
        *out = h.release();
        return TN_OK;
    } catch (const TnError &e) {
        return (tn_status)e.code;
    } catch (...) {
        return TN_ERR_HIP;
    }
}

tn_status tn_destroy(tn_handle *h) {
    if (!h) return TN_ERR_INVALID;
    try {
        (void)hipSetDevice(h->device);
        if (h->E) {
            free_set(*h->E, h->cache);
            unstage(*h->E, h->cache_peps);
        }
        h->E.reset();
    } catch (...) {
    }
    delete h;
    return TN_OK;
}

tn_status tn_boundary_contract(tn_handle *h, const tn_peps *p, const tn_opts *o, double *logabs, double *arg) {
    try {
        begin(h, o);
        validate(p, o);
        if (!logabs || !arg) throw TnError(ST_INVALID, "null output");
        if (o->direction == 0) {
            const BoundarySet &S = cached_set(h, p, o, true);
            LView V = make_view(h->cache_peps, 0);
            norm_close(*h->E, V, S, logabs, arg);
        } else {
            PepsDev P = stage(*h->E, p);
            LView V = make_view(P, o->direction);
            BoundarySet S;
            try {
                S = boundary_set(*h->E, V, fit_opts(o), (o->direction == 1 || o->direction == 3) ? 1 : 0);
                norm_close(*h->E, V, S, logabs, arg);
            } catch (...) {
                free_set(*h->E, S);
                unstage(*h->E, P);
                throw;
            }
            free_set(*h->E, S);
            unstage(*h->E, P);
        }
        return TN_OK;
    } catch (const TnError &e) {
        return fail(h, e);
    } catch (const std::exception &e) {
        return fail(h, TnError(ST_HIP, e.what()));
    }
}

tn_status tn_environments(tn_handle *h, const tn_peps *p, const tn_opts *o, double *rho1, double *zz_h,
                          double *zz_v, double *p2_h, double *p2_v) {
    try {
        begin(h, o);
        validate(p, o);
        if (!rho1) throw TnError(ST_INVALID, "null rho1");
        // the bottom-up boundary set is shared with the norm and the sampler (cached)
        const BoundarySet &S = cached_set(h, p, o, false);
        environments(*h->E, h->cache_peps, fit_opts(o), &S, rho1, zz_h, zz_v, p2_h, p2_v);
        return TN_OK;
    } catch (const TnError &e) {
        return fail(h, e);
    } catch (const std::exception &e) {
        return fail(h, TnError(ST_HIP, e.what()));
    }
}

tn_status tn_sample(tn_handle *h, const tn_peps *p, const tn_opts *o, uint64_t seed, uint64_t first, int64_t n,
                    const double *uniforms, uint8_t *bits, double *log_q, double *log_p, int32_t *chi_x_used) {
    try {
        begin(h, o);
        validate(p, o);
        if (n < 0) throw TnError(ST_INVALID, "n must be >= 0");
        if (n == 0) return TN_OK;
        if (!bits || !log_q) throw TnError(ST_INVALID, "null output");
        const BoundarySet &S = cached_set(h, p, o, false);
        SampleOpts so;
        so.chi_x = o->chi_x;
        so.sweeps = o->sweeps;
        so.force_fit = o->init == 1;
        so.init_seed = o->init_seed;
        so.seed = seed;
        so.svd_cutoff = o->svd_cutoff;
        so.chi_x_min = o->chi_x_min;
        so.wave = h->sample_wave;
        so.rows_limit = h->sample_rows_limit;
        so.log_cond = h->sample_log_cond;
        so.graphs = h->sample_graphs;
        if (so.svd_cutoff > 0 && o->chi_x > tnk::SVD_NMAX)
            throw TnError(ST_UNSUPPORTED, "svd_cutoff needs chi_x <= " + std::to_string(tnk::SVD_NMAX));
        sample(*h->E, h->cache_peps, S, so, first, n, uniforms, bits, log_q, log_p, chi_x_used);
        return TN_OK;
    } catch (const TnError &e) {
        return fail(h, e);
    } catch (const std::exception &e) {
        return fail(h, TnError(ST_HIP, e.what()));
    }
}

tn_status tn_simple_update(tn_handle *h, const tn_peps *p, void *const *site_out, int n_gates,
                           const int32_t *gate_sites, const double *gates, int gate_stride, int bp_max_sweeps,
                           double bp_tol, double *eps, double *fidelity, const void *messages_in,
                           void *messages_out) {
    try {
        begin(h, nullptr);
        tn_opts dflt;
        tn_default_opts(&dflt);
        validate(p, &dflt);
        if (n_gates < 0) throw TnError(ST_INVALID, "n_gates must be >= 0");
        if (!site_out || (n_gates > 0 && (!gate_sites || !gates || !eps)))
            throw TnError(ST_INVALID, "null pointer");
        if (gate_stride != 0 && gate_stride != 16) throw TnError(ST_INVALID, "gate_stride must be 0 or 16");
        if (bp_max_sweeps < 1 || !(bp_tol >= 0.0)) throw TnError(ST_INVALID, "bp_max_sweeps >= 1 and bp_tol >= 0");
        const int rows = p->rows, cols = p->cols;
        std::vector<SuGate> gl((size_t)n_gates);
        for (int g = 0; g < n_gates; ++g) {
            const int32_t *q = gate_sites + (size_t)g * 5;
            SuGate x{q[0], q[1], q[2], q[3], q[4]};
            const bool h_ok = x.r2 == x.r && x.c2 == x.c + 1, v_ok = x.c2 == x.c && x.r2 == x.r + 1;
            if (!(h_ok || v_ok) || x.r < 0 || x.c < 0 || x.r2 >= rows || x.c2 >= cols)
                throw TnError(ST_INVALID, "gate " + std::to_string(g) + ": sites must be (r, c) and (r, c+1) or (r+1, c)");
            if (p->phys[x.r * cols + x.c] != 2 || p->phys[x.r2 * cols + x.c2] != 2)
                throw TnError(ST_INVALID, "gate " + std::to_string(g) + ": both sites must hold qubits");
            gl[(size_t)g] = x;
        }
        Engine &E = *h->E;
        E.set_prec(tnk::P_FP64);
        PepsDev P = stage(E, p);
        try {
            SuOpts so;
            so.bp_max_sweeps = bp_max_sweeps;
            so.bp_tol = bp_tol;
            simple_update(E, P, gl, gates, gate_stride, so, eps, messages_in, messages_out);
            const int dst_esz = p->dtype == TN_C128 ? 16 : 8;
            for (int i = 0; i < rows * cols; ++i) {
                const Ten &t = P.site[(size_t)i];
                if (!site_out[i]) throw TnError(ST_INVALID, "null output site");
                TN_HIP(tnk::launch_convert(t.p, 16, site_out[i], dst_esz, t.numel(), E.s));
            }
            E.sync();
        } catch (...) {
            unstage(E, P);
            throw;
        }
        unstage(E, P);
        if (fidelity) {
            double f = 1.0;
            for (int g = 0; g < n_gates; ++g) f *= 1.0 - eps[g];
            *fidelity = f;
        }
        return TN_OK;
    } catch (const TnError &e) {
        return fail(h, e);
    } catch (const std::exception &e) {
        return fail(h, TnError(ST_HIP, e.what()));
    }
}

tn_status tn_bp(tn_handle *h, const tn_peps *p, int max_sweeps, double tol, double *log_abs_Z, double *arg_Z,
                int *sweeps, double *last_change, double *eps_mean, double *eps_loops, int eps_capacity,
                int *n_loops, void *messages) {
    try {
        begin(h, nullptr);
        tn_opts dflt;
        tn_default_opts(&dflt);
        validate(p, &dflt);
        if (max_sweeps < 1 || !(tol >= 0.0)) throw TnError(ST_INVALID, "max_sweeps must be >= 1 and tol >= 0");
        if (!log_abs_Z || !arg_Z) throw TnError(ST_INVALID, "null output");
        if (eps_loops && eps_capacity < 0) throw TnError(ST_INVALID, "eps_capacity must be >= 0");
        Engine &E = *h->E;
        E.set_prec(tnk::P_FP64);
        PepsDev P = stage(E, p);
        BpOpts bo;
        bo.max_sweeps = max_sweeps;
        bo.tol = tol;
        bo.loops = eps_mean || eps_loops || n_loops;
        bo.messages = messages;
        BpResult r;
        try {
            bp_contract(E, P, bo, r);
        } catch (...) {
            unstage(E, P);
            throw;
        }
        unstage(E, P);
        E.sync();
        *log_abs_Z = r.log_abs;
        *arg_Z = r.arg;
        if (sweeps) *sweeps = r.sweeps;
        if (last_change) *last_change = r.delta;
        if (eps_mean) *eps_mean = r.eps_mean;
        if (n_loops) *n_loops = (int)r.eps.size();
        if (r.eig_info) throw TnError(ST_NUMERIC, "loop eigenvalue iteration did not converge");
        if (eps_loops) {
            if ((int)r.eps.size() > eps_capacity)
                throw TnError(ST_INVALID, "eps_loops holds " + std::to_string(eps_capacity) + " entries, " +
                                              std::to_string(r.eps.size()) + " loops found");
            std::copy(r.eps.begin(), r.eps.end(), eps_loops);
        }
        return TN_OK;
    } catch (const TnError &e) {
        return fail(h, e);
    } catch (const std::exception &e) {
        return fail(h, TnError(ST_HIP, e.what()));
    }
}

tn_status tn_amplitude(tn_handle *h, const tn_peps *p, const tn_opts *o, uint64_t first, int64_t n,
                       const uint8_t *bits, double *log_p, double *arg) {
    try {
        begin(h, o);
        validate(p, o);
        if (n < 0) throw TnError(ST_INVALID, "n must be >= 0");
        if (n == 0) return TN_OK;
        if (!bits || !log_p) throw TnError(ST_INVALID, "null bits or log_p");
        SampleOpts so;
        so.chi_x = o->chi_x;
        so.sweeps = o->sweeps;
        so.force_fit = o->init == 1;
        so.init_seed = o->init_seed;
        so.init_tag = 4;
        PepsDev P = stage(*h->E, p);
        try {
            amplitude(*h->E, P, so, first, n, bits, log_p, arg);
        } catch (...) {
            unstage(*h->E, P);
            throw;
        }
        unstage(*h->E, P);
        return TN_OK;
    } catch (const TnError &e) {
        return fail(h, e);
    } catch (const std::exception &e) {
        return fail(h, TnError(ST_HIP, e.what()));
    }
}

tn_status tn_sample_stats(tn_handle *h, int64_t n, int32_t n_qubits, const uint8_t *bits, const double *log_q,
                          const double *log_p, double log_Z, double *out, double *z_is) {
    try {
        if (!h || !h->E) throw TnError(ST_INVALID, "null handle");
        h->err.clear();
        TN_HIP(hipSetDevice(h->device));
        if (n <= 0) throw TnError(ST_INVALID, "n must be > 0");
        if (!log_q || !log_p || !out) throw TnError(ST_INVALID, "null log_q, log_p or out");
        if (z_is && (!bits || n_qubits <= 0)) throw TnError(ST_INVALID, "z_is needs bits and n_qubits > 0");
        Engine &E = *h->E;
        double *dev = reinterpret_cast<double *>(E.raw(3 * sizeof(double)));
        void *ws = E.raw(tnk::stats_workspace_bytes(n, n_qubits, z_is != nullptr));
        try {
            TN_HIP(tnk::launch_sample_stats(log_q, log_p, n, log_Z, z_is ? bits : nullptr, n_qubits, dev, z_is, ws,
                                            E.s));
            TN_HIP(hipMemcpyAsync(out, dev, 3 * sizeof(double), hipMemcpyDeviceToHost, E.s));
            E.sync();
        } catch (...) {
            E.unraw(dev);
            E.unraw(ws);
            throw;
        }
        E.unraw(dev);
        E.unraw(ws);
        return TN_OK;
    } catch (const TnError &e) {
        return fail(h, e);
    } catch (const std::exception &e) {
        return fail(h, TnError(ST_HIP, e.what()));
    }
}

tn_status tn_sample_stats_noalloc(tn_handle *h, int64_t n, int32_t n_qubits, const uint8_t *bits,
                                  const double *log_q, const double *log_p, double log_Z, double *out, double *z_is) {
    try {
        if (!h || !h->E) throw TnError(ST_INVALID, "null handle");
        h->err.clear();
        TN_HIP(hipSetDevice(h->device));
        if (n <= 0) throw TnError(ST_INVALID, "n must be > 0");
        if (!log_q || !log_p || !out) throw TnError(ST_INVALID, "null log_q, log_p or out");
        if (z_is && (!bits || n_qubits <= 0)) throw TnError(ST_INVALID, "z_is needs bits and n_qubits > 0");
        const size_t need = tnk::stats_workspace_bytes(n, z_is ? n_qubits : 0, z_is != nullptr);
        if (need > NOALLOC_SCRATCH_BYTES)
            throw TnError(ST_INVALID, "tn_sample_stats_noalloc: n_qubits = " + std::to_string(n_qubits) + " needs " +
                                          std::to_string(need) + " bytes of scratch, the fixed scratch holds " +
                                          std::to_string(NOALLOC_SCRATCH_BYTES) + " (at most " +
                                          std::to_string(TN_NOALLOC_MAX_QUBITS) + " qubits)");
        void *ws = scratch_on(h->device);
        TN_HIP(tnk::launch_sample_stats(log_q, log_p, n, log_Z, z_is ? bits : nullptr, n_qubits, out, z_is, ws,
                                        h->E->s));
        return TN_OK;
    } catch (const TnError &e) {
        return fail(h, e);
    } catch (const std::exception &e) {
        return fail(h, TnError(ST_HIP, e.what()));
    }
}

const char *tn_last_error(const tn_handle *h) { return h ? h->err.c_str() : "null handle"; }

tn_status tn_get_counters(const tn_handle *h, double *gemm_flops, int64_t *gemm_launches, double *gemm_ms,
                          double *qr_ms, int64_t *qr_launches, double *qr_gemm_flops, int64_t *masked_launches,
                          double *masked_ms, double *gemm_bytes, int64_t *graph_launches) {
    if (!h || !h->E) return TN_ERR_INVALID;
    try {
        const_cast<Engine *>(h->E.get())->collect_timing();
    } catch (const TnError &e) {
        return (tn_status)e.code;
    }
    const Counters &c = h->E->ctr;
    if (gemm_flops) *gemm_flops = c.gemm_flops;
    if (gemm_launches) *gemm_launches = c.gemm_launches;
    if (gemm_ms) *gemm_ms = c.gemm_ms;
    if (qr_ms) *qr_ms = c.qr_ms;
    if (qr_launches) *qr_launches = c.qr_launches;
    if (qr_gemm_flops) *qr_gemm_flops = c.qr_gemm_flops;
    if (masked_launches) *masked_launches = c.masked_launches;
    if (masked_ms) *masked_ms = c.masked_ms;
    if (gemm_bytes) *gemm_bytes = c.gemm_bytes;
    if (graph_launches) *graph_launches = c.graph_launches;
    return TN_OK;
}

tn_status tn_plan_report(const tn_handle *h, int top, char *buf, size_t len) {
    if (!h || !h->E || !buf || len == 0) return TN_ERR_INVALID;
    try {
        const_cast<Engine *>(h->E.get())->collect_timing();
    } catch (const TnError &e) {
        return (tn_status)e.code;
    }
    const std::string s = h->E->plan_report(top);
    const size_t n = std::min(len - 1, s.size());
    std::memcpy(buf, s.data(), n);
    buf[n] = 0;
    return TN_OK;
}

tn_status tn_set_timing(tn_handle *h, int enable) {
    if (!h || !h->E) return TN_ERR_INVALID;
    h->E->timing = enable != 0;
    return TN_OK;
}

tn_status tn_set_autotune(tn_handle *h, int enable, const char *cache_path) {
    if (!h || !h->E) return TN_ERR_INVALID;
    try {
        h->err.clear();
        h->E->set_autotune(enable != 0, cache_path ? std::string(cache_path) : std::string());
        return TN_OK;
    } catch (const TnError &e) {
        h->err = e.what();
        return (tn_status)e.code;
    } catch (const std::exception &e) {
        h->err = e.what();
        return TN_ERR_INVALID;
    }
}

// ---------------------------------------------------------------- test hooks

tn_status tn_test_contract(tn_handle *h, int prec, const char *ia, const void *A, const int32_t *adims, int conjA,
                           const char *ib, const void *B, const int32_t *bdims, int conjB, const char *ic,
                           void *C, const int32_t *cdims, int accumulate, int cfg, int ksplit) {
    try {
        if (!h) throw TnError(ST_INVALID, "null handle");
        h->err.clear();
        TN_HIP(hipSetDevice(h->device));
        h->E->set_prec(prec);
        auto mk = [&](const void *p, const int32_t *d, const char *idx) {
            Ten t;
            t.p = const_cast<void *>(p);
            t.esz = h->E->esz;
            t.d.assign(d, d + std::strlen(idx));
            return t;
        };
        Ten a = mk(A, adims, ia), b = mk(B, bdims, ib), c = mk(C, cdims, ic);
        h->E->force_cfg = cfg;
        h->E->force_ksplit = ksplit;
        try {
            h->E->contract(op(a, ia, conjA != 0), op(b, ib, conjB != 0), op(c, ic), accumulate != 0);
        } catch (...) {
            h->E->force_cfg = -1;
            throw;
        }
        h->E->force_cfg = -1;
        return TN_OK;
    } catch (const TnError &e) {
        return fail(h, e);
    }
}

tn_status tn_test_qr(tn_handle *h, int m, int n, int batch, int esz, const void *A, void *Q, void *R, int method) {
    try {
        if (!h) throw TnError(ST_INVALID, "null handle");
        h->err.clear();
        TN_HIP(hipSetDevice(h->device));
        const int k = m < n ? m : n;
        tnk::QrArgs a{};
        a.m = m; a.n = n; a.batch = batch;
        a.A = A; a.a_esz = esz; a.a_bs = (int64_t)m * n; a.a_rs = n; a.a_cs = 1;
        a.Q = Q; a.q_esz = esz; a.q_bs = (int64_t)m * k; a.q_rs = k; a.q_cs = 1;
        a.R = R; a.r_esz = esz; a.r_bs = (int64_t)k * n; a.r_rs = n; a.r_cs = 1;
        if (method == 2) {
            // LQ layout: A holds the conjugate transpose (batch x n x m), Q is
            // written the same way (rows orthonormal), as the fit's LQ moves do
            if (R || m < n) throw TnError(ST_INVALID, "tn_test_qr: the LQ layout takes no R and needs m >= n");
            a.a_rs = 1; a.a_cs = m; a.a_conj = 1;
            a.q_rs = 1; a.q_cs = m; a.q_conj = 1;
            a.R = nullptr;
        }
        if (method == 0) h->E->qr(a);
        else h->E->orthonormalise(a);
        return TN_OK;
    } catch (const TnError &e) {
        return fail(h, e);
    }
}

tn_status tn_test_sample_config(tn_handle *h, int wave, int rows_limit, double *log_cond, int graphs) {
    if (!h || !h->E) return TN_ERR_INVALID;
    if (wave < 0 || rows_limit < 0 || graphs < 0 || graphs > 1) {
        h->err = "tn_test_sample_config: wave and rows_limit must be >= 0, graphs 0 or 1";
        return TN_ERR_INVALID;
    }
    h->sample_wave = wave;
    h->sample_rows_limit = rows_limit;
    h->sample_log_cond = log_cond;
    h->sample_graphs = graphs;
    return TN_OK;
}

tn_status tn_test_eig(tn_handle *h, int n, int batch, const void *A, void *lam, double *eps, int32_t *info) {
    try {
        if (!h || !h->E) throw TnError(ST_INVALID, "null handle");
        h->err.clear();
        TN_HIP(hipSetDevice(h->device));
        if (n < 1 || n > tnk::BP_EIG_NMAX || batch < 0) throw TnError(ST_INVALID, "tn_test_eig: bad n or batch");
        if (!A || !lam || !eps || !info) throw TnError(ST_INVALID, "tn_test_eig: null pointer");
        Engine &E = *h->E;
        const size_t bytes = (size_t)batch * n * n * 16;
        void *w = E.raw(bytes);
        TN_HIP(hipMemcpyAsync(w, A, bytes, hipMemcpyDeviceToDevice, E.s));
        const hipError_t e = tnk::launch_eig(w, n, batch, lam, eps, info, E.s);
        E.unraw(w);
        TN_HIP(e);
        return TN_OK;
    } catch (const TnError &e) {
        return fail(h, e);
    } catch (const std::exception &e) {
        return fail(h, TnError(ST_HIP, e.what()));
    }
}

tn_status tn_test_set_mask(tn_handle *h, const int32_t *mask, char letter) {
    if (!h || !h->E) return TN_ERR_INVALID;
    if (mask) h->E->set_mask(mask, letter);
    else h->E->clear_mask();
    return TN_OK;
}

tn_status tn_test_svd(tn_handle *h, int n, int batch, const void *R, double cutoff, int chi_min, void *U, void *SV,
                      int esz, int32_t *k) {
    try {
        if (!h) throw TnError(ST_INVALID, "null handle");
        h->err.clear();
        TN_HIP(hipSetDevice(h->device));
        if (n < 1 || n > tnk::SVD_NMAX || batch < 0 || (esz != 8 && esz != 16))
            throw TnError(ST_INVALID, "tn_test_svd: bad n, batch or esz");
        if (!R || !U || !SV || !k) throw TnError(ST_INVALID, "tn_test_svd: null pointer");
        const size_t wsb = tnk::svd_trunc_workspace_bytes(n, batch);
        void *ws = wsb ? h->E->raw(wsb) : nullptr;
        const hipError_t e = tnk::launch_svd_trunc(static_cast<const double *>(R), n, batch, cutoff, chi_min, U, SV,
                                                   esz, k, ws, h->E->s);
        if (ws) h->E->unraw(ws);
        TN_HIP(e);
        return TN_OK;
    } catch (const TnError &e) {
        return fail(h, e);
    }
}

}  // extern "C"

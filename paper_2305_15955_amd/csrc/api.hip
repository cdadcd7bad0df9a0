// C ABI of the CD-WAC library: validation, workspace plan and stage order
// (Sec. 3.4: wmatrix(F_im) -> wmatrix(F_real) -> AC -> QP iteration).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <random>
#include <string>
#include <vector>

#include "../../include/cdwac.h"
#include "common.h"
#include "kernels.h"

using namespace cdwac;

// Fixed device scratch of the allocation-free fit entry point
// (cdwac_pade_fit_eval_noalloc): the coefficients and nodes of up to
// kNoAllocFitPoints = n_fit * n_pts complex values each, then the term counts
// of up to kNoAllocFitPoints fits.  One copy per device, kept until the
// process ends.  Host code never passes this name to a kernel: it is a
// host-side stand-in; the device address comes from hipGetSymbolAddress.
namespace {
constexpr int64_t kNoAllocFitPoints = (int64_t)1 << 19;
constexpr size_t kNoAllocPlane = sizeof(double) * 2 * (size_t)kNoAllocFitPoints;
constexpr size_t kNoAllocBytes = 2 * kNoAllocPlane + sizeof(int) * (size_t)kNoAllocFitPoints;
}  // namespace
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
// Device address of `scratch` on each device, looked up once per device
// (with that device current) by the first context created on it.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_address(int device, void** out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}
}  // namespace

namespace {

// Device memory for the prescaled polarizability operands (batched over the
// weight vectors so that large systems stay within a fixed budget).
constexpr size_t kPrescaleBudget = (size_t)48 << 30;
constexpr size_t kPiListPad = 8 * 128;

// Fit ranges are widened by the Z-factor step of the root search so that
// every self-energy evaluation of the solver finds a Pade model.
constexpr double kFitMargin = 1e-4;

// Largest accepted sampled residual of an inversion, max|eps^-1 eps_j - e_j|
// relative to max(|eps^-1| |eps_j|): a backward-stable inverse stays within a
// small multiple of the unit roundoff (about 1e-15 measured); element growth
// in the unpivoted sweep of an indefinite eps(x + i eta) raises it by the
// growth factor.  Above this the inverse has lost more than half its digits.
constexpr double kFactTol = 1e-8;

struct Region {
    size_t off = 0, bytes = 0;
};

struct Plan {
    // sizes
    int n_mo, n_occ, n_virt, n_aux, S, n_freq, n_im, n_re, n_pts, n_f, prec;
    int npad, cpad, cfpad, ni, n_fit, nblk, nb, n_tpi, n_tw, n_twf;
    int n_imp;    // imaginary-axis planes (every node, or the skeleton nodes)
    bool nr64;    // 16-bit mode with the near-real planes of Pi on the FP64 path
    int64_t K, kpad;
    // persistent regions
    Region eps, eps_g, freq, weight, ref_re, ref_im, state_idx, vxc, sigx, win_lo, win_hi, m0, m1, fit_off, fit_s,
        fit_m, w_im, w_re, coef, node, nterm, qpout, err, hedin, w0;
    // transient regions (prepare only)
    Region zr, zi, part, idflag, amax, sf, cw, cw64, x64, xh, xl, E, dinv_r, pbuf_r, qbuf_r, dinv_c, pbuf_c, qbuf_c,
        dscr_r, lh, ll,
        bt64, bh, bl, bf64, bfh, bfl, partial_im, partial_re, rowsel, ref_u, ref_w, x32, yh, yl, t_pi, t_w,
        t_wf, pmap, imnode, imrest, tmat, rowsum, fcols, fcolidx, fres;
    size_t total = 0;
};

size_t add(Plan& p, Region& r, size_t bytes) {
    r.off = p.total;
    r.bytes = bytes;
    p.total += (bytes + 255) / 256 * 256;
    return r.off;
}

struct HostState {
    std::vector<int> state_idx, m0, m1, fit_off, fit_s, fit_m;
    std::vector<double> eps, vxc, win_lo, win_hi;
    double eps_f = 0.0, eta = 0.0, qp_tol = 1e-10;
    int qp_maxit = 100, use_mlp = 0;
    double mlp_accept = 0.0;
    bool vxc_is_sigx = false;
    bool fit_all = false;
    bool quad_limit = false;
    // imaginary nodes with a plane (ascending), the others, and the
    // interpolation of W at the others: W_rest[r] = sum_j T[r][j] W_node[j]
    std::vector<int> node, rest;
    std::vector<double> T;
    double omega_lo = 0.0, omega_hi = 0.0;   // excitation range the decomposition assumes
};

}  // namespace

struct cdwac_ctx {
    int device = 0;
    int n_cu = 256;   // compute units of the device
    std::vector<int2> pi_work[2];   // polarizability work lists of the last prepare
    hipStream_t stream = nullptr;
    std::string err;
    void* ws_user = nullptr;
    size_t ws_user_bytes = 0;
    void* ws_own = nullptr;
    size_t ws_own_bytes = 0;
    char* ws = nullptr;
    bool prepared = false;
    Plan plan{};
    HostState hs;
    // learned seed
    float* mlp_theta = nullptr;
    bool have_mlp = false;
    float mlp_mu[8] = {}, mlp_sd[8] = {}, mlp_out_mu = 0.f, mlp_out_sd = 1.f;
    // MLP scratch
    void* mlp_scratch = nullptr;
    size_t mlp_scratch_bytes = 0;
    // second stream (default priority) for the complex-plane sweep, and the
    // events that fork it from and join it to the context's stream
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    // tables of a batch of systems (cdwac_solve_batch)
    void* batch = nullptr;
    size_t batch_bytes = 0;
    // stage timing: segments of kernels bracketed by event pairs on the stream
    bool timing = false;
    struct Seg {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Seg> segs;
    std::vector<hipEvent_t> pool;
    size_t pool_used = 0;
    double stage_ms[CDWAC_N_STAGES] = {};
    int32_t stage_n[CDWAC_N_STAGES] = {};
    // sampled residual of the inversions of the last preparation
    double fact_ratio = 0.0;
    int32_t fact_mat = -1;
    // device address of the fixed scratch on this context's device
    char* scratch = nullptr;
};

namespace {

int fail(cdwac_ctx* c, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

#define HIPCK(call)                                                                              \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) return fail(ctx, CDWAC_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define LAUNCHCK()                                                                                  \
    do {                                                                                            \
        hipError_t e_ = hipGetLastError();                                                          \
        if (e_ != hipSuccess) return fail(ctx, CDWAC_EHIP, "kernel launch: %s", hipGetErrorString(e_)); \
    } while (0)

bool finite_all(const double* v, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

int validate_system(cdwac_ctx* ctx, const cdwac_system* s) {
    if (!s) return fail(ctx, CDWAC_EINVAL, "system is NULL");
    if (s->n_mo < 2 || s->n_occ < 1 || s->n_occ >= s->n_mo)
        return fail(ctx, CDWAC_EINVAL, "need 1 <= n_occ < n_mo (n_occ=%d, n_mo=%d)", s->n_occ, s->n_mo);
    if (s->n_aux < 1) return fail(ctx, CDWAC_EINVAL, "n_aux must be >= 1");
    if (s->n_states < 1) return fail(ctx, CDWAC_EINVAL, "n_states must be >= 1");
    if (!s->state_idx || !s->eps || !s->o_ia || !s->o_nm) return fail(ctx, CDWAC_EINVAL, "NULL array in system");
    if (!finite_all(s->eps, s->n_mo)) return fail(ctx, CDWAC_EINVAL, "non-finite orbital energy");
    for (int m = 1; m < s->n_mo; ++m)
        if (!(s->eps[m] > s->eps[m - 1]))
            return fail(ctx, CDWAC_EINVAL, "orbital energies must be strictly ascending (index %d)", m);
    for (int j = 0; j < s->n_states; ++j)
        if (s->state_idx[j] < 0 || s->state_idx[j] >= s->n_mo)
            return fail(ctx, CDWAC_EINVAL, "state_idx[%d] = %d out of range", j, s->state_idx[j]);
    if (s->vxc && !finite_all(s->vxc, s->n_states)) return fail(ctx, CDWAC_EINVAL, "non-finite vxc");
    if (!(s->spin > 0.0) || !std::isfinite(s->spin)) return fail(ctx, CDWAC_EINVAL, "spin factor must be > 0");
    int64_t K = (int64_t)s->n_occ * (s->n_mo - s->n_occ);
    if (K > (int64_t)1 << 31) return fail(ctx, CDWAC_EINVAL, "n_occ * n_virt too large");
    return CDWAC_OK;
}

int validate_params(cdwac_ctx* ctx, const cdwac_system* s, const cdwac_params* p) {
    if (!p) return fail(ctx, CDWAC_EINVAL, "params is NULL");
    if (p->n_freq < 1 || p->n_freq > qp_max_freq())
        return fail(ctx, CDWAC_EINVAL, "n_freq must be in [1, %d]", qp_max_freq());
    if (!p->freq || !p->weight) return fail(ctx, CDWAC_EINVAL, "NULL frequency grid");
    for (int k = 0; k < p->n_freq; ++k)
        if (!(p->freq[k] > 0.0) || !std::isfinite(p->freq[k]) || !std::isfinite(p->weight[k]))
            return fail(ctx, CDWAC_EINVAL, "frequency node %d must be finite and > 0", k);
    if (p->n_ref_im < 0 || p->n_ref_re < 0) return fail(ctx, CDWAC_EINVAL, "negative reference count");
    if (p->n_ref_im + p->n_ref_re < 1 || p->n_ref_im + p->n_ref_re > kMaxPade)
        return fail(ctx, CDWAC_EINVAL, "Pade reference count must be in [1, %d]", kMaxPade);
    if (p->n_ref_im > 0 && !p->ref_im_idx) return fail(ctx, CDWAC_EINVAL, "ref_im_idx is NULL");
    std::vector<char> seen(p->n_freq, 0);
    for (int j = 0; j < p->n_ref_im; ++j) {
        int k = p->ref_im_idx[j];
        if (k < 0 || k >= p->n_freq || seen[k]) return fail(ctx, CDWAC_EINVAL, "ref_im_idx must be distinct grid indices");
        seen[k] = 1;
    }
    if (p->n_ref_re > 0) {
        if (!p->ref_re) return fail(ctx, CDWAC_EINVAL, "ref_re is NULL");
        for (int j = 0; j < p->n_ref_re; ++j)
            if (!(p->ref_re[j] >= 0.0) || !std::isfinite(p->ref_re[j]))
                return fail(ctx, CDWAC_EINVAL, "ref_re[%d] must be finite and >= 0", j);
        if (!(p->eta_ref > 0.0) || !std::isfinite(p->eta_ref)) return fail(ctx, CDWAC_EINVAL, "eta_ref must be > 0");
    }
    if (!(p->eta >= 0.0) || !std::isfinite(p->eta)) return fail(ctx, CDWAC_EINVAL, "eta must be >= 0");
    if (!(p->pade_tol >= 0.0)) return fail(ctx, CDWAC_EINVAL, "pade_tol must be >= 0");
    if (!p->win_lo || !p->win_hi) return fail(ctx, CDWAC_EINVAL, "NULL QP window");
    for (int j = 0; j < s->n_states; ++j) {
        if (!std::isfinite(p->win_lo[j]) || !std::isfinite(p->win_hi[j]) || !(p->win_lo[j] < p->win_hi[j]))
            return fail(ctx, CDWAC_EINVAL, "QP window %d must satisfy lo < hi", j);
        // the root search starts at eps_n (Eq. qp_eq)
        const double e_n = s->eps[s->state_idx[j]];
        if (!(p->win_lo[j] <= e_n && e_n <= p->win_hi[j]))
            return fail(ctx, CDWAC_EINVAL, "QP window %d [%g, %g] does not contain its state's energy %g", j,
                        p->win_lo[j], p->win_hi[j], e_n);
    }
    if (!(p->qp_tol > 0.0) || p->qp_maxit < 1) return fail(ctx, CDWAC_EINVAL, "qp_tol > 0 and qp_maxit >= 1 required");
    if (p->prec < CDWAC_P64 || p->prec > CDWAC_F16) return fail(ctx, CDWAC_EINVAL, "unknown precision %d", p->prec);
    if (p->use_mlp_seed != 0 && p->use_mlp_seed != 1) return fail(ctx, CDWAC_EINVAL, "use_mlp_seed must be 0 or 1");
    if (p->use_mlp_seed && !(p->mlp_accept >= 0.0)) return fail(ctx, CDWAC_EINVAL, "mlp_accept must be >= 0");
    if (!(p->freq_rank_tol >= 0.0 && p->freq_rank_tol < 1.0))
        return fail(ctx, CDWAC_EINVAL, "freq_rank_tol must be in [0, 1)");
    if (p->fit_all != 0 && p->fit_all != 1) return fail(ctx, CDWAC_EINVAL, "fit_all must be 0 or 1");
    if (p->near_real_f64 != 0 && p->near_real_f64 != 1)
        return fail(ctx, CDWAC_EINVAL, "near_real_f64 must be 0 or 1");
    if (p->quad_limit != 0 && p->quad_limit != 1) return fail(ctx, CDWAC_EINVAL, "quad_limit must be 0 or 1");
    return CDWAC_OK;
}

// Orbitals whose residue can enter the window [lo, hi] (Eq. ffact):
// occupied m with eps_m >= lo and virtual m with eps_m <= hi, a range [m0, m1).
void fit_range(const double* eps, int n_mo, int n_occ, double lo, double hi, int& m0, int& m1) {
    m0 = (int)(std::lower_bound(eps, eps + n_occ, lo) - eps);
    m1 = n_occ + (int)(std::upper_bound(eps + n_occ, eps + n_mo, hi) - (eps + n_occ));
}

// ---- frequency decomposition of W on the imaginary axis -------------------
// With the RPA excitation energies Omega_s and weights w_s >= 0 (Woodbury
// form of Eq. bigLambda), W^c_nm(i w) = -sum_s w_s / (w^2 + Omega_s^2): every
// W^c_nm lies in the span of the family h_w(Omega) = 1 / (w^2 + Omega^2),
// Omega in [Omega_lo, Omega_hi].  A row interpolative decomposition
// h_f ~= sum_j T[f][j] h_{node j} of that family therefore interpolates every
// W^c_nm(i w_f) from its values at the skeleton nodes, which are the only
// nodes that need Pi, the inversion and the W contraction.  The decomposition
// is taken on a logarithmic grid of Omega by column-pivoted Gram-Schmidt with
// re-orthogonalisation, starting from the largest node (whose plane the caller
// uses to check Omega_hi); the rank is the smallest for which every
// interpolated function is reproduced on the grid to tol times its maximum.
// Returns false if no rank below n meets tol.
struct FreqId {
    std::vector<int> skel, rest;   // skeleton ascending
    std::vector<double> T;         // [rest.size()][skel.size()], columns in skel order
};

bool freq_id(const double* w, int n, double lo, double hi, double tol, FreqId& out) {
    const int m = 2048;
    std::vector<double> G((size_t)m * n), A, scale(n, 0.0);
    for (int f = 0; f < n; ++f) {
        for (int j = 0; j < m; ++j) {
            const double om = lo * std::pow(hi / lo, (double)j / (m - 1));
            const double g = 1.0 / (w[f] * w[f] + om * om);
            G[(size_t)f * m + j] = g;
            scale[f] = std::max(scale[f], g);
        }
        for (int j = 0; j < m; ++j) G[(size_t)f * m + j] /= scale[f];
    }
    A = G;
    std::vector<int> piv(n);
    for (int i = 0; i < n; ++i) piv[i] = i;
    std::vector<double> R((size_t)n * n, 0.0);   // R[k * n + i], columns in pivot order
    auto col = [&](int c) { return &A[(size_t)c * m]; };
    const int fmax = (int)(std::max_element(w, w + n) - w);
    int steps = 0;
    for (int k = 0; k < n; ++k) {
        int best = -1;
        double bn = 0.0;
        for (int i = k; i < n; ++i) {
            const double* a = col(piv[i]);
            double s2 = 0.0;
            for (int j = 0; j < m; ++j) s2 += a[j] * a[j];
            if (k == 0 && piv[i] == fmax) { best = i; bn = s2; break; }
            if (s2 > bn) { bn = s2; best = i; }
        }
        if (best < 0 || !(bn > 1e-300)) break;
        std::swap(piv[k], piv[best]);
        for (int r = 0; r < k; ++r) std::swap(R[(size_t)r * n + k], R[(size_t)r * n + best]);
        double* q = col(piv[k]);
        const double nq = std::sqrt(bn);
        for (int j = 0; j < m; ++j) q[j] /= nq;
        R[(size_t)k * n + k] = nq;
        for (int i = k + 1; i < n; ++i) {
            double* a = col(piv[i]);
            double tot = 0.0;
            for (int pass = 0; pass < 2; ++pass) {
                double d = 0.0;
                for (int j = 0; j < m; ++j) d += q[j] * a[j];
                for (int j = 0; j < m; ++j) a[j] -= d * q[j];
                tot += d;
            }
            R[(size_t)k * n + i] = tot;
        }
        steps = k + 1;
    }
    for (int k = 1; k < steps; ++k) {
        const int nr = n - k;
        std::vector<double> T((size_t)nr * k);
        double worst = 0.0;
        for (int i = k; i < n && worst <= tol; ++i) {
            double* t = &T[(size_t)(i - k) * k];
            for (int r = k - 1; r >= 0; --r) {   // R11 t = R12(:, i)
                double v = R[(size_t)r * n + i];
                for (int c = r + 1; c < k; ++c) v -= R[(size_t)r * n + c] * t[c];
                t[r] = v / R[(size_t)r * n + r];
            }
            const double* g = &G[(size_t)piv[i] * m];
            for (int j = 0; j < m; ++j) {
                double v = g[j];
                for (int c = 0; c < k; ++c) v -= t[c] * G[(size_t)piv[c] * m + j];
                worst = std::max(worst, std::fabs(v));
            }
        }
        if (worst <= tol) {
            // skeleton in ascending node order; T columns follow it
            std::vector<int> order(k);
            for (int c = 0; c < k; ++c) order[c] = c;
            std::sort(order.begin(), order.end(), [&](int a, int b) { return piv[a] < piv[b]; });
            out.skel.resize(k);
            for (int c = 0; c < k; ++c) out.skel[c] = piv[order[c]];
            out.rest.assign(piv.begin() + k, piv.end());
            out.T.assign((size_t)nr * k, 0.0);
            for (int r = 0; r < nr; ++r)
                for (int c = 0; c < k; ++c)
                    out.T[(size_t)r * k + c] =
                        T[(size_t)r * k + order[c]] * scale[out.rest[r]] / scale[piv[order[c]]];
            return true;
        }
    }
    return false;
}

// Assumed bound of the RPA excitation energies for the decomposition: the
// lowest is >= the lowest transition energy (Omega^2 = eig(D^2 + positive
// semidefinite)); the highest is taken as 4 times the highest transition
// energy and checked after Pi is known (cdwac_prepare falls back to every
// node if the check fails).
constexpr double kOmegaHiFactor = 4.0;

Plan make_plan(const cdwac_system* s, const cdwac_params* p, HostState* hs, bool allow_id = true) {
    Plan P{};
    P.n_mo = s->n_mo;
    P.n_occ = s->n_occ;
    P.n_virt = s->n_mo - s->n_occ;
    P.n_aux = s->n_aux;
    P.S = s->n_states;
    P.n_freq = p->n_freq;
    P.n_im = p->n_ref_im;
    P.n_re = p->n_ref_re;
    P.n_pts = P.n_im + P.n_re;
    P.prec = p->prec;
    // imaginary nodes with a plane
    std::vector<int> node, rest;
    std::vector<double> T;
    double om_lo = 0.0, om_hi = 0.0;
    if (allow_id && P.prec != CDWAC_P64 && p->freq_rank_tol > 0.0 && P.n_freq >= 4) {
        // transition energies span [min virt - max occ, max - min] (the
        // energies need not be sorted inside a block, e.g. QP energies of evGW)
        const double* e = s->eps;
        om_lo = *std::min_element(e + s->n_occ, e + s->n_mo) - *std::max_element(e, e + s->n_occ);
        om_hi = kOmegaHiFactor * (*std::max_element(e, e + s->n_mo) - *std::min_element(e, e + s->n_mo));
        FreqId fid;
        if (freq_id(p->freq, P.n_freq, om_lo, om_hi, p->freq_rank_tol, fid)) {
            node = fid.skel;
            rest = fid.rest;
            T = fid.T;
        }
    }
    if (node.empty())
        for (int f = 0; f < P.n_freq; ++f) node.push_back(f);
    P.n_imp = (int)node.size();
    P.n_f = P.n_imp + 2 * P.n_re;
    P.K = (int64_t)P.n_occ * P.n_virt;
    P.kpad = round_up(P.K, 32);
    P.npad = (int)round_up(P.n_aux, kGemmRows);
    P.nblk = P.npad / kNb;
    P.cpad = (int)round_up((int64_t)P.S * P.n_mo, kGemmCols);
    P.ni = w_partial_blocks(P.prec, P.npad);
    // fit list
    std::vector<int> m0(P.S), m1(P.S), off(P.S), fs, fm;
    for (int j = 0; j < P.S; ++j) {
        if (p->fit_all) {
            m0[j] = 0;
            m1[j] = P.n_mo;
        } else {
            fit_range(s->eps, P.n_mo, P.n_occ, p->win_lo[j] - kFitMargin, p->win_hi[j] + kFitMargin, m0[j], m1[j]);
        }
        off[j] = (int)fs.size();
        for (int m = m0[j]; m < m1[j]; ++m) {
            fs.push_back(j);
            fm.push_back(m);
        }
    }
    P.n_fit = (int)fs.size();
    P.cfpad = (int)round_up(std::max(P.n_fit, 1), kGemmCols);
    if (hs) {
        hs->node = node;
        hs->rest = rest;
        hs->T = T;
        hs->omega_lo = om_lo;
        hs->omega_hi = om_hi;
        hs->m0 = m0;
        hs->m1 = m1;
        hs->fit_off = off;
        hs->fit_s = fs;
        hs->fit_m = fm;
    }
    const bool f64 = P.prec == CDWAC_P64;
    P.nr64 = !f64 && p->near_real_f64 && P.n_re > 0;
    const int64_t n2 = (int64_t)P.npad * P.npad;
    const int64_t blk = (int64_t)kNb * kNb;
    // persistent
    add(P, P.eps, sizeof(double) * P.n_mo);
    add(P, P.eps_g, sizeof(double) * P.n_mo);
    add(P, P.freq, sizeof(double) * P.n_freq);
    add(P, P.weight, sizeof(double) * P.n_freq);
    add(P, P.ref_re, sizeof(double) * std::max(P.n_re, 1));
    add(P, P.ref_im, sizeof(int) * std::max(P.n_im, 1));
    add(P, P.state_idx, sizeof(int) * P.S);
    add(P, P.vxc, sizeof(double) * P.S);
    add(P, P.sigx, sizeof(double) * P.S);
    add(P, P.win_lo, sizeof(double) * P.S);
    add(P, P.win_hi, sizeof(double) * P.S);
    add(P, P.m0, sizeof(int) * P.S);
    add(P, P.m1, sizeof(int) * P.S);
    add(P, P.fit_off, sizeof(int) * P.S);
    add(P, P.fit_s, sizeof(int) * std::max(P.n_fit, 1));
    add(P, P.fit_m, sizeof(int) * std::max(P.n_fit, 1));
    add(P, P.w_im, sizeof(double) * (size_t)P.S * P.n_mo * P.n_freq);
    add(P, P.w_re, sizeof(double) * 2 * (size_t)std::max(P.n_fit, 1) * std::max(P.n_re, 1));
    add(P, P.coef, sizeof(double) * 2 * (size_t)std::max(P.n_fit, 1) * P.n_pts);
    add(P, P.node, sizeof(double) * 2 * (size_t)std::max(P.n_fit, 1) * P.n_pts);
    add(P, P.nterm, sizeof(int) * std::max(P.n_fit, 1));
    add(P, P.qpout, sizeof(QpOut) * P.S);
    // G_dH W0: evaluation points eps_n, Sigma_n(eps_n), shifts dH_n
    add(P, P.hedin, sizeof(double) * 3 * (size_t)P.S);
    // W at a_m = 0 of every fit (analytic limit of the integral term)
    add(P, P.w0, sizeof(double) * std::max(P.n_fit, 1));
    add(P, P.err, sizeof(int) * 4);
    // transient
    add(P, P.zr, sizeof(double) * P.n_f);
    add(P, P.zi, sizeof(double) * P.n_f);
    add(P, P.part, sizeof(int) * P.n_f);
    add(P, P.idflag, sizeof(int) * P.n_f);
    add(P, P.pmap, sizeof(int) * P.n_f);
    add(P, P.imnode, sizeof(int) * P.n_freq);
    add(P, P.imrest, sizeof(int) * P.n_freq);
    add(P, P.tmat, sizeof(double) * (size_t)P.n_freq * P.n_freq);
    add(P, P.rowsum, sizeof(double) * P.npad);
    // residual check of the inversions: sampled columns of every plane of eps
    add(P, P.fcols, sizeof(double) * (size_t)P.n_f * kFactCols * P.npad);
    add(P, P.fcolidx, sizeof(int) * kFactCols);
    add(P, P.fres, sizeof(unsigned long long) * 2 * (size_t)(P.n_imp + P.n_re) * kFactCols);
    // operand maxima: [0] |O^ia|, [1] |O^nm|, [2..2+F) |c_f|, [2+F..2+2F) |Lambda_f|
    add(P, P.amax, sizeof(uint32_t) * (2 + 2 * (size_t)P.n_f));
    // scales: [0] x, [1] B, cfac[F], pi_unscale[F], lam_scale[F], w_unscale[F]
    add(P, P.sf, sizeof(double) * (2 + 4 * (size_t)P.n_f));
    add(P, P.cw, (f64 ? sizeof(double) : sizeof(float)) * (size_t)P.n_f * P.kpad);
    add(P, P.cw64, P.nr64 ? sizeof(double) * (size_t)P.n_f * P.kpad : 0);
    if (f64 || P.nr64) add(P, P.x64, sizeof(double) * (size_t)P.npad * P.kpad);
    if (!f64) {
        // one-product Pi (CDWAC_F16) needs no lo planes of X and Y
        const size_t n_pl = P.prec == CDWAC_F16 ? 1 : 2;
        add(P, P.xh, sizeof(uint16_t) * (size_t)P.npad * P.kpad);
        add(P, P.xl, n_pl == 2 ? sizeof(uint16_t) * (size_t)P.npad * P.kpad : 0);
        add(P, P.x32, sizeof(float) * (size_t)P.npad * P.kpad);
        // prescaled operands X diag(c_f) for a batch of nb weight vectors
        const size_t per_f = sizeof(uint16_t) * (size_t)P.npad * P.kpad;
        P.nb = (int)std::max<size_t>(1, std::min<size_t>(P.n_f, kPrescaleBudget / (n_pl * per_f)));
        add(P, P.yh, per_f * P.nb);
        add(P, P.yl, n_pl == 2 ? per_f * P.nb : 0);
        P.n_tpi = pi_tile_count(P.npad);
        P.n_tw = (int)w_tiles(P.npad, P.cpad).size();
        P.n_twf = (int)w_tiles(P.npad, P.cfpad).size();
        // work lists of a full batch and of the last one, each padded by at
        // most 8 rounds of one tile per CU (up to 128 CUs per XCD)
        add(P, P.t_pi, sizeof(int2) * 2 * ((size_t)P.nb * P.n_tpi + kPiListPad));
        add(P, P.t_w, sizeof(int2) * P.n_tw);
        add(P, P.t_wf, sizeof(int2) * P.n_twf);
    }
    add(P, P.E, sizeof(double) * (size_t)P.n_f * n2);
    // real planes: sweeps with 128-wide pivots (64 x 128 panel blocks, and a
    // 128 x 128 copy of each pivot block, swept with 64-wide pivots for its
    // inverse); complex planes: 64-wide pivots
    add(P, P.dinv_r, sizeof(double) * (size_t)std::max(P.n_imp, 1) * blk);
    add(P, P.pbuf_r, sizeof(double) * 2 * (size_t)P.n_imp * P.nblk * blk);
    add(P, P.qbuf_r, sizeof(double) * 2 * (size_t)P.n_imp * P.nblk * blk);
    add(P, P.dinv_c, sizeof(double) * 2 * (size_t)std::max(P.n_re, 1) * blk);
    add(P, P.pbuf_c, sizeof(double) * 2 * (size_t)P.n_re * P.nblk * blk);
    add(P, P.qbuf_c, sizeof(double) * 2 * (size_t)P.n_re * P.nblk * blk);
    add(P, P.dscr_r, sizeof(double) * 4 * (size_t)std::max(P.n_imp, 1) * blk);
    if (!f64) {
        add(P, P.lh, sizeof(uint16_t) * (size_t)P.n_f * n2);
        add(P, P.ll, sizeof(uint16_t) * (size_t)P.n_f * n2);
    }
    add(P, P.bt64, sizeof(double) * (size_t)P.cpad * P.npad);
    add(P, P.bf64, sizeof(double) * (size_t)P.cfpad * P.npad);
    if (!f64) {
        add(P, P.bh, sizeof(uint16_t) * (size_t)P.cpad * P.npad);
        add(P, P.bl, sizeof(uint16_t) * (size_t)P.cpad * P.npad);
        add(P, P.bfh, sizeof(uint16_t) * (size_t)P.cfpad * P.npad);
        add(P, P.bfl, sizeof(uint16_t) * (size_t)P.cfpad * P.npad);
    }
    add(P, P.partial_im, sizeof(double) * (size_t)P.n_imp * P.ni * P.cpad);
    add(P, P.partial_re, sizeof(double) * 2 * (size_t)std::max(P.n_re, 1) * P.ni * P.cfpad);
    add(P, P.rowsel, sizeof(int) * std::max(P.n_fit, 1));
    add(P, P.ref_u, sizeof(double) * 2 * (size_t)std::max(P.n_fit, 1) * P.n_pts);
    add(P, P.ref_w, sizeof(double) * 2 * (size_t)std::max(P.n_fit, 1) * P.n_pts);
    return P;
}

template <typename T>
T* at(cdwac_ctx* c, const Region& r) {
    return reinterpret_cast<T*>(c->ws + r.off);
}

int ensure_workspace(cdwac_ctx* ctx, size_t bytes) {
    if (ctx->ws_user) {
        if (ctx->ws_user_bytes < bytes)
            return fail(ctx, CDWAC_ENOMEM, "workspace too small: %zu bytes given, %zu needed", ctx->ws_user_bytes,
                        bytes);
        ctx->ws = (char*)ctx->ws_user;
        return CDWAC_OK;
    }
    if (ctx->ws_own_bytes < bytes) {
        if (ctx->ws_own) {
            HIPCK(hipStreamSynchronize(ctx->stream));
            HIPCK(hipFree(ctx->ws_own));
            ctx->ws_own = nullptr;
            ctx->ws_own_bytes = 0;
        }
        if (hipMalloc(&ctx->ws_own, bytes) != hipSuccess) {
            ctx->ws_own = nullptr;
            (void)hipGetLastError();
            return fail(ctx, CDWAC_ENOMEM, "cannot allocate %zu bytes of workspace", bytes);
        }
        ctx->ws_own_bytes = bytes;
    }
    ctx->ws = (char*)ctx->ws_own;
    return CDWAC_OK;
}

template <typename T>
int upload(cdwac_ctx* ctx, T* dst, const T* src, size_t n) {
    if (n == 0) return CDWAC_OK;
    HIPCK(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyHostToDevice, ctx->stream));
    return CDWAC_OK;
}

#define TRY(x)                       \
    do {                             \
        int r_ = (x);                \
        if (r_ != CDWAC_OK) return r_; \
    } while (0)

// Takes an event from the context's pool (handles are copied out: the pool
// vector may reallocate when it grows).
int next_event(cdwac_ctx* ctx, hipEvent_t* out) {
    if (ctx->pool_used == ctx->pool.size()) {
        hipEvent_t e;
        HIPCK(hipEventCreate(&e));
        ctx->pool.push_back(e);
    }
    *out = ctx->pool[ctx->pool_used++];
    return CDWAC_OK;
}

// Opens a timed segment of `stage` (closed by seg_end) when timing is on.
int seg_begin(cdwac_ctx* ctx, int stage) {
    if (!ctx->timing) return CDWAC_OK;
    hipEvent_t a, b;
    TRY(next_event(ctx, &a));
    TRY(next_event(ctx, &b));
    HIPCK(hipEventRecord(a, ctx->stream));
    ctx->segs.push_back({stage, a, b});
    return CDWAC_OK;
}

int seg_end(cdwac_ctx* ctx) {
    if (!ctx->timing) return CDWAC_OK;
    HIPCK(hipEventRecord(ctx->segs.back().b, ctx->stream));
    return CDWAC_OK;
}

// After the stream has synchronised: adds every segment to its stage total.
int seg_collect(cdwac_ctx* ctx) {
    for (auto& g : ctx->segs) {
        float ms = 0.f;
        HIPCK(hipEventElapsedTime(&ms, g.a, g.b));
        ctx->stage_ms[g.stage] += ms;
        ctx->stage_n[g.stage] += 1;
    }
    ctx->segs.clear();
    ctx->pool_used = 0;
    return CDWAC_OK;
}

QpArgs qp_args(cdwac_ctx* c) {
    const Plan& P = c->plan;
    QpArgs a{};
    a.n_mo = P.n_mo;
    a.n_states = P.S;
    a.n_freq = P.n_freq;
    a.n_pts = P.n_pts;
    a.eps = at<double>(c, P.eps_g);
    a.eps_n = at<double>(c, P.eps);
    a.freq = at<double>(c, P.freq);
    a.weight = at<double>(c, P.weight);
    a.w_im = at<double>(c, P.w_im);
    a.coef = at<double>(c, P.coef);
    a.node = at<double>(c, P.node);
    a.nterm = at<int>(c, P.nterm);
    a.fit_off = at<int>(c, P.fit_off);
    a.m0 = at<int>(c, P.m0);
    a.m1 = at<int>(c, P.m1);
    a.state_idx = at<int>(c, P.state_idx);
    a.sigx = at<double>(c, P.sigx);
    a.vxc = at<double>(c, P.vxc);
    a.win_lo = at<double>(c, P.win_lo);
    a.win_hi = at<double>(c, P.win_hi);
    a.eta = c->hs.eta;
    a.eps_f = c->hs.eps_f;
    a.qp_tol = c->hs.qp_tol;
    a.qp_maxit = c->hs.qp_maxit;
    a.use_mlp = c->hs.use_mlp;
    a.mlp_accept = c->hs.mlp_accept;
    a.mlp_theta = c->mlp_theta;
    for (int i = 0; i < 8; ++i) {
        a.mlp_mu[i] = c->mlp_mu[i];
        a.mlp_sd[i] = c->mlp_sd[i];
    }
    a.mlp_out_mu = c->mlp_out_mu;
    a.mlp_out_sd = c->mlp_out_sd;
    a.w0 = c->hs.quad_limit ? at<double>(c, P.w0) : nullptr;
    return a;
}

}  // namespace

extern "C" {

int cdwac_ctx_create(cdwac_ctx** out, int device, void* hip_stream) {
    if (!out) return CDWAC_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return CDWAC_EINVAL;
    cdwac_ctx* ctx = new cdwac_ctx();
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    if (hipSetDevice(device) != hipSuccess || hipMalloc(&ctx->mlp_theta, sizeof(float) * kMlpParams) != hipSuccess ||
        hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->join, hipEventDisableTiming) != hipSuccess ||
        hipDeviceGetAttribute(&ctx->n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        ctx->n_cu < 1 || scratch_address(device, (void**)&ctx->scratch) != hipSuccess || !ctx->scratch) {
        if (ctx->mlp_theta) (void)hipFree(ctx->mlp_theta);
        if (ctx->side) (void)hipStreamDestroy(ctx->side);
        if (ctx->fork) (void)hipEventDestroy(ctx->fork);
        delete ctx;
        return CDWAC_EHIP;
    }
    *out = ctx;
    return CDWAC_OK;
}

void cdwac_ctx_destroy(cdwac_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->ws_own) (void)hipFree(ctx->ws_own);
    for (auto& e : ctx->pool) (void)hipEventDestroy(e);
    if (ctx->mlp_theta) (void)hipFree(ctx->mlp_theta);
    if (ctx->mlp_scratch) (void)hipFree(ctx->mlp_scratch);
    if (ctx->batch) (void)hipFree(ctx->batch);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    if (ctx->fork) (void)hipEventDestroy(ctx->fork);
    if (ctx->join) (void)hipEventDestroy(ctx->join);
    delete ctx;
}

const char* cdwac_last_error(const cdwac_ctx* ctx) { return ctx ? ctx->err.c_str() : "NULL context"; }

size_t cdwac_workspace_bytes(const cdwac_system* sys, const cdwac_params* prm) {
    if (validate_system(nullptr, sys) != CDWAC_OK || validate_params(nullptr, sys, prm) != CDWAC_OK) return 0;
    return make_plan(sys, prm, nullptr).total;
}

int cdwac_set_workspace(cdwac_ctx* ctx, void* dev_ptr, size_t bytes) {
    if (!ctx) return CDWAC_EINVAL;
    if (dev_ptr && ((uintptr_t)dev_ptr % 256) != 0) return fail(ctx, CDWAC_EINVAL, "workspace must be 256-byte aligned");
    ctx->ws_user = dev_ptr;
    ctx->ws_user_bytes = dev_ptr ? bytes : 0;
    ctx->prepared = false;
    return CDWAC_OK;
}

namespace {
// Destination of a batched preparation's fit inputs: the reference data of the
// system's fits go to u, w (fits are then left to one launch for the batch).
struct FitSink {
    double* u = nullptr;
    double* w = nullptr;
};
int prepare_impl(cdwac_ctx* ctx, const cdwac_system* sys, const cdwac_params* prm, bool allow_id,
                 const FitSink* sink = nullptr);
}

int cdwac_prepare(cdwac_ctx* ctx, const cdwac_system* sys, const cdwac_params* prm) {
    if (!ctx) return CDWAC_EINVAL;
    ctx->prepared = false;
    TRY(validate_system(ctx, sys));
    TRY(validate_params(ctx, sys, prm));
    if (prm->use_mlp_seed && !ctx->have_mlp) return fail(ctx, CDWAC_EINVAL, "use_mlp_seed set but no model installed");
    return prepare_impl(ctx, sys, prm, true);
}

namespace {
int prepare_impl(cdwac_ctx* ctx, const cdwac_system* sys, const cdwac_params* prm, bool allow_id,
                 const FitSink* sink) {
    HIPCK(hipSetDevice(ctx->device));
    HostState hs;
    Plan P = make_plan(sys, prm, &hs, allow_id);
    const bool use_id = !hs.rest.empty();
    TRY(ensure_workspace(ctx, P.total));
    ctx->plan = P;
    hipStream_t st = ctx->stream;
    const bool f64 = P.prec == CDWAC_P64;
    const int64_t n2 = (int64_t)P.npad * P.npad;

    // host state
    hs.state_idx.assign(sys->state_idx, sys->state_idx + P.S);
    hs.eps.assign(sys->eps, sys->eps + P.n_mo);
    hs.win_lo.assign(prm->win_lo, prm->win_lo + P.S);
    hs.win_hi.assign(prm->win_hi, prm->win_hi + P.S);
    hs.eps_f = std::isnan(sys->eps_fermi) ? 0.5 * (sys->eps[P.n_occ - 1] + sys->eps[P.n_occ]) : sys->eps_fermi;
    hs.eta = prm->eta;
    hs.qp_tol = prm->qp_tol;
    hs.qp_maxit = prm->qp_maxit;
    hs.use_mlp = prm->use_mlp_seed;
    hs.mlp_accept = prm->mlp_accept;
    hs.vxc_is_sigx = sys->vxc == nullptr;
    hs.fit_all = prm->fit_all != 0;
    hs.quad_limit = prm->quad_limit != 0;
    if (sys->vxc) hs.vxc.assign(sys->vxc, sys->vxc + P.S);

    // weight vectors: imaginary nodes, then (Re, Im) of every near-real point
    std::vector<double> zr(P.n_f), zi(P.n_f);
    std::vector<int> part(P.n_f), idf(P.n_f);
    for (int k = 0; k < P.n_imp; ++k) {
        zr[k] = 0.0;
        zi[k] = prm->freq[hs.node[k]];
        part[k] = 0;
        idf[k] = 1;
    }
    for (int j = 0; j < P.n_re; ++j)
        for (int q = 0; q < 2; ++q) {
            int f = P.n_imp + 2 * j + q;
            zr[f] = prm->ref_re[j];
            zi[f] = prm->eta_ref;
            part[f] = q;
            idf[f] = q == 0;
        }
    std::vector<int> rowsel(std::max(P.n_fit, 1), 0);
    for (int f = 0; f < P.n_fit; ++f) rowsel[f] = hs.fit_s[f] * P.n_mo + hs.fit_m[f];

    TRY(upload(ctx, at<double>(ctx, P.eps), sys->eps, P.n_mo));
    TRY(upload(ctx, at<double>(ctx, P.eps_g), sys->eps, P.n_mo));
    TRY(upload(ctx, at<double>(ctx, P.freq), prm->freq, P.n_freq));
    TRY(upload(ctx, at<double>(ctx, P.weight), prm->weight, P.n_freq));
    if (P.n_re) TRY(upload(ctx, at<double>(ctx, P.ref_re), prm->ref_re, P.n_re));
    if (P.n_im) TRY(upload(ctx, at<int>(ctx, P.ref_im), prm->ref_im_idx, P.n_im));
    TRY(upload(ctx, at<int>(ctx, P.state_idx), sys->state_idx, P.S));
    TRY(upload(ctx, at<double>(ctx, P.win_lo), prm->win_lo, P.S));
    TRY(upload(ctx, at<double>(ctx, P.win_hi), prm->win_hi, P.S));
    TRY(upload(ctx, at<int>(ctx, P.m0), hs.m0.data(), P.S));
    TRY(upload(ctx, at<int>(ctx, P.m1), hs.m1.data(), P.S));
    TRY(upload(ctx, at<int>(ctx, P.fit_off), hs.fit_off.data(), P.S));
    if (P.n_fit) {
        TRY(upload(ctx, at<int>(ctx, P.fit_s), hs.fit_s.data(), P.n_fit));
        TRY(upload(ctx, at<int>(ctx, P.fit_m), hs.fit_m.data(), P.n_fit));
    }
    TRY(upload(ctx, at<int>(ctx, P.rowsel), rowsel.data(), rowsel.size()));
    TRY(upload(ctx, at<double>(ctx, P.zr), zr.data(), P.n_f));
    TRY(upload(ctx, at<double>(ctx, P.zi), zi.data(), P.n_f));
    TRY(upload(ctx, at<int>(ctx, P.part), part.data(), P.n_f));
    TRY(upload(ctx, at<int>(ctx, P.idflag), idf.data(), P.n_f));
    std::vector<int> pmap(P.n_f);
    for (int f = 0; f < P.n_f; ++f) pmap[f] = f;
    TRY(upload(ctx, at<int>(ctx, P.pmap), pmap.data(), pmap.size()));
    TRY(upload(ctx, at<int>(ctx, P.imnode), hs.node.data(), hs.node.size()));
    if (use_id) {
        TRY(upload(ctx, at<int>(ctx, P.imrest), hs.rest.data(), hs.rest.size()));
        TRY(upload(ctx, at<double>(ctx, P.tmat), hs.T.data(), hs.T.size()));
        HIPCK(hipMemsetAsync(at<double>(ctx, P.rowsum), 0, sizeof(double) * P.npad, st));
    }
    int* err = at<int>(ctx, P.err);
    HIPCK(hipMemsetAsync(err, 0, sizeof(int) * 4, st));
    for (double& x : ctx->stage_ms) x = 0.0;
    for (int32_t& x : ctx->stage_n) x = 0;
    ctx->segs.clear();
    ctx->pool_used = 0;

    // (a0) staging: weights, operand maxima and scales, the O^{ia} operand
    TRY(seg_begin(ctx, 0));
    const int et = prec_elem(P.prec);
    const bool pi_split = P.prec != CDWAC_F16;
    uint32_t* amax = at<uint32_t>(ctx, P.amax);
    double* sf = at<double>(ctx, P.sf);
    double* pi_unscale = sf + 2 + P.n_f;
    double* lam_scale = sf + 2 + 2 * P.n_f;
    double* w_unscale = sf + 2 + 3 * P.n_f;
    HIPCK(hipMemsetAsync(amax, 0, sizeof(uint32_t) * (2 + 2 * (size_t)P.n_f), st));
    launch_absmax(st, sys->o_ia, P.K, P.n_aux, P.K, amax, err);
    launch_absmax(st, sys->o_nm, P.n_mo, P.S * P.n_aux, P.n_mo, amax + 1, err);
    launch_weights(st, at<double>(ctx, P.eps), P.n_occ, P.n_virt, sys->spin, at<double>(ctx, P.zr),
                   at<double>(ctx, P.zi), at<int>(ctx, P.part), P.n_f, P.kpad,
                   f64 ? at<double>(ctx, P.cw) : (P.nr64 ? at<double>(ctx, P.cw64) : nullptr),
                   f64 ? nullptr : at<float>(ctx, P.cw), amax + 2);
    LAUNCHCK();
    if (f64 || P.nr64) launch_pad_f64(st, sys->o_ia, P.K, P.n_aux, P.K, at<double>(ctx, P.x64), P.npad, P.kpad);
    if (!f64) {
        launch_scales_pi(st, amax, P.n_f, sf);
        launch_split_panel(st, et, sys->o_ia, 0, 1, P.K, P.n_aux, P.K, sf, at<uint16_t>(ctx, P.xh),
                           pi_split ? at<uint16_t>(ctx, P.xl) : nullptr, at<float>(ctx, P.x32), P.npad, P.kpad);
        std::vector<int2> tw = w_tiles(P.npad, P.cpad), twf = w_tiles(P.npad, P.cfpad);
        TRY(upload(ctx, at<int2>(ctx, P.t_w), tw.data(), tw.size()));
        TRY(upload(ctx, at<int2>(ctx, P.t_wf), twf.data(), twf.size()));
    }
    LAUNCHCK();
    TRY(seg_end(ctx));
    // (a1) eps_f = I - Pi_f for every weight vector
    if (f64) {
        TRY(seg_begin(ctx, 1));
        launch_pi_f64(st, P.npad, P.kpad, P.n_f, at<double>(ctx, P.x64), at<double>(ctx, P.cw), at<int>(ctx, P.idflag),
                      at<double>(ctx, P.E));
        LAUNCHCK();
        TRY(seg_end(ctx));
    } else {
        const int* pm = at<int>(ctx, P.pmap);
        const int n_pi16 = P.nr64 ? P.n_imp : P.n_f;   // planes on the 16-bit path
        const int per_batch = pi_batch_size(n_pi16, P.nb, P.n_tpi, ctx->n_cu);
        // work lists of a full batch and of the last batch (kept in the context
        // until the next prepare, as the source of the asynchronous upload)
        const int cu_x = std::max(1, ctx->n_cu / 8);
        const int last = n_pi16 - per_batch * ((n_pi16 - 1) / per_batch);
        ctx->pi_work[0] = pi_worklist(P.npad, per_batch, cu_x);
        ctx->pi_work[1] = last != per_batch ? pi_worklist(P.npad, last, cu_x) : std::vector<int2>();
        const size_t cap = (size_t)P.nb * P.n_tpi + kPiListPad;
        if (ctx->pi_work[0].size() > cap || ctx->pi_work[1].size() > cap)
            return fail(ctx, CDWAC_EINVAL, "polarizability work list exceeds its buffer (more than 128 CUs per XCD)");
        int2* wl = at<int2>(ctx, P.t_pi);
        TRY(upload(ctx, wl, ctx->pi_work[0].data(), ctx->pi_work[0].size()));
        TRY(upload(ctx, wl + cap, ctx->pi_work[1].data(), ctx->pi_work[1].size()));
        for (int f0 = 0; f0 < n_pi16; f0 += per_batch) {
            const int nfb = std::min(per_batch, n_pi16 - f0);
            const int li = nfb == per_batch ? 0 : 1;
            TRY(seg_begin(ctx, 7));
            launch_prescale(st, et, at<float>(ctx, P.x32), P.npad, P.kpad, at<float>(ctx, P.cw), sf + 2, pm + f0, nfb,
                            at<uint16_t>(ctx, P.yh), pi_split ? at<uint16_t>(ctx, P.yl) : nullptr);
            LAUNCHCK();
            TRY(seg_end(ctx));
            TRY(seg_begin(ctx, 1));
            launch_pi_gemm(st, P.prec, P.npad, P.kpad, pm + f0, at<uint16_t>(ctx, P.xh),
                           at<uint16_t>(ctx, pi_split ? P.xl : P.xh), at<uint16_t>(ctx, P.yh),
                           at<uint16_t>(ctx, pi_split ? P.yl : P.yh), wl + li * cap, (int)ctx->pi_work[li].size(),
                           pi_unscale, at<int>(ctx, P.idflag), at<double>(ctx, P.E));
            LAUNCHCK();
            TRY(seg_end(ctx));
        }
        if (P.nr64) {
            TRY(seg_begin(ctx, 1));
            launch_pi_f64(st, P.npad, P.kpad, 2 * P.n_re, at<double>(ctx, P.x64),
                          at<double>(ctx, P.cw64) + (size_t)P.n_imp * P.kpad, at<int>(ctx, P.idflag) + P.n_imp,
                          at<double>(ctx, P.E) + (size_t)P.n_imp * n2);
            LAUNCHCK();
            TRY(seg_end(ctx));
        }
    }
    if (use_id) {
        // Gershgorin bound of -Pi at the largest node (always a skeleton node),
        // for the check of the assumed excitation range
        const int fslot = (int)(std::max_element(hs.node.begin(), hs.node.end(),
                                                 [&](int a, int b) { return prm->freq[a] < prm->freq[b]; }) -
                                hs.node.begin());
        launch_rowabs(st, at<double>(ctx, P.E) + (int64_t)fslot * n2, P.npad, at<double>(ctx, P.rowsum));
        LAUNCHCK();
    }
    // (a2) eps^-1 by blocked sweeps, Lambda = eps^-1 - I
    TRY(seg_begin(ctx, 2));
    {
        // columns of eps kept for the residual check of the inverses
        int cols[kFactCols];
        for (int c = 0; c < kFactCols; ++c) cols[c] = (int)((int64_t)c * (P.n_aux - 1) / (kFactCols - 1));
        TRY(upload(ctx, at<int>(ctx, P.fcolidx), cols, kFactCols));
        HIPCK(hipMemsetAsync(at<unsigned long long>(ctx, P.fres), 0, P.fres.bytes, st));
        launch_fact_gather(st, at<double>(ctx, P.E), P.npad, P.n_f, at<int>(ctx, P.fcolidx), at<double>(ctx, P.fcols));
        LAUNCHCK();
    }
    if (P.n_re > 0) {
        // the complex planes on the second stream, with 64-wide pivots (eps is
        // complex symmetric and indefinite there and no pivoting is done, so
        // the smaller pivot blocks keep the element growth down); their small
        // per-step kernels overlap the real planes' updates and vice versa
        HIPCK(hipEventRecord(ctx->fork, st));
        HIPCK(hipStreamWaitEvent(ctx->side, ctx->fork, 0));
        // (16-bit modes: complex products in three real ones, whose rounding
        // stays far below the error the 16-bit contraction leaves in eps)
        launch_sweep(ctx->side, at<double>(ctx, P.E), P.npad, 0, P.n_re, P.n_imp, at<double>(ctx, P.dinv_r),
                     at<double>(ctx, P.pbuf_r), at<double>(ctx, P.qbuf_r), at<double>(ctx, P.dinv_c),
                     at<double>(ctx, P.pbuf_c), at<double>(ctx, P.qbuf_c), err, !f64);
        LAUNCHCK();
    }
    // the real (positive definite) planes with 128-wide pivots
    launch_sweep2(st, at<double>(ctx, P.E), P.npad, P.n_imp, 0, P.n_imp, at<double>(ctx, P.dscr_r), nullptr,
                  at<double>(ctx, P.dinv_r), at<double>(ctx, P.pbuf_r), at<double>(ctx, P.qbuf_r), nullptr, nullptr,
                  nullptr, err);
    LAUNCHCK();
    if (P.n_re > 0) {
        HIPCK(hipEventRecord(ctx->join, ctx->side));
        HIPCK(hipStreamWaitEvent(st, ctx->join, 0));
    }
    TRY(seg_end(ctx));
    TRY(seg_begin(ctx, 3));
    launch_finalize_lambda(st, at<double>(ctx, P.E), P.npad, P.n_f, at<int>(ctx, P.idflag),
                           f64 ? nullptr : amax + 2 + P.n_f);
    LAUNCHCK();
    launch_fact_residual(st, at<double>(ctx, P.E), P.npad, P.n_imp, P.n_re, P.n_imp, at<int>(ctx, P.fcolidx),
                         at<double>(ctx, P.fcols), at<unsigned long long>(ctx, P.fres));
    LAUNCHCK();
    if (!f64) {
        launch_scales_w(st, amax + 2 + P.n_f, P.n_f, sf, lam_scale, w_unscale);
        launch_split_panel(st, et, at<double>(ctx, P.E), (int64_t)P.npad * P.npad, P.n_f, P.npad, P.npad, P.npad,
                           lam_scale, at<uint16_t>(ctx, P.lh), at<uint16_t>(ctx, P.ll), nullptr, P.npad, P.npad);
        LAUNCHCK();
    }
    TRY(seg_end(ctx));
    // (a3) W^c_nm: all (n, m) at the imaginary nodes, fitted (n, m) at the near-real points
    TRY(seg_begin(ctx, 4));
    const double* bscale = f64 ? nullptr : sf + 1;
    launch_transpose_b(st, et, sys->o_nm, P.S, P.n_aux, P.n_mo, nullptr, P.S * P.n_mo, bscale, at<double>(ctx, P.bt64),
                       f64 ? nullptr : at<uint16_t>(ctx, P.bh), f64 ? nullptr : at<uint16_t>(ctx, P.bl), P.cpad,
                       P.npad, nullptr, err);
    LAUNCHCK();
    if (P.n_re > 0 && P.n_fit > 0) {
        launch_transpose_b(st, et, sys->o_nm, P.S, P.n_aux, P.n_mo, at<int>(ctx, P.rowsel), P.n_fit, bscale,
                           at<double>(ctx, P.bf64), f64 ? nullptr : at<uint16_t>(ctx, P.bfh),
                           f64 ? nullptr : at<uint16_t>(ctx, P.bfl), P.cfpad, P.npad, nullptr, err);
        LAUNCHCK();
    }
    launch_w(st, P.prec, P.npad, 0, P.n_imp, at<double>(ctx, P.E), f64 ? nullptr : at<uint16_t>(ctx, P.lh),
             f64 ? nullptr : at<uint16_t>(ctx, P.ll), at<double>(ctx, P.bt64), f64 ? nullptr : at<uint16_t>(ctx, P.bh),
             f64 ? nullptr : at<uint16_t>(ctx, P.bl), P.cpad, f64 ? nullptr : at<int2>(ctx, P.t_w), P.n_tw, w_unscale,
             at<double>(ctx, P.partial_im));
    LAUNCHCK();
    if (P.n_re > 0 && P.n_fit > 0) {
        launch_w(st, P.prec, P.npad, P.n_imp, 2 * P.n_re, at<double>(ctx, P.E),
                 f64 ? nullptr : at<uint16_t>(ctx, P.lh), f64 ? nullptr : at<uint16_t>(ctx, P.ll),
                 at<double>(ctx, P.bf64), f64 ? nullptr : at<uint16_t>(ctx, P.bfh),
                 f64 ? nullptr : at<uint16_t>(ctx, P.bfl), P.cfpad, f64 ? nullptr : at<int2>(ctx, P.t_wf), P.n_twf,
                 w_unscale, at<double>(ctx, P.partial_re));
        LAUNCHCK();
    }
    launch_reduce_w(st, at<double>(ctx, P.partial_im), at<double>(ctx, P.partial_re), P.ni, P.cpad, P.cfpad,
                    P.n_imp, at<int>(ctx, P.imnode), P.n_freq, P.n_re, P.S * P.n_mo, P.n_re > 0 ? P.n_fit : 0,
                    at<double>(ctx, P.w_im), at<double>(ctx, P.w_re));
    LAUNCHCK();
    if (use_id) {
        launch_interp_w(st, at<double>(ctx, P.w_im), P.n_freq, P.S * P.n_mo, P.n_imp, at<int>(ctx, P.imnode),
                        (int)hs.rest.size(), at<int>(ctx, P.imrest), at<double>(ctx, P.tmat));
        LAUNCHCK();
    }
    TRY(seg_end(ctx));
    // (a4) Sigma^x and v^xc
    TRY(seg_begin(ctx, 5));
    launch_exchange(st, sys->o_nm, P.S, P.n_aux, P.n_mo, P.n_occ, at<double>(ctx, P.sigx));
    LAUNCHCK();
    if (sys->vxc) TRY(upload(ctx, at<double>(ctx, P.vxc), sys->vxc, P.S));
    else HIPCK(hipMemcpyAsync(at<double>(ctx, P.vxc), at<double>(ctx, P.sigx), sizeof(double) * P.S,
                              hipMemcpyDeviceToDevice, st));
    // (a5) greedy Thiele fits over F_wac
    if (P.n_fit > 0) {
        double* ru = sink ? sink->u : at<double>(ctx, P.ref_u);
        double* rw = sink ? sink->w : at<double>(ctx, P.ref_w);
        launch_gather_refs(st, P.n_fit, at<int>(ctx, P.fit_s), at<int>(ctx, P.fit_m), P.n_mo, P.n_freq,
                           at<double>(ctx, P.w_im), at<double>(ctx, P.w_re), at<double>(ctx, P.freq),
                           at<int>(ctx, P.ref_im), P.n_im, at<double>(ctx, P.ref_re), P.n_re, prm->eta_ref, ru, rw);
        LAUNCHCK();
        if (!sink) {
            launch_thiele_fit(st, P.n_fit, P.n_pts, ru, rw, prm->pade_tol, at<double>(ctx, P.coef),
                              at<double>(ctx, P.node), at<int>(ctx, P.nterm));
            LAUNCHCK();
            if (hs.quad_limit) {
                launch_w0_from_fits(st, P.n_fit, P.n_pts, at<double>(ctx, P.coef), at<double>(ctx, P.node),
                                    at<int>(ctx, P.nterm), prm->eta, at<double>(ctx, P.w0));
                LAUNCHCK();
            }
        }
    }
    TRY(seg_end(ctx));
    int herr[4] = {0, 0, 0, 0};
    HIPCK(hipMemcpyAsync(herr, err, sizeof herr, hipMemcpyDeviceToHost, st));
    std::vector<unsigned long long> fres(P.fres.bytes / sizeof(unsigned long long));
    HIPCK(hipMemcpyAsync(fres.data(), at<unsigned long long>(ctx, P.fres), P.fres.bytes, hipMemcpyDeviceToHost, st));
    std::vector<double> rows(use_id ? P.npad : 0);
    if (use_id) HIPCK(hipMemcpyAsync(rows.data(), at<double>(ctx, P.rowsum), sizeof(double) * P.npad,
                                     hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    TRY(seg_collect(ctx));
    if (herr[0] & 2) return fail(ctx, CDWAC_EINVAL, "non-finite value in the RI coefficients");
    if (use_id) {
        // Omega_max^2 <= D_max^2 + lambda_max(A A^T) and A A^T <= (w_max^2 + D_max^2) (-Pi(i w_max)),
        // lambda_max(-Pi) <= its largest absolute row sum
        const double g = *std::max_element(rows.begin(), rows.end());
        const double dmax = *std::max_element(sys->eps, sys->eps + P.n_mo) - *std::min_element(sys->eps, sys->eps + P.n_mo);
        const double wmax = *std::max_element(prm->freq, prm->freq + P.n_freq);
        const double om_bound = std::sqrt(dmax * dmax + (wmax * wmax + dmax * dmax) * g);
        if (!(om_bound <= hs.omega_hi)) return prepare_impl(ctx, sys, prm, false, sink);
    }
    if (herr[0] & 1) return fail(ctx, CDWAC_ENOTPD, "zero or non-finite pivot while inverting eps = I - Pi");
    // sampled residual of every inversion (a NaN counts as a failure)
    ctx->fact_ratio = 0.0;
    ctx->fact_mat = -1;
    for (int m = 0; m < P.n_imp + P.n_re; ++m)
        for (int c = 0; c < kFactCols; ++c) {
            double r, b;
            std::memcpy(&r, &fres[2 * ((size_t)m * kFactCols + c)], sizeof r);
            std::memcpy(&b, &fres[2 * ((size_t)m * kFactCols + c) + 1], sizeof b);
            const double q = r == 0.0 ? 0.0 : r / b;
            if (!(q <= ctx->fact_ratio)) {
                ctx->fact_ratio = std::isnan(q) ? INFINITY : q;
                ctx->fact_mat = m;
            }
        }
    if (!(ctx->fact_ratio <= kFactTol))
        return fail(ctx, CDWAC_EFACT,
                    "inverse of eps failed its residual check: max|eps^-1 eps_j - e_j| = %.3g of |eps^-1||eps_j| "
                    "(matrix %d; %s), above %.0e", ctx->fact_ratio, ctx->fact_mat,
                    ctx->fact_mat >= P.n_imp ? "near-real reference, complex symmetric" : "imaginary node",
                    kFactTol);
    ctx->hs = hs;
    ctx->prepared = true;
    return CDWAC_OK;
}
}

int cdwac_qp(cdwac_ctx* ctx, const double* vxc, cdwac_state_out* out) {
    if (!ctx) return CDWAC_EINVAL;
    if (!ctx->prepared) return fail(ctx, CDWAC_ESTATE, "cdwac_qp called before cdwac_prepare");
    if (!out) return fail(ctx, CDWAC_EINVAL, "out is NULL");
    const Plan& P = ctx->plan;
    if (vxc && !finite_all(vxc, P.S)) return fail(ctx, CDWAC_EINVAL, "non-finite vxc");
    if (ctx->hs.use_mlp && !ctx->have_mlp) return fail(ctx, CDWAC_EINVAL, "no MLP model installed");
    HIPCK(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    if (vxc) TRY(upload(ctx, at<double>(ctx, P.vxc), vxc, P.S));
    QpArgs a = qp_args(ctx);
    ctx->stage_ms[6] = 0.0;
    ctx->stage_n[6] = 0;
    TRY(seg_begin(ctx, 6));
    launch_qp(st, a, at<QpOut>(ctx, P.qpout));
    LAUNCHCK();
    TRY(seg_end(ctx));
    static_assert(sizeof(QpOut) == sizeof(cdwac_state_out), "output layout");
    HIPCK(hipMemcpyAsync(out, at<QpOut>(ctx, P.qpout), sizeof(QpOut) * P.S, hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    TRY(seg_collect(ctx));
    for (int j = 0; j < P.S; ++j)
        if (out[j].flags & CDWAC_FLAG_NOROOT) return CDWAC_WNOROOT;
    return CDWAC_OK;
}

int cdwac_qp_hedin(cdwac_ctx* ctx, const double* vxc, cdwac_state_out* out, double* shift) {
    if (!ctx) return CDWAC_EINVAL;
    if (!ctx->prepared) return fail(ctx, CDWAC_ESTATE, "cdwac_qp_hedin called before cdwac_prepare");
    if (!out) return fail(ctx, CDWAC_EINVAL, "out is NULL");
    if (!ctx->hs.fit_all)
        return fail(ctx, CDWAC_EINVAL, "the shifted G needs a preparation with fit_all = 1 (a model for every m)");
    const Plan& P = ctx->plan;
    if (vxc && !finite_all(vxc, P.S)) return fail(ctx, CDWAC_EINVAL, "non-finite vxc");
    if (ctx->hs.use_mlp && !ctx->have_mlp) return fail(ctx, CDWAC_EINVAL, "no MLP model installed");
    HIPCK(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    if (vxc) TRY(upload(ctx, at<double>(ctx, P.vxc), vxc, P.S));
    // dH_n = Re Sigma_n(eps_n) - v^xc_n with the unshifted G, before the QP iteration
    double* hv = at<double>(ctx, P.hedin);
    std::vector<double> e_n(P.S), sig(P.S), vx(P.S), dh(P.S);
    for (int j = 0; j < P.S; ++j) e_n[j] = ctx->hs.eps[ctx->hs.state_idx[j]];
    TRY(upload(ctx, hv, e_n.data(), P.S));
    QpArgs a = qp_args(ctx);
    launch_sigma(st, a, 1, hv, hv + P.S, nullptr, nullptr);
    LAUNCHCK();
    HIPCK(hipMemcpyAsync(sig.data(), hv + P.S, sizeof(double) * P.S, hipMemcpyDeviceToHost, st));
    HIPCK(hipMemcpyAsync(vx.data(), at<double>(ctx, P.vxc), sizeof(double) * P.S, hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    for (int j = 0; j < P.S; ++j) dh[j] = sig[j] - vx[j];
    TRY(upload(ctx, hv + 2 * P.S, dh.data(), P.S));
    a.g_shift = hv + 2 * P.S;
    launch_qp(st, a, at<QpOut>(ctx, P.qpout));
    LAUNCHCK();
    HIPCK(hipMemcpyAsync(out, at<QpOut>(ctx, P.qpout), sizeof(QpOut) * P.S, hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    if (shift) std::copy(dh.begin(), dh.end(), shift);
    for (int j = 0; j < P.S; ++j)
        if (out[j].flags & CDWAC_FLAG_NOROOT) return CDWAC_WNOROOT;
    return CDWAC_OK;
}

int cdwac_solve(cdwac_ctx* ctx, const cdwac_system* sys, const cdwac_params* prm, cdwac_state_out* out) {
    if (!out) return fail(ctx, CDWAC_EINVAL, "out is NULL");
    TRY(cdwac_prepare(ctx, sys, prm));
    return cdwac_qp(ctx, nullptr, out);
}

namespace {
// Per-system tables of a batch, copied out of the workspace after the
// system's preparation (offsets into the batch buffer).
struct BatchSys {
    size_t w_im, eps, freq, weight, state_idx, sigx, vxc, win_lo, win_hi, m0, m1, fit_off;
    int fit0;
    QpArgs args;
};

// Context-owned device buffer of at least `bytes` (grown on demand, kept).
int ensure_batch(cdwac_ctx* ctx, size_t bytes) {
    if (ctx->batch_bytes >= bytes) return CDWAC_OK;
    if (ctx->batch) {
        HIPCK(hipStreamSynchronize(ctx->stream));
        HIPCK(hipFree(ctx->batch));
        ctx->batch = nullptr;
        ctx->batch_bytes = 0;
    }
    if (hipMalloc(&ctx->batch, bytes) != hipSuccess) {
        ctx->batch = nullptr;
        (void)hipGetLastError();
        return fail(ctx, CDWAC_ENOMEM, "cannot allocate %zu bytes of batch tables", bytes);
    }
    ctx->batch_bytes = bytes;
    return CDWAC_OK;
}

size_t bump(size_t& total, size_t bytes) {
    size_t off = total;
    total += (bytes + 255) / 256 * 256;
    return off;
}

int copy_d2d(cdwac_ctx* ctx, size_t dst_off, const void* src, size_t bytes) {
    if (bytes == 0) return CDWAC_OK;
    HIPCK(hipMemcpyAsync((char*)ctx->batch + dst_off, src, bytes, hipMemcpyDeviceToDevice, ctx->stream));
    return CDWAC_OK;
}
}  // namespace

int cdwac_solve_batch(cdwac_ctx* ctx, int32_t n_sys, const cdwac_system* sys, const cdwac_params* prm,
                      cdwac_state_out* out) {
    if (!ctx) return CDWAC_EINVAL;
    ctx->prepared = false;
    if (n_sys < 1 || !sys || !prm || !out) return fail(ctx, CDWAC_EINVAL, "bad batch arguments");
    // every argument is checked before any launch
    size_t ws_max = 0;
    int n_pts = 0, s_tot = 0, f_tot = 0;
    std::vector<int> n_fit(n_sys);
    for (int j = 0; j < n_sys; ++j) {
        TRY(validate_system(ctx, &sys[j]));
        TRY(validate_params(ctx, &sys[j], &prm[j]));
        if (prm[j].use_mlp_seed && !ctx->have_mlp)
            return fail(ctx, CDWAC_EINVAL, "system %d: use_mlp_seed set but no model installed", j);
        const int m = prm[j].n_ref_im + prm[j].n_ref_re;
        if (j == 0) n_pts = m;
        if (m != n_pts || prm[j].pade_tol != prm[0].pade_tol)
            return fail(ctx, CDWAC_EINVAL, "system %d: every system needs the same Pade point count and pade_tol", j);
        const Plan P = make_plan(&sys[j], &prm[j], nullptr);
        ws_max = std::max(ws_max, P.total);
        n_fit[j] = P.n_fit;
        s_tot += P.S;
        f_tot += P.n_fit;
    }
    HIPCK(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    // batch buffer layout
    std::vector<BatchSys> bs(n_sys);
    size_t total = 0;
    for (int j = 0; j < n_sys; ++j) {
        const cdwac_system& y = sys[j];
        const int S = y.n_states;
        BatchSys& b = bs[j];
        b.w_im = bump(total, sizeof(double) * (size_t)S * y.n_mo * prm[j].n_freq);
        b.eps = bump(total, sizeof(double) * y.n_mo);
        b.freq = bump(total, sizeof(double) * prm[j].n_freq);
        b.weight = bump(total, sizeof(double) * prm[j].n_freq);
        b.state_idx = bump(total, sizeof(int) * S);
        b.sigx = bump(total, sizeof(double) * S);
        b.vxc = bump(total, sizeof(double) * S);
        b.win_lo = bump(total, sizeof(double) * S);
        b.win_hi = bump(total, sizeof(double) * S);
        b.m0 = bump(total, sizeof(int) * S);
        b.m1 = bump(total, sizeof(int) * S);
        b.fit_off = bump(total, sizeof(int) * S);
    }
    const size_t fits = (size_t)std::max(f_tot, 1) * n_pts * 2 * sizeof(double);
    const size_t o_u = bump(total, fits), o_w = bump(total, fits), o_coef = bump(total, fits),
                 o_node = bump(total, fits);
    const size_t o_nterm = bump(total, sizeof(int) * std::max(f_tot, 1));
    const size_t o_w0 = bump(total, sizeof(double) * std::max(f_tot, 1));
    const size_t o_args = bump(total, sizeof(QpArgs) * n_sys);
    const size_t o_map = bump(total, sizeof(int2) * s_tot);
    const size_t o_out = bump(total, sizeof(QpOut) * s_tot);
    TRY(ensure_batch(ctx, total));
    TRY(ensure_workspace(ctx, ws_max));
    char* base = (char*)ctx->batch;
    double ms[CDWAC_N_STAGES] = {};
    int32_t cnt[CDWAC_N_STAGES] = {};
    // (a0)-(a4) per system; the fits' reference data go to the batch buffer
    int fit0 = 0;
    for (int j = 0; j < n_sys; ++j) {
        const size_t fo = (size_t)fit0 * n_pts * 2;
        FitSink sink{(double*)(base + o_u) + fo, (double*)(base + o_w) + fo};
        const int rc = prepare_impl(ctx, &sys[j], &prm[j], true, &sink);
        ctx->prepared = false;             // the workspace holds no fits
        if (rc != CDWAC_OK) return rc;
        for (int i = 0; i < CDWAC_N_STAGES; ++i) {
            ms[i] += ctx->stage_ms[i];
            cnt[i] += ctx->stage_n[i];
        }
        const Plan& P = ctx->plan;
        BatchSys& b = bs[j];
        TRY(copy_d2d(ctx, b.w_im, at<double>(ctx, P.w_im), sizeof(double) * (size_t)P.S * P.n_mo * P.n_freq));
        TRY(copy_d2d(ctx, b.eps, at<double>(ctx, P.eps), sizeof(double) * P.n_mo));
        TRY(copy_d2d(ctx, b.freq, at<double>(ctx, P.freq), sizeof(double) * P.n_freq));
        TRY(copy_d2d(ctx, b.weight, at<double>(ctx, P.weight), sizeof(double) * P.n_freq));
        TRY(copy_d2d(ctx, b.state_idx, at<int>(ctx, P.state_idx), sizeof(int) * P.S));
        TRY(copy_d2d(ctx, b.sigx, at<double>(ctx, P.sigx), sizeof(double) * P.S));
        TRY(copy_d2d(ctx, b.vxc, at<double>(ctx, P.vxc), sizeof(double) * P.S));
        TRY(copy_d2d(ctx, b.win_lo, at<double>(ctx, P.win_lo), sizeof(double) * P.S));
        TRY(copy_d2d(ctx, b.win_hi, at<double>(ctx, P.win_hi), sizeof(double) * P.S));
        TRY(copy_d2d(ctx, b.m0, at<int>(ctx, P.m0), sizeof(int) * P.S));
        TRY(copy_d2d(ctx, b.m1, at<int>(ctx, P.m1), sizeof(int) * P.S));
        TRY(copy_d2d(ctx, b.fit_off, at<int>(ctx, P.fit_off), sizeof(int) * P.S));
        QpArgs a = qp_args(ctx);
        a.eps = (const double*)(base + b.eps);
        a.eps_n = a.eps;
        a.freq = (const double*)(base + b.freq);
        a.weight = (const double*)(base + b.weight);
        a.w_im = (const double*)(base + b.w_im);
        a.coef = (const double*)(base + o_coef) + fo;
        a.node = (const double*)(base + o_node) + fo;
        a.nterm = (const int*)(base + o_nterm) + fit0;
        a.fit_off = (const int*)(base + b.fit_off);
        a.m0 = (const int*)(base + b.m0);
        a.m1 = (const int*)(base + b.m1);
        a.state_idx = (const int*)(base + b.state_idx);
        a.sigx = (const double*)(base + b.sigx);
        a.vxc = (const double*)(base + b.vxc);
        a.win_lo = (const double*)(base + b.win_lo);
        a.win_hi = (const double*)(base + b.win_hi);
        a.w0 = prm[j].quad_limit ? (const double*)(base + o_w0) + fit0 : nullptr;
        b.args = a;
        b.fit0 = fit0;
        fit0 += n_fit[j];
    }
    ctx->segs.clear();
    ctx->pool_used = 0;
    for (int i = 0; i < CDWAC_N_STAGES; ++i) {
        ctx->stage_ms[i] = ms[i];
        ctx->stage_n[i] = cnt[i];
    }
    // (a5) the greedy fits of every system in one launch
    TRY(seg_begin(ctx, 5));
    launch_thiele_fit(st, f_tot, n_pts, (const double*)(base + o_u), (const double*)(base + o_w), prm[0].pade_tol,
                      (double*)(base + o_coef), (double*)(base + o_node), (int*)(base + o_nterm));
    LAUNCHCK();
    // W at a_m = 0 for the systems with the analytic limit of I_n (each its own eta)
    for (int j = 0; j < n_sys; ++j) {
        if (!prm[j].quad_limit || n_fit[j] == 0) continue;
        const size_t fo = (size_t)bs[j].fit0 * n_pts * 2;
        launch_w0_from_fits(st, n_fit[j], n_pts, (const double*)(base + o_coef) + fo,
                            (const double*)(base + o_node) + fo, (const int*)(base + o_nterm) + bs[j].fit0,
                            prm[j].eta, (double*)(base + o_w0) + bs[j].fit0);
        LAUNCHCK();
    }
    TRY(seg_end(ctx));
    // (a6)-(a8) the QP roots of every state in one launch
    std::vector<QpArgs> args(n_sys);
    std::vector<int2> map;
    map.reserve(s_tot);
    for (int j = 0; j < n_sys; ++j) {
        args[j] = bs[j].args;
        for (int q = 0; q < sys[j].n_states; ++q) map.push_back(make_int2(j, q));
    }
    TRY(upload(ctx, (QpArgs*)(base + o_args), args.data(), args.size()));
    TRY(upload(ctx, (int2*)(base + o_map), map.data(), map.size()));
    TRY(seg_begin(ctx, 6));
    launch_qp_batch(st, s_tot, (const QpArgs*)(base + o_args), (const int2*)(base + o_map), (QpOut*)(base + o_out));
    LAUNCHCK();
    TRY(seg_end(ctx));
    static_assert(sizeof(QpOut) == sizeof(cdwac_state_out), "output layout");
    HIPCK(hipMemcpyAsync(out, base + o_out, sizeof(QpOut) * s_tot, hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    TRY(seg_collect(ctx));
    for (int j = 0; j < s_tot; ++j)
        if (out[j].flags & CDWAC_FLAG_NOROOT) return CDWAC_WNOROOT;
    return CDWAC_OK;
}

int cdwac_set_g_energies(cdwac_ctx* ctx, const double* eps_g, double eps_fermi) {
    if (!ctx) return CDWAC_EINVAL;
    if (!ctx->prepared) return fail(ctx, CDWAC_ESTATE, "cdwac_set_g_energies called before cdwac_prepare");
    if (!ctx->hs.fit_all)
        return fail(ctx, CDWAC_EINVAL, "G energies need a preparation with fit_all = 1 (a model for every m)");
    const Plan& P = ctx->plan;
    if (!eps_g || !finite_all(eps_g, P.n_mo)) return fail(ctx, CDWAC_EINVAL, "eps_g must hold n_mo finite values");
    if (!std::isnan(eps_fermi) && !std::isfinite(eps_fermi)) return fail(ctx, CDWAC_EINVAL, "eps_fermi not finite");
    HIPCK(hipSetDevice(ctx->device));
    TRY(upload(ctx, at<double>(ctx, P.eps_g), eps_g, P.n_mo));
    HIPCK(hipStreamSynchronize(ctx->stream));
    ctx->hs.eps_f = std::isnan(eps_fermi) ? 0.5 * (eps_g[P.n_occ - 1] + eps_g[P.n_occ]) : eps_fermi;
    return CDWAC_OK;
}

int cdwac_evgw(cdwac_ctx* ctx, const cdwac_system* sys, const cdwac_params* prm, int32_t mode, int32_t max_iter,
               double tol, double* eps_out, int32_t* n_iter, cdwac_state_out* out) {
    if (!ctx) return CDWAC_EINVAL;
    ctx->prepared = false;
    TRY(validate_system(ctx, sys));
    TRY(validate_params(ctx, sys, prm));
    if (mode != 0 && mode != 1) return fail(ctx, CDWAC_EINVAL, "mode must be 0 (evGW0) or 1 (evGW)");
    if (max_iter < 1 || !(tol > 0.0)) return fail(ctx, CDWAC_EINVAL, "max_iter >= 1 and tol > 0 required");
    if (!eps_out || !out) return fail(ctx, CDWAC_EINVAL, "eps_out / out is NULL");
    const int n_mo = sys->n_mo, n_occ = sys->n_occ, S = sys->n_states;
    std::vector<double> ks(sys->eps, sys->eps + n_mo), cur = ks;
    cdwac_params p1 = *prm;
    p1.fit_all = 1;                   // G energies move: every m needs a model
    p1.use_mlp_seed = 0;
    cdwac_system s1 = *sys;
    s1.eps_fermi = NAN;               // the Fermi level follows the G energies
    int it = 0;
    for (; it < max_iter; ++it) {
        if (mode == 1 || it == 0) {
            // evGW: Pi and W from the current energies (eps_ia = cur_a - cur_i > 0 checked)
            double occ_max = *std::max_element(cur.begin(), cur.begin() + n_occ);
            double virt_min = *std::min_element(cur.begin() + n_occ, cur.end());
            if (!(occ_max < virt_min))
                return fail(ctx, CDWAC_EINVAL, "iteration %d: an occupied QP energy rose above a virtual one", it);
            s1.eps = cur.data();
            TRY(prepare_impl(ctx, &s1, &p1, true));
            const Plan& P = ctx->plan;
            TRY(upload(ctx, at<double>(ctx, P.eps), ks.data(), n_mo));   // eps_n of the QP equation stays KS
        }
        TRY(cdwac_set_g_energies(ctx, cur.data(), NAN));
        const int rc = cdwac_qp(ctx, nullptr, out);
        if (rc != CDWAC_OK && rc != CDWAC_WNOROOT) return rc;
        double delta = 0.0;
        std::vector<double> nxt = cur;
        for (int j = 0; j < S; ++j)
            if (!(out[j].flags & CDWAC_FLAG_NOROOT)) {
                nxt[sys->state_idx[j]] = out[j].qp;
                delta = std::max(delta, std::fabs(out[j].qp - cur[sys->state_idx[j]]));
            }
        cur = nxt;
        if (delta < tol) {
            ++it;
            break;
        }
    }
    std::copy(cur.begin(), cur.end(), eps_out);
    if (n_iter) *n_iter = it;
    for (int j = 0; j < S; ++j)
        if (out[j].flags & CDWAC_FLAG_NOROOT) return CDWAC_WNOROOT;
    return CDWAC_OK;
}

int cdwac_sigma_cd(cdwac_ctx* ctx, const cdwac_system* sys, const cdwac_params* prm, int32_t state, double omega,
                   double* out, int32_t* n_res) {
    if (!ctx) return CDWAC_EINVAL;
    ctx->prepared = false;
    TRY(validate_system(ctx, sys));
    TRY(validate_params(ctx, sys, prm));
    if (state < 0 || state >= sys->n_states) return fail(ctx, CDWAC_EINVAL, "state %d out of range", state);
    if (!std::isfinite(omega)) return fail(ctx, CDWAC_EINVAL, "omega is not finite");
    if (!out) return fail(ctx, CDWAC_EINVAL, "out is NULL");
    const int n_mo = sys->n_mo, n_occ = sys->n_occ;
    const double ef = std::isnan(sys->eps_fermi) ? 0.5 * (sys->eps[n_occ - 1] + sys->eps[n_occ]) : sys->eps_fermi;
    auto theta = [](double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? 0.0 : 0.5); };
    // residues of Eq. (Rn_term): every m with f_m(omega) != 0 (Eq. ffact)
    std::vector<int> rm;
    std::vector<double> rf, rx;
    for (int m = 0; m < n_mo; ++m) {
        const double em = sys->eps[m];
        const double fm = -theta(ef - em) * theta(em - omega) + theta(em - ef) * theta(omega - em);
        if (fm == 0.0) continue;
        rm.push_back(m);
        rf.push_back(fm);
        rx.push_back(std::fabs(em - omega));
    }
    if (rm.empty()) {          // no residue: one placeholder point with weight 0
        rm.push_back(0);
        rf.push_back(0.0);
        rx.push_back(0.0);
    }
    const int nr = (int)rm.size();
    if (n_res) *n_res = rf[0] == 0.0 && nr == 1 ? 0 : nr;
    // One preparation holds at most kMaxPade near-real planes, so the residues
    // go through in chunks of kMaxPade - 1; the first chunk also carries the
    // point i eta (a_m = 0) of the analytic limit and gives I_n and Sigma^x,
    // every chunk its share of R_n.  The imaginary-axis part is computed
    // again for each chunk.
    const int per = kMaxPade - 1;
    hipStream_t st = ctx->stream;
    const size_t o_rm = 0, o_rf = (sizeof(int) * per + 255) / 256 * 256,
                 o_out = o_rf + (sizeof(double) * per + 255) / 256 * 256;
    double first[3] = {0.0, 0.0, 0.0}, r_rest = 0.0;
    for (int c0 = 0; c0 < nr; c0 += per) {
        const int cn = std::min(per, nr - c0);
        const bool lim = c0 == 0 && prm->quad_limit;
        const int n_pts_re = cn + (lim ? 1 : 0);
        std::vector<double> px(rx.begin() + c0, rx.begin() + c0 + cn);
        if (lim) px.push_back(0.0);
        // one state; the residues are the near-real points (eta_ref = eta); every m fitted
        cdwac_system s1 = *sys;
        s1.n_states = 1;
        s1.state_idx = sys->state_idx + state;
        s1.o_nm = sys->o_nm + (size_t)state * sys->n_aux * n_mo;
        s1.vxc = sys->vxc ? sys->vxc + state : nullptr;
        s1.eps_fermi = ef;
        cdwac_params p1 = *prm;
        p1.n_ref_im = 0;
        p1.ref_im_idx = nullptr;
        p1.n_ref_re = n_pts_re;
        p1.ref_re = px.data();
        p1.eta_ref = prm->eta > 0.0 ? prm->eta : 1e-3;
        p1.win_lo = prm->win_lo + state;
        p1.win_hi = prm->win_hi + state;
        p1.use_mlp_seed = 0;
        p1.fit_all = 1;
        p1.quad_limit = lim ? 1 : 0;      // I_n is taken from the first chunk only
        const int rc = prepare_impl(ctx, &s1, &p1, true);
        ctx->prepared = false;             // a residue set, not a CD-WAC model
        if (rc != CDWAC_OK) return rc;
        TRY(ensure_batch(ctx, o_out + 256));
        char* base = (char*)ctx->batch;
        TRY(upload(ctx, (int*)(base + o_rm), rm.data() + c0, cn));
        TRY(upload(ctx, (double*)(base + o_rf), rf.data() + c0, cn));
        const Plan& P = ctx->plan;
        if (lim) {
            launch_w0_from_points(st, P.n_fit, at<double>(ctx, P.w_re), n_pts_re, cn, at<double>(ctx, P.w0));
            LAUNCHCK();
        }
        launch_sigma_direct(st, qp_args(ctx), omega, at<double>(ctx, P.w_re), n_pts_re, cn,
                            (const int*)(base + o_rm), (const double*)(base + o_rf), (double*)(base + o_out));
        LAUNCHCK();
        double part[3];
        HIPCK(hipMemcpyAsync(part, base + o_out, sizeof(double) * 3, hipMemcpyDeviceToHost, st));
        HIPCK(hipStreamSynchronize(st));
        if (c0 == 0) std::copy(part, part + 3, first);
        else r_rest += part[1];
    }
    out[0] = first[0] + r_rest;
    out[1] = first[1] + r_rest;
    out[2] = first[2];
    return CDWAC_OK;
}

namespace {
// Without fit_all only the orbitals whose residue can enter a state's window
// have Pade models (Eq. ffact): an omega outside the window (widened by the
// Z-factor step) would silently drop residues, so it is rejected.
int check_omega_in_fit_range(cdwac_ctx* ctx, int32_t n_omega, const double* omega) {
    if (ctx->hs.fit_all || n_omega == 0) return CDWAC_OK;
    const int S = ctx->plan.S;
    std::vector<double> om((size_t)S * n_omega);
    HIPCK(hipMemcpyAsync(om.data(), omega, sizeof(double) * om.size(), hipMemcpyDeviceToHost, ctx->stream));
    HIPCK(hipStreamSynchronize(ctx->stream));
    for (int j = 0; j < S; ++j) {
        const double lo = ctx->hs.win_lo[j] - kFitMargin, hi = ctx->hs.win_hi[j] + kFitMargin;
        for (int k = 0; k < n_omega; ++k) {
            const double w = om[(size_t)j * n_omega + k];
            if (!(lo <= w && w <= hi))
                return fail(ctx, CDWAC_EINVAL,
                            "omega[%d][%d] = %g lies outside the fitted window [%g, %g] of its state (prepare "
                            "with fit_all = 1 to evaluate anywhere)", j, k, w, lo, hi);
        }
    }
    return CDWAC_OK;
}
}  // namespace

int cdwac_sigma(cdwac_ctx* ctx, int32_t n_omega, const double* omega, double* sigma, double* i_term,
                double* r_term) {
    if (!ctx) return CDWAC_EINVAL;
    if (!ctx->prepared) return fail(ctx, CDWAC_ESTATE, "cdwac_sigma called before cdwac_prepare");
    if (n_omega < 0 || (n_omega > 0 && (!omega || !sigma))) return fail(ctx, CDWAC_EINVAL, "bad omega/sigma");
    if (n_omega > 65535) return fail(ctx, CDWAC_EINVAL, "n_omega must be <= 65535");
    HIPCK(hipSetDevice(ctx->device));
    TRY(check_omega_in_fit_range(ctx, n_omega, omega));
    QpArgs a = qp_args(ctx);
    launch_sigma(ctx->stream, a, n_omega, omega, sigma, i_term, r_term);
    LAUNCHCK();
    HIPCK(hipStreamSynchronize(ctx->stream));
    return CDWAC_OK;
}

int cdwac_spectral(cdwac_ctx* ctx, int32_t n_omega, const double* omega, const double* vxc, double* spectral,
                   double* sigma_re, double* sigma_im) {
    if (!ctx) return CDWAC_EINVAL;
    if (!ctx->prepared) return fail(ctx, CDWAC_ESTATE, "cdwac_spectral called before cdwac_prepare");
    if (n_omega < 0 || (n_omega > 0 && (!omega || !spectral))) return fail(ctx, CDWAC_EINVAL, "bad omega/spectral");
    if (n_omega > 65535) return fail(ctx, CDWAC_EINVAL, "n_omega must be <= 65535");
    if (vxc)
        for (int j = 0; j < ctx->plan.S; ++j)
            if (!std::isfinite(vxc[j])) return fail(ctx, CDWAC_EINVAL, "vxc[%d] is not finite", j);
    HIPCK(hipSetDevice(ctx->device));
    TRY(check_omega_in_fit_range(ctx, n_omega, omega));
    if (vxc) TRY(upload(ctx, at<double>(ctx, ctx->plan.vxc), vxc, ctx->plan.S));
    QpArgs a = qp_args(ctx);
    launch_spectral(ctx->stream, a, n_omega, omega, spectral, sigma_re, sigma_im);
    LAUNCHCK();
    HIPCK(hipStreamSynchronize(ctx->stream));
    return CDWAC_OK;
}

int cdwac_w_table(cdwac_ctx* ctx, double* w_im, double* w_re, double* sigma_x) {
    if (!ctx) return CDWAC_EINVAL;
    if (!ctx->prepared) return fail(ctx, CDWAC_ESTATE, "cdwac_w_table called before cdwac_prepare");
    const Plan& P = ctx->plan;
    HIPCK(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    if (w_im)
        HIPCK(hipMemcpyAsync(w_im, at<double>(ctx, P.w_im), sizeof(double) * (size_t)P.S * P.n_mo * P.n_freq,
                             hipMemcpyDeviceToDevice, st));
    if (w_re && P.n_re > 0 && P.n_fit > 0)
        HIPCK(hipMemcpyAsync(w_re, at<double>(ctx, P.w_re), sizeof(double) * 2 * (size_t)P.n_fit * P.n_re,
                             hipMemcpyDeviceToDevice, st));
    if (sigma_x)
        HIPCK(hipMemcpyAsync(sigma_x, at<double>(ctx, P.sigx), sizeof(double) * P.S, hipMemcpyDeviceToDevice, st));
    HIPCK(hipStreamSynchronize(st));
    return CDWAC_OK;
}

int cdwac_fit_ranges(cdwac_ctx* ctx, int32_t* m0, int32_t* m1, int32_t* n_fit_total) {
    if (!ctx) return CDWAC_EINVAL;
    if (!ctx->prepared) return fail(ctx, CDWAC_ESTATE, "cdwac_fit_ranges called before cdwac_prepare");
    for (int j = 0; j < ctx->plan.S; ++j) {
        if (m0) m0[j] = ctx->hs.m0[j];
        if (m1) m1[j] = ctx->hs.m1[j];
    }
    if (n_fit_total) *n_fit_total = ctx->plan.n_fit;
    return CDWAC_OK;
}

int cdwac_polarizability(cdwac_ctx* ctx, const cdwac_system* sys, int32_t prec, int32_t n_z, const double* z_re,
                         const double* z_im, double* pi_re, double* pi_im) {
    if (!ctx) return CDWAC_EINVAL;
    TRY(validate_system(ctx, sys));
    if (prec < CDWAC_P64 || prec > CDWAC_F16) return fail(ctx, CDWAC_EINVAL, "unknown precision %d", prec);
    if (n_z < 1 || !z_re || !z_im || !pi_re) return fail(ctx, CDWAC_EINVAL, "bad z list or output");
    bool all_imag = true;
    for (int j = 0; j < n_z; ++j) {
        if (!std::isfinite(z_re[j]) || !std::isfinite(z_im[j])) return fail(ctx, CDWAC_EINVAL, "non-finite z");
        if (z_re[j] != 0.0) all_imag = false;
    }
    if (!all_imag && !pi_im) return fail(ctx, CDWAC_EINVAL, "pi_im required for z off the imaginary axis");
    HIPCK(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const int n_virt = sys->n_mo - sys->n_occ;
    const int64_t K = (int64_t)sys->n_occ * n_virt, kpad = round_up(K, 32);
    const int npad = (int)round_up(sys->n_aux, kGemmRows);
    const int nf = 2 * n_z;
    const bool f64 = prec == CDWAC_P64;
    std::vector<double> zr(nf), zi(nf);
    std::vector<int> part(nf), idf(nf, 0);
    for (int j = 0; j < n_z; ++j)
        for (int q = 0; q < 2; ++q) {
            zr[2 * j + q] = z_re[j];
            zi[2 * j + q] = z_im[j];
            part[2 * j + q] = q;
        }
    size_t bytes = 0;
    auto take = [&](size_t b) {
        size_t o = bytes;
        bytes += (b + 255) / 256 * 256;
        return o;
    };
    size_t o_eps = take(sizeof(double) * sys->n_mo), o_zr = take(sizeof(double) * nf), o_zi = take(sizeof(double) * nf),
           o_part = take(sizeof(int) * nf), o_id = take(sizeof(int) * nf), o_err = take(sizeof(int) * 4),
           o_amax = take(sizeof(uint32_t) * (2 + 2 * (size_t)nf)), o_sf = take(sizeof(double) * (2 + 4 * (size_t)nf)),
           o_cw = take((f64 ? 8 : 4) * (size_t)nf * kpad), o_x = take(8 * (size_t)npad * kpad),
           o_y = take(f64 ? 0 : 4 * (size_t)nf * npad * kpad), o_E = take(sizeof(double) * (size_t)nf * npad * npad);
    const std::vector<int2> tiles = f64 ? std::vector<int2>() : pi_worklist(npad, nf, std::max(1, ctx->n_cu / 8));
    size_t o_t = take(sizeof(int2) * std::max<size_t>(1, tiles.size()));
    size_t o_map = take(sizeof(int) * nf);
    std::vector<int> fmap(nf);
    for (int f = 0; f < nf; ++f) fmap[f] = f;
    char* buf = nullptr;
    if (hipMalloc(&buf, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, CDWAC_ENOMEM, "cannot allocate %zu bytes", bytes);
    }
    int rc = CDWAC_OK;
    do {
        if (hipMemcpyAsync(buf + o_eps, sys->eps, sizeof(double) * sys->n_mo, hipMemcpyHostToDevice, st) ||
            hipMemcpyAsync(buf + o_zr, zr.data(), sizeof(double) * nf, hipMemcpyHostToDevice, st) ||
            hipMemcpyAsync(buf + o_zi, zi.data(), sizeof(double) * nf, hipMemcpyHostToDevice, st) ||
            hipMemcpyAsync(buf + o_part, part.data(), sizeof(int) * nf, hipMemcpyHostToDevice, st) ||
            hipMemcpyAsync(buf + o_id, idf.data(), sizeof(int) * nf, hipMemcpyHostToDevice, st) ||
            hipMemsetAsync(buf + o_err, 0, sizeof(int) * 4, st) ||
            hipMemsetAsync(buf + o_amax, 0, sizeof(uint32_t) * (2 + 2 * (size_t)nf), st)) {
            rc = fail(ctx, CDWAC_EHIP, "upload failed");
            break;
        }
        int* err = (int*)(buf + o_err);
        uint32_t* amax = (uint32_t*)(buf + o_amax);
        double* sf = (double*)(buf + o_sf);
        launch_absmax(st, sys->o_ia, K, sys->n_aux, K, amax, err);
        launch_weights(st, (double*)(buf + o_eps), sys->n_occ, n_virt, sys->spin, (double*)(buf + o_zr),
                       (double*)(buf + o_zi), (int*)(buf + o_part), nf, kpad, f64 ? (double*)(buf + o_cw) : nullptr,
                       f64 ? nullptr : (float*)(buf + o_cw), amax + 2);
        uint16_t* xh = (uint16_t*)(buf + o_x);
        uint16_t* xl = xh + (size_t)npad * kpad;
        float* x32 = (float*)(xl + (size_t)npad * kpad);
        uint16_t* yh = (uint16_t*)(buf + o_y);
        uint16_t* yl = yh + (size_t)nf * npad * kpad;
        if (f64) {
            launch_pad_f64(st, sys->o_ia, K, sys->n_aux, K, (double*)(buf + o_x), npad, kpad);
            launch_pi_f64(st, npad, kpad, nf, (double*)(buf + o_x), (double*)(buf + o_cw), (int*)(buf + o_id),
                          (double*)(buf + o_E));
        } else {
            const int et = prec_elem(prec);
            if (hipMemcpyAsync(buf + o_t, tiles.data(), sizeof(int2) * tiles.size(), hipMemcpyHostToDevice, st) ||
                hipMemcpyAsync(buf + o_map, fmap.data(), sizeof(int) * nf, hipMemcpyHostToDevice, st)) {
                rc = fail(ctx, CDWAC_EHIP, "upload failed");
                break;
            }
            launch_scales_pi(st, amax, nf, sf);
            const bool split = prec != CDWAC_F16;
            launch_split_panel(st, et, sys->o_ia, 0, 1, K, sys->n_aux, K, sf, xh, split ? xl : nullptr, x32, npad,
                               kpad);
            launch_prescale(st, et, x32, npad, kpad, (float*)(buf + o_cw), sf + 2, (int*)(buf + o_map), nf, yh,
                            split ? yl : nullptr);
            launch_pi_gemm(st, prec, npad, kpad, (int*)(buf + o_map), xh, xl, yh, yl, (int2*)(buf + o_t),
                           (int)tiles.size(), sf + 2 + nf, (int*)(buf + o_id), (double*)(buf + o_E));
        }
        if (hipGetLastError() != hipSuccess) {
            rc = fail(ctx, CDWAC_EHIP, "kernel launch failed");
            break;
        }
        // E holds -Pi on the lower tiles; mirror to full symmetric outputs
        const double* E = (const double*)(buf + o_E);
        launch_extract_pi(st, E, npad, sys->n_aux, n_z, 0, pi_re);
        if (pi_im) launch_extract_pi(st, E, npad, sys->n_aux, n_z, 1, pi_im);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
            rc = fail(ctx, CDWAC_EHIP, "extract failed");
            break;
        }
        int herr = 0;
        if (rc == CDWAC_OK && (hipMemcpy(&herr, err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess))
            rc = fail(ctx, CDWAC_EHIP, "copy failed");
        if (rc == CDWAC_OK && (herr & 2)) rc = fail(ctx, CDWAC_EINVAL, "non-finite value in the RI coefficients");
    } while (false);
    (void)hipStreamSynchronize(st);
    (void)hipFree(buf);
    return rc;
}

int cdwac_pade_fit_eval(cdwac_ctx* ctx, int32_t n_fit, int32_t n_pts, const double* u, const double* w, double tol,
                        int32_t n_x, const double* x, double* out, int32_t* n_terms) {
    if (!ctx) return CDWAC_EINVAL;
    if (n_fit < 0 || n_pts < 1 || n_pts > kMaxPade || n_x < 0 || !(tol >= 0.0))
        return fail(ctx, CDWAC_EINVAL, "bad fit sizes (n_pts must be in [1, %d])", kMaxPade);
    if (n_fit == 0) return CDWAC_OK;
    if (!u || !w || (n_x > 0 && (!x || !out))) return fail(ctx, CDWAC_EINVAL, "NULL array");
    HIPCK(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    size_t cb = sizeof(double) * 2 * (size_t)n_fit * n_pts;
    char* buf = nullptr;
    if (hipMalloc(&buf, 2 * cb + sizeof(int) * (size_t)n_fit + 512) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, CDWAC_ENOMEM, "cannot allocate fit buffers");
    }
    double* coef = (double*)buf;
    double* node = (double*)(buf + cb);
    int* nt = (int*)(buf + 2 * cb);
    launch_thiele_fit(st, n_fit, n_pts, u, w, tol, coef, node, nt);
    launch_thiele_eval(st, n_fit, n_pts, coef, node, nt, n_x, x, out);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && n_terms) e = hipMemcpyAsync(n_terms, nt, sizeof(int) * n_fit, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(buf);
    if (e != hipSuccess) return fail(ctx, CDWAC_EHIP, "pade fit: %s", hipGetErrorString(e));
    return CDWAC_OK;
}

int cdwac_pade_fit_eval_noalloc(cdwac_ctx* ctx, int32_t n_fit, int32_t n_pts, const double* u, const double* w,
                                double tol, int32_t n_x, const double* x, double* out, int32_t* n_terms) {
    if (!ctx) return CDWAC_EINVAL;
    if (n_fit < 0 || n_pts < 1 || n_pts > kMaxPade || n_x < 0 || !(tol >= 0.0))
        return fail(ctx, CDWAC_EINVAL, "bad fit sizes (n_pts must be in [1, %d])", kMaxPade);
    if ((int64_t)n_fit * n_pts > kNoAllocFitPoints)
        return fail(ctx, CDWAC_EINVAL, "n_fit * n_pts = %lld exceeds the fixed scratch (%lld)",
                    (long long)n_fit * n_pts, (long long)kNoAllocFitPoints);
    if (n_fit == 0) return CDWAC_OK;
    if (!u || !w || (n_x > 0 && (!x || !out))) return fail(ctx, CDWAC_EINVAL, "NULL array");
    HIPCK(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    // every coefficient, node and term count the evaluation reads is written
    // by the fit kernel of this call, so nothing in the scratch is cleared
    double* coef = (double*)ctx->scratch;
    double* node = (double*)(ctx->scratch + kNoAllocPlane);
    int* nt = (int*)(ctx->scratch + 2 * kNoAllocPlane);
    launch_thiele_fit(st, n_fit, n_pts, u, w, tol, coef, node, nt);
    launch_thiele_eval(st, n_fit, n_pts, coef, node, nt, n_x, x, out);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && n_terms) e = hipMemcpyAsync(n_terms, nt, sizeof(int) * n_fit, hipMemcpyDeviceToDevice, st);
    // while the stream is being captured into a graph the launches and the
    // copy are recorded, not run: the results appear when the graph runs
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (e == hipSuccess) e = hipStreamIsCapturing(st, &cap);
    if (e == hipSuccess && cap == hipStreamCaptureStatusNone) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(ctx, CDWAC_EHIP, "pade fit (fixed scratch): %s", hipGetErrorString(e));
    return CDWAC_OK;
}

int cdwac_set_timing(cdwac_ctx* ctx, int on) {
    if (!ctx) return CDWAC_EINVAL;
    ctx->timing = on != 0;
    return CDWAC_OK;
}

int cdwac_get_timing(const cdwac_ctx* ctx, double* ms, int32_t n) {
    if (!ctx || !ms || n < 0) return CDWAC_EINVAL;
    for (int i = 0; i < n && i < CDWAC_N_STAGES; ++i) ms[i] = ctx->stage_ms[i];
    return CDWAC_OK;
}

int cdwac_freq_decomposition(int32_t n_freq, const double* freq, double dmin, double dmax, double tol,
                             int32_t* n_skel, int32_t* skel, int32_t* rest, double* T) {
    if (n_freq < 1 || !freq || !n_skel || !skel || !rest || !T) return CDWAC_EINVAL;
    if (!(dmin > 0.0) || !(dmax > dmin) || !std::isfinite(dmax) || !(tol > 0.0 && tol < 1.0)) return CDWAC_EINVAL;
    for (int f = 0; f < n_freq; ++f)
        if (!(freq[f] > 0.0) || !std::isfinite(freq[f])) return CDWAC_EINVAL;
    FreqId fid;
    if (!freq_id(freq, n_freq, dmin, dmax, tol, fid)) {
        *n_skel = n_freq;
        for (int f = 0; f < n_freq; ++f) skel[f] = f;
        return CDWAC_OK;
    }
    *n_skel = (int32_t)fid.skel.size();
    std::copy(fid.skel.begin(), fid.skel.end(), skel);
    std::copy(fid.rest.begin(), fid.rest.end(), rest);
    std::copy(fid.T.begin(), fid.T.end(), T);
    return CDWAC_OK;
}

int cdwac_plane_counts(const cdwac_ctx* ctx, int32_t* n_imag, int32_t* n_planes) {
    if (!ctx || !n_imag || !n_planes) return CDWAC_EINVAL;
    if (!ctx->prepared) return CDWAC_ESTATE;
    *n_imag = ctx->plan.n_imp;
    *n_planes = ctx->plan.n_f;
    return CDWAC_OK;
}

int cdwac_inversion_residual(const cdwac_ctx* ctx, double* worst, int32_t* matrix) {
    if (!ctx) return CDWAC_EINVAL;
    if (worst) *worst = ctx->fact_ratio;
    if (matrix) *matrix = ctx->fact_mat;
    return CDWAC_OK;
}

int cdwac_get_timing_segments(const cdwac_ctx* ctx, int32_t* count, int32_t n) {
    if (!ctx || !count || n < 0) return CDWAC_EINVAL;
    for (int i = 0; i < n && i < CDWAC_N_STAGES; ++i) count[i] = ctx->stage_n[i];
    return CDWAC_OK;
}

int cdwac_mlp_set_model(cdwac_ctx* ctx, const float* theta, const float* mu, const float* sd, float out_mu,
                        float out_sd) {
    if (!ctx) return CDWAC_EINVAL;
    if (!theta || !mu || !sd) return fail(ctx, CDWAC_EINVAL, "NULL model array");
    for (int i = 0; i < 8; ++i)
        if (!(sd[i] > 0.f) || !std::isfinite(mu[i])) return fail(ctx, CDWAC_EINVAL, "feature scale must be > 0");
    if (!(out_sd > 0.f) || !std::isfinite(out_sd) || !std::isfinite(out_mu))
        return fail(ctx, CDWAC_EINVAL, "out_sd must be finite and > 0, out_mu finite");
    HIPCK(hipSetDevice(ctx->device));
    HIPCK(hipMemcpy(ctx->mlp_theta, theta, sizeof(float) * kMlpParams, hipMemcpyHostToDevice));
    memcpy(ctx->mlp_mu, mu, sizeof ctx->mlp_mu);
    memcpy(ctx->mlp_sd, sd, sizeof ctx->mlp_sd);
    ctx->mlp_out_mu = out_mu;
    ctx->mlp_out_sd = out_sd;
    ctx->have_mlp = true;
    return CDWAC_OK;
}

int cdwac_mlp_forward(cdwac_ctx* ctx, const float* theta, int32_t n, const float* x, float* y) {
    if (!ctx) return CDWAC_EINVAL;
    if (n < 0 || (n > 0 && (!theta || !x || !y))) return fail(ctx, CDWAC_EINVAL, "bad MLP forward arguments");
    HIPCK(hipSetDevice(ctx->device));
    launch_mlp_forward(ctx->stream, theta, n, x, y);
    LAUNCHCK();
    HIPCK(hipStreamSynchronize(ctx->stream));
    return CDWAC_OK;
}

namespace {
int mlp_scratch(cdwac_ctx* ctx, size_t bytes, char** out) {
    if (ctx->mlp_scratch_bytes < bytes) {
        if (ctx->mlp_scratch) {
            HIPCK(hipStreamSynchronize(ctx->stream));
            HIPCK(hipFree(ctx->mlp_scratch));
            ctx->mlp_scratch = nullptr;
            ctx->mlp_scratch_bytes = 0;
        }
        if (hipMalloc(&ctx->mlp_scratch, bytes) != hipSuccess) {
            ctx->mlp_scratch = nullptr;
            (void)hipGetLastError();
            return fail(ctx, CDWAC_ENOMEM, "cannot allocate MLP scratch");
        }
        ctx->mlp_scratch_bytes = bytes;
    }
    *out = (char*)ctx->mlp_scratch;
    return CDWAC_OK;
}
}  // namespace

int cdwac_mlp_grad(cdwac_ctx* ctx, const float* theta, int32_t n, const float* x, const float* t, float* grad,
                   float* loss) {
    if (!ctx) return CDWAC_EINVAL;
    if (n < 1 || !theta || !x || !t || !grad || !loss) return fail(ctx, CDWAC_EINVAL, "bad MLP grad arguments");
    HIPCK(hipSetDevice(ctx->device));
    int nb = mlp_grad_blocks(n);
    char* s = nullptr;
    TRY(mlp_scratch(ctx, sizeof(float) * ((size_t)nb * kMlpParams + nb) + 256, &s));
    launch_mlp_grad(ctx->stream, theta, n, x, t, (float*)s, (float*)s + (size_t)nb * kMlpParams, grad, loss);
    LAUNCHCK();
    HIPCK(hipStreamSynchronize(ctx->stream));
    return CDWAC_OK;
}

int cdwac_mlp_adam(cdwac_ctx* ctx, float* theta, const float* grad, float* m, float* v, int32_t step, float lr,
                   float beta1, float beta2, float adam_eps) {
    if (!ctx) return CDWAC_EINVAL;
    if (!theta || !grad || !m || !v || step < 1) return fail(ctx, CDWAC_EINVAL, "bad Adam arguments");
    HIPCK(hipSetDevice(ctx->device));
    launch_mlp_adam(ctx->stream, theta, grad, m, v, step, lr, beta1, beta2, adam_eps);
    LAUNCHCK();
    HIPCK(hipStreamSynchronize(ctx->stream));
    return CDWAC_OK;
}

int cdwac_mlp_train(cdwac_ctx* ctx, float* theta, float* m, float* v, int32_t n, const float* x, const float* t,
                    int32_t epochs, int32_t batch, float lr, uint64_t seed, float* loss_curve) {
    if (!ctx) return CDWAC_EINVAL;
    if (n < 1 || epochs < 1 || batch < 1 || batch > 1024 || !theta || !m || !v || !x || !t)
        return fail(ctx, CDWAC_EINVAL, "bad MLP train arguments");
    HIPCK(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const int nb = mlp_grad_blocks(batch);
    const int nbatch = (n + batch - 1) / batch;
    size_t o_part = 0, o_lp = o_part + sizeof(float) * (size_t)nb * kMlpParams;
    size_t o_grad = round_up(o_lp + sizeof(float) * nb, 256);
    size_t o_loss = round_up(o_grad + sizeof(float) * kMlpParams, 256);
    size_t o_xb = round_up(o_loss + sizeof(float) * (size_t)nbatch, 256);
    size_t o_tb = round_up(o_xb + sizeof(float) * 8 * (size_t)batch, 256);
    size_t o_perm = round_up(o_tb + sizeof(float) * (size_t)batch, 256);
    size_t total = round_up(o_perm + sizeof(int) * (size_t)n, 256);
    char* s = nullptr;
    TRY(mlp_scratch(ctx, total, &s));
    std::vector<int> perm(n);
    std::vector<float> losses(nbatch);
    std::mt19937_64 rng(seed);
    int step = 0;
    for (int e = 0; e < epochs; ++e) {
        for (int i = 0; i < n; ++i) perm[i] = i;
        for (int i = n - 1; i > 0; --i) {
            int j = (int)(rng() % (uint64_t)(i + 1));
            std::swap(perm[i], perm[j]);
        }
        HIPCK(hipMemcpyAsync(s + o_perm, perm.data(), sizeof(int) * n, hipMemcpyHostToDevice, st));
        for (int b = 0; b < nbatch; ++b) {
            int nbt = std::min(batch, n - b * batch);
            launch_mlp_gather(st, x, t, (int*)(s + o_perm) + (size_t)b * batch, nbt, (float*)(s + o_xb),
                              (float*)(s + o_tb));
            launch_mlp_grad(st, theta, nbt, (float*)(s + o_xb), (float*)(s + o_tb), (float*)(s + o_part),
                            (float*)(s + o_lp), (float*)(s + o_grad), (float*)(s + o_loss) + b);
            launch_mlp_adam(st, theta, (float*)(s + o_grad), m, v, ++step, lr, 0.9f, 0.999f, 1e-8f);
        }
        LAUNCHCK();
        if (loss_curve) {
            HIPCK(hipMemcpyAsync(losses.data(), s + o_loss, sizeof(float) * nbatch, hipMemcpyDeviceToHost, st));
            HIPCK(hipStreamSynchronize(st));
            double acc = 0.0;
            for (int b = 0; b < nbatch; ++b) acc += (double)losses[b] * std::min(batch, n - b * batch);
            loss_curve[e] = (float)(acc / n);
        }
    }
    HIPCK(hipStreamSynchronize(st));
    return CDWAC_OK;
}

}  // extern "C"

// Host logic of the library under the address and undefined-behaviour
// sanitizers (host side only; no GPU call is made): argument validation,
// the workspace plan of many shapes and settings, the skeleton-node
// decomposition, the fit ranges, the polarizability work list and batch
// sizes.  Every source of the library is compiled into this one translation
// unit so that the functions of api.hip's anonymous namespace are callable.
// Exit status 0 on success; a sanitizer finding aborts with its report.
#include "../../paper_2305_15955_amd/csrc/k_stage.hip"
#include "../../paper_2305_15955_amd/csrc/k_dense.hip"
#include "../../paper_2305_15955_amd/csrc/k_sweep.hip"
#include "../../paper_2305_15955_amd/csrc/k_thiele.hip"
#include "../../paper_2305_15955_amd/csrc/k_qp.hip"
#include "../../paper_2305_15955_amd/csrc/k_mlp.hip"
#include "../../paper_2305_15955_amd/csrc/api.hip"

#include <cstdio>
#include <random>
#include <vector>

namespace {

int bad = 0;

void expect(bool ok, const char* what) {
    if (!ok) {
        ++bad;
        std::printf("FAILED: %s\n", what);
    }
}

struct Shape {
    int n_mo, n_occ, n_aux, n_states, n_freq, n_im, n_re, prec, fit_all, near_real_f64;
    double rank_tol;
};

// A system and settings whose host arrays live in the struct (the device
// pointers are never dereferenced on the host).
struct Case {
    std::vector<double> eps, vxc, freq, weight, ref_re, lo, hi;
    std::vector<int32_t> state_idx, ref_im;
    cdwac_system sys{};
    cdwac_params prm{};

    explicit Case(const Shape& s, std::mt19937_64& rng) {
        std::uniform_real_distribution<double> u01(0.0, 1.0);
        eps.resize(s.n_mo);
        for (int m = 0; m < s.n_mo; ++m) eps[m] = m < s.n_occ ? -11.0 + 0.02 * m : 0.02 + 0.01 * (m - s.n_occ);
        for (int j = 0; j < s.n_states; ++j) state_idx.push_back(j % s.n_occ);
        vxc.assign(s.n_states, -0.3);
        for (int k = 0; k < s.n_freq; ++k) {
            const double x = -1.0 + (2.0 * k + 1.0) / s.n_freq;
            freq.push_back((1.0 + x) / (1.0 - x));
            weight.push_back(0.1 + u01(rng));
        }
        for (int j = 0; j < s.n_im; ++j) ref_im.push_back((int)((int64_t)j * (s.n_freq - 1) / std::max(s.n_im - 1, 1)));
        for (int j = 0; j < s.n_re; ++j) ref_re.push_back(0.5 * j);
        for (int j = 0; j < s.n_states; ++j) {
            lo.push_back(eps[state_idx[j]] - 1.1);
            hi.push_back(eps[state_idx[j]] + 1.1);
        }
        sys.n_mo = s.n_mo;
        sys.n_occ = s.n_occ;
        sys.n_aux = s.n_aux;
        sys.n_states = s.n_states;
        sys.state_idx = state_idx.data();
        sys.eps = eps.data();
        sys.vxc = vxc.data();
        sys.o_ia = reinterpret_cast<const double*>(0x1000);
        sys.o_nm = reinterpret_cast<const double*>(0x2000);
        sys.spin = 2.0;
        sys.eps_fermi = NAN;
        prm.n_freq = s.n_freq;
        prm.freq = freq.data();
        prm.weight = weight.data();
        prm.n_ref_im = s.n_im;
        prm.ref_im_idx = ref_im.data();
        prm.n_ref_re = s.n_re;
        prm.ref_re = ref_re.data();
        prm.eta_ref = 1e-3;
        prm.eta = 1e-3;
        prm.pade_tol = 1e-9;
        prm.win_lo = lo.data();
        prm.win_hi = hi.data();
        prm.qp_tol = 1e-10;
        prm.qp_maxit = 100;
        prm.prec = s.prec;
        prm.freq_rank_tol = s.rank_tol;
        prm.fit_all = s.fit_all;
        prm.near_real_f64 = s.near_real_f64;
    }
};

// Regions of a plan: 256-byte aligned, inside the total, pairwise disjoint.
void check_plan(const Plan& P, const char* what) {
    const Region* regs[] = {&P.eps, &P.eps_g, &P.freq, &P.weight, &P.ref_re, &P.ref_im, &P.state_idx, &P.vxc,
                            &P.sigx, &P.win_lo, &P.win_hi, &P.m0, &P.m1, &P.fit_off, &P.fit_s, &P.fit_m, &P.w_im,
                            &P.w_re, &P.coef, &P.node, &P.nterm, &P.qpout, &P.err, &P.hedin, &P.zr, &P.zi,
                            &P.part, &P.idflag, &P.amax, &P.sf, &P.cw, &P.cw64, &P.x64, &P.xh, &P.xl, &P.E,
                            &P.dinv_r, &P.pbuf_r, &P.qbuf_r, &P.dinv_c, &P.pbuf_c, &P.qbuf_c, &P.dscr_r, &P.lh,
                            &P.ll, &P.bt64, &P.bh, &P.bl, &P.bf64, &P.bfh, &P.bfl, &P.partial_im, &P.partial_re,
                            &P.rowsel, &P.ref_u, &P.ref_w, &P.x32, &P.yh, &P.yl, &P.t_pi, &P.t_w, &P.t_wf,
                            &P.pmap, &P.imnode, &P.imrest, &P.tmat, &P.rowsum, &P.fcols, &P.fcolidx, &P.fres, &P.w0};
    std::vector<std::pair<size_t, size_t>> iv;
    for (const Region* r : regs) {
        if (r->bytes == 0) continue;
        expect(r->off % 256 == 0, what);
        expect(r->off + r->bytes <= P.total, what);
        iv.push_back({r->off, r->off + r->bytes});
    }
    std::sort(iv.begin(), iv.end());
    for (size_t i = 1; i < iv.size(); ++i) expect(iv[i].first >= iv[i - 1].second, what);
    expect(P.n_imp >= 1 && P.n_imp <= P.n_freq, what);
    expect(P.n_f == P.n_imp + 2 * P.n_re, what);
    expect(P.npad % 256 == 0 && P.npad >= P.n_aux, what);
    expect(P.kpad % 32 == 0 && P.kpad >= P.K, what);
}

}  // namespace

int main() {
    std::mt19937_64 rng(7);
    const Shape shapes[] = {
        {60, 10, 200, 1, 32, 8, 8, CDWAC_P64, 0, 0, 0.0},
        {90, 15, 300, 3, 48, 12, 12, CDWAC_F16X3, 0, 0, 0.0},
        {90, 15, 300, 3, 48, 12, 12, CDWAC_F16, 1, 1, 1e-6},
        {600, 100, 2000, 6, 64, 12, 12, CDWAC_B16X3, 0, 0, 0.0},
        {1500, 250, 5000, 16, 64, 12, 12, CDWAC_B16X3, 0, 0, 0.0},
        {1500, 250, 5000, 16, 64, 12, 12, CDWAC_F16, 0, 0, 1e-6},
        {2, 1, 1, 1, 8, 1, 1, CDWAC_P64, 1, 0, 0.0},
        {3, 1, 2, 1, 8, 0, 1, CDWAC_B16, 0, 0, 1e-8},
        {200, 40, 660, 12, 200, 200, 40, CDWAC_P64, 0, 0, 0.0},
    };
    for (const Shape& s : shapes) {
        Case c(s, rng);
        expect(validate_system(nullptr, &c.sys) == CDWAC_OK, "valid system rejected");
        expect(validate_params(nullptr, &c.sys, &c.prm) == CDWAC_OK, "valid params rejected");
        HostState hs;
        const Plan P = make_plan(&c.sys, &c.prm, &hs);
        check_plan(P, "plan layout");
        expect((int)hs.m0.size() == s.n_states && (int)hs.fit_s.size() == P.n_fit, "fit lists");
        for (int j = 0; j < s.n_states; ++j)
            expect(0 <= hs.m0[j] && hs.m0[j] <= hs.m1[j] && hs.m1[j] <= s.n_mo, "fit range bounds");
        expect(cdwac_workspace_bytes(&c.sys, &c.prm) == P.total, "workspace bytes");
        // invalid arguments are rejected before anything else
        Case d(s, rng);
        d.eps[s.n_mo - 1] = d.eps[s.n_mo - 2];
        expect(validate_system(nullptr, &d.sys) == CDWAC_EINVAL, "non-ascending energies");
        Case e(s, rng);
        e.lo[0] = e.eps[e.state_idx[0]] + 0.01;
        expect(validate_params(nullptr, &e.sys, &e.prm) == CDWAC_EINVAL, "window without eps_n");
        Case f(s, rng);
        f.freq[0] = -1.0;
        expect(validate_params(nullptr, &f.sys, &f.prm) == CDWAC_EINVAL, "negative node");
        Case g(s, rng);
        g.prm.n_ref_re = 300;
        expect(validate_params(nullptr, &g.sys, &g.prm) == CDWAC_EINVAL, "too many references");
        Case g2(s, rng);
        g2.prm.n_ref_re = kMaxPade + 1 - g2.prm.n_ref_im;
        expect(g2.prm.n_ref_re < 0 || validate_params(nullptr, &g2.sys, &g2.prm) == CDWAC_EINVAL,
               "one reference point beyond the limit");
        Case g3(s, rng);
        g3.prm.n_freq = qp_max_freq() + 1;
        expect(validate_params(nullptr, &g3.sys, &g3.prm) == CDWAC_EINVAL, "one imaginary node beyond the limit");
        Case h(s, rng);
        h.state_idx[0] = s.n_mo;
        expect(validate_system(nullptr, &h.sys) == CDWAC_EINVAL, "state index out of range");
        expect(cdwac_workspace_bytes(&h.sys, &h.prm) == 0, "workspace of an invalid system");
    }
    expect(validate_system(nullptr, nullptr) == CDWAC_EINVAL, "NULL system");
    // skeleton-node decomposition over random grids and excitation ranges
    std::uniform_real_distribution<double> u01(0.0, 1.0);
    for (int t = 0; t < 40; ++t) {
        const int n = 4 + (int)(u01(rng) * 120);
        std::vector<double> w(n);
        for (int k = 0; k < n; ++k) {
            const double x = -1.0 + (2.0 * k + 1.0) / n;
            w[k] = (1.0 + x) / (1.0 - x);
        }
        const double lo = 0.01 + u01(rng), hi = lo * (2.0 + 100.0 * u01(rng));
        const double tol = std::pow(10.0, -(4.0 + 8.0 * u01(rng)));
        FreqId id;
        const bool ok = freq_id(w.data(), n, lo, hi, tol, id);
        if (ok) {
            expect(id.skel.size() + id.rest.size() == (size_t)n, "skeleton partition");
            expect(id.T.size() == id.rest.size() * id.skel.size(), "interpolation size");
        }
        std::vector<int32_t> skel(n), rest(n);
        std::vector<double> T((size_t)n * n);
        int32_t ns = 0;
        expect(cdwac_freq_decomposition(n, w.data(), lo, hi, tol, &ns, skel.data(), rest.data(), T.data()) ==
                   CDWAC_OK && ns >= 1 && ns <= n, "decomposition entry point");
    }
    // fit ranges against a direct count
    std::vector<double> eps(50);
    for (int m = 0; m < 50; ++m) eps[m] = m < 12 ? -10.0 + 0.3 * m : 0.1 * (m - 11);
    for (int t = 0; t < 200; ++t) {
        const double a = -12.0 + 16.0 * u01(rng), b = a + 4.0 * u01(rng);
        int m0, m1;
        fit_range(eps.data(), 50, 12, a, b, m0, m1);
        int c0 = 0, c1 = 12;
        while (c0 < 12 && eps[c0] < a) ++c0;
        while (c1 < 50 && eps[c1] <= b) ++c1;
        expect(m0 == c0 && m1 == c1, "fit range");
    }
    // polarizability work lists and batch sizes
    for (int npad : {256, 1280, 5120})
        for (int nfb : {1, 6, 12})
            for (int cu : {1, 32}) {
                const std::vector<int2> wl = pi_worklist(npad, nfb, cu);
                const int n = npad / 256;
                long tiles = 0;
                for (const int2 x : wl) tiles += x.x >= 0;
                expect(tiles == (long)nfb * n * (n + 1) / 2, "work list size");
            }
    for (int np : {1, 48, 88}) expect(pi_batch_size(np, 7, 210, 256) <= 7, "batch size");
    std::printf("%s\n", bad ? "FAIL" : "ok");
    return bad != 0;
}

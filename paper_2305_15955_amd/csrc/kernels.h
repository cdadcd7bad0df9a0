// Launchers of the gfx950 kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace cdwac {

constexpr int CDWAC_FLAG_NOROOT_DEV = 1;
constexpr int CDWAC_FLAG_FALLBACK_DEV = 2;
constexpr int CDWAC_FLAG_MLP_ACCEPTED_DEV = 4;

// Everything the self-energy / root kernels read (device pointers unless noted).
struct QpArgs {
    int n_mo, n_states, n_freq, n_pts;
    const double* eps;       // [n_mo] energies of G (the KS ones unless replaced)
    const double* eps_n;     // [n_mo] KS energies: eps_n of the QP equation
    const double* freq;
    const double* weight;
    const double* w_im;      // [S][n_mo][n_freq]
    const double* coef;      // [n_fit][n_pts][2]
    const double* node;      // [n_fit][n_pts][2]
    const int* nterm;        // [n_fit]
    const int* fit_off;      // [S]
    const int* m0;           // [S]
    const int* m1;           // [S]
    const int* state_idx;    // [S]
    const double* sigx;      // [S]
    const double* vxc;       // [S]
    const double* win_lo;    // [S]
    const double* win_hi;    // [S]
    const double* g_shift;   // [S] shift of G's energies per state (G_dH W0), or nullptr
    const double* w0;        // [n_fit] W_nm at a_m = 0 for the analytic limit of I_n, or nullptr
    double eta, eps_f, qp_tol;
    int qp_maxit;
    int use_mlp;
    double mlp_accept;
    const float* mlp_theta;  // [4801]
    float mlp_mu[8], mlp_sd[8];
    float mlp_out_mu, mlp_out_sd;
};

struct QpOut {
    double qp, z, sigma_x, sigma_c, residual;
    int32_t n_evals, flags, n_rounds;
};

// precision codes (same values as cdwac_prec)
constexpr int PREC_P64 = 0, PREC_B16X3 = 1, PREC_B16 = 2, PREC_F16X3 = 3, PREC_F16 = 4;
inline int prec_elem(int prec) { return prec == PREC_F16X3 || prec == PREC_F16 ? 1 : 0; }

// k_stage.hip
void launch_absmax(hipStream_t s, const double* src, int64_t lds, int rows, int64_t cols, uint32_t* amax, int* err);
void launch_weights(hipStream_t s, const double* eps, int n_occ, int n_virt, double spin, const double* zr,
                    const double* zi, const int* part, int n_f, int64_t kpad, double* cw64, float* cw32,
                    uint32_t* cmax);
void launch_scales_pi(hipStream_t s, const uint32_t* amax, int n_f, double* sf);
void launch_prescale(hipStream_t s, int et, const float* x32, int npad, int64_t kpad, const float* cw32,
                     const double* ys, const int* fmap, int nfb, uint16_t* yh, uint16_t* yl);
void launch_scales_w(hipStream_t s, const uint32_t* lmax, int n_f, double* sf, double* lam_scale, double* w_unscale);
void launch_pad_f64(hipStream_t s, const double* src, int64_t lds, int rows, int64_t cols, double* f64, int rpad,
                    int64_t cpad);
// nz planes src + z * sstride, scaled by scale[z], to hi/lo panel planes (panel_off)
void launch_split_panel(hipStream_t s, int et, const double* src, int64_t sstride, int nz, int64_t lds, int rows,
                        int64_t cols, const double* scale, uint16_t* hi, uint16_t* lo, float* f32, int rpad,
                        int64_t cpad);
void launch_transpose_b(hipStream_t s, int et, const double* onm, int S, int N, int n_mo, const int* rowsel,
                        int nrows, const double* scale, double* bt64, uint16_t* bh, uint16_t* bl, int cpad,
                        int npad, uint32_t* bmax, int* err);
void launch_exchange(hipStream_t s, const double* onm, int S, int N, int n_mo, int n_occ, double* sx);
void launch_finalize_lambda(hipStream_t s, double* E, int npad, int n_f, const int* idflag, uint32_t* lmax);
// W at the imaginary nodes without a plane, from the nodes with one
void launch_interp_w(hipStream_t s, double* w_im, int n_freq, int ncols, int n_imp, const int* node, int n_rest,
                     const int* rest, const double* T);
// rowsum[P] += sum_Q |E_PQ - delta_PQ| (lower-triangle storage; rowsum zeroed by the caller)
void launch_rowabs(hipStream_t s, const double* E, int npad, double* rowsum);
void launch_extract_pi(hipStream_t s, const double* E, int npad, int n, int n_z, int q, double* out);
void launch_reduce_w(hipStream_t s, const double* partial_im, const double* partial_re, int ni, int cpad,
                     int cfpad, int n_imp, const int* node, int n_freq, int n_re, int ncols, int nfit, double* w_im,
                     double* w_re);

// k_dense.hip
constexpr int kGemmRows = 256;   // row block of the 16-bit contraction (A operand)
constexpr int kGemmCols = 256;   // column block (B operand rows)
int pi_tile_count(int npad);
int pi_batch_size(int n_planes, int nb, int n_tiles, int n_cu);
std::vector<int2> pi_worklist(int npad, int nfb, int cu_per_xcd);
std::vector<int2> w_tiles(int npad, int cpad);
void launch_pi_f64(hipStream_t s, int npad, int64_t kpad, int n_f, const double* x64, const double* cw64,
                   const int* idflag, double* E);
void launch_pi_gemm(hipStream_t s, int prec, int npad, int64_t kpad, const int* fmap, const uint16_t* xh,
                    const uint16_t* xl, const uint16_t* yh, const uint16_t* yl, const int2* work, int n_work,
                    const double* pi_unscale, const int* idflag, double* E);
int w_partial_blocks(int prec, int npad);
void launch_w(hipStream_t s, int prec, int npad, int f0, int nf, const double* lam64, const uint16_t* lh,
              const uint16_t* ll, const double* bt64, const uint16_t* bh, const uint16_t* bl, int cpad,
              const int2* tiles, int n_tiles, const double* w_unscale, double* partial);

// k_sweep.hip
void launch_sweep(hipStream_t s, double* E, int npad, int n_real, int n_cplx, int cbase, double* dinv_r,
                  double* pbuf_r, double* qbuf_r, double* dinv_c, double* pbuf_c, double* qbuf_c, int* err,
                  bool gauss3 = false);
void launch_sweep2(hipStream_t s, double* E, int npad, int n_real, int n_cplx, int cbase, double* dscr_r,
                   double* dscr_c, double* dinv_r, double* pbuf_r, double* qbuf_r, double* dinv_c, double* pbuf_c,
                   double* qbuf_c, int* err);
// residual check of the inverses: kFactCols sampled columns of every plane of
// eps (before the sweep), then {max|eps^-1 eps_j - e_j|, max |eps^-1||eps_j|}
// per matrix and column into res [n_real + n_cplx][kFactCols][2]
constexpr int kFactCols = 4;
void launch_fact_gather(hipStream_t s, const double* E, int npad, int n_f, const int* cols, double* out);
void launch_fact_residual(hipStream_t s, const double* E, int npad, int n_real, int n_cplx, int cbase,
                          const int* cols, const double* saved, unsigned long long* res);

// k_thiele.hip
void launch_thiele_fit(hipStream_t s, int n_fit, int n_pts, const double* u, const double* w, double tol,
                       double* coef, double* node, int* nterm);
void launch_thiele_eval(hipStream_t s, int n_fit, int n_pts, const double* coef, const double* node,
                        const int* nterm, int n_x, const double* x, double* out);
// w0[f] = Re T_f((i eta)^2), the model's value at the residue point of a_m = 0
void launch_w0_from_fits(hipStream_t s, int n_fit, int n_pts, const double* coef, const double* node, const int* nterm,
                         double eta, double* w0);
// w0[f] = Re w_re[f][j] (near-real point j of every fit)
void launch_w0_from_points(hipStream_t s, int n_fit, const double* w_re, int stride, int j, double* w0);
void launch_gather_refs(hipStream_t s, int n_fit, const int* fit_s, const int* fit_m, int n_mo, int n_freq,
                        const double* w_im, const double* w_re, const double* freq, const int* ref_im_idx,
                        int n_im, const double* ref_re, int n_re, double eta_ref, double* u, double* w);

// k_qp.hip
int qp_max_freq();
void launch_sigma_direct(hipStream_t s, const QpArgs& a, double omega, const double* w_re, int stride, int n_res,
                         const int* rm, const double* rf, double* out);
void launch_qp_batch(hipStream_t s, int n_blocks, const QpArgs* args, const int2* map, QpOut* out);
void launch_qp(hipStream_t s, const QpArgs& a, QpOut* out);
void launch_sigma(hipStream_t s, const QpArgs& a, int n_omega, const double* omega, double* sigma,
                  double* iterm, double* rterm);
void launch_spectral(hipStream_t s, const QpArgs& a, int n_omega, const double* omega, double* spec, double* sre,
                     double* sim);

// k_mlp.hip
constexpr int kMlpParams = 4801;
int mlp_grad_blocks(int n);
void launch_mlp_forward(hipStream_t s, const float* theta, int n, const float* x, float* y);
void launch_mlp_grad(hipStream_t s, const float* theta, int n, const float* x, const float* t, float* partial,
                     float* loss_partial, float* grad, float* loss);
void launch_mlp_adam(hipStream_t s, float* theta, const float* grad, float* m, float* v, int step, float lr,
                     float b1, float b2, float eps);
void launch_mlp_gather(hipStream_t s, const float* x, const float* t, const int* idx, int n, float* xb,
                       float* tb);

}  // namespace cdwac

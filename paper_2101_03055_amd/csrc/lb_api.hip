// lb_api.hip -- host runtime behind the C ABI of include/lb.h.
//
// Owns the handle (parameters, kernel parameter blocks, workspace layout,
// time counter and AA parity), validates inputs, stages host data through
// the caller's workspace and enqueues the kernels of lb_kernels.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lb_internal.h"

using namespace lbk;

namespace {

thread_local std::string g_err;

lb_status fail(lb_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
lb_status fail(lb_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHK(expr)                                                                               \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(LB_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                        __LINE__);                                                                 \
    } while (0)

constexpr uint64_t kMagic = 0x4c42434446303032ull;  // "LBCDF002"

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t elem_bytes(int storage) {
    return storage == LB_STORE_F64 ? 8 : (storage == LB_STORE_F32 ? 4 : 2);
}
size_t arith_bytes(int storage) { return storage == LB_STORE_F64 ? 8 : 4; }

int source_mask(const lb_params& p) {
    if (p.model == LB_MODEL_CHEMOTAXIS) return 2;
    int mask = 0;
    for (int a = 0; a < p.m; ++a)
        for (int b = 0; b < p.m; ++b)
            if (p.K[a * p.m + b] != 0.0) mask |= 1 << a;
    return mask;
}

// gamma of D-bar acts (gamma != 0 for a species that carries a source)
bool gamma_on(const lb_params& p) {
    const int mask = source_mask(p);
    for (int a = 0; a < p.m; ++a)
        if ((mask >> a & 1) && p.gamma_s[a] != 0.0) return true;
    return false;
}

Layout make_layout(const lb_params& p) {
    Layout L{};
    L.N = (size_t)p.nx * (size_t)p.ny;
    L.elem = elem_bytes(p.storage);
    // populations in blocks of 64 nodes (see pidx in lb_device.h)
    L.plane = round_up(L.N, 64);
    const size_t pb = round_up(L.plane * L.elem, 256);
    const bool cde = p.model == LB_MODEL_CDE;
    L.npop = (cde ? 0 : 9) + 5 * (size_t)p.m;
    L.nsrc = (size_t)__builtin_popcount(source_mask(p));
    L.naux = cde ? 2 + (size_t)p.m : 0;
    size_t off = 0;
    L.pop_off = off;
    off += L.npop * pb;
    off = round_up(off, 256);
    L.sold_off = off;
    L.aux_off = off + L.nsrc * L.N * arith_bytes(p.storage);
    off += round_up((L.nsrc + L.naux) * L.N * arith_bytes(p.storage), 256);
    L.snap_off = off;
    off += round_up((size_t)(p.m + 2) * L.N * 8, 256);
    L.stage_off = off;
    off += round_up((size_t)(p.m + 3) * L.N * 8, 256);
    L.part_off = off;
    off += round_up((size_t)kRedBlocks * kRedWidth * 8, 256);
    L.res_off = off;
    off += 256 * 8;
    L.pref_off = off;
    off += round_up((size_t)p.ny * 8, 256);
    L.tstep_off = off;
    off += 256;
    L.pop2_off = L.pop_off;
    L.sold2_off = L.sold_off;
    if (gamma_on(p) && p.fused_steps != 2) {
        L.sold2_off = off;
        off += round_up(L.nsrc * L.N * arith_bytes(p.storage), 256);
    }
    if (p.fused_steps == 2) {
        off = round_up(off, 4096);
        L.pop2_off = off;
        off += L.npop * pb;
        off = round_up(off, 256);
        L.sold2_off = off;
        off += round_up(L.nsrc * L.N * arith_bytes(p.storage), 256);
    }
    L.total = off;
    return L;
}

bool finite_all(const double* v, size_t n) {
    for (size_t k = 0; k < n; ++k)
        if (!std::isfinite(v[k])) return false;
    return true;
}

// eigenvalues of a small real matrix (m <= 4): characteristic polynomial by
// Faddeev-LeVerrier, roots by Durand-Kerner iteration
void eigenvalues(int m, const double* A, std::complex<double>* lam) {
    double c[LB_MAX_M + 1];  // monic: x^m + c[1] x^{m-1} + ... + c[m]
    double Mk[LB_MAX_M * LB_MAX_M], AM[LB_MAX_M * LB_MAX_M];
    c[0] = 1.0;
    std::memset(Mk, 0, sizeof Mk);
    for (int k = 1; k <= m; ++k) {
        // M_k = A M_{k-1} + c_{k-1} I ; c_k = -tr(A M_k)/k
        double Mn[LB_MAX_M * LB_MAX_M];
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                double s = (i == j) ? c[k - 1] : 0.0;
                for (int l = 0; l < m; ++l) s += A[i * m + l] * Mk[l * m + j];
                Mn[i * m + j] = s;
            }
        std::memcpy(Mk, Mn, sizeof Mn);
        double tr = 0.0;
        for (int i = 0; i < m; ++i)
            for (int l = 0; l < m; ++l) tr += A[i * m + l] * Mk[l * m + i];
        (void)AM;
        c[k] = -tr / k;
    }
    std::complex<double> z[LB_MAX_M];
    const std::complex<double> seed(0.4, 0.9);
    double scale = 0.0;
    for (int k = 0; k < m * m; ++k) scale = std::max(scale, std::fabs(A[k]));
    scale = std::max(scale, 1e-300);
    for (int k = 0; k < m; ++k) z[k] = scale * std::pow(seed, k);
    for (int it = 0; it < 500; ++it) {
        for (int k = 0; k < m; ++k) {
            std::complex<double> num = 1.0;
            for (int j = 1; j <= m; ++j) num = num * z[k] + c[j];
            std::complex<double> den = 1.0;
            for (int j = 0; j < m; ++j)
                if (j != k) den *= (z[k] - z[j]);
            if (std::abs(den) > 0) z[k] -= num / den;
        }
    }
    for (int k = 0; k < m; ++k) lam[k] = z[k];
}

// inverse of a small row-major matrix by Gauss-Jordan with partial pivoting
bool invert(int m, const double* A, double* out) {
    double w[LB_MAX_M][2 * LB_MAX_M];
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < 2 * m; ++j) w[i][j] = j < m ? A[i * m + j] : (j - m == i ? 1.0 : 0.0);
    for (int k = 0; k < m; ++k) {
        int pv = k;
        for (int i = k + 1; i < m; ++i)
            if (std::fabs(w[i][k]) > std::fabs(w[pv][k])) pv = i;
        if (w[pv][k] == 0.0) return false;
        for (int j = 0; j < 2 * m; ++j) std::swap(w[k][j], w[pv][j]);
        const double d = w[k][k];
        for (int j = 0; j < 2 * m; ++j) w[k][j] /= d;
        for (int i = 0; i < m; ++i)
            if (i != k) {
                const double s = w[i][k];
                for (int j = 0; j < 2 * m; ++j) w[i][j] -= s * w[k][j];
            }
    }
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) out[i * m + j] = w[i][m + j];
    return true;
}

// lambda of Eq. feq-phi as given (all zeros: the identity); returns whether it differs from I
bool lambda_matrix(const lb_params& p, double* lam) {
    const int m = p.m;
    bool zero = true, ident = true;
    for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) {
            const double v = p.lam[a * m + b];
            zero = zero && v == 0.0;
            ident = ident && v == (a == b ? 1.0 : 0.0);
        }
    for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) lam[a * m + b] = zero ? (a == b ? 1.0 : 0.0) : p.lam[a * m + b];
    return !(zero || ident);
}

// D lambda^-1 (Eq. omega-D: omega^-1 = 3 D lambda^-1 + I/2); false if lambda is singular
bool d_lambda_inv(const lb_params& p, double* out) {
    const int m = p.m;
    double lam[LB_MAX_M * LB_MAX_M], li[LB_MAX_M * LB_MAX_M];
    lambda_matrix(p, lam);
    if (!invert(m, lam, li)) return false;
    for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) {
            double s = 0.0;
            for (int c = 0; c < m; ++c) s += p.D[a * m + c] * li[c * m + b];
            out[a * m + b] = s;
        }
    return true;
}

lb_status validate(const lb_params* p) {
    if (!p) return fail(LB_EINVAL, "params is NULL");
    if (p->nx < 2 || p->ny < 2) return fail(LB_EINVAL, "grid %d x %d: each side must be >= 2", p->nx, p->ny);
    if ((long long)p->nx * p->ny > (1ll << 31) - 1) return fail(LB_EINVAL, "grid too large");
    if (p->m < 1 || p->m > LB_MAX_M) return fail(LB_EINVAL, "m = %d outside 1..%d", p->m, LB_MAX_M);
    // neighbour offsets within a row are formed in 32-bit arithmetic
    if (((long long)p->nx + 64) * (9 + 5 * p->m) > (1ll << 31) - 1)
        return fail(LB_EINVAL, "grid %d wide: (nx + 64) (9 + 5m) must stay below 2^31", p->nx);
    if (p->model != LB_MODEL_LINEAR && p->model != LB_MODEL_CHEMOTAXIS && p->model != LB_MODEL_CDE)
        return fail(LB_EINVAL, "unknown model");
    if (p->model == LB_MODEL_CDE) {
        if (p->storage == LB_STORE_F16) return fail(LB_EINVAL, "no-fluid model: storage must be F64 or F32");
        if (p->collision != LB_COLL_BGK) return fail(LB_EINVAL, "no-fluid model: collision must be BGK (no fluid)");
        if (p->fused_steps == 2) return fail(LB_EINVAL, "no-fluid model: one step per launch only");
        if (p->F0[0] != 0.0 || p->F0[1] != 0.0) return fail(LB_EINVAL, "no-fluid model: no body force");
        for (int a = 0; a < LB_MAX_M; ++a)
            if (p->Fphi[a][0] != 0.0 || p->Fphi[a][1] != 0.0) return fail(LB_EINVAL, "no-fluid model: no body force");
    }
    if (p->model == LB_MODEL_CHEMOTAXIS && p->m != 2) return fail(LB_EINVAL, "chemotaxis model needs m = 2");
    if (p->storage < LB_STORE_F64 || p->storage > LB_STORE_F16) return fail(LB_EINVAL, "unknown storage");
    if (p->collision != LB_COLL_BGK && p->collision != LB_COLL_MRT) return fail(LB_EINVAL, "unknown collision");
    if (p->r_kind != LB_R_STEP && p->r_kind != LB_R_SMOOTH) return fail(LB_EINVAL, "unknown r_kind");
    if (p->fused_steps < 0 || p->fused_steps > 2) return fail(LB_EINVAL, "fused_steps must be 0, 1 or 2");
    if (!(p->tau_f > 0.5) || !std::isfinite(p->tau_f)) return fail(LB_EINVAL, "tau_f = %g must be > 1/2", p->tau_f);
    if (!std::isfinite(p->rho0)) return fail(LB_EINVAL, "rho0 not finite");
    for (int s = 0; s < 4; ++s) {
        if (p->fluid_bc[s] < 0 || p->fluid_bc[s] > 2) return fail(LB_EINVAL, "fluid_bc[%d] invalid", s);
        for (int a = 0; a < p->m; ++a) {
            if (p->scalar_bc[s][a] < 0 || p->scalar_bc[s][a] > 2) return fail(LB_EINVAL, "scalar_bc[%d][%d] invalid", s, a);
            if (!std::isfinite(p->wall[s][a])) return fail(LB_EINVAL, "wall[%d][%d] not finite", s, a);
        }
    }
    for (int axis = 0; axis < 2; ++axis) {
        const int s0 = 2 * axis, s1 = s0 + 1;
        const bool per = p->fluid_bc[s0] == LB_BC_PERIODIC;
        if ((p->fluid_bc[s1] == LB_BC_PERIODIC) != per)
            return fail(LB_EINVAL, "periodic fluid sides must come in pairs (axis %d)", axis);
        for (int a = 0; a < p->m; ++a)
            if ((p->scalar_bc[s0][a] == LB_SBC_PERIODIC) != per || (p->scalar_bc[s1][a] == LB_SBC_PERIODIC) != per)
                return fail(LB_EINVAL, "scalar %d periodicity on axis %d must match the fluid", a, axis);
    }
    if (p->collision == LB_COLL_MRT)
        for (int k = 0; k < 9; ++k)
            if (!(p->mrt_s[k] > 0.0 && p->mrt_s[k] < 2.0) && k != 7 && k != 8)
                return fail(LB_EINVAL, "mrt_s[%d] = %g outside (0, 2)", k, p->mrt_s[k]);
    const int m = p->m;
    for (int k = 0; k < m * m; ++k)
        if (!std::isfinite(p->D[k]) || !std::isfinite(p->K[k]) || !std::isfinite(p->lam[k]))
            return fail(LB_EINVAL, "D, K or lambda not finite");
    if (!std::isfinite(p->varphi)) return fail(LB_EINVAL, "varphi not finite");
    if (p->varphi != 0.0 && p->collision != LB_COLL_BGK)
        return fail(LB_EINVAL, "varphi != 0 needs BGK (its pressure correction uses the single fluid rate)");
    if (p->varphi != 0.0 && p->model == LB_MODEL_CDE) return fail(LB_EINVAL, "no-fluid model: varphi must be 0");
    for (int a = 0; a < p->m; ++a)
        if (!std::isfinite(p->gamma_s[a])) return fail(LB_EINVAL, "gamma_s[%d] not finite", a);
    if (gamma_on(*p) && (p->model == LB_MODEL_CDE || p->fused_steps == 2))
        return fail(LB_EINVAL, "gamma != 0 needs the linear or chemotaxis model and one step per launch");
    double lamm[LB_MAX_M * LB_MAX_M];
    const bool lam_on = lambda_matrix(*p, lamm);
    if (lam_on && p->model == LB_MODEL_CHEMOTAXIS)
        return fail(LB_EINVAL, "chemotaxis model: lambda must be the identity");
    if (lam_on) {
        std::complex<double> ev[LB_MAX_M];
        eigenvalues(m, lamm, ev);
        for (int k = 0; k < m; ++k)
            if (!(ev[k].real() > 0.0 && ev[k].real() < 1.5))
                return fail(LB_EINVAL, "lambda has an eigenvalue with real part %g outside (0, 3/2): "
                            "the rest weight of the equilibrium would not be positive", ev[k].real());
    }
    if (p->model == LB_MODEL_LINEAR || p->model == LB_MODEL_CDE) {
        double dl[LB_MAX_M * LB_MAX_M];
        if (!d_lambda_inv(*p, dl)) return fail(LB_EINVAL, "lambda is singular");
        std::complex<double> lam[LB_MAX_M];
        eigenvalues(m, dl, lam);
        for (int k = 0; k < m; ++k)
            if (!(lam[k].real() > 0.0))
                return fail(LB_EINVAL, "D lambda^-1 has an eigenvalue with real part %g <= 0: eig(omega) leaves (0, 2)",
                            lam[k].real());
    } else {
        if (!(p->D[0] > 0.0 && p->D[3] > 0.0)) return fail(LB_EINVAL, "chemotaxis: D00, D11 must be > 0");
        if (p->D[2] != 0.0) return fail(LB_EINVAL, "chemotaxis: D10 must be 0 (upper-triangular D)");
        if (!(p->chi >= 0.0) || !(p->beta >= 0.0)) return fail(LB_EINVAL, "chemotaxis: chi, beta must be >= 0");
        if (p->r_kind == LB_R_SMOOTH && !(p->eps > 0.0)) return fail(LB_EINVAL, "smooth r(c) needs eps > 0");
    }
    if (p->storage == LB_STORE_F16 && !(p->fp16_scale > 0.0 && std::isfinite(p->fp16_scale) &&
                                        p->fp16_scale_h > 0.0 && std::isfinite(p->fp16_scale_h)))
        return fail(LB_EINVAL, "fp16_scale and fp16_scale_h must be finite and > 0");
    return LB_OK;
}

template <class T>
void fill_kparams(const lb_params& p, const Layout& L, KParams<T>& k) {
    std::memset(&k, 0, sizeof k);
    const bool shifted = p.storage != LB_STORE_F64;
    k.nx = p.nx;
    k.ny = p.ny;
    k.px = p.fluid_bc[0] == LB_BC_PERIODIC;
    k.py = p.fluid_bc[2] == LB_BC_PERIODIC;
    for (int s = 0; s < 4; ++s) {
        k.fbc[s] = p.fluid_bc[s];
        for (int a = 0; a < LB_MAX_M; ++a) {
            k.sbc[s][a] = a < p.m ? p.scalar_bc[s][a] : 0;
            const double ref = shifted && a < p.m ? p.phi_ref[a] : 0.0;
            k.wallr[s][a] = T(a < p.m ? p.wall[s][a] - ref : 0.0);
        }
    }
    k.r_kind = p.r_kind;
    k.src_mask = source_mask(p);
    k.omega_f = T(1.0 / p.tau_f);
    k.rho0_eff = T(shifted ? 0.0 : p.rho0);
    k.h0_shift = T(shifted ? p.rho0 : 0.0);
    const int m = p.m;
    if (p.model == LB_MODEL_LINEAR || p.model == LB_MODEL_CDE) {
        // Eq. omega-D: omega = (3 D lambda^-1 + I/2)^-1 (lambda = I: (3 D + I/2)^-1)
        double A[LB_MAX_M * LB_MAX_M], om[LB_MAX_M * LB_MAX_M], dl[LB_MAX_M * LB_MAX_M];
        double lam[LB_MAX_M * LB_MAX_M];
        k.lam_on = lambda_matrix(p, lam) ? 1 : 0;
        if (k.lam_on) {
            d_lambda_inv(p, dl);
        } else {
            for (int q = 0; q < m * m; ++q) dl[q] = p.D[q];
        }
        for (int a = 0; a < m; ++a)
            for (int b = 0; b < m; ++b) A[a * m + b] = 3.0 * dl[a * m + b] + (a == b ? 0.5 : 0.0);
        invert(m, A, om);
        for (int q = 0; q < m * m; ++q) k.omega[q] = T(om[q]);
        for (int a = 0; a < m; ++a)
            for (int b = 0; b < m; ++b) k.lamm[a * m + b] = T(lam[a * m + b] - (a == b ? 1.0 : 0.0));
    } else {
        for (int q = 0; q < 4; ++q) k.Dc[q] = T(p.D[q]);
    }
    for (int q = 0; q < m * m; ++q) {
        k.K[q] = T(p.K[q]);
        k.Dflux[q] = T(p.D[q]);
    }
    k.F0[0] = T(p.F0[0]);
    k.F0[1] = T(p.F0[1]);
    for (int a = 0; a < m; ++a) {
        k.Fphi[a][0] = T(p.Fphi[a][0]);
        k.Fphi[a][1] = T(p.Fphi[a][1]);
        k.phi_ref[a] = T(shifted ? p.phi_ref[a] : 0.0);
    }
    k.chi = T(p.chi);
    k.beta = T(p.beta);
    k.cstar = T(p.cstar);
    k.eps = T(p.eps);
    for (int q = 0; q < 9; ++q) k.mrt_s[q] = T(p.mrt_s[q]);
    k.scale = T(p.storage == LB_STORE_F16 ? p.fp16_scale : 1.0);
    k.inv_scale = T(p.storage == LB_STORE_F16 ? 1.0 / p.fp16_scale : 1.0);
    k.scale_h = T(p.storage == LB_STORE_F16 ? p.fp16_scale_h : 1.0);
    k.inv_scale_h = T(p.storage == LB_STORE_F16 ? 1.0 / p.fp16_scale_h : 1.0);
    k.varphi = T(p.varphi);
    k.vp_p = T((p.tau_f - 0.5) * (4.0 / 3.0) * p.varphi);
    k.gam_on = gamma_on(p) ? 1 : 0;
    for (int a = 0; a < m; ++a) k.gam12[a] = T(k.gam_on ? p.gamma_s[a] / 12.0 : 0.0);
}

}  // namespace

struct lb_handle {
    lb_params p;
    Layout L;
    KParams<double> kd;
    KParams<float> kf;
    void* ws;
    size_t ws_bytes;
    hipStream_t stream;
    int64_t t;           // steps taken
    int parity;          // 0: canonical layout (own slots); 1: layout left by an even step
    int has_snapshot;
    int device;          // device current at lb_init (the workspace's)
    Launch lc;
    // cached graph of kGraphSteps single-step launches (one step per launch);
    // rebuilt when the tile shape changes
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    Launch glc{0, 0};
    size_t gsold = 0;    // source buffer the graph's first launch reads (gamma != 0 alternates two)
    int href = 0;        // a fluid reference pressure per row is in use (kd.pref / kf.pref set)
    ~lb_handle() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

namespace {
// one row segment of 256 nodes per workgroup on wide grids (measured ~1.5 %
// faster at 4096^2), 64 x 4 otherwise (measured best on 512 x 256)
constexpr int kGraphSteps = 64;  // launches per replayed step graph (even)

// working sets up to this size (population bytes) take the non-temporal
// population accesses: measured faster while the state fits the 256 MB MALL,
// slower on grids far beyond it
constexpr size_t kNtMaxBytes = size_t(64) << 20;

// non-temporal hint bits (Launch::nt): even steps always (own-slot accesses,
// aligned runs), odd steps only for small states (their shifted accesses share
// cache lines between neighbouring wavefronts)
int hint_bits(size_t state_bytes) { return state_bytes <= kNtMaxBytes ? 3 : 1; }

int small_state(const lb_params& p) {
    const size_t q = (p.model == LB_MODEL_CDE ? 0 : 9) + 5 * (size_t)p.m;
    return hint_bits(q * (size_t)p.nx * (size_t)p.ny * elem_bytes(p.storage));
}

Launch default_launch(const lb_params& p) {
    const int nt = small_state(p);
    return p.nx >= 1024 ? Launch{256, 1, nt} : Launch{64, 4, nt};
}

void* at(void* ws, size_t off) { return static_cast<char*>(ws) + off; }

struct StateHeader {
    uint64_t magic;
    int64_t t;
    int64_t parity;
    int64_t has_snapshot;
    uint64_t param_hash;
    uint64_t pop_bytes, sold_bytes, snap_bytes;
    int64_t href;        // the fluid reference pressure (ny values of the arithmetic type) follows the snapshot
};

uint64_t fnv(const void* data, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(data);
    uint64_t h = 1469598103934665603ull;
    for (size_t k = 0; k < n; ++k) {
        h ^= b[k];
        h *= 1099511628211ull;
    }
    return h;
}

size_t sold_bytes(const lb_handle* h) { return (h->L.nsrc + h->L.naux) * h->L.N * arith_bytes(h->p.storage); }
size_t snap_bytes(const lb_handle* h) { return (size_t)(h->p.m + 2) * h->L.N * 8; }
size_t pop_bytes(const lb_handle* h) { return h->L.npop * h->L.plane * h->L.elem; }
size_t pref_bytes(const lb_handle* h) { return (size_t)h->p.ny * arith_bytes(h->p.storage); }

// point the kernels' parameter blocks at the reference array (on) or at none;
// the cached step graph holds the parameter blocks by value and is rebuilt
void set_pref(lb_handle* h, bool on) {
    h->kd.pref = on ? (const double*)at(h->ws, h->L.pref_off) : nullptr;
    h->kf.pref = on ? (const float*)at(h->ws, h->L.pref_off) : nullptr;
    h->href = on ? 1 : 0;
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    h->gexec = nullptr;
    h->graph = nullptr;
}
}  // namespace

extern "C" {

const char* lb_last_error(void) { return g_err.c_str(); }

size_t lb_params_bytes(void) { return sizeof(lb_params); }

lb_status lb_workspace_bytes(const lb_params* params, size_t* bytes) {
    lb_status st = validate(params);
    if (st != LB_OK) return st;
    if (!bytes) return fail(LB_EINVAL, "bytes is NULL");
    *bytes = make_layout(*params).total;
    return LB_OK;
}

// ---- library-held reduction scratch (lb_residual_noalloc) -------------------
// Partial records of the first reduction pass (at most kRedBlocks of kRedWidth
// doubles) and the result record, for callers that cannot allocate.  Each GPU
// holds its own copy; host code reaches it only through the device address
// that hipGetSymbolAddress returns for that GPU (the array's name is a host
// stand-in there).
constexpr size_t kScratchDoubles = (size_t)kRedBlocks * kRedWidth + 64;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;                    // guards the table
double* g_scratch[kMaxDevices] = {};        // device address of `scratch` per device
std::mutex g_scratch_use[kMaxDevices];      // one lb_residual_noalloc at a time per device
}  // namespace

// Looks up the device address of `scratch` on `dev` once (with dev current).
static hipError_t scratch_setup(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[dev]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch[dev] = static_cast<double*>(ptr);
    return hipSuccess;
}

static double* scratch_ptr(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch[dev];
}

lb_status lb_init(const lb_params* params, void* dev_workspace, size_t workspace_bytes, void* hip_stream,
                  const double* phi0, const double* u0, const double* p0, lb_handle** out) {
    if (!out) return fail(LB_EINVAL, "out is NULL");
    *out = nullptr;
    lb_status st = validate(params);
    if (st != LB_OK) return st;
    const Layout L = make_layout(*params);
    if (!dev_workspace) return fail(LB_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(dev_workspace) % 256) return fail(LB_EINVAL, "workspace not 256-byte aligned");
    if (workspace_bytes < L.total)
        return fail(LB_ENOMEM, "workspace has %zu bytes, %zu needed", workspace_bytes, L.total);
    if (!phi0 || !u0) return fail(LB_EINVAL, "phi0 and u0 are required");
    const size_t N = L.N, m = (size_t)params->m;
    if (!finite_all(phi0, m * N) || !finite_all(u0, 2 * N) || (p0 && !finite_all(p0, N)))
        return fail(LB_ENONFINITE, "initial fields contain non-finite values");

    lb_handle* h = new (std::nothrow) lb_handle();
    if (!h) return fail(LB_ENOMEM, "host allocation failed");
    h->p = *params;
    h->L = L;
    fill_kparams(h->p, L, h->kd);
    fill_kparams(h->p, L, h->kf);
    h->ws = dev_workspace;
    h->ws_bytes = workspace_bytes;
    h->stream = static_cast<hipStream_t>(hip_stream);
    h->t = 0;
    h->parity = 0;
    h->has_snapshot = 0;
    h->lc = default_launch(h->p);
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return fail(LB_EDEVICE, "lb_init: hipGetDevice failed");
    }
    if (scratch_setup(h->device) != hipSuccess) {
        delete h;
        return fail(LB_EDEVICE, "lb_init: device address of the reduction scratch array not available");
    }

    double* stage = (double*)at(h->ws, L.stage_off);
    hipError_t e = hipMemcpyAsync(stage, phi0, m * N * 8, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(stage + m * N, u0, 2 * N * 8, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess && p0) e = hipMemcpyAsync(stage + (m + 2) * N, p0, N * 8, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
        e = h->p.model == LB_MODEL_CDE ? launch_cde_init(h->p, L, h->ws, h->kd, h->kf, h->stream)
                                       : launch_init(h->p, L, h->ws, h->kd, h->kf, p0 ? 1 : 0, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        delete h;
        return fail(LB_EDEVICE, "lb_init: %s", hipGetErrorString(e));
    }
    *out = h;
    return LB_OK;
}

lb_status lb_step(lb_handle* h, int64_t n) {
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    if (n < 0) return fail(LB_EINVAL, "n = %lld < 0", (long long)n);
    if (h->p.model == LB_MODEL_CDE) {
        // long runs: replay a prebuilt graph of kGraphSteps launches, as for the fluid model
        if (n >= kGraphSteps + (h->parity ? 1 : 0)) {
            if (h->parity) {
                hipError_t e = launch_cde_step(h->p, h->L, h->ws, h->kd, h->kf, true, h->lc, h->stream);
                if (e != hipSuccess) return fail(LB_EDEVICE, "lb_step launch: %s", hipGetErrorString(e));
                h->t += 1;
                h->parity = 0;
                n -= 1;
            }
            if (!h->gexec || h->glc.tile_x != h->lc.tile_x || h->glc.tile_y != h->lc.tile_y) {
                if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
                if (h->graph) (void)hipGraphDestroy(h->graph);
                h->gexec = nullptr;
                h->graph = nullptr;
                hipError_t e = build_cde_step_graph(h->p, h->L, h->ws, h->kd, h->kf, h->lc, kGraphSteps, &h->graph);
                if (e == hipSuccess) e = hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0);
                if (e != hipSuccess) return fail(LB_EDEVICE, "lb_step graph: %s", hipGetErrorString(e));
                h->glc = h->lc;
            }
            for (; n >= kGraphSteps; n -= kGraphSteps) {
                hipError_t e = hipGraphLaunch(h->gexec, h->stream);
                if (e != hipSuccess) return fail(LB_EDEVICE, "lb_step graph launch: %s", hipGetErrorString(e));
                h->t += kGraphSteps;
            }
        }
        for (int64_t s = 0; s < n; ++s) {
            hipError_t e = launch_cde_step(h->p, h->L, h->ws, h->kd, h->kf, h->parity != 0, h->lc, h->stream);
            if (e != hipSuccess) return fail(LB_EDEVICE, "lb_step launch: %s", hipGetErrorString(e));
            h->t += 1;
            h->parity ^= 1;
        }
        return LB_OK;
    }
    if (h->p.fused_steps == 2) {
        // finish a pending AA odd step, then two steps per launch, a last single even step if n is odd
        if (h->parity && n > 0) {
            hipError_t e = launch_step(h->p, h->L, h->ws, h->kd, h->kf, true, h->lc, h->t, h->stream);
            if (e != hipSuccess) return fail(LB_EDEVICE, "lb_step launch: %s", hipGetErrorString(e));
            h->t += 1;
            h->parity = 0;
            n -= 1;
        }
        for (; n >= 2; n -= 2) {
            hipError_t e = launch_step2(h->p, h->L, h->ws, h->kd, h->kf, h->t, h->stream);
            if (e != hipSuccess) return fail(LB_EDEVICE, "lb_step two-step launch: %s", hipGetErrorString(e));
            std::swap(h->L.pop_off, h->L.pop2_off);
            std::swap(h->L.sold_off, h->L.sold2_off);
            h->t += 2;
        }
    }
    // long runs of single steps: replay a prebuilt graph of kGraphSteps
    // launches (one host call instead of kGraphSteps), which keeps small grids
    // from being limited by the host's launch rate
    if (h->p.fused_steps != 2 && n >= kGraphSteps + (h->parity ? 1 : 0)) {
        if (h->parity) {
            hipError_t e = launch_step(h->p, h->L, h->ws, h->kd, h->kf, true, h->lc, h->t, h->stream);
            if (e != hipSuccess) return fail(LB_EDEVICE, "lb_step launch: %s", hipGetErrorString(e));
            if (h->kd.gam_on) std::swap(h->L.sold_off, h->L.sold2_off);
            h->t += 1;
            h->parity = 0;
            n -= 1;
        }
        if (!h->gexec || h->glc.tile_x != h->lc.tile_x || h->glc.tile_y != h->lc.tile_y ||
            h->gsold != h->L.sold_off) {
            if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
            if (h->graph) (void)hipGraphDestroy(h->graph);
            h->gexec = nullptr;
            h->graph = nullptr;
            hipError_t e = build_step_graph(h->p, h->L, h->ws, h->kd, h->kf, h->lc, kGraphSteps,
                                            (const long long*)at(h->ws, h->L.tstep_off), &h->graph);
            if (e == hipSuccess) e = hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0);
            if (e != hipSuccess) return fail(LB_EDEVICE, "lb_step graph: %s", hipGetErrorString(e));
            h->glc = h->lc;
            h->gsold = h->L.sold_off;
        }
        for (; n >= kGraphSteps; n -= kGraphSteps) {
            hipError_t e = hipSuccess;
            if (h->p.storage == LB_STORE_F16)   // the replay's stochastic-rounding salts follow the step count
                e = launch_set_step((long long*)at(h->ws, h->L.tstep_off), h->t, h->stream);
            if (e == hipSuccess) e = hipGraphLaunch(h->gexec, h->stream);
            if (e != hipSuccess) return fail(LB_EDEVICE, "lb_step graph launch: %s", hipGetErrorString(e));
            h->t += kGraphSteps;
        }
    }
    for (int64_t s = 0; s < n; ++s) {
        const bool odd = h->parity != 0;
        hipError_t e = launch_step(h->p, h->L, h->ws, h->kd, h->kf, odd, h->lc, h->t, h->stream);
        if (e != hipSuccess) return fail(LB_EDEVICE, "lb_step launch: %s", hipGetErrorString(e));
        // gamma != 0: the launch wrote the new source field into the second buffer
        if (h->kd.gam_on) std::swap(h->L.sold_off, h->L.sold2_off);
        h->t += 1;
        h->parity ^= 1;
    }
    return LB_OK;
}

// first and second reduction pass of either model
static hipError_t reduce_any(lb_handle* h, int mode, hipStream_t s) {
    return h->p.model == LB_MODEL_CDE ? launch_cde_reduce(h->p, h->L, h->ws, h->kd, h->kf, h->parity != 0, mode, s)
                                      : launch_reduce(h->p, h->L, h->ws, h->kd, h->kf, h->parity != 0, mode, s);
}

lb_status lb_moments_device(lb_handle* h, double* d_phi, double* d_u, double* d_p) {
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    hipError_t e = h->p.model == LB_MODEL_CDE
                       ? launch_cde_moments(h->p, h->L, h->ws, h->kd, h->kf, h->parity != 0, d_phi, d_u, d_p, h->stream)
                       : launch_moments(h->p, h->L, h->ws, h->kd, h->kf, h->parity != 0, d_phi, d_u, d_p, h->stream);
    if (e != hipSuccess) return fail(LB_EDEVICE, "lb_moments_device: %s", hipGetErrorString(e));
    return LB_OK;
}

lb_status lb_moments(lb_handle* h, double* phi, double* u, double* p) {
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    const size_t N = h->L.N, m = (size_t)h->p.m;
    double* stage = (double*)at(h->ws, h->L.stage_off);
    double* dphi = stage;
    double* du = stage + m * N;
    double* dp = stage + (m + 2) * N;
    lb_status st = lb_moments_device(h, phi ? dphi : nullptr, u ? du : nullptr, p ? dp : nullptr);
    if (st != LB_OK) return st;
    if (phi) HIPCHK(hipMemcpyAsync(phi, dphi, m * N * 8, hipMemcpyDeviceToHost, h->stream));
    if (u) HIPCHK(hipMemcpyAsync(u, du, 2 * N * 8, hipMemcpyDeviceToHost, h->stream));
    if (p) HIPCHK(hipMemcpyAsync(p, dp, N * 8, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return LB_OK;
}

lb_status lb_residual(lb_handle* h, double* res) {
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    if (!res) return fail(LB_EINVAL, "res is NULL");
    const int Q = h->p.m + 2;
    const int mode = h->has_snapshot ? 0 : 1;
    hipError_t e = reduce_any(h, mode, h->stream);
    if (e != hipSuccess) return fail(LB_EDEVICE, "lb_residual: %s", hipGetErrorString(e));
    double out[64];
    HIPCHK(hipMemcpyAsync(out, at(h->ws, h->L.res_off), sizeof(double) * (3 * Q + 1), hipMemcpyDeviceToHost,
                          h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    for (int q = 0; q < Q; ++q) res[q] = mode == 0 ? out[2 * Q + 1 + q] : HUGE_VAL;
    h->has_snapshot = 1;
    if (out[2 * Q] != 0.0) return fail(LB_ENONFINITE, "non-finite values at %.0f nodes", out[2 * Q]);
    return LB_OK;
}

lb_status lb_residual_noalloc(lb_handle* h, double* res) {
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    if (!res) return fail(LB_EINVAL, "res is NULL");
    const int Q = h->p.m + 2;
    const size_t need = (size_t)reduce_blocks(h->L.N) * kRedWidth + (size_t)(3 * Q + 1);
    if (need > kScratchDoubles)
        return fail(LB_EINVAL, "lb_residual_noalloc: %zu doubles of scratch needed, the array holds %zu", need,
                    kScratchDoubles);
    double* sp = scratch_ptr(h->device);
    if (!sp) return fail(LB_EDEVICE, "lb_residual_noalloc: no scratch address for device %d", h->device);
    double* part = sp;
    double* rec = sp + (size_t)kRedBlocks * kRedWidth;
    // the array is shared by every call on this device: hold it until this
    // call's stream has finished reading it
    std::lock_guard<std::mutex> use(g_scratch_use[h->device]);
    const int mode = h->has_snapshot ? 0 : 1;
    hipError_t e = h->p.model == LB_MODEL_CDE
                       ? launch_cde_reduce(h->p, h->L, h->ws, h->kd, h->kf, h->parity != 0, mode, h->stream, part, rec)
                       : launch_reduce(h->p, h->L, h->ws, h->kd, h->kf, h->parity != 0, mode, h->stream, part, rec);
    if (e != hipSuccess) return fail(LB_EDEVICE, "lb_residual_noalloc: %s", hipGetErrorString(e));
    double out[64];
    HIPCHK(hipMemcpyAsync(out, rec, sizeof(double) * (3 * Q + 1), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    for (int q = 0; q < Q; ++q) res[q] = mode == 0 ? out[2 * Q + 1 + q] : HUGE_VAL;
    h->has_snapshot = 1;
    if (out[2 * Q] != 0.0) return fail(LB_ENONFINITE, "non-finite values at %.0f nodes", out[2 * Q]);
    return LB_OK;
}

lb_status lb_solve_steady(lb_handle* h, double tol, int64_t check_every, int64_t max_steps, int64_t* steps_out,
                          double* res_out) {
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    if (!(tol > 0.0) || check_every < 1 || max_steps < 0) return fail(LB_EINVAL, "tol > 0, check_every >= 1 required");
    double res[LB_MAX_M + 2];
    const int Q = h->p.m + 2;
    int64_t done = 0;
    lb_status st = LB_OK;
    if (!h->has_snapshot) {
        st = lb_residual(h, res);
        if (st != LB_OK) goto out;
    }
    st = LB_ESTATE;
    while (done < max_steps) {
        const int64_t k = std::min(check_every, max_steps - done);
        lb_status s2 = lb_step(h, k);
        if (s2 != LB_OK) { st = s2; break; }
        done += k;
        s2 = lb_residual(h, res);
        if (s2 != LB_OK) { st = s2; break; }
        double r = 0.0;
        for (int q = 0; q < Q; ++q) r = std::max(r, res[q]);
        if (k == check_every && r < tol) { st = LB_OK; break; }
    }
    if (st == LB_ESTATE) fail(LB_ESTATE, "not converged after %lld steps", (long long)done);
out:
    if (steps_out) *steps_out = done;
    if (res_out)
        for (int q = 0; q < Q; ++q) res_out[q] = res[q];
    return st;
}

lb_status lb_wall_flux(lb_handle* h, int32_t side, double* flux) {
    if (!h || !flux) return fail(LB_EINVAL, "NULL argument");
    if (side < 0 || side > 3) return fail(LB_EINVAL, "side must be 0..3");
    if (h->p.model == LB_MODEL_CDE) return fail(LB_EINVAL, "lb_wall_flux: not available for the no-fluid model");
    for (int a = 0; a < h->p.m; ++a)
        if (h->p.scalar_bc[side][a] != LB_SBC_DIRICHLET)
            return fail(LB_EINVAL, "side %d is not a Dirichlet wall for species %d", side, a);
    const int depth = side < 2 ? h->p.nx : h->p.ny;
    if (depth < 2) return fail(LB_EINVAL, "need two nodes across the cavity");
    double* dev = (double*)at(h->ws, h->L.res_off);
    hipError_t e = launch_wall_flux(h->p, h->L, h->ws, h->kd, h->kf, h->parity != 0, side, dev, h->stream);
    if (e != hipSuccess) return fail(LB_EDEVICE, "lb_wall_flux: %s", hipGetErrorString(e));
    HIPCHK(hipMemcpyAsync(flux, dev, sizeof(double) * h->p.m, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return LB_OK;
}

lb_status lb_mass(lb_handle* h, double* mass) {
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    if (!mass) return fail(LB_EINVAL, "mass is NULL");
    const int Q = h->p.m + 2;
    hipError_t e = reduce_any(h, 2, h->stream);
    if (e != hipSuccess) return fail(LB_EDEVICE, "lb_mass: %s", hipGetErrorString(e));
    double out[64];
    HIPCHK(hipMemcpyAsync(out, at(h->ws, h->L.res_off), sizeof(double) * (2 * Q + 1), hipMemcpyDeviceToHost,
                          h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    for (int a = 0; a <= h->p.m; ++a) mass[a] = out[a];
    if (out[2 * Q] != 0.0) return fail(LB_ENONFINITE, "non-finite values at %.0f nodes", out[2 * Q]);
    return LB_OK;
}

lb_status lb_populations(lb_handle* h, double* f, double* hpop) {
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    if (h->p.model == LB_MODEL_CDE) {  // scalar planes only; no fluid populations
        const size_t N = h->L.N;
        if (hpop) std::memset(hpop, 0, 9 * N * sizeof(double));
        if (!f) return LB_OK;
        const int chunk = h->p.m + 3, total = 5 * h->p.m;
        double* stage = (double*)at(h->ws, h->L.stage_off);
        for (int b = 0; b < total; b += chunk) {
            const int cnt = std::min(chunk, total - b);
            hipError_t e = launch_cde_export(h->p, h->L, h->ws, h->kd, h->kf, h->parity != 0, b, cnt, stage, h->stream);
            if (e != hipSuccess) return fail(LB_EDEVICE, "lb_populations: %s", hipGetErrorString(e));
            HIPCHK(hipMemcpyAsync(f + (size_t)b * N, stage, (size_t)cnt * N * 8, hipMemcpyDeviceToHost, h->stream));
            HIPCHK(hipStreamSynchronize(h->stream));
        }
        return LB_OK;
    }
    const size_t N = h->L.N, m = (size_t)h->p.m;
    const int chunk = h->p.m + 3;  // planes the staging area holds
    const int total = 9 + 5 * h->p.m;
    double* stage = (double*)at(h->ws, h->L.stage_off);
    for (int b = 0; b < total; b += chunk) {
        const int cnt = std::min(chunk, total - b);
        const bool want_h = hpop && b < 9, want_f = f && b + cnt > 9;
        if (!want_h && !want_f) continue;
        hipError_t e = launch_export(h->p, h->L, h->ws, h->kd, h->kf, h->parity != 0, b, cnt, stage, h->stream);
        if (e != hipSuccess) return fail(LB_EDEVICE, "lb_populations: %s", hipGetErrorString(e));
        for (int k = b; k < b + cnt; ++k) {
            double* dst = k < 9 ? (hpop ? hpop + (size_t)k * N : nullptr) : (f ? f + (size_t)(k - 9) * N : nullptr);
            if (dst) HIPCHK(hipMemcpyAsync(dst, stage + (size_t)(k - b) * N, N * 8, hipMemcpyDeviceToHost, h->stream));
        }
        HIPCHK(hipStreamSynchronize(h->stream));
    }
    (void)m;
    return LB_OK;
}

lb_status lb_fluid_reference(lb_handle* h, int32_t mode) {
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    if (mode != 0 && mode != 1) return fail(LB_EINVAL, "mode must be 0 (none) or 1 (row means of the pressure)");
    if (h->p.model == LB_MODEL_CDE) return fail(LB_EINVAL, "lb_fluid_reference: the no-fluid model has no fluid");
    if (h->p.fused_steps == 2) return fail(LB_EINVAL, "lb_fluid_reference: not with two steps per launch");
    if (mode == 0 && !h->href) return LB_OK;
    const size_t ny = (size_t)h->p.ny;
    double* rows = (double*)at(h->ws, h->L.stage_off);   // row means (FP64), then the new reference
    void* pnew = rows + ny;                               // in the arithmetic type
    hipError_t e = hipSuccess;
    if (mode == 1) {
        e = launch_row_pressure(h->p, h->L, h->ws, h->kd, h->kf, h->parity != 0, rows, h->stream);
        if (e == hipSuccess) {
            if (h->p.storage == LB_STORE_F64)
                e = hipMemcpyAsync(pnew, rows, ny * 8, hipMemcpyDeviceToDevice, h->stream);
            else
                e = launch_to_float(rows, (float*)pnew, (long long)ny, h->stream);
        }
    } else {
        e = hipMemsetAsync(pnew, 0, ny * arith_bytes(h->p.storage), h->stream);
    }
    if (e == hipSuccess) e = launch_reref(h->p, h->L, h->ws, h->kd, h->kf, pnew, h->stream);
    if (e == hipSuccess && mode == 1)
        e = hipMemcpyAsync(at(h->ws, h->L.pref_off), pnew, ny * arith_bytes(h->p.storage), hipMemcpyDeviceToDevice,
                           h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail(LB_EDEVICE, "lb_fluid_reference: %s", hipGetErrorString(e));
    set_pref(h, mode == 1);
    return LB_OK;
}

lb_status lb_time(lb_handle* h, int64_t* t) {
    if (!h || !t) return fail(LB_EINVAL, "NULL argument");
    *t = h->t;
    return LB_OK;
}

lb_status lb_state_bytes(lb_handle* h, size_t* bytes) {
    if (!h || !bytes) return fail(LB_EINVAL, "NULL argument");
    *bytes = sizeof(StateHeader) + pop_bytes(h) + sold_bytes(h) + snap_bytes(h) + pref_bytes(h);
    return LB_OK;
}

lb_status lb_save(lb_handle* h, void* host_buf, size_t bytes) {
    size_t need = 0;
    lb_status st = lb_state_bytes(h, &need);
    if (st != LB_OK) return st;
    if (!host_buf || bytes < need) return fail(LB_EINVAL, "buffer of %zu bytes, %zu needed", bytes, need);
    StateHeader hd{kMagic, h->t, h->parity, h->has_snapshot, fnv(&h->p, sizeof h->p), pop_bytes(h), sold_bytes(h), snap_bytes(h),
                   h->href};
    char* b = static_cast<char*>(host_buf);
    std::memcpy(b, &hd, sizeof hd);
    b += sizeof hd;
    HIPCHK(hipMemcpyAsync(b, at(h->ws, h->L.pop_off), hd.pop_bytes, hipMemcpyDeviceToHost, h->stream));
    b += hd.pop_bytes;
    if (hd.sold_bytes) HIPCHK(hipMemcpyAsync(b, at(h->ws, h->L.sold_off), hd.sold_bytes, hipMemcpyDeviceToHost, h->stream));
    b += hd.sold_bytes;
    HIPCHK(hipMemcpyAsync(b, at(h->ws, h->L.snap_off), hd.snap_bytes, hipMemcpyDeviceToHost, h->stream));
    b += hd.snap_bytes;
    if (h->href) HIPCHK(hipMemcpyAsync(b, at(h->ws, h->L.pref_off), pref_bytes(h), hipMemcpyDeviceToHost, h->stream));
    else std::memset(b, 0, pref_bytes(h));
    HIPCHK(hipStreamSynchronize(h->stream));
    return LB_OK;
}

lb_status lb_load(lb_handle* h, const void* host_buf, size_t bytes) {
    size_t need = 0;
    lb_status st = lb_state_bytes(h, &need);
    if (st != LB_OK) return st;
    if (!host_buf || bytes < need) return fail(LB_EINVAL, "buffer of %zu bytes, %zu needed", bytes, need);
    StateHeader hd;
    const char* b = static_cast<const char*>(host_buf);
    std::memcpy(&hd, b, sizeof hd);
    if (hd.magic != kMagic) return fail(LB_EINVAL, "not a state blob");
    if (hd.param_hash != fnv(&h->p, sizeof h->p) || hd.pop_bytes != pop_bytes(h) || hd.sold_bytes != sold_bytes(h) ||
        hd.snap_bytes != snap_bytes(h))
        return fail(LB_EINVAL, "state blob was saved with different parameters");
    b += sizeof hd;
    HIPCHK(hipMemcpyAsync(at(h->ws, h->L.pop_off), b, hd.pop_bytes, hipMemcpyHostToDevice, h->stream));
    b += hd.pop_bytes;
    if (hd.sold_bytes) HIPCHK(hipMemcpyAsync(at(h->ws, h->L.sold_off), b, hd.sold_bytes, hipMemcpyHostToDevice, h->stream));
    b += hd.sold_bytes;
    HIPCHK(hipMemcpyAsync(at(h->ws, h->L.snap_off), b, hd.snap_bytes, hipMemcpyHostToDevice, h->stream));
    b += hd.snap_bytes;
    if (hd.href) HIPCHK(hipMemcpyAsync(at(h->ws, h->L.pref_off), b, pref_bytes(h), hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if ((hd.href != 0) != (h->href != 0)) set_pref(h, hd.href != 0);
    h->t = hd.t;
    h->parity = (int)hd.parity;
    h->has_snapshot = (int)hd.has_snapshot;
    return LB_OK;
}

lb_status lb_copy_state(lb_handle* dst, lb_handle* src) {
    if (!dst || !src) return fail(LB_EINVAL, "handle is NULL");
    if (dst->p.model == LB_MODEL_CDE || src->p.model == LB_MODEL_CDE)
        return fail(LB_EINVAL, "lb_copy_state: not available for the no-fluid model");
    lb_params a = dst->p, b = src->p;
    a.storage = b.storage = 0;
    for (int k = 0; k < LB_MAX_M; ++k) a.phi_ref[k] = b.phi_ref[k] = 0.0;
    a.fp16_scale = b.fp16_scale = a.fp16_scale_h = b.fp16_scale_h = 0.0;
    a.fused_steps = b.fused_steps = 0;
    if (std::memcmp(&a, &b, sizeof a) != 0)
        return fail(LB_EINVAL, "lb_copy_state: handles differ in more than storage, phi_ref, scales and fused_steps");
    HIPCHK(hipStreamSynchronize(src->stream));
    const int total = 9 + 5 * dst->p.m;
    const int chunk = dst->p.m + 3;
    double* stage = (double*)at(dst->ws, dst->L.stage_off);
    for (int b0 = 0; b0 < total; b0 += chunk) {
        const int cnt = std::min(chunk, total - b0);
        hipError_t e = launch_export(src->p, src->L, src->ws, src->kd, src->kf, src->parity != 0, b0, cnt, stage,
                                     dst->stream);
        if (e == hipSuccess) e = launch_import(dst->p, dst->L, dst->ws, dst->kd, dst->kf, b0, cnt, stage, dst->stream);
        if (e != hipSuccess) return fail(LB_EDEVICE, "lb_copy_state: %s", hipGetErrorString(e));
    }
    hipError_t e = launch_copy_sold(src->p, src->L, src->ws, dst->p, dst->L, dst->ws, dst->stream);
    if (e != hipSuccess) return fail(LB_EDEVICE, "lb_copy_state: %s", hipGetErrorString(e));
    HIPCHK(hipStreamSynchronize(dst->stream));
    dst->t = src->t;
    dst->parity = 0;
    dst->has_snapshot = 0;
    return LB_OK;
}

lb_status lb_set_tile(lb_handle* h, int32_t tile_x, int32_t tile_y) {
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    if (tile_x == 0 && tile_y == 0) {
        h->lc = default_launch(h->p);
        return LB_OK;
    }
    if (tile_x < 64 || tile_x % 64 || tile_y < 1 || tile_x * tile_y > 256)
        return fail(LB_EINVAL, "tile %d x %d: tile_x must be a multiple of 64, tile_x * tile_y <= 256", tile_x, tile_y);
    h->lc = Launch{tile_x, tile_y, h->lc.nt};
    return LB_OK;
}

lb_status lb_free(lb_handle* h) {
    delete h;
    return LB_OK;
}

}  // extern "C"

// ============================================================================
// batched sweep
// ============================================================================
namespace {
constexpr int kTileCand[][2] = {{32, 4}, {32, 8}, {64, 2}, {64, 4}, {128, 1}, {128, 2}, {256, 1}};
constexpr int kStatusRunning = 0, kStatusConverged = 1, kStatusDiverged = 2;
}  // namespace

struct lbb_handle {
    int count;
    lb_params p0;                    // shared template fields (m, model, storage, collision)
    std::vector<lb_params> p;
    std::vector<Layout> L;           // absolute offsets from ws
    std::vector<KParams<double>> kd;
    std::vector<KParams<float>> kf;
    std::vector<CavRec> cav;
    void* ws;
    size_t ws_bytes;
    hipStream_t stream;
    size_t kp_off, cav_off, tiles_off, ranges_off, part_off, out_off, stage_off, tstep_off, max_tiles;
    std::vector<int> status, parity, has_snap;
    std::vector<int64_t> steps;
    int cur_parity;
    int64_t t;
    Launch lc;
    std::vector<int2> tiles;
    std::vector<int2> ctile;         // tile shape of each cavity (all of lc's workgroup size)
    std::vector<int4> ranges;
    std::vector<double> out;
    int64_t tiles_gen = 0;           // bumped whenever the device tile list changes
    hipGraph_t graph = nullptr;      // cached graph of kGraphSteps batched steps (FP32/FP64)
    hipGraphExec_t gexec = nullptr;
    int64_t g_gen = -1;
    Launch g_lc{0, 0};
    ~lbb_handle() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

namespace {
bool same_template(const lb_params& a, const lb_params& b) {
    return a.m == b.m && a.model == b.model && a.storage == b.storage && a.collision == b.collision &&
           a.r_kind == b.r_kind;
}

size_t batch_max_tiles(const lb_params* params, int count) {
    size_t total = 0;   // each cavity may take any of the shapes
    for (int c = 0; c < count; ++c) {
        size_t most = 0;
        for (const auto& tc : kTileCand)
            most = std::max(most, (size_t)((params[c].nx + tc[0] - 1) / tc[0]) * (size_t)((params[c].ny + tc[1] - 1) / tc[1]));
        total += most;
    }
    return total;
}

// workspace plan: shared arrays first, then each cavity's own region
size_t batch_plan(const lb_params* params, int count, lbb_handle* b) {
    size_t N_max = 0;
    for (int c = 0; c < count; ++c) N_max = std::max(N_max, (size_t)params[c].nx * params[c].ny);
    const size_t maxt = batch_max_tiles(params, count);
    const size_t kpb = params[0].storage == LB_STORE_F64 ? sizeof(KParams<double>) : sizeof(KParams<float>);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = round_up(off + bytes, 256);
        return o;
    };
    const size_t kp_off = take(kpb * count), cav_off = take(sizeof(CavRec) * count);
    const size_t tiles_off = take(sizeof(int2) * maxt), ranges_off = take(sizeof(int4) * count);
    const size_t part_off = take(sizeof(double) * kRedWidth * maxt), out_off = take(sizeof(double) * 64 * count);
    const size_t stage_off = take(sizeof(double) * (params[0].m + 3) * N_max);
    const size_t tstep_off = take(sizeof(long long));   // step count read by replayed FP16 step graphs
    if (b) {
        b->kp_off = kp_off; b->cav_off = cav_off; b->tiles_off = tiles_off; b->ranges_off = ranges_off;
        b->part_off = part_off; b->out_off = out_off; b->stage_off = stage_off; b->tstep_off = tstep_off;
        b->max_tiles = maxt;
    }
    for (int c = 0; c < count; ++c) {
        Layout Lc = make_layout(params[c]);
        const size_t base = off;
        const size_t own = Lc.stage_off;  // populations, S_old and snapshot precede the staging area
        if (b) {
            Lc.pop_off += base;
            Lc.sold_off += base;
            Lc.snap_off += base;
            Lc.stage_off = stage_off;
            Lc.part_off = part_off;
            Lc.res_off = out_off;
            b->L.push_back(Lc);
        }
        off = round_up(base + own, 4096);
    }
    return off;
}

void batch_build_tiles(lbb_handle* b) {
    b->tiles.clear();
    b->ranges.clear();
    for (int c = 0; c < b->count; ++c) {
        if (b->status[c] != kStatusRunning) continue;
        const int2 sh = b->ctile[c];
        const int tx = (b->p[c].nx + sh.x - 1) / sh.x;
        const int ty = (b->p[c].ny + sh.y - 1) / sh.y;
        b->cav[c].tiles_x = tx;
        b->cav[c].tiles_y = ty;
        b->cav[c].tile_x = sh.x;
        b->cav[c].tile_y = sh.y;
        b->ranges.push_back(int4{c, (int)b->tiles.size(), tx * ty, 0});
        for (int k = 0; k < tx * ty; ++k) b->tiles.push_back(int2{c, k});
    }
}

lb_status batch_upload(lbb_handle* b) {
    char* w = static_cast<char*>(b->ws);
    b->tiles_gen += 1;
    HIPCHK(hipMemcpyAsync(w + b->cav_off, b->cav.data(), sizeof(CavRec) * b->count, hipMemcpyHostToDevice, b->stream));
    if (!b->tiles.empty())
        HIPCHK(hipMemcpyAsync(w + b->tiles_off, b->tiles.data(), sizeof(int2) * b->tiles.size(), hipMemcpyHostToDevice,
                              b->stream));
    if (!b->ranges.empty())
        HIPCHK(hipMemcpyAsync(w + b->ranges_off, b->ranges.data(), sizeof(int4) * b->ranges.size(),
                              hipMemcpyHostToDevice, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));  // host vectors may change after return
    return LB_OK;
}

const void* batch_kparams(lbb_handle* b) { return static_cast<char*>(b->ws) + b->kp_off; }

lb_status batch_reduce(lbb_handle* b, int mode) {
    char* w = static_cast<char*>(b->ws);
    hipError_t e = launch_breduce(b->p0, b->ws, batch_kparams(b), (const CavRec*)(w + b->cav_off),
                                  (const int2*)(w + b->tiles_off), (int)b->tiles.size(),
                                  (const int4*)(w + b->ranges_off), (int)b->ranges.size(), b->cur_parity != 0, b->lc,
                                  mode, (double*)(w + b->part_off), (double*)(w + b->out_off), b->stream);
    if (e != hipSuccess) return fail(LB_EDEVICE, "batched reduction: %s", hipGetErrorString(e));
    HIPCHK(hipMemcpyAsync(b->out.data(), w + b->out_off, sizeof(double) * 64 * b->count, hipMemcpyDeviceToHost,
                          b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    return LB_OK;
}
}  // namespace

extern "C" {

lb_status lbb_workspace_bytes(const lb_params* params, int32_t count, size_t* bytes) {
    if (!params || count < 1 || !bytes) return fail(LB_EINVAL, "params, count >= 1 and bytes required");
    for (int c = 0; c < count; ++c) {
        lb_status st = validate(&params[c]);
        if (st != LB_OK) return fail(st, "cavity %d: %s", c, g_err.c_str());
        if (!same_template(params[0], params[c]))
            return fail(LB_EINVAL, "cavity %d: m, model, storage, collision and r_kind must match cavity 0", c);
        if (params[c].fused_steps == 2) return fail(LB_EINVAL, "cavity %d: the batched sweep takes one step per launch", c);
        if (params[c].model == LB_MODEL_CDE) return fail(LB_EINVAL, "cavity %d: the no-fluid model is not batched", c);
        if (gamma_on(params[c])) return fail(LB_EINVAL, "cavity %d: gamma != 0 is not batched", c);
    }
    *bytes = batch_plan(params, count, nullptr);
    return LB_OK;
}

lb_status lbb_init(const lb_params* params, int32_t count, void* dev_workspace, size_t workspace_bytes,
                   void* hip_stream, const double* const* phi0, const double* const* u0, const double* const* p0,
                   lbb_handle** out) {
    if (!out) return fail(LB_EINVAL, "out is NULL");
    *out = nullptr;
    size_t need = 0;
    lb_status st = lbb_workspace_bytes(params, count, &need);
    if (st != LB_OK) return st;
    if (!dev_workspace || reinterpret_cast<uintptr_t>(dev_workspace) % 256)
        return fail(LB_EINVAL, "workspace NULL or not 256-byte aligned");
    if (workspace_bytes < need) return fail(LB_ENOMEM, "workspace has %zu bytes, %zu needed", workspace_bytes, need);
    if (!phi0 || !u0) return fail(LB_EINVAL, "phi0 and u0 are required");
    for (int c = 0; c < count; ++c) {
        const size_t N = (size_t)params[c].nx * params[c].ny;
        if (!phi0[c] || !u0[c]) return fail(LB_EINVAL, "cavity %d: phi0 and u0 are required", c);
        if (!finite_all(phi0[c], params[c].m * N) || !finite_all(u0[c], 2 * N) || (p0 && p0[c] && !finite_all(p0[c], N)))
            return fail(LB_ENONFINITE, "cavity %d: initial fields contain non-finite values", c);
    }
    lbb_handle* b = new (std::nothrow) lbb_handle();
    if (!b) return fail(LB_ENOMEM, "host allocation failed");
    b->count = count;
    b->p0 = params[0];
    b->p.assign(params, params + count);
    b->ws = dev_workspace;
    b->ws_bytes = workspace_bytes;
    b->stream = static_cast<hipStream_t>(hip_stream);
    batch_plan(params, count, b);
    b->kd.resize(count);
    b->kf.resize(count);
    b->cav.resize(count);
    b->status.assign(count, kStatusRunning);
    b->parity.assign(count, 0);
    b->has_snap.assign(count, 0);
    b->steps.assign(count, 0);
    b->out.assign((size_t)64 * count, 0.0);
    b->cur_parity = 0;
    b->t = 0;
    size_t state = 0;
    for (int c = 0; c < count; ++c) state += b->L[c].npop * b->L[c].plane * b->L[c].elem;
    b->lc = Launch{64, 4, hint_bits(state)};
    b->ctile.assign(count, int2{64, 4});
    char* w = static_cast<char*>(b->ws);
    for (int c = 0; c < count; ++c) {
        fill_kparams(b->p[c], b->L[c], b->kd[c]);
        fill_kparams(b->p[c], b->L[c], b->kf[c]);
        b->cav[c] = CavRec{(long long)b->L[c].pop_off, (long long)b->L[c].sold_off, (long long)b->L[c].snap_off, 1, 1};
    }
    hipError_t e = b->p0.storage == LB_STORE_F64
                       ? hipMemcpyAsync(w + b->kp_off, b->kd.data(), sizeof(KParams<double>) * count,
                                        hipMemcpyHostToDevice, b->stream)
                       : hipMemcpyAsync(w + b->kp_off, b->kf.data(), sizeof(KParams<float>) * count,
                                        hipMemcpyHostToDevice, b->stream);
    for (int c = 0; c < count && e == hipSuccess; ++c) {
        const size_t N = b->L[c].N, m = (size_t)b->p[c].m;
        double* stage = (double*)(w + b->stage_off);
        e = hipMemcpyAsync(stage, phi0[c], m * N * 8, hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(stage + m * N, u0[c], 2 * N * 8, hipMemcpyHostToDevice, b->stream);
        const bool hp = p0 && p0[c];
        if (e == hipSuccess && hp) e = hipMemcpyAsync(stage + (m + 2) * N, p0[c], N * 8, hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess) e = launch_init(b->p[c], b->L[c], b->ws, b->kd[c], b->kf[c], hp ? 1 : 0, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);  // the staging area is reused
    }
    if (e != hipSuccess) {
        delete b;
        return fail(LB_EDEVICE, "lbb_init: %s", hipGetErrorString(e));
    }
    batch_build_tiles(b);
    st = batch_upload(b);
    if (st != LB_OK) {
        delete b;
        return st;
    }
    *out = b;
    return LB_OK;
}

lb_status lbb_step(lbb_handle* b, int64_t n) {
    if (!b) return fail(LB_EINVAL, "handle is NULL");
    if (n < 0) return fail(LB_EINVAL, "n < 0");
    char* w = static_cast<char*>(b->ws);
    int64_t left = n;
    // long runs: replay a prebuilt graph of kGraphSteps launches (rebuilt when
    // the tile list or the tile shape changes)
    if (!b->tiles.empty() && left >= kGraphSteps + (b->cur_parity ? 1 : 0)) {
        if (b->cur_parity) {
            hipError_t e = launch_bstep(b->p0, b->ws, batch_kparams(b), (const CavRec*)(w + b->cav_off),
                                        (const int2*)(w + b->tiles_off), (int)b->tiles.size(), true, b->lc, b->t,
                                        b->stream);
            if (e != hipSuccess) return fail(LB_EDEVICE, "lbb_step: %s", hipGetErrorString(e));
            b->cur_parity = 0;
            b->t += 1;
            left -= 1;
        }
        if (!b->gexec || b->g_gen != b->tiles_gen || b->g_lc.tile_x != b->lc.tile_x || b->g_lc.tile_y != b->lc.tile_y) {
            if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
            if (b->graph) (void)hipGraphDestroy(b->graph);
            b->gexec = nullptr;
            b->graph = nullptr;
            hipError_t e = build_bstep_graph(b->p0, b->ws, batch_kparams(b), (const CavRec*)(w + b->cav_off),
                                             (const int2*)(w + b->tiles_off), (int)b->tiles.size(), b->lc, kGraphSteps,
                                             (const long long*)(w + b->tstep_off), &b->graph);
            if (e == hipSuccess) e = hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0);
            if (e != hipSuccess) return fail(LB_EDEVICE, "lbb_step graph: %s", hipGetErrorString(e));
            b->g_gen = b->tiles_gen;
            b->g_lc = b->lc;
        }
        for (; left >= kGraphSteps; left -= kGraphSteps) {
            hipError_t e = hipSuccess;
            if (b->p0.storage == LB_STORE_F16)   // the replay's stochastic-rounding salts follow the step count
                e = launch_set_step((long long*)(w + b->tstep_off), b->t, b->stream);
            if (e == hipSuccess) e = hipGraphLaunch(b->gexec, b->stream);
            if (e != hipSuccess) return fail(LB_EDEVICE, "lbb_step graph launch: %s", hipGetErrorString(e));
            b->t += kGraphSteps;
        }
    }
    for (int64_t s = 0; s < left; ++s) {
        hipError_t e = launch_bstep(b->p0, b->ws, batch_kparams(b), (const CavRec*)(w + b->cav_off),
                                    (const int2*)(w + b->tiles_off), (int)b->tiles.size(), b->cur_parity != 0, b->lc,
                                    b->t, b->stream);
        if (e != hipSuccess) return fail(LB_EDEVICE, "lbb_step: %s", hipGetErrorString(e));
        b->cur_parity ^= 1;
        b->t += 1;
    }
    for (int c = 0; c < b->count; ++c)
        if (b->status[c] == kStatusRunning) {
            b->steps[c] += n;
            b->parity[c] = b->cur_parity;
        }
    return LB_OK;
}

lb_status lbb_run(lbb_handle* b, double tol, int64_t check_every, int64_t max_steps, int64_t* steps_out,
                  int32_t* status_out, double* res_out) {
    if (!b) return fail(LB_EINVAL, "handle is NULL");
    if (!(tol > 0.0) || check_every < 1 || max_steps < 0) return fail(LB_EINVAL, "tol > 0, check_every >= 1 required");
    check_every += check_every & 1;  // even windows keep every running cavity at the same AA parity
    const int Q = b->p0.m + 2;
    lb_status st = batch_reduce(b, 1);  // snapshots of every running cavity
    if (st != LB_OK) return st;
    for (int c = 0; c < b->count; ++c)
        if (b->status[c] == kStatusRunning) b->has_snap[c] = 1;
    int64_t done = 0;
    while (!b->tiles.empty() && done < max_steps) {
        const int64_t k = std::min(check_every, max_steps - done);
        st = lbb_step(b, k);
        if (st != LB_OK) return st;
        done += k;
        st = batch_reduce(b, 0);
        if (st != LB_OK) return st;
        bool changed = false;
        for (int c = 0; c < b->count; ++c) {
            if (b->status[c] != kStatusRunning) continue;
            const double* o = &b->out[(size_t)64 * c];
            double r = 0.0;
            for (int q = 0; q < Q; ++q) r = std::max(r, o[2 * Q + 1 + q]);
            if (o[2 * Q] != 0.0) {
                b->status[c] = kStatusDiverged;
                changed = true;
            } else if (k == check_every && r < tol) {
                b->status[c] = kStatusConverged;
                changed = true;
            }
        }
        if (changed) {
            batch_build_tiles(b);
            st = batch_upload(b);
            if (st != LB_OK) return st;
        }
    }
    for (int c = 0; c < b->count; ++c) {
        if (steps_out) steps_out[c] = b->steps[c];
        if (status_out) status_out[c] = b->status[c];
        if (res_out)
            for (int q = 0; q < Q; ++q) res_out[(size_t)c * Q + q] = b->out[(size_t)64 * c + 2 * Q + 1 + q];
    }
    return LB_OK;
}

lb_status lbb_moments(lbb_handle* b, int32_t i, double* phi, double* u, double* p) {
    if (!b || i < 0 || i >= b->count) return fail(LB_EINVAL, "bad handle or cavity index");
    const Layout& L = b->L[i];
    const size_t N = L.N, m = (size_t)b->p[i].m;
    double* stage = (double*)(static_cast<char*>(b->ws) + b->stage_off);
    hipError_t e = launch_moments(b->p[i], L, b->ws, b->kd[i], b->kf[i], b->parity[i] != 0, stage, stage + m * N,
                                  stage + (m + 2) * N, b->stream);
    if (e != hipSuccess) return fail(LB_EDEVICE, "lbb_moments: %s", hipGetErrorString(e));
    if (phi) HIPCHK(hipMemcpyAsync(phi, stage, m * N * 8, hipMemcpyDeviceToHost, b->stream));
    if (u) HIPCHK(hipMemcpyAsync(u, stage + m * N, 2 * N * 8, hipMemcpyDeviceToHost, b->stream));
    if (p) HIPCHK(hipMemcpyAsync(p, stage + (m + 2) * N, N * 8, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    return LB_OK;
}

lb_status lbb_set_tile(lbb_handle* b, int32_t tile_x, int32_t tile_y) {
    if (!b) return fail(LB_EINVAL, "handle is NULL");
    bool ok = false;
    for (const auto& tc : kTileCand) ok |= (tc[0] == tile_x && tc[1] == tile_y);
    if (!ok) return fail(LB_EINVAL, "tile %d x %d is not one of the supported batch tiles", tile_x, tile_y);
    b->lc = Launch{tile_x, tile_y, b->lc.nt};
    b->ctile.assign(b->count, int2{tile_x, tile_y});
    batch_build_tiles(b);
    return batch_upload(b);
}

lb_status lbb_set_cavity_tile(lbb_handle* b, int32_t i, int32_t tile_x, int32_t tile_y) {
    if (!b || i < 0 || i >= b->count) return fail(LB_EINVAL, "bad handle or cavity index");
    bool ok = false;
    for (const auto& tc : kTileCand) ok |= (tc[0] == tile_x && tc[1] == tile_y);
    if (!ok) return fail(LB_EINVAL, "tile %d x %d is not one of the supported batch tiles", tile_x, tile_y);
    if (tile_x * tile_y != b->lc.tile_x * b->lc.tile_y)
        return fail(LB_EINVAL, "tile %d x %d: every cavity's tile has the batch's workgroup size, %d threads", tile_x,
                    tile_y, b->lc.tile_x * b->lc.tile_y);
    b->ctile[i] = int2{tile_x, tile_y};
    batch_build_tiles(b);
    return batch_upload(b);
}

lb_status lbb_cavity_tile(lbb_handle* b, int32_t i, int32_t* tile_x, int32_t* tile_y) {
    if (!b || i < 0 || i >= b->count || !tile_x || !tile_y) return fail(LB_EINVAL, "bad handle, index or pointer");
    *tile_x = b->ctile[i].x;
    *tile_y = b->ctile[i].y;
    return LB_OK;
}

lb_status lbb_autotune(lbb_handle* b, int32_t trial_steps, int32_t* tile_x, int32_t* tile_y, double* us_per_step) {
    if (!b) return fail(LB_EINVAL, "handle is NULL");
    if (trial_steps < 2) trial_steps = 2;
    trial_steps += trial_steps & 1;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    struct EventPair {   // released on every return path
        hipEvent_t* a;
        hipEvent_t* b;
        ~EventPair() {
            if (*a) (void)hipEventDestroy(*a);
            if (*b) (void)hipEventDestroy(*b);
        }
    } events{&e0, &e1};
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    // wall time of trial_steps steps of the batch as it is set up (after two untimed ones)
    auto trial = [&](float* ms) -> lb_status {
        lb_status st = lbb_step(b, 2);
        if (st != LB_OK) return st;
        HIPCHK(hipEventRecord(e0, b->stream));
        st = lbb_step(b, trial_steps);
        if (st != LB_OK) return st;
        HIPCHK(hipEventRecord(e1, b->stream));
        HIPCHK(hipEventSynchronize(e1));
        HIPCHK(hipEventElapsedTime(ms, e0, e1));
        return LB_OK;
    };
    // 1. one shape for every cavity
    float best = 1e30f;
    Launch best_lc = b->lc;
    for (const auto& tc : kTileCand) {
        lb_status st = lbb_set_tile(b, tc[0], tc[1]);
        float ms = 0.f;
        if (st == LB_OK) st = trial(&ms);
        if (st != LB_OK) return st;
        if (ms < best) {
            best = ms;
            best_lc = b->lc;
        }
    }
    lb_status st = lbb_set_tile(b, best_lc.tile_x, best_lc.tile_y);
    if (st != LB_OK) return st;
    // 2. per cavity width, the other shapes of the same workgroup size, one width at a time
    //    against a fresh timing of the current setting; a change is kept when it saves more
    //    than 1 % of the batch's step time (below that the timings do not tell them apart)
    std::vector<int> widths;
    for (int c = 0; c < b->count; ++c)
        if (b->status[c] == kStatusRunning && std::find(widths.begin(), widths.end(), b->p[c].nx) == widths.end())
            widths.push_back(b->p[c].nx);
    std::sort(widths.begin(), widths.end());
    const int threads = best_lc.tile_x * best_lc.tile_y;
    for (int w : widths) {
        if (widths.size() < 2) break;
        float cur = 0.f;
        if ((st = trial(&cur)) != LB_OK) return st;
        int2 keep = int2{best_lc.tile_x, best_lc.tile_y};
        for (int c = 0; c < b->count; ++c)
            if (b->p[c].nx == w) keep = b->ctile[c];
        for (const auto& tc : kTileCand) {
            if (tc[0] * tc[1] != threads || (tc[0] == keep.x && tc[1] == keep.y)) continue;
            for (int c = 0; c < b->count; ++c)
                if (b->p[c].nx == w) b->ctile[c] = int2{tc[0], tc[1]};
            batch_build_tiles(b);
            if ((st = batch_upload(b)) != LB_OK) return st;
            float ms = 0.f;
            if ((st = trial(&ms)) != LB_OK) return st;
            if (ms < 0.99f * cur) {
                cur = ms;
                keep = int2{tc[0], tc[1]};
            }
        }
        for (int c = 0; c < b->count; ++c)
            if (b->p[c].nx == w) b->ctile[c] = keep;
        batch_build_tiles(b);
        if ((st = batch_upload(b)) != LB_OK) return st;
        best = std::min(best, cur);
    }
    if (tile_x) *tile_x = best_lc.tile_x;
    if (tile_y) *tile_y = best_lc.tile_y;
    if (us_per_step) *us_per_step = 1e3 * best / trial_steps;
    return LB_OK;
}

lb_status lbb_copy_cavity(lbb_handle* dst, int32_t i, lbb_handle* src, int32_t j) {
    if (!dst || !src || i < 0 || i >= dst->count || j < 0 || j >= src->count)
        return fail(LB_EINVAL, "bad handle or cavity index");
    if (dst->cur_parity != 0) return fail(LB_ESTATE, "destination batch is between an even and an odd step");
    lb_params a = dst->p[i], c = src->p[j];
    a.storage = c.storage = 0;
    for (int k = 0; k < LB_MAX_M; ++k) a.phi_ref[k] = c.phi_ref[k] = 0.0;
    a.fp16_scale = c.fp16_scale = a.fp16_scale_h = c.fp16_scale_h = 0.0;
    if (std::memcmp(&a, &c, sizeof a) != 0)
        return fail(LB_EINVAL, "cavities differ in more than storage, phi_ref and scales");
    HIPCHK(hipStreamSynchronize(src->stream));
    const int total = 9 + 5 * dst->p[i].m, chunk = dst->p[i].m + 3;
    double* stage = (double*)(static_cast<char*>(dst->ws) + dst->stage_off);
    for (int b0 = 0; b0 < total; b0 += chunk) {
        const int cnt = std::min(chunk, total - b0);
        hipError_t e = launch_export(src->p[j], src->L[j], src->ws, src->kd[j], src->kf[j], src->parity[j] != 0, b0,
                                     cnt, stage, dst->stream);
        if (e == hipSuccess)
            e = launch_import(dst->p[i], dst->L[i], dst->ws, dst->kd[i], dst->kf[i], b0, cnt, stage, dst->stream);
        if (e != hipSuccess) return fail(LB_EDEVICE, "lbb_copy_cavity: %s", hipGetErrorString(e));
    }
    hipError_t e = launch_copy_sold(src->p[j], src->L[j], src->ws, dst->p[i], dst->L[i], dst->ws, dst->stream);
    if (e != hipSuccess) return fail(LB_EDEVICE, "lbb_copy_cavity: %s", hipGetErrorString(e));
    HIPCHK(hipStreamSynchronize(dst->stream));
    dst->steps[i] = src->steps[j];
    dst->parity[i] = 0;
    dst->has_snap[i] = 0;
    if (dst->status[i] != kStatusRunning) {
        dst->status[i] = kStatusRunning;
        batch_build_tiles(dst);
        return batch_upload(dst);
    }
    return LB_OK;
}

lb_status lbb_time(lbb_handle* b, int32_t i, int64_t* steps, int32_t* status) {
    if (!b || i < 0 || i >= b->count) return fail(LB_EINVAL, "bad handle or cavity index");
    if (steps) *steps = b->steps[i];
    if (status) *status = b->status[i];
    return LB_OK;
}

lb_status lbb_free(lbb_handle* b) {
    delete b;
    return LB_OK;
}

}  // extern "C"
